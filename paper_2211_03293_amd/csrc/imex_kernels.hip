// imex_kernels.hip -- kernels of the IMEX-MRI-GARK slow step (Sec. 2.1 with
// f^S = f^I + f^E): the combination of slow evaluations into forcing planes or
// the right-hand side of a solve-decoupled stage, and a conjugate-gradient
// solve of (I - a D lap) Y = b on the periodic grid, one independent CG per
// component (the implicit diffusion of Sec. 3.2 / Sec. 6).
//
// All reductions run in a fixed order (per-block partial sums, then one block
// per component over the partials in index order): a solve is bitwise
// reproducible.

#include <hip/hip_runtime.h>

#include "imex_dev.h"

namespace {

// out[k][comp][cell] = (base ? base[comp][cell] : 0)
//                      + sum_j (coef.e[k][j] FE[j][comp][cell] + coef.i[k][j] FI[j][comp][cell])
// for cells < n_cells, components < n; planes are [n][ld] with stride `plane`.
__global__ void __launch_bounds__(256)
    k_imex_combine(int n_cells, int ld, long long plane, int n_out, int nj,
                   const double *__restrict__ FE, const double *__restrict__ FI, ImexCoef coef,
                   const double *__restrict__ base, double *__restrict__ out)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells) return;
    const long long e = (long long)blockIdx.y * ld + cell;
    double fe[IMEX_JMAX], fi[IMEX_JMAX];
#pragma unroll
    for (int j = 0; j < IMEX_JMAX; ++j)
        if (j < nj) {
            fe[j] = FE[j * plane + e];
            fi[j] = FI[j * plane + e];
        }
    const double b0 = base ? base[e] : 0.0;
#pragma unroll
    for (int k = 0; k < IMEX_KMAX; ++k) {
        if (k < n_out) {
            double acc = b0;
#pragma unroll
            for (int j = 0; j < IMEX_JMAX; ++j)
                if (j < nj) {
                    acc = fma(coef.i[k][j], fi[j], acc);
                    acc = fma(coef.e[k][j], fe[j], acc);
                }
            out[k * plane + e] = acc;
        }
    }
}

// Sum over the block (fixed order: lanes by shuffles within each wave, then
// the waves' sums in index order); the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += lds[i];
    return s;
}

// q = p - a D lap(p) on the periodic grid (7-point stencil, the tiling of the
// advection-diffusion kernel: a block owns CG_TX x CG_TY cells of one
// component and marches over CG_TZ planes of z) and the block's partial sum of
// p . q into part[comp * nb + block].  Components whose CG has converged are
// skipped (block-uniform: a block holds one component).
constexpr int CG_TX = 64, CG_TY = 8, CG_TZ = 4, CG_NT = CG_TX * CG_TY;

__global__ void __launch_bounds__(CG_NT)
    k_cg_apply(int nx, int ny, int nz, int ld, double aD, double dx,
               const double *__restrict__ p_all, double *__restrict__ q_all,
               const int *__restrict__ done, double *__restrict__ part)
{
    __shared__ double tile[CG_TY + 2][CG_TX + 2];
    __shared__ double red[CG_NT / 64];
    const int nzc = (nz + CG_TZ - 1) / CG_TZ;
    const int comp = blockIdx.z / nzc, z0 = (blockIdx.z % nzc) * CG_TZ;
    const int nb = gridDim.x * gridDim.y * nzc;
    const int blk = (blockIdx.z % nzc) * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x;
    if (done[comp]) return;
    const int tx = threadIdx.x % CG_TX, ty = threadIdx.x / CG_TX;
    const int x0 = blockIdx.x * CG_TX, y0 = blockIdx.y * CG_TY;
    const int z1 = min(nz, z0 + CG_TZ);
    const int x = x0 + tx, yy = y0 + ty;
    const bool in = x < nx && yy < ny;
    const double *p = p_all + (size_t)comp * ld;
    double *q = q_all + (size_t)comp * ld;
    const long long row = nx, plane = (long long)nx * ny;
    const double c = aD / (dx * dx);
    const int xm = x0 == 0 ? nx - 1 : x0 - 1;
    const int ym = y0 == 0 ? ny - 1 : y0 - 1;
    auto at = [&](int z, int yy_, int x_) { return p[(long long)z * plane + (long long)yy_ * row + x_]; };
    double pzm = 0.0, c0 = 0.0, pzp = 0.0, dot = 0.0;
    if (in) {
        pzm = at(z0 == 0 ? nz - 1 : z0 - 1, yy, x);
        c0 = at(z0, yy, x);
    }
    for (int z = z0; z < z1; ++z) {
        const int zp = z == nz - 1 ? 0 : z + 1;
        if (in) {
            pzp = at(zp, yy, x);
            tile[ty + 1][tx + 1] = c0;
        }
        if (tx < 2 && y0 + ty < ny) {
            const int lastx = min(CG_TX, nx - x0);
            const int hx = tx == 0 ? xm : (x0 + lastx == nx ? 0 : x0 + lastx);
            tile[ty + 1][tx == 0 ? 0 : lastx + 1] = at(z, y0 + ty, hx);
        }
        if (ty < 2 && x < nx) {
            const int lasty = min(CG_TY, ny - y0);
            const int hy = ty == 0 ? ym : (y0 + lasty == ny ? 0 : y0 + lasty);
            tile[ty == 0 ? 0 : lasty + 1][tx + 1] = at(z, hy, x);
        }
        __syncthreads();
        if (in) {
            const double pxm = tile[ty + 1][tx], pxp = tile[ty + 1][tx + 2];
            const double pym = tile[ty][tx + 1], pyp = tile[ty + 2][tx + 1];
            const double lap = pxp + pxm + pyp + pym + pzp + pzm - 6.0 * c0;
            const double qv = fma(-c, lap, c0);
            q[(long long)z * plane + (long long)yy * row + x] = qv;
            dot = fma(c0, qv, dot);
        }
        __syncthreads();
        pzm = c0;
        c0 = pzp;
    }
    const double s = block_sum<CG_NT>(dot, red);
    if (threadIdx.x == 0) part[(size_t)comp * nb + blk] = s;
}

// r = b - q, p = r; partial sums of r . r and b . b.
constexpr int CG_VT = 256;
__global__ void __launch_bounds__(CG_VT)
    k_cg_init(int n_cells, int ld, const double *__restrict__ b, const double *__restrict__ q,
              double *__restrict__ r, double *__restrict__ p, double *__restrict__ part_rr,
              double *__restrict__ part_bb)
{
    __shared__ double red[CG_VT / 64];
    const int comp = blockIdx.y, nb = gridDim.x;
    const int cell = blockIdx.x * CG_VT + threadIdx.x;
    double rr = 0.0, bb = 0.0;
    if (cell < n_cells) {
        const size_t e = (size_t)comp * ld + cell;
        const double bv = b[e], rv = bv - q[e];
        r[e] = rv;
        p[e] = rv;
        rr = rv * rv;
        bb = bv * bv;
    }
    double s = block_sum<CG_VT>(rr, red);
    if (threadIdx.x == 0) part_rr[(size_t)comp * nb + blockIdx.x] = s;
    __syncthreads();
    s = block_sum<CG_VT>(bb, red);
    if (threadIdx.x == 0) part_bb[(size_t)comp * nb + blockIdx.x] = s;
}

// x += alpha p, r -= alpha q; partial sums of the new r . r.
__global__ void __launch_bounds__(CG_VT)
    k_cg_update(int n_cells, int ld, const CgScalars *__restrict__ sc, const int *__restrict__ done,
                double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
                const double *__restrict__ q, double *__restrict__ part)
{
    __shared__ double red[CG_VT / 64];
    const int comp = blockIdx.y, nb = gridDim.x;
    if (done[comp]) return;
    const double alpha = sc[comp].alpha;
    const int cell = blockIdx.x * CG_VT + threadIdx.x;
    double rr = 0.0;
    if (cell < n_cells) {
        const size_t e = (size_t)comp * ld + cell;
        x[e] = fma(alpha, p[e], x[e]);
        const double rv = fma(-alpha, q[e], r[e]);
        r[e] = rv;
        rr = rv * rv;
    }
    const double s = block_sum<CG_VT>(rr, red);
    if (threadIdx.x == 0) part[(size_t)comp * nb + blockIdx.x] = s;
}

// p = r + beta p.
__global__ void __launch_bounds__(CG_VT)
    k_cg_dir(int n_cells, int ld, const CgScalars *__restrict__ sc, const int *__restrict__ done,
             const double *__restrict__ r, double *__restrict__ p)
{
    const int comp = blockIdx.y;
    if (done[comp]) return;
    const int cell = blockIdx.x * CG_VT + threadIdx.x;
    if (cell >= n_cells) return;
    const size_t e = (size_t)comp * ld + cell;
    p[e] = fma(sc[comp].beta, p[e], r[e]);
}

// One block per component: the partial sums in index order, then the CG
// scalars of that component (mode 0: start, 1: step length, 2: direction
// update and convergence test ||r|| <= tol ||b||).
__global__ void __launch_bounds__(256)
    k_cg_reduce(int mode, int nb, const double *__restrict__ part,
                const double *__restrict__ part2, double tol2, CgScalars *__restrict__ sc,
                int *__restrict__ done)
{
    __shared__ double red[4];
    const int comp = blockIdx.x;
    if (mode != 0 && done[comp]) return;
    double v = 0.0, v2 = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        v += part[(size_t)comp * nb + i];
        if (mode == 0) v2 += part2[(size_t)comp * nb + i];
    }
    const double s = block_sum<256>(v, red);
    __syncthreads();
    const double s2 = mode == 0 ? block_sum<256>(v2, red) : 0.0;
    if (threadIdx.x != 0) return;
    CgScalars &c = sc[comp];
    if (mode == 0) {
        c.rr = s;
        c.bb = s2;
        done[comp] = !(s > tol2 * s2);
    } else if (mode == 1) {
        if (s > 0.0) {
            c.alpha = c.rr / s;
        } else {
            c.alpha = 0.0;        // p . Ap = 0 only when p = 0: nothing left to do
            done[comp] = 1;
        }
    } else {
        c.beta = s / c.rr;
        c.rr = s;
        done[comp] = !(s > tol2 * c.bb);
    }
}

__global__ void k_copy_planes(int n_cells, int ld, const double *__restrict__ src,
                              double *__restrict__ dst)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells) return;
    const size_t e = (size_t)blockIdx.y * ld + cell;
    dst[e] = src[e];
}

__global__ void k_fill_i32(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_imex_combine(int n, int n_cells, int ld, int n_out, int nj, const double *FE,
                               const double *FI, const ImexCoef &coef, const double *base,
                               double *out, hipStream_t s)
{
    if (n_cells == 0 || n == 0) return hipSuccess;
    const long long plane = (long long)n * ld;
    hipLaunchKernelGGL(k_imex_combine, dim3((unsigned)((n_cells + 255) / 256), (unsigned)n),
                       dim3(256), 0, s, n_cells, ld, plane, n_out, nj, FE, FI, coef, base, out);
    return hipGetLastError();
}

int cg_apply_blocks(int nx, int ny, int nz)
{
    return ((nx + CG_TX - 1) / CG_TX) * ((ny + CG_TY - 1) / CG_TY) * ((nz + CG_TZ - 1) / CG_TZ);
}

int cg_vec_blocks(int n_cells) { return (n_cells + CG_VT - 1) / CG_VT; }

hipError_t launch_cg_apply(int nx, int ny, int nz, int n_comp, int ld, double aD, double dx,
                           const double *p, double *q, const int *done, double *part,
                           hipStream_t s)
{
    const long long gz = (long long)n_comp * ((nz + CG_TZ - 1) / CG_TZ);
    const long long gy = (ny + CG_TY - 1) / CG_TY;
    if (gz > 65535 || gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg_apply, dim3((unsigned)((nx + CG_TX - 1) / CG_TX), (unsigned)gy,
                                        (unsigned)gz),
                       dim3(CG_NT), 0, s, nx, ny, nz, ld, aD, dx, p, q, done, part);
    return hipGetLastError();
}

hipError_t launch_cg_init(int n_comp, int n_cells, int ld, const double *b, const double *q,
                          double *r, double *p, double *part_rr, double *part_bb, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)cg_vec_blocks(n_cells), (unsigned)n_comp),
                       dim3(CG_VT), 0, s, n_cells, ld, b, q, r, p, part_rr, part_bb);
    return hipGetLastError();
}

hipError_t launch_cg_update(int n_comp, int n_cells, int ld, const CgScalars *sc, const int *done,
                            double *x, double *r, const double *p, const double *q, double *part,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update, dim3((unsigned)cg_vec_blocks(n_cells), (unsigned)n_comp),
                       dim3(CG_VT), 0, s, n_cells, ld, sc, done, x, r, p, q, part);
    return hipGetLastError();
}

hipError_t launch_cg_dir(int n_comp, int n_cells, int ld, const CgScalars *sc, const int *done,
                         const double *r, double *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_dir, dim3((unsigned)cg_vec_blocks(n_cells), (unsigned)n_comp),
                       dim3(CG_VT), 0, s, n_cells, ld, sc, done, r, p);
    return hipGetLastError();
}

hipError_t launch_cg_reduce(int mode, int n_comp, int nb, const double *part, const double *part2,
                            double tol2, CgScalars *sc, int *done, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_reduce, dim3((unsigned)n_comp), dim3(256), 0, s, mode, nb, part, part2,
                       tol2, sc, done);
    return hipGetLastError();
}

hipError_t launch_copy_planes(int n_comp, int n_cells, int ld, const double *src, double *dst,
                              hipStream_t s)
{
    if (n_cells == 0 || n_comp == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_planes, dim3((unsigned)((n_cells + 255) / 256), (unsigned)n_comp),
                       dim3(256), 0, s, n_cells, ld, src, dst);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int n, int v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
