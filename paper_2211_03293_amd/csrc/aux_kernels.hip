// aux_kernels.hip -- memory-bound helpers of the MRI slow step: forcing
// assembly, the advection-diffusion slow RHS, a linear slow RHS for tests,
// status reduction and small fills.
#include "mri_dev.h"
#include "mri_math.h"

namespace {

// Forcing coefficients of one slow stage (Sec. 2.1 step 2a):
// rho_k = sum_{j < i} (Gamma^(k)_ij / dc_i) F_j, the 1/dc_i folded into coef.
__global__ void __launch_bounds__(256)
    k_forcing(long long n_elem, int n_gamma, int nj, const double *__restrict__ F,
              long long F_stride, ForcingCoef coef, double *__restrict__ rho)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    double f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < nj) f[j] = F[j * F_stride + e];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < n_gamma) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < nj) acc = fma(coef.c[k * 8 + j], f[j], acc);
            rho[k * n_elem + e] = acc;
        }
    }
}

// f = -u . grad(phi) + D lap(phi), 2nd-order centred, periodic; one thread per
// (component, cell).  Neighbour reads hit L2 / L1: x neighbours are
// contiguous, y and z neighbours are one row / plane away.
// 2.5D blocking: a block owns a tile of ADV_TX x ADV_TY cells of one component
// and marches through ADV_TZ planes of z, each thread keeping the z-1, z and
// z+1 values of its column in registers; the x- and y-neighbours of the
// current plane come from an LDS tile with a one-cell halo (periodic wrap), so
// every value is read from memory about once.  The arithmetic is that of the
// plain 7-point formula, term for term.
// Tile shape measured on MI355X (64^3 x 22 / 128^3 x 54 fields): 8 rows x 4
// planes 22.1 / 472 us; 4 x 16: 25.9 / 505; 8 x 16: 24.9 / 492; 8 x 32: 40.6
// / 527 -- short z marches keep more blocks in flight.
#ifndef MRI_ADV_TY
#define MRI_ADV_TY 8
#endif
#ifndef MRI_ADV_TZ
#define MRI_ADV_TZ 4
#endif
constexpr int ADV_TX = 64, ADV_TY = MRI_ADV_TY, ADV_TZ = MRI_ADV_TZ;

__global__ void __launch_bounds__(ADV_TX *ADV_TY)
    k_advdiff(int nx, int ny, int nz, int n_comp, int ld, double ux, double uy, double uz,
              double D, double dx, const double *__restrict__ y, double *__restrict__ fy)
{
    __shared__ double tile[ADV_TY + 2][ADV_TX + 2];
    const int tx = threadIdx.x % ADV_TX, ty = threadIdx.x / ADV_TX;
    const int x0 = blockIdx.x * ADV_TX, y0 = blockIdx.y * ADV_TY;
    const int nzc = (nz + ADV_TZ - 1) / ADV_TZ;
    const int comp = blockIdx.z / nzc, z0 = (blockIdx.z % nzc) * ADV_TZ;
    const int z1 = min(nz, z0 + ADV_TZ);
    const int x = x0 + tx, yy = y0 + ty;
    const bool in = x < nx && yy < ny;
    const double *p = y + (size_t)comp * ld;
    const long long row = nx, plane = (long long)nx * ny;
    const double inv2dx = 1.0 / (2.0 * dx), invdx2 = 1.0 / (dx * dx);
    // halo cells of the tile: x halo (2 per tile row), y halo (2 per tile column)
    const int xm = x0 == 0 ? nx - 1 : x0 - 1;
    const int ym = y0 == 0 ? ny - 1 : y0 - 1;
    auto at = [&](int z, int yy_, int x_) { return p[(long long)z * plane + (long long)yy_ * row + x_]; };
    double pzm = 0.0, c0 = 0.0, pzp = 0.0;
    if (in) {
        pzm = at(z0 == 0 ? nz - 1 : z0 - 1, yy, x);
        c0 = at(z0, yy, x);
    }
    for (int z = z0; z < z1; ++z) {
        const int zp = z == nz - 1 ? 0 : z + 1;
        if (in) {
            pzp = at(zp, yy, x);
            tile[ty + 1][tx + 1] = c0;   // cells outside the grid would overwrite a halo
        }
        // x halo: the wrapped neighbours of the tile's first and last column
        if (tx < 2 && y0 + ty < ny) {
            const int lastx = min(ADV_TX, nx - x0);     // columns present in this tile
            const int hx = tx == 0 ? xm : (x0 + lastx == nx ? 0 : x0 + lastx);
            tile[ty + 1][tx == 0 ? 0 : lastx + 1] = at(z, y0 + ty, hx);
        }
        // y halo: the wrapped neighbours of the tile's first and last row
        if (ty < 2 && x < nx) {
            const int lasty = min(ADV_TY, ny - y0);
            const int hy = ty == 0 ? ym : (y0 + lasty == ny ? 0 : y0 + lasty);
            tile[ty == 0 ? 0 : lasty + 1][tx + 1] = at(z, hy, x);
        }
        __syncthreads();
        if (in) {
            const double pxm = tile[ty + 1][tx], pxp = tile[ty + 1][tx + 2];
            const double pym = tile[ty][tx + 1], pyp = tile[ty + 2][tx + 1];
            const double adv = (ux * (pxp - pxm) + uy * (pyp - pym) + uz * (pzp - pzm)) * inv2dx;
            const double lap = (pxp + pxm + pyp + pym + pzp + pzm - 6.0 * c0) * invdx2;
            fy[(size_t)comp * ld + (long long)z * plane + (long long)yy * row + x] =
                fma(D, lap, -adv);
        }
        __syncthreads();
        pzm = c0;
        c0 = pzp;
    }
}

__global__ void __launch_bounds__(256)
    k_lin_apply(int n, const double *__restrict__ A, int n_cells, int ld,
                const double *__restrict__ y, double *__restrict__ fy)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells) return;
    double v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (c < n) v[c] = y[(size_t)c * ld + cell];
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (r < n) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < n) s = fma(A[r * n + c], v[c], s);
            fy[(size_t)r * ld + cell] = s;
        }
}

__global__ void __launch_bounds__(256)
    k_status_count(const int32_t *__restrict__ st, int n, int32_t mask,
                   unsigned long long *count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = (i < n) && ((st[i] & mask) != 0);
    const unsigned long long m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

__global__ void __launch_bounds__(256) k_exp2(const double *__restrict__ x, double *__restrict__ y,
                                             int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = mri_exp2(x[i]);
}

__constant__ double exp2_tab_src[256] = MRI_EXP2_T256;

// 2^x by the table-driven exponential of the specialized kernels (u = 256 x is
// exact), with the table staged in LDS as those kernels do
__global__ void __launch_bounds__(256) k_exp2_t256(const double *__restrict__ x,
                                                  double *__restrict__ y, int n)
{
    __shared__ double tab[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) tab[i] = exp2_tab_src[i];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = mri_exp2_t256(256.0 * x[i], tab);
}

__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Step-doubling error of an adaptive slow step, reduced per block: for every
// cell and component w = scale (y_half - y_full) / (atol_c + rtol |y_half|),
// atol_c = atol_T for the last component (temperature) of chemistry states;
// part_w2[block] = sum of w^2 over the block's cells, part_steps[block] = sum
// of the fast substeps of the two half steps.  The block reduction runs in a
// fixed tree order; the host sums the partials in block order.
__global__ void __launch_bounds__(256)
    k_step_err(int n, int t_comp, int n_cells, int ld, const double *__restrict__ y_half,
               const double *__restrict__ y_full, double scale, double rtol, double atol,
               double atol_t, const int32_t *__restrict__ sp_a, const int32_t *__restrict__ sp_b,
               double *part_w2, long long *part_steps)
{
    __shared__ double w2s[256];
    __shared__ long long sts[256];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    long long nst = 0;
    if (cell < n_cells) {
        for (int c = 0; c < n; ++c) {
            const size_t o = (size_t)c * ld + cell;
            const double yh = y_half[o];
            const double w = scale * (yh - y_full[o]) / ((c == t_comp ? atol_t : atol) + rtol * fabs(yh));
            acc = fma(w, w, acc);
        }
        if (sp_a) nst += sp_a[cell];
        if (sp_b) nst += sp_b[cell];
    }
    w2s[threadIdx.x] = acc;
    sts[threadIdx.x] = nst;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            w2s[threadIdx.x] += w2s[threadIdx.x + h];
            sts[threadIdx.x] += sts[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_w2[blockIdx.x] = w2s[0];
        part_steps[blockIdx.x] = sts[0];
    }
}

// status_out[cell] |= st_a[cell] | st_b[cell] (flags of an accepted step)
__global__ void __launch_bounds__(256)
    k_status_merge(int n_cells, const int32_t *__restrict__ st_a, const int32_t *__restrict__ st_b,
                   int32_t *status_out)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell < n_cells) status_out[cell] |= st_a[cell] | st_b[cell];
}

}  // namespace

hipError_t launch_step_err(int n, int t_comp, int n_cells, int ld, const double *y_half,
                           const double *y_full, double scale, double rtol, double atol,
                           double atol_t, const int32_t *sp_a, const int32_t *sp_b,
                           double *part_w2, long long *part_steps, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(k_step_err, dim3(step_err_blocks(n_cells)), dim3(block), 0, s, n, t_comp,
                       n_cells, ld, y_half, y_full, scale, rtol, atol, atol_t, sp_a, sp_b, part_w2,
                       part_steps);
    return hipGetLastError();
}

hipError_t launch_status_merge(int n_cells, const int32_t *st_a, const int32_t *st_b,
                               int32_t *status_out, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(k_status_merge, dim3((unsigned)(((long long)n_cells + block - 1) / block)), dim3(block), 0, s,
                       n_cells, st_a, st_b, status_out);
    return hipGetLastError();
}

hipError_t launch_forcing(long long n_elem, int n_gamma, int nj, const double *F,
                          long long F_stride, ForcingCoef coef, double *rho, hipStream_t s)
{
    const int block = 256;
    const long long grid = (n_elem + block - 1) / block;
    hipLaunchKernelGGL(k_forcing, dim3((unsigned)grid), dim3(block), 0, s, n_elem, n_gamma, nj, F,
                       F_stride, coef, rho);
    return hipGetLastError();
}

hipError_t launch_advdiff(int nx, int ny, int nz, int n_comp, int ld, const double *u,
                          double D, double dx, const double *y, double *fy, hipStream_t s)
{
    const long long gz = (long long)n_comp * ((nz + ADV_TZ - 1) / ADV_TZ);
    const long long gy = (ny + ADV_TY - 1) / ADV_TY;
    if (gz > 65535 || gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_advdiff, dim3((unsigned)((nx + ADV_TX - 1) / ADV_TX), (unsigned)gy,
                                       (unsigned)gz),
                       dim3(ADV_TX * ADV_TY), 0, s, nx, ny, nz, n_comp, ld, u[0], u[1], u[2], D,
                       dx, y, fy);
    return hipGetLastError();
}

hipError_t launch_lin_apply(int n, const double *A, int n_cells, int ld, const double *y,
                            double *fy, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(k_lin_apply, dim3((unsigned)(((long long)n_cells + block - 1) / block)), dim3(block), 0, s, n, A,
                       n_cells, ld, y, fy);
    return hipGetLastError();
}

hipError_t launch_status_count(const int32_t *status, int n_cells, int32_t mask,
                               unsigned long long *count, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(k_status_count, dim3((unsigned)(((long long)n_cells + block - 1) / block)), dim3(block), 0, s,
                       status, n_cells, mask, count);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(((long long)n + block - 1) / block)), dim3(block), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_exp2_t256(const double *x, double *y, int n, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(k_exp2_t256, dim3((unsigned)(((long long)n + block - 1) / block)), dim3(block), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_exp2(const double *x, double *y, int n, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(k_exp2, dim3((unsigned)(((long long)n + block - 1) / block)), dim3(block), 0, s, x, y, n);
    return hipGetLastError();
}
