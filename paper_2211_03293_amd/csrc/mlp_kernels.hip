// mlp_kernels.hip -- surrogate MLP kernels: BF16 MFMA GEMM for training,
// training elementwise kernels (bias + SiLU, MSE gradient, SiLU backward,
// bias gradient, Adam), feature construction, the fused four-layer inference
// kernel, the step-doubling gate with compaction, and gather / scatter.
//
// MFMA: v_mfma_f32_16x16x32_bf16 (gfx950).  Operand layout, lane l, g = l / 16:
//   A[i][k]: i = l % 16, k = 8 g + e (e = 0..7, one 16-byte register quad)
//   B[k][j]: j = l % 16, k = 8 g + e
//   D[i][j]: j = l % 16, i = 4 g + r (r = 0..3, four f32)
#include "mlp_dev.h"

#include <algorithm>
#include <utility>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x)
{
    __bf16 b = static_cast<__bf16>(x);   // round to nearest even
    return __builtin_bit_cast(uint16_t, b);
}

// The features are computed in FP64, rounded to FP32 and then to bfloat16
// (nearest even at each step).  The second rounding is done on the FP32 bit
// pattern: a plain conversion of an FP32 value that was just narrowed from
// FP64 may be folded by the compiler into one FP64 -> bfloat16 rounding, which
// differs from the two-step rounding where the FP64 value lies within half an
// FP32 ulp of a bfloat16 midpoint.
__device__ __forceinline__ uint16_t f2bf_bits(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t u)
{
    return __builtin_bit_cast(float, (uint32_t)u << 16);
}

// SiLU with the hardware exponential and reciprocal (about 1 ulp each in FP32;
// the result is rounded to bfloat16 next)
__device__ __forceinline__ float silu_f(float z)
{
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

__device__ __forceinline__ float silu_grad_f(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// C[M x N] (f32, ldc) = op(A)[M x K] * op(B)[K x N], bf16 operands.
// op(A)[m][k] = transA ? A[k*lda + m] : A[m*lda + k]
// op(B)[k][n] = transB ? B[n*ldb + k] : B[k*ldb + n]
// Block 256 threads = 4 waves, tile 64 x 64, each wave 32 x 32 (2 x 2 MFMA tiles).
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 32, GPAD = 8;

__global__ void __launch_bounds__(256)
    k_gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A, int lda, int transA,
                const uint16_t *__restrict__ B, int ldb, int transB, float *__restrict__ C,
                int ldc, int k_chunk)
{
    // split K: block z handles [z k_chunk, (z + 1) k_chunk) and writes its own
    // partial product at C + z M ldc
    const int kbeg = blockIdx.z * k_chunk, kend = min(K, kbeg + k_chunk);
    C += (size_t)blockIdx.z * M * ldc;
    __shared__ __attribute__((aligned(16))) uint16_t As[GT][GK + GPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GK + GPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int g = lane >> 4, i16 = lane & 15;
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        for (int e = tid; e < GT * GK; e += 256) {
            const int r = e / GK, k = e % GK;
            const int m = m0 + r, kk = k0 + k;
            uint16_t va = 0;
            if (m < M && kk < kend) va = transA ? A[(size_t)kk * lda + m] : A[(size_t)m * lda + kk];
            As[r][k] = va;
            const int n = n0 + r;
            uint16_t vb = 0;
            if (n < N && kk < kend) vb = transB ? B[(size_t)n * ldb + kk] : B[(size_t)kk * ldb + n];
            Bs[r][k] = vb;
        }
        __syncthreads();
        bf16x8 af[2], bfr[2];
        for (int t = 0; t < 2; ++t) {
            af[t] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * t + i16][8 * g]);
            bfr[t] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * t + i16][8 * g]);
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma(af[a], bfr[b], acc[a][b]);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * a + 4 * g + r, n = n0 + wn + 16 * b + i16;
                if (m < M && n < N) C[(size_t)m * ldc + n] = acc[a][b][r];
            }
}

// Z [rows x N] += bias; A = bf16(silu(Z)) when act != 0.
__global__ void __launch_bounds__(256)
    k_bias_act(int rows, int N, float *__restrict__ Z, const float *__restrict__ bias, int act,
               uint16_t *__restrict__ Aout)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * N) return;
    const int n = (int)(e % N);
    const float z = Z[e] + bias[n];
    Z[e] = z;
    if (act) Aout[e] = f2bf(silu_f(z));
}

// dZ = 2 (Y - T) / (rows * N) in f32, its bf16 copy, and the loss sum (f64).
__global__ void __launch_bounds__(256)
    k_mse_grad(int rows, int N, const float *__restrict__ Y, const float *__restrict__ T,
               float *__restrict__ dZ, uint16_t *__restrict__ dZq, double *loss)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)rows * N;
    double l = 0.0;
    if (e < tot) {
        const float d = Y[e] - T[e];
        const float s = 1.0f / (float)((double)rows * N);
        const float g = 2.0f * d * s;
        dZ[e] = g;
        dZq[e] = f2bf(g);
        l = (double)d * (double)d / (double)tot;
    }
    // wave reduction, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, l);
}

// dZ = dA * silu'(Z) (f32) and its bf16 copy.
__global__ void __launch_bounds__(256)
    k_silu_bwd(long long n, const float *__restrict__ dA, const float *__restrict__ Z,
               float *__restrict__ dZ, uint16_t *__restrict__ dZq)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float g = dA[e] * silu_grad_f(Z[e]);
    dZ[e] = g;
    dZq[e] = f2bf(g);
}

// out[e] = sum_z part[z][e], fixed order (deterministic split-K reduction).
__global__ void __launch_bounds__(256)
    k_sum_parts(long long n, int parts, const float *__restrict__ part, float *__restrict__ out)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.0f;
    for (int z = 0; z < parts; ++z) s += part[z * n + e];
    out[e] = s;
}

// Partial column sums: part[z][n] = sum over rows [z rc, (z + 1) rc) of dZ[r][n].
__global__ void __launch_bounds__(256)
    k_colsum_part(int rows, int N, int rc, const float *__restrict__ dZ, float *__restrict__ part)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int r0 = blockIdx.y * rc, r1 = min(rows, r0 + rc);
    float s = 0.0f;
    for (int r = r0; r < r1; ++r) s += dZ[(size_t)r * N + n];
    part[(size_t)blockIdx.y * N + n] = s;
}

__global__ void __launch_bounds__(256)
    k_adam(long long n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
           float *__restrict__ v, uint16_t *__restrict__ wq, float lr, float b1, float b2,
           float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (wq) wq[i] = f2bf(wi);
}

__global__ void __launch_bounds__(256)
    k_to_bf16(long long n, const float *__restrict__ x, uint16_t *__restrict__ y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// ---------------------------------------------------------------------------
// Raw feature k of one sample read straight from SoA arrays (no private
// arrays, so per-lane feature indices cost no scratch memory):
//   k < NS: log max(Y_k, 1e-30); k = NS: T; then the forcing coefficient p of
//   component c for k = NS + 1 + p NC + c (zero for p >= n_poly); last: log L
//   (L is the stage length).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double raw_feature(int k, const double *__restrict__ y,
                                              const double *__restrict__ rho, long long ld,
                                              long long s, int n_poly, double L)
{
    // species logarithms in FP32: every feature is rounded to bfloat16 afterwards
    if (k < MLP_NS) return (double)__logf((float)fmax(y[k * ld + s], 1e-30));
    if (k == MLP_NS) return y[MLP_NS * ld + s];
    if (k < MLP_NS + 1 + MLP_NPOLY * MLP_NC) {
        const int q = k - MLP_NS - 1, p = q / MLP_NC;
        return (p < n_poly) ? rho[(long long)q * ld + s] : 0.0;
    }
    if (k == MLP_FEAT - 1) return log(L);
    return 0.0;
}

__device__ __forceinline__ float std_feature(int k, const double *__restrict__ y,
                                             const double *__restrict__ rho, long long ld,
                                             long long s, int n_poly, double L,
                                             const double *__restrict__ stats)
{
    if (k >= MLP_FEAT) return 0.0f;
    return (float)((raw_feature(k, y, rho, ld, s, n_poly, L) - stats[k]) * stats[MLP_FEAT + k]);
}

// Raw target of component c: log-increment for species, plain increment for T.
__device__ __forceinline__ double raw_target(int c, double y0, double y1)
{
    if (c == MLP_NS) return y1 - y0;
    return log(fmax(y1, 0.0) + MLP_EPS) - log(fmax(y0, 0.0) + MLP_EPS);
}

// Inverse of raw_target: the end state from the start state and the increment.
__device__ __forceinline__ double apply_target(int c, double y0, double d)
{
    if (c == MLP_NS) return y0 + d;
    return (fmax(y0, 0.0) + MLP_EPS) * exp(d) - MLP_EPS;
}

// Training / evaluation features.  Samples are SoA with leading dimension ld:
// Y0[c*ld + s] (c < NC), RHO[(p*NC + c)*ld + s] (p < n_poly), Lv[s], Yb and Y1
// like Y0.  idx (nullable) picks the samples of this batch.  X: bf16
// [B][MLP_KPAD] standardized features of (Y0, RHO, Lv); T (nullable): f32
// [B][MLP_NC] standardized targets (raw_target(Yb, Y1) - y_mean) / y_std, the
// correction from the base state Yb to Y1.
__global__ void __launch_bounds__(256)
    k_featurize(int B, const int *__restrict__ idx, long long ld, const double *__restrict__ Y0,
                int n_poly, const double *__restrict__ RHO, const double *__restrict__ Lv,
                const double *__restrict__ Yb, const double *__restrict__ Y1,
                const double *__restrict__ stats, uint16_t *__restrict__ X,
                float *__restrict__ T)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const long long s = idx ? idx[b] : b;
    const double L = Lv[s];
    for (int k = 0; k < MLP_KPAD; ++k)
        X[(size_t)b * MLP_KPAD + k] = f2bf_bits(std_feature(k, Y0, RHO, ld, s, n_poly, L, stats));
    if (T) {
        const double *ym = stats + 2 * MLP_FEAT, *yi = stats + 2 * MLP_FEAT + MLP_NC;
        for (int c = 0; c < MLP_NC; ++c)
            T[(size_t)b * MLP_NC + c] =
                (float)((raw_target(c, Yb[c * ld + s], Y1[c * ld + s]) - ym[c]) * yi[c]);
    }
}

// Per-block partial sums for feature / target statistics (FP64): part[block]
// holds sum and sum of squares of the MLP_FEAT raw features and MLP_NC raw
// targets over the block's samples.
__global__ void __launch_bounds__(256)
    k_stats_partial(long long N, long long ld, const double *__restrict__ Y0, int n_poly,
                    const double *__restrict__ RHO, const double *__restrict__ Lv,
                    const double *__restrict__ Yb, const double *__restrict__ Y1,
                    double *__restrict__ part)
{
    constexpr int NV = MLP_FEAT + MLP_NC;
    __shared__ double red[256];
    const long long per = (N + gridDim.x - 1) / gridDim.x;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(N, s0 + per);
    for (int v = 0; v < NV; ++v) {
        double sum = 0.0, sq = 0.0;
        for (long long s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
            const double x = (v < MLP_FEAT)
                                 ? raw_feature(v, Y0, RHO, ld, s, n_poly, Lv[s])
                                 : raw_target(v - MLP_FEAT, Yb[(v - MLP_FEAT) * ld + s],
                                              Y1[(v - MLP_FEAT) * ld + s]);
            sum += x;
            sq += x * x;
        }
        red[threadIdx.x] = sum;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * 2 * NV + v] = red[0];
        __syncthreads();
        red[threadIdx.x] = sq;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * 2 * NV + NV + v] = red[0];
        __syncthreads();
    }
}

// stats = [x_mean (FEAT), x_inv_std (FEAT), y_mean (NC), y_inv_std (NC), y_std (NC)]
__global__ void k_stats_final(int n_blocks, long long N, const double *__restrict__ part,
                              double *__restrict__ stats)
{
    constexpr int NV = MLP_FEAT + MLP_NC;
    const int v = threadIdx.x;
    if (v >= NV) return;
    double sum = 0.0, sq = 0.0;
    for (int b = 0; b < n_blocks; ++b) {
        sum += part[(size_t)b * 2 * NV + v];
        sq += part[(size_t)b * 2 * NV + NV + v];
    }
    const double mean = sum / (double)N;
    const double var = fmax(sq / (double)N - mean * mean, 0.0);
    const double sd = sqrt(var);
    const double inv = (sd > 1e-30 * fmax(1.0, fabs(mean))) ? 1.0 / sd : 1.0;
    if (v < MLP_FEAT) {
        stats[v] = mean;
        stats[MLP_FEAT + v] = inv;
    } else {
        const int c = v - MLP_FEAT;
        stats[2 * MLP_FEAT + c] = mean;
        stats[2 * MLP_FEAT + MLP_NC + c] = inv;
        stats[2 * MLP_FEAT + 2 * MLP_NC + c] = (sd > 0.0) ? sd : 1.0;
    }
}

// ---------------------------------------------------------------------------
// Residual check of the surrogate, G = max(D, I), on FP64 data:
//   Ve = vc + rich (vc - vh), the Richardson extrapolation of the coarse stage
//   vc (n substeps) and vh (n / 2 substeps), rich = 1 / (2^p - 1) for a fast
//   method of order p: an estimate of the fine stage from FP64 work alone;
//   D = max_c |vn_c - Ve_c| / max(|Ve_c|, floor_c) (floor 1e-8 for mass
//   fractions, 0 for T), vn the network's correction of vc;
//   I = the residual of the mass-sum invariant of vn: the chemistry conserves
//   sum_k Y_k, so over the stage sum_k (vn_k - y0_k) must equal
//   L sum_p sum_k rho_(p,k) / (p + 1), relative to sum_k |y0_k|.
// A cell is accepted when G <= tol and neither coarse solve flagged it
// (status_c, nullable); it takes vn and status 0.  Rejected cells are appended
// to the fallback list (one atomic per wave, ranks from the ballot mask).
// gate_cell is the check of cell i (vn_at(c) gives vn's component c); k_gate
// and the fused inference-and-check run the same code.
template <bool PRELOAD, typename VN>
__device__ __forceinline__ bool gate_cell(long long i, long long ld, const double *yin,
                                          const double *rho, int n_poly, double L,
                                          const double *vc, const double *vh, VN vn_at,
                                          const int *status_c, double rich, double tol, double &G)
{
    // PRELOAD (few waves per SIMD): every load of the cell is issued before
    // the arithmetic; the arithmetic is the same, in component order
    double va[MLP_NC], vb[MLP_NC], vv[MLP_NC], vy[MLP_NS];
    if constexpr (PRELOAD) {
#pragma unroll
        for (int c = 0; c < MLP_NC; ++c) {
            va[c] = vc[c * ld + i];
            vb[c] = vh[c * ld + i];
            vv[c] = vn_at(c);
            if (c < MLP_NS) vy[c] = yin[c * ld + i];
        }
    }
    double D = 0.0, dsum = 0.0, y0sum = 0.0, fsum = 0.0;
    bool nan = false;
#pragma unroll PRELOAD ? MLP_NC : 1
    for (int c = 0; c < MLP_NC; ++c) {
        const double a = PRELOAD ? va[c] : vc[c * ld + i];
        const double h = PRELOAD ? vb[c] : vh[c * ld + i];
        const double ve = a + rich * (a - h);
        const double fl = (c < MLP_NS) ? 1e-8 : 0.0;
        const double v = PRELOAD ? vv[c] : vn_at(c);
        const double e = fabs(v - ve) / fmax(fabs(ve), fl);
        nan = nan || (e != e);
        D = (e > D) ? e : D;
        if (c < MLP_NS) {
            const double y0 = PRELOAD ? vy[c] : yin[c * ld + i];
            dsum += v - y0;
            y0sum += fabs(y0);
            for (int p = 0; p < n_poly; ++p)
                fsum += rho[((long long)p * MLP_NC + c) * ld + i] / (double)(p + 1);
        }
    }
    const double I = fabs(dsum - L * fsum) / fmax(y0sum, 1e-300);
    nan = nan || (I != I);
    G = nan ? __builtin_nan("") : fmax(D, I);
    return nan || !(G <= tol) || (status_c && status_c[i] != 0);
}

// Appends the wave's rejected cells to the fallback list: one atomic per wave,
// ranks from the ballot mask (every lane of the wave calls it).
__device__ __forceinline__ void append_rejected(bool reject, int i, int *list,
                                                unsigned int *count)
{
    const unsigned long long m = __ballot(reject);
    const int lane = threadIdx.x & 63;
    unsigned int basepos = 0;
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        if (lane == leader) basepos = atomicAdd(count, (unsigned int)__popcll(m));
        basepos = __shfl(basepos, leader);
        if (reject) list[basepos + __popcll(m & ((1ull << lane) - 1ull))] = i;
    }
}

// Fused inference: y_out = apply_target(base, y_mean + y_std * MLP(features(y_in,
// rho', L'))): the network reads the stage start state and predicts the
// correction of `base` (the coarse FP64 stage result; y_in itself for an
// increment over the stage).
// One wave owns 32 cells (two 16-cell MFMA column tiles); activations stay in
// registers between layers: the D layout of one layer is the B layout of the
// next once the next layer's input columns are permuted (done on the host):
// logical K index 32 t + 8 g + e of a layer holds the previous layer's output
// 32 t + (e < 4 ? 4 g + e : 16 + 4 g + e - 4).
// ---------------------------------------------------------------------------
struct InferArgs {
    const double *yin;
    const double *base;         // state the predicted correction applies to
    double *yout;
    // the residual check fused after the inference (k_infer<true>): base is
    // the coarse stage vc, vh the half-resolution one; the other fields as
    // for k_gate
    const double *vh;
    const int *status_c;
    double rich, tol;
    int *used_fallback;
    double *gval;
    int *status;
    int *list;
    unsigned int *count;
    const double *rho;
    const uint16_t *W[4];       // [out_pad][in_pad] bf16, permuted inputs
    const float *b[4];          // [out_pad]
    const double *stats;
    long long ld;
    int n_cells;
    int n_poly;
    double L;
};

// Weights stream through LDS in chunks of RB = 32 output rows with all their
// input columns (16 KB for a hidden layer), shared by the block's four waves.
// Each chunk yields two finished row tiles, whose SiLU (for the next layer's
// input) overlaps the matrix products of the following chunk.  The chunks are
// copied by direct global -> LDS loads (no register staging) into a ring of
// three buffers, two chunks ahead of the one being multiplied.  In a buffer,
// row r holds its P = kin / 8 pieces of 16 bytes (8 bf16 each), piece p at slot
// r P + (p ^ (r & 15)): the 16 lanes that read one A fragment (16 rows, one
// piece index) hit 16 distinct 16-byte bank groups, so the reads are free of
// bank conflicts for 128- and 256-byte bank widths alike.
constexpr int RB = 32;
constexpr int WCHUNK = RB * MLP_HID;    // bf16 elements of one chunk buffer (16 KB)
constexpr int N_BUF = 3;

typedef __attribute__((address_space(3))) void lds_void_t;

// The weight stream of one inference: 8 row blocks of the first layer (input
// rows padded to MLP_K0_IN columns), 8 of each hidden layer, 1 of the output
// layer (32 padded rows).
constexpr int N_CHUNKS = 8 + 8 + 8 + 1;
__host__ __device__ constexpr int chunk_layer(int c) { return c < 24 ? c / 8 : 3; }
__host__ __device__ constexpr int chunk_rb(int c) { return c < 24 ? c % 8 : 0; }
__host__ __device__ constexpr int layer_kin(int l) { return l == 0 ? MLP_K0_IN : MLP_HID; }
__host__ __device__ constexpr int layer_kb(int l) { return l == 0 ? MLP_KPAD / 32 : MLP_HID / 32; }
// direct-to-LDS loads one wave issues per chunk (the same for all four waves)
__host__ __device__ constexpr int chunk_loads(int c)
{
    return RB * (layer_kin(chunk_layer(c)) / 8) / 256;
}

// Byte offset, within a chunk's rows, of the piece that wave w's direct-to-LDS
// load i writes to slot 256 i + 64 w + lane of a buffer with P pieces per row.
template <int P>
__device__ __forceinline__ unsigned chunk_src_off(int i, int w, int lane)
{
    const int slot = 256 * i + 64 * w + lane;
    const int row = slot / P, p = (slot % P) ^ (row & 15);
    return 2u * (unsigned)(row * 8 * P + 8 * p);
}

// Per-lane offsets of the direct-to-LDS loads (the same for every chunk with
// the same row length) and the lane bases of the A-fragment reads.
//
// A-fragment piece 4 kb + g of row 16 mi + j of a buffer with P pieces per
// row sits at slot (16 mi + j) P + ((4 kb + g) ^ j).  As (4 kb + g) ^ j =
// 4 (kb ^ (j >> 2)) + (g ^ (j & 3)) and kb ^ (j >> 2) = (kb & ~3) +
// ((kb & 3) ^ (j >> 2)), that slot is rd[kb & 3] + 16 mi P + 4 (kb & ~3): four
// lane bases per row length and a compile-time offset per fragment.
struct Slots {
    unsigned ld16[2], ld32[4];   // chunk_src_off for P = 16 (2 loads), 32 (4 loads)
    int rd16[4], rd32[4];        // A-fragment lane bases (slots) for P = 16, 32
};

// Issues the direct-to-LDS loads of chunk C into buffer `buf` (wave `w`): wave
// w's load i fills slots 256 i + 64 w + lane.  `zs` is a scalar zero produced
// after the preceding barrier (the loads must not move above it).
template <int C>
__device__ __forceinline__ void chunk_issue(const InferArgs &a, uint16_t *buf, int w,
                                            const Slots &sl, int zs)
{
    constexpr int l = chunk_layer(C), kin = layer_kin(l), P = kin / 8;
    static_assert(P == 16 || P == 32, "row lengths of the stream");
    static_assert(chunk_loads(C) == (P == 16 ? 2 : 4), "loads per chunk");
    const char *W =
        reinterpret_cast<const char *>(a.W[l] + (size_t)(RB * chunk_rb(C)) * kin) + zs;
#pragma unroll
    for (int i = 0; i < chunk_loads(C); ++i) {
        const unsigned off = (P == 16) ? sl.ld16[i] : sl.ld32[i];
        __builtin_amdgcn_global_load_lds((const void *)(W + off),
                                         (lds_void_t *)(buf + 8 * (256 * i + 64 * w)), 16, 0, 0);
    }
}

// Waits until at most N of this wave's vector-memory loads are outstanding
// (loads complete in issue order) and all of its LDS reads have returned (the
// buffer they read is refilled after this barrier), then joins the block
// barrier.  Returns a zero that the compiler cannot see through, produced
// after the barrier, in a vector register (z) and in a scalar one (zs): LDS
// reads and direct-to-LDS loads whose addresses add it cannot be scheduled
// before the barrier.
template <int N>
__device__ __forceinline__ int wait_loads_and_barrier(int &zs)
{
    static_assert(N >= 0 && N <= 15, "vmcnt field");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((N & 0xf) | (0x7 << 4));   // vmcnt(N), lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    int z = 0;
    asm volatile("" : "+v"(z)::"memory");
    zs = 0;
    asm volatile("" : "+s"(zs)::"memory");
    return z;
}

constexpr int XROW = MLP_KPAD + 8;     // padded LDS feature row (bf16), 208 bytes

// Column tiles (16 cells each) per wave, and the waves-per-SIMD target.
#ifndef MLP_NT
#define MLP_NT 2
#endif
#ifndef MLP_WPE
#define MLP_WPE 2
#endif
constexpr int NT = MLP_NT;
constexpr int CELLS_PER_BLOCK = 4 * 16 * NT;

// The ring: three distinct LDS objects, so that the compiler can tell a read
// of one buffer from the direct-to-LDS loads still in flight into another (it
// then needs no wait for those loads before the read).
struct Ring {
    uint16_t *b0, *b1, *b2;
    template <int I>
    __device__ __forceinline__ uint16_t *get() const
    {
        if constexpr (I % N_BUF == 0) return b0;
        else if constexpr (I % N_BUF == 1) return b1;
        else return b2;
    }
};

// Activations of one inference, per lane: the first layer's input (3 k-blocks
// of features), and two 8-k-block arrays that alternate as input and output of
// the hidden layers; two sets of accumulators (one row block each) alternate
// between chunks.
struct Act {
    bf16x8 x0[MLP_KPAD / 32][NT];
    bf16x8 ha[8][NT], hb[8][NT];
    f32x4 acc[2][2][NT];
};

template <int L>
__device__ __forceinline__ auto &layer_in(Act &s)
{
    if constexpr (L == 0) return s.x0;
    else if constexpr (L == 2) return s.hb;
    else return s.ha;
}
template <int L>
__device__ __forceinline__ auto &layer_out(Act &s)
{
    if constexpr (L == 1) return s.hb;
    else return s.ha;
}

// SiLU + bf16 repack of chunk C's two row tiles into k-block rb of the next
// layer's input (the MFMA output layout is the next layer's B layout once its
// input columns are permuted on the host).
template <int C>
__device__ __forceinline__ void chunk_activate(Act &s)
{
    constexpr int l = chunk_layer(C), rb = chunk_rb(C);
    auto &out = layer_out<l>(s);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        bf16x8 v;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[4 * h + r] = static_cast<__bf16>(silu_f(s.acc[C & 1][h][t][r]));
        out[rb][t] = v;
    }
}

// One step of the weight stream: wait for chunk C (the loads of chunk C + 1
// stay in flight), barrier, issue chunk C + 2 into the buffer that chunk C - 1
// used, multiply chunk C into its accumulator set, and activate chunk C - 1
// (before the products when chunk C starts a layer, which needs it as input).
template <int C>
__device__ __forceinline__ void weight_step(const InferArgs &a, const Ring &ring,
                                            const float *bias, int w, int g, const Slots &sl,
                                            Act &s)
{
    constexpr int l = chunk_layer(C), KB = layer_kb(l), P = layer_kin(l) / 8;
    constexpr bool prev_hidden = C > 0 && chunk_layer(C - 1) < 3;
    constexpr bool layer_start = C > 0 && chunk_layer(C - 1) != l;
    int zs;
    const int z = wait_loads_and_barrier < C + 1 < N_CHUNKS ? chunk_loads(C + 1) : 0 > (zs);
    if constexpr (C + 2 < N_CHUNKS) chunk_issue<C + 2>(a, ring.get<C + 2>(), w, sl, zs);
    if constexpr (prev_hidden && layer_start) chunk_activate<C - 1>(s);
    const uint16_t *buf = ring.get<C>();
    auto &in = layer_in<l>(s);
    // hidden layers: the accumulators start from the bias (lane (j, g) holds
    // rows 4 g .. 4 g + 3 of each row tile), so the activation needs no add
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        f32x4 b0 = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (l < 3)
            b0 = *reinterpret_cast<const f32x4 *>(bias + MLP_HID * l + RB * chunk_rb(C) + 16 * mi +
                                                  4 * g);
#pragma unroll
        for (int t = 0; t < NT; ++t) s.acc[C & 1][mi][t] = b0;
    }
    // All A fragments of the chunk are requested before the first product, so
    // the products start as soon as the first fragments arrive (LDS returns
    // in order).  The buffer is written only by direct-to-LDS loads, which the
    // compiler does not see as stores to it, so it would be free to move these
    // reads above the barrier that orders them after the other waves' loads of
    // the chunk: their addresses depend on `z`, which the barrier produces.
    static_assert(P == 16 || P == 32, "row lengths of the stream");
    const int *lb = (P == 16) ? sl.rd16 : sl.rd32;
    const uint16_t *bq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[q] = buf + 8 * lb[q] + z;
    bf16x8 af[KB][2];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
            af[kb][mi] = *reinterpret_cast<const bf16x8 *>(
                bq[kb & 3] + 8 * (16 * mi * P + 4 * (kb & ~3)));
    __builtin_amdgcn_sched_barrier(0);       // keep every read ahead of the products
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                s.acc[C & 1][mi][t] = mfma(af[kb][mi], in[kb][t], s.acc[C & 1][mi][t]);
    if constexpr (prev_hidden && !layer_start) {
        chunk_activate<C - 1>(s);
#ifndef MLP_NO_INTERLEAVE
        // The activation of chunk C - 1 does not depend on chunk C's
        // products: interleave them (one product, then a few vector
        // instructions), so the vector ALU works while the matrix core runs.
        constexpr int NM = KB * 2 * NT, PER = (16 * NT * 6 + NM - 1) / NM;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);     // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);   // VALU
        }
#endif
    }
}

template <int... C>
__device__ __forceinline__ void weight_stream(const InferArgs &a, const Ring &ring,
                                              const float *bias, int w, int g, const Slots &sl,
                                              Act &s, std::integer_sequence<int, C...>)
{
    (weight_step<C>(a, ring, bias, w, g, sl, s), ...);
}

// GATE: the residual check follows in the same launch (the network states go
// through LDS to one lane per cell, which runs gate_cell exactly as k_gate).
template <bool GATE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MLP_WPE)))
    k_infer(InferArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t wb0[WCHUNK];
    __shared__ __attribute__((aligned(16))) uint16_t wb1[WCHUNK];
    __shared__ __attribute__((aligned(16))) uint16_t wb2[WCHUNK];
    __shared__ __attribute__((aligned(16))) uint16_t xs[CELLS_PER_BLOCK * XROW];
    const Ring ring{wb0, wb1, wb2};
    __shared__ __attribute__((aligned(16))) float bias[3 * MLP_HID];   // hidden-layer biases
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, j = lane & 15;
    Slots sl;
#pragma unroll
    for (int i = 0; i < 2; ++i) sl.ld16[i] = chunk_src_off<16>(i, w, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) sl.ld32[i] = chunk_src_off<32>(i, w, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lp = 4 * (q ^ (j >> 2)) + (g ^ (j & 3));
        sl.rd16[q] = 16 * j + lp;
        sl.rd32[q] = 32 * j + lp;
    }
    // the first two weight chunks are in flight while the features are built
    chunk_issue<0>(a, ring.get<0>(), w, sl, 0);
    chunk_issue<1>(a, ring.get<1>(), w, sl, 0);
    for (int e = threadIdx.x; e < 3 * MLP_HID; e += 256) bias[e] = a.b[e / MLP_HID][e % MLP_HID];
    // every wave takes part in the block's barriers; idle cells are clamped
    const long long block0 = (long long)blockIdx.x * CELLS_PER_BLOCK;
    const long long base = block0 + w * 16 * NT;
    const double L = a.L;
    // ---- features of the block's cells, computed cooperatively: thread
    // groups take interleaved features (the feature index is uniform per wave,
    // so its source plane is a scalar address and the loads are coalesced)
    {
        constexpr int GROUPS = 256 / CELLS_PER_BLOCK;
        constexpr int PER = MLP_KPAD / GROUPS;           // features per thread
        const int c = threadIdx.x % CELLS_PER_BLOCK;
        const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / CELLS_PER_BLOCK);
        long long cell = block0 + c;
        if (cell >= a.n_cells) cell = a.n_cells - 1;
        // each feature is one unconditional load (the state, a forcing plane or
        // a dummy for log L and the padding) plus selects.  Loads go out in
        // batches of FB before any of them is used.
        // The statistics are read through the constant address space
        // (scalar loads: the feature index is uniform per wave and the
        // statistics are not written during the launch).
        constexpr int FB = PER % 48 == 0 ? 48 : (PER % 16 == 0 ? 16 : 8);
        static_assert(PER % FB == 0, "feature batches");
        typedef const __attribute__((address_space(4))) double cdouble;
        cdouble *cst = (cdouble *)a.stats;
        const double logL = log(L);
        for (int b0 = 0; b0 < PER; b0 += FB) {
            double v[FB];
#pragma unroll
            for (int i = 0; i < FB; ++i) {
                const int k = grp + GROUPS * (b0 + i);
                const bool isy = k <= MLP_NS;
                const bool isr = (k > MLP_NS) && (k - MLP_NS - 1 < a.n_poly * MLP_NC);
                const double *src = isy ? a.yin + (long long)k * a.ld
                                        : (isr ? a.rho + (long long)(k - MLP_NS - 1) * a.ld
                                               : a.yin);
                v[i] = src[cell];
            }
#pragma unroll
            for (int i = 0; i < FB; ++i) {
                const int k = grp + GROUPS * (b0 + i);
                const bool isy = k <= MLP_NS;
                const bool isr = (k > MLP_NS) && (k - MLP_NS - 1 < a.n_poly * MLP_NC);
                // species logarithms in FP32 (the feature is rounded to bfloat16
                // next); T, the forcing and log L as they are
                double raw = (k < MLP_NS) ? (double)__logf((float)fmax(v[i], 1e-30)) : v[i];
                if (k == MLP_FEAT - 1) raw = logL;
                const bool live = isy || isr || (k == MLP_FEAT - 1);
                const int kk = min(k, MLP_FEAT - 1);
                const float z = live ? (float)((raw - cst[kk]) * cst[MLP_FEAT + kk]) : 0.0f;
                xs[c * XROW + k] = f2bf_bits(z);
            }
        }
    }
    __syncthreads();
    Act st;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int kb = 0; kb < MLP_KPAD / 32; ++kb)
            st.x0[kb][t] = *reinterpret_cast<const bf16x8 *>(
                xs + (w * 16 * NT + 16 * t + j) * XROW + 32 * kb + 8 * g);
    // ---- three hidden layers and the output layer, one weight stream
    weight_stream(a, ring, bias, w, g, sl, st, std::make_integer_sequence<int, N_CHUNKS>{});
    // the output layer is chunk N_CHUNKS - 1 (accumulator set 0)
    static_assert(((N_CHUNKS - 1) & 1) == 0, "output accumulator set");
    const f32x4 (&acc)[2][NT] = st.acc[0];
    // ---- output: lane (j, g) holds components 4 g + r (and 16 + 4 g + r) of
    // cell 16 t + j; the start states are loaded before any is used
    const double *ym = a.stats + 2 * MLP_FEAT, *ysd = a.stats + 2 * MLP_FEAT + 2 * MLP_NC;
    double y0[NT][2][4], mean[2][4], sd[2][4];
    float bo[2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            const int c = min(16 * mi + 4 * g + r4, MLP_NC - 1);
            mean[mi][r4] = ym[c];
            sd[mi][r4] = ysd[c];
            bo[mi][r4] = a.b[3][c];
        }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const long long cell = min(base + 16 * t + j, (long long)a.n_cells - 1);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int c = min(16 * mi + 4 * g + r4, MLP_NC - 1);
                y0[t][mi][r4] = a.base[c * a.ld + cell];
            }
    }
    // the network states of the wave's cells: to y_out, or (GATE) to LDS,
    // [component][cell of the block] in the feature buffer, which no wave
    // reads any more
    double *vl = reinterpret_cast<double *>(xs);
    static_assert(sizeof(double) * MLP_NC * CELLS_PER_BLOCK <= sizeof(xs), "gate staging");
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const long long cell = base + 16 * t + j;
        if (cell >= a.n_cells) continue;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int c = 16 * mi + 4 * g + r4;
                if (c >= MLP_NC) continue;
                const double d = mean[mi][r4] + sd[mi][r4] * (double)(acc[mi][t][r4] + bo[mi][r4]);
                const double v = apply_target(c, y0[t][mi][r4], d);
                if constexpr (GATE)
                    vl[c * CELLS_PER_BLOCK + w * 16 * NT + 16 * t + j] = v;
                else
                    a.yout[c * a.ld + cell] = v;
            }
    }
    if constexpr (GATE) {
        __syncthreads();
        // lane l < 16 NT checks cell base + l of its wave
        const long long i = base + lane;
        bool reject = false;
        if (lane < 16 * NT && i < a.n_cells) {
            const double *vrow = vl + w * 16 * NT + lane;
            double G;
            reject = gate_cell<true>(i, a.ld, a.yin, a.rho, a.n_poly, a.L, a.base, a.vh,
                                     [&](int c) { return vrow[c * CELLS_PER_BLOCK]; },
                                     a.status_c, a.rich, a.tol, G);
            if (!reject)
                for (int c = 0; c < MLP_NC; ++c) a.yout[c * a.ld + i] = vrow[c * CELLS_PER_BLOCK];
            if (a.used_fallback) a.used_fallback[i] = reject ? 1 : 0;
            if (a.gval) a.gval[i] = G;
            if (a.status && !reject) a.status[i] = 0;
        }
        append_rejected(reject, (int)i, a.list, a.count);
    }
}

__global__ void __launch_bounds__(256)
    k_gate(int n_cells, long long ld, const double *__restrict__ yin,
           const double *__restrict__ rho, int n_poly, double L, const double *__restrict__ vc,
           const double *__restrict__ vh, const double *__restrict__ vn,
           const int *__restrict__ status_c, double rich, double tol, double *__restrict__ yout,
           int *__restrict__ used_fallback, double *__restrict__ gval, int *__restrict__ status,
           int *__restrict__ list, unsigned int *count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool reject = false;
    if (i < n_cells) {
        double G;
        reject = gate_cell<false>(i, ld, yin, rho, n_poly, L, vc, vh,
                                  [&](int c) { return vn[c * ld + i]; }, status_c, rich, tol, G);
        if (!reject)
            for (int c = 0; c < MLP_NC; ++c) yout[c * ld + i] = vn[c * ld + i];
        if (used_fallback) used_fallback[i] = reject ? 1 : 0;
        if (gval) gval[i] = G;
        if (status && !reject) status[i] = 0;
    }
    append_rejected(reject, i, list, count);
}

// dst[c*ldd + k] = src[c*lds + list[k]] for planes c < n_planes, k < *count.
__global__ void __launch_bounds__(256)
    k_gather(int n_planes, const unsigned int *count, const int *__restrict__ list,
             const double *__restrict__ src, long long lds, double *__restrict__ dst,
             long long ldd)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)*count) return;
    const int cell = list[k];
    for (int c = 0; c < n_planes; ++c) dst[c * ldd + k] = src[c * lds + cell];
}

__global__ void __launch_bounds__(256)
    k_scatter(int n_planes, const unsigned int *count, const int *__restrict__ list,
              const double *__restrict__ src, long long lds, double *__restrict__ dst,
              long long ldd)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)*count) return;
    const int cell = list[k];
    for (int c = 0; c < n_planes; ++c) dst[c * ldd + cell] = src[c * lds + k];
}

// dst[list[k]] = src[k] for k < *count (the fallback cells' status words).
__global__ void __launch_bounds__(256)
    k_scatter_i32(const unsigned int *count, const int *__restrict__ list,
                  const int *__restrict__ src, int *__restrict__ dst)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)*count) return;
    dst[list[k]] = src[k];
}

__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

inline dim3 grid1(long long n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

}  // namespace

hipError_t mlp_gemm(int M, int N, int K, const uint16_t *A, int lda, int transA, const uint16_t *B,
                    int ldb, int transB, float *C, int ldc, hipStream_t s, float *part,
                    size_t part_elems)
{
    // few output tiles and a long K: split K over up to 32 blocks per tile into
    // `part` and reduce in a fixed order (deterministic)
    const int tiles = ((N + GT - 1) / GT) * ((M + GT - 1) / GT);
    int splits = 1;
    if (part && ldc == N && tiles < 128 && K >= 8 * GK) {
        splits = std::min(32, std::max(1, 256 / tiles));
        while (splits > 1 && (size_t)splits * M * N > part_elems) --splits;
    }
    const int k_chunk = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    splits = (K + k_chunk - 1) / k_chunk;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
    float *dst = splits > 1 ? part : C;
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, lda, transA, B, ldb,
                       transB, dst, ldc, k_chunk);
    if (splits > 1)
        hipLaunchKernelGGL(k_sum_parts, grid1((long long)M * N, 256), dim3(256), 0, s,
                           (long long)M * N, splits, part, C);
    return hipGetLastError();
}

hipError_t mlp_bias_act(int rows, int N, float *Z, const float *bias, int act, uint16_t *Aout,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_bias_act, grid1((long long)rows * N, 256), dim3(256), 0, s, rows, N, Z,
                       bias, act, Aout);
    return hipGetLastError();
}

hipError_t mlp_mse_grad(int rows, int N, const float *Y, const float *T, float *dZ, uint16_t *dZq,
                        double *loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_mse_grad, grid1((long long)rows * N, 256), dim3(256), 0, s, rows, N, Y, T,
                       dZ, dZq, loss);
    return hipGetLastError();
}

hipError_t mlp_silu_bwd(long long n, const float *dA, const float *Z, float *dZ, uint16_t *dZq,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_silu_bwd, grid1(n, 256), dim3(256), 0, s, n, dA, Z, dZ, dZq);
    return hipGetLastError();
}

hipError_t mlp_colsum(int rows, int N, const float *dZ, float *db, hipStream_t s, float *part,
                      size_t part_elems)
{
    int chunks = std::max(1, std::min(64, rows / 64));
    while (chunks > 1 && (size_t)chunks * N > part_elems) --chunks;
    const int rc = (rows + chunks - 1) / chunks;
    chunks = (rows + rc - 1) / rc;
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 255) / 256, chunks), dim3(256), 0, s, rows, N, rc,
                       dZ, chunks > 1 ? part : db);
    if (chunks > 1)
        hipLaunchKernelGGL(k_sum_parts, grid1(N, 256), dim3(256), 0, s, (long long)N, chunks,
                           part, db);
    return hipGetLastError();
}

hipError_t mlp_adam(long long n, float *w, const float *g, float *m, float *v, uint16_t *wq,
                    float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, grid1(n, 256), dim3(256), 0, s, n, w, g, m, v, wq, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(long long n, const float *x, uint16_t *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_bf16, grid1(n, 256), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

hipError_t mlp_featurize(int B, const int *idx, long long ld, const double *Y0, int n_poly,
                         const double *RHO, const double *Lv, const double *Yb,
                         const double *Y1, const double *stats, uint16_t *X, float *T,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_featurize, grid1(B, 256), dim3(256), 0, s, B, idx, ld, Y0, n_poly, RHO,
                       Lv, Yb ? Yb : Y0, Y1, stats, X, T);
    return hipGetLastError();
}

hipError_t mlp_stats(long long N, long long ld, const double *Y0, int n_poly, const double *RHO,
                     const double *Lv, const double *Yb, const double *Y1, double *part,
                     int n_blocks, double *stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_partial, dim3(n_blocks), dim3(256), 0, s, N, ld, Y0, n_poly, RHO,
                       Lv, Yb ? Yb : Y0, Y1, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(128), 0, s, n_blocks, N, part, stats);
    return hipGetLastError();
}

hipError_t mlp_infer(const double *yin, const double *base, double *yout, const double *rho,
                     const uint16_t *const *W, const float *const *b, const double *stats,
                     long long ld, int n_cells, int n_poly, double L, hipStream_t s)
{
    InferArgs a{};
    a.yin = yin;
    a.base = base ? base : yin;
    a.yout = yout;
    a.rho = rho;
    for (int l = 0; l < 4; ++l) {
        a.W[l] = W[l];
        a.b[l] = b[l];
    }
    a.stats = stats;
    a.ld = ld;
    a.n_cells = n_cells;
    a.n_poly = n_poly;
    a.L = L;
    hipLaunchKernelGGL(k_infer<false>, grid1(n_cells, CELLS_PER_BLOCK), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t mlp_infer_gate(const double *yin, const double *vc, const double *vh,
                          const double *rho, const uint16_t *const *W, const float *const *b,
                          const double *stats, long long ld, int n_cells, int n_poly, double L,
                          const int *status_c, double rich, double tol, double *yout,
                          int *used_fallback, double *gval, int *status, int *list,
                          unsigned int *count, hipStream_t s)
{
    InferArgs a{};
    a.yin = yin;
    a.base = vc;
    a.yout = yout;
    a.rho = rho;
    for (int l = 0; l < 4; ++l) {
        a.W[l] = W[l];
        a.b[l] = b[l];
    }
    a.stats = stats;
    a.ld = ld;
    a.n_cells = n_cells;
    a.n_poly = n_poly;
    a.L = L;
    a.vh = vh;
    a.status_c = status_c;
    a.rich = rich;
    a.tol = tol;
    a.used_fallback = used_fallback;
    a.gval = gval;
    a.status = status;
    a.list = list;
    a.count = count;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, count);
    hipLaunchKernelGGL(k_infer<true>, grid1(n_cells, CELLS_PER_BLOCK), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t mlp_gate(int n_cells, long long ld, const double *yin, const double *rho, int n_poly,
                    double L, const double *vc, const double *vh, const double *vn,
                    const int *status_c, double rich, double tol, double *yout, int *used_fallback,
                    double *gval, int *status, int *list, unsigned int *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, count);
    hipLaunchKernelGGL(k_gate, grid1(n_cells, 256), dim3(256), 0, s, n_cells, ld, yin, rho,
                       n_poly, L, vc, vh, vn, status_c, rich, tol, yout, used_fallback, gval,
                       status, list, count);
    return hipGetLastError();
}

hipError_t mlp_gather(int n_planes, const unsigned int *count, const int *list, long long n_max,
                      const double *src, long long lds, double *dst, long long ldd, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, grid1(n_max, 256), dim3(256), 0, s, n_planes, count, list, src,
                       lds, dst, ldd);
    return hipGetLastError();
}

hipError_t mlp_scatter(int n_planes, const unsigned int *count, const int *list, long long n_max,
                       const double *src, long long lds, double *dst, long long ldd, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, grid1(n_max, 256), dim3(256), 0, s, n_planes, count, list, src,
                       lds, dst, ldd);
    return hipGetLastError();
}

hipError_t mlp_scatter_i32(const unsigned int *count, const int *list, long long n_max,
                           const int *src, int *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter_i32, grid1(n_max, 256), dim3(256), 0, s, count, list, src, dst);
    return hipGetLastError();
}

hipError_t mlp_zero_u32(unsigned int *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}
