// fast_generic.hip -- fast-stage kernels compiled once for every mechanism.
//
// One cell per lane.  The mechanism coefficients are staged in LDS by each
// block (broadcast reads: every lane of a wave reads the same word).  Because
// species indices are data, the per-lane concentration factors Z_k and the
// production rates live in LDS columns owned by the lane ([k][64] per wave,
// conflict-free 8-byte accesses); the state, the RK accumulator and the stage
// input stay in VGPRs with compile-time-bounded loops (NMAX).
//
// Rate evaluation: see mri_dev.h (kappa and Z factorization of
// k_f C_a C_b - k_r C_c C_d, R + S exponentials per RHS), in base 2 with the
// polynomial 2^t of mri_math.h (the host scales the exponent coefficients by
// log2 e when it copies the mechanism to the device).
#include "mri_dev.h"
#include "mri_math.h"

namespace {

struct LdsView {
    const double *sp;
    const double *rx;
    const uint32_t *rxi;
    double *Z;      // [S][64] this wave
    double *Wd;     // [S][64] this wave
};

__device__ __forceinline__ LdsView stage_mechanism(const GenMech &gm)
{
    extern __shared__ double lds[];
    const int S = gm.S, R = gm.R;
    double *sp = lds;
    double *rx = sp + GEN_SP_STRIDE * S;
    uint32_t *rxi = reinterpret_cast<uint32_t *>(rx + 3 * R);
    double *wave_base = rx + 3 * R + (R + 1) / 2;
    for (int i = threadIdx.x; i < GEN_SP_STRIDE * S; i += blockDim.x) sp[i] = gm.sp[i];
    for (int i = threadIdx.x; i < 3 * R; i += blockDim.x) rx[i] = gm.rx[i];
    for (int i = threadIdx.x; i < R; i += blockDim.x) rxi[i] = gm.rxi[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    LdsView v;
    v.sp = sp;
    v.rx = rx;
    v.rxi = rxi;
    v.Z = wave_base + (size_t)wave * 2 * S * 64;
    v.Wd = v.Z + (size_t)S * 64;
    return v;
}

__device__ __forceinline__ void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Species rates (left in Wd, already multiplied by W/rho) and the temperature
// rate for the stage input whose mass fractions the caller stored in the Z
// columns and whose temperature is T.  Z is overwritten with the factors Z_k.
template <int NMAX>
__device__ __forceinline__ double gen_rhs(const LdsView &m, int S, int R, double T_ref, double T,
                                          int lane)
{
    const double invT = 1.0 / T;
    const double l2T = log2(T);
    double den = 0.0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < S) {
            const double *p = m.sp + k * GEN_SP_STRIDE;
            const double Yk = m.Z[k * 64 + lane];
            m.Z[k * 64 + lane] = (Yk * p[0]) * mri_exp2(fma(p[2], invT, p[3]));
            m.Wd[k * 64 + lane] = 0.0;
            den = fma(Yk, p[5], den);
        }
    }
    for (int j = 0; j < R; ++j) {
        const double lna = m.rx[3 * j], be = m.rx[3 * j + 1], th = m.rx[3 * j + 2];
        const uint32_t id = m.rxi[j];
        const int a = (id & 255u) * 64 + lane, b = ((id >> 8) & 255u) * 64 + lane;
        const int c = ((id >> 16) & 255u) * 64 + lane, d = (id >> 24) * 64 + lane;
        const double kap = mri_exp2(fma(-th, invT, fma(be, l2T, lna)));
        const double q = kap * fma(-m.Z[c], m.Z[d], m.Z[a] * m.Z[b]);
        // LDS atomic adds (no return): the four updates need no read-modify-
        // write round trip, so consecutive reactions do not wait on each
        // other; a lane's adds to its own column land in program order, giving
        // the same sums as plain updates.
        lds_add(&m.Wd[a], -q);
        lds_add(&m.Wd[b], -q);
        lds_add(&m.Wd[c], q);
        lds_add(&m.Wd[d], q);
    }
    double num = 0.0;
    const double dT = T - T_ref;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < S) {
            const double *p = m.sp + k * GEN_SP_STRIDE;
            const double w = m.Wd[k * 64 + lane] * p[1];
            m.Wd[k * 64 + lane] = w;
            num = fma(fma(p[5], dT, p[4]), w, num);
        }
    }
    return -num / den;
}

template <int NP>
__device__ __forceinline__ double gen_forcing(const double *__restrict__ rho, size_t plane,
                                              size_t off, double tau)
{
    if (NP == 0) return 0.0;
    double r = rho[(NP - 1) * plane + off];
#pragma unroll
    for (int k = NP - 2; k >= 0; --k) r = fma(r, tau, rho[k * plane + off]);
    return r;
}

template <int NMAX>
__device__ __forceinline__ int gen_flags(const double (&Ys)[NMAX], double T, int S)
{
    double s = T;
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) s += Ys[k];
    int st = 0;
    if (!isfinite(s)) st |= 1;
    if (!(T >= 200.0 && T <= 6000.0)) st |= 4;
    return st;
}

template <int NMAX, int NP>
__global__ void __launch_bounds__(256)
    k_gen_rk4(GenMech gm, ErkCoef e, int n_cells, int ld, const double *__restrict__ yin,
              double *yout, const double *__restrict__ rho, double L, int n_sub, int *status,
              int *steps, int accumulate, const unsigned int *n_live)
{
    const LdsView m = stage_mechanism(gm);
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    // no barrier below this point
    if (cell >= n_cells || (n_live && (unsigned int)cell >= *n_live)) return;
    const int S = gm.S, R = gm.R, lane = threadIdx.x & 63;
    const size_t plane = (size_t)(S + 1) * ld;
    const size_t offT = (size_t)S * ld + cell;
    double y0[NMAX], acc[NMAX];
    double y0T = yin[offT], accT, YcT;
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) y0[k] = yin[(size_t)k * ld + cell];
    const double h = L / n_sub;
    const double inv_nsub = 1.0 / n_sub;
    for (int it = 0; it < n_sub; ++it) {
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < S) {
                acc[k] = 0.0;
                m.Z[k * 64 + lane] = y0[k];
            }
        accT = 0.0;
        YcT = y0T;
#pragma unroll 1
        for (int st = 0; st < e.s; ++st) {
            const double cn = e.c[st], bw = e.b[st], ah = e.a[st] * h;
            const double tau = (it + cn) * inv_nsub;
            const double Tdot = gen_rhs<NMAX>(m, S, R, gm.T_ref, YcT, lane);
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < S) {
                    const double kc =
                        m.Wd[k * 64 + lane] + gen_forcing<NP>(rho, plane, (size_t)k * ld + cell, tau);
                    acc[k] = fma(bw, kc, acc[k]);
                    m.Z[k * 64 + lane] = fma(ah, kc, y0[k]);
                }
            const double kT = Tdot + gen_forcing<NP>(rho, plane, offT, tau);
            accT = fma(bw, kT, accT);
            YcT = fma(ah, kT, y0T);
        }
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < S) y0[k] = fma(h, acc[k], y0[k]);
        y0T = fma(h, accT, y0T);
    }
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) yout[(size_t)k * ld + cell] = y0[k];
    yout[offT] = y0T;
    const int fl = gen_flags<NMAX>(y0, y0T, S);
    if (status) status[cell] = accumulate ? (status[cell] | fl) : fl;
    if (steps) steps[cell] = accumulate ? (steps[cell] + n_sub) : n_sub;
}

// General explicit RK tableau (at most ERK_SMAX stages), n_sub uniform
// substeps: stage st takes y0 + h sum_j a[st][j] k_j.  The stage loop is not
// unrolled (one inlined rate evaluation); the stage derivatives stay in
// registers with static indices: the input sum runs over every stored
// derivative (a[st][j] = 0 for j >= st, and the slots start at zero) and a
// new derivative is written by select.
template <int NMAX, int NP>
__global__ void __launch_bounds__(256)
    k_gen_erk(GenMech gm, ErkFull e, int n_cells, int ld, const double *__restrict__ yin,
              double *yout, const double *__restrict__ rho, double L, int n_sub, int *status,
              int *steps, int accumulate, const unsigned int *n_live)
{
    constexpr int NK = ERK_SMAX - 1;   // derivatives a later stage can read
    const LdsView m = stage_mechanism(gm);
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    // no barrier below this point
    if (cell >= n_cells || (n_live && (unsigned int)cell >= *n_live)) return;
    const int S = gm.S, R = gm.R, lane = threadIdx.x & 63;
    const size_t plane = (size_t)(S + 1) * ld;
    const size_t offT = (size_t)S * ld + cell;
    double y0[NMAX], acc[NMAX], kst[NK][NMAX], kT[NK];
    double y0T = yin[offT], accT;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < S) y0[k] = yin[(size_t)k * ld + cell];
#pragma unroll
        for (int j = 0; j < NK; ++j) kst[j][k] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) kT[j] = 0.0;
    const double h = L / n_sub;
    const double inv_nsub = 1.0 / n_sub;
    for (int it = 0; it < n_sub; ++it) {
#pragma unroll
        for (int k = 0; k < NMAX; ++k) acc[k] = 0.0;
        accT = 0.0;
#pragma unroll 1
        for (int st = 0; st < e.s; ++st) {
            double ah[NK];
#pragma unroll
            for (int j = 0; j < NK; ++j) ah[j] = h * e.a[st][j];
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < S) {
                    double v = y0[k];
#pragma unroll
                    for (int j = 0; j < NK; ++j) v = fma(ah[j], kst[j][k], v);
                    m.Z[k * 64 + lane] = v;
                }
            double YcT = y0T;
#pragma unroll
            for (int j = 0; j < NK; ++j) YcT = fma(ah[j], kT[j], YcT);
            const double bw = e.b[st];
            const double tau = (it + e.c[st]) * inv_nsub;
            const double Tdot = gen_rhs<NMAX>(m, S, R, gm.T_ref, YcT, lane);
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < S) {
                    const double kc =
                        m.Wd[k * 64 + lane] + gen_forcing<NP>(rho, plane, (size_t)k * ld + cell, tau);
                    acc[k] = fma(bw, kc, acc[k]);
#pragma unroll
                    for (int j = 0; j < NK; ++j) kst[j][k] = (j == st) ? kc : kst[j][k];
                }
            const double kc = Tdot + gen_forcing<NP>(rho, plane, offT, tau);
            accT = fma(bw, kc, accT);
#pragma unroll
            for (int j = 0; j < NK; ++j) kT[j] = (j == st) ? kc : kT[j];
        }
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < S) y0[k] = fma(h, acc[k], y0[k]);
        y0T = fma(h, accT, y0T);
    }
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) yout[(size_t)k * ld + cell] = y0[k];
    yout[offT] = y0T;
    const int fl = gen_flags<NMAX>(y0, y0T, S);
    if (status) status[cell] = accumulate ? (status[cell] | fl) : fl;
    if (steps) steps[cell] = accumulate ? (steps[cell] + n_sub) : n_sub;
}

// One attempted Zonneveld 4(3) step (RK4 + stage 5 at c = 3/4, embedded
// third-order estimate); returns the WRMS error, writes the RK4 solution.
template <int NMAX, int NP>
__device__ __forceinline__ double gen_zv_try(const LdsView &m, const GenMech &gm,
                                             const double (&v)[NMAX], double vT,
                                             double (&vn)[NMAX], double &vnT, double t, double h,
                                             double invL, const double *__restrict__ rho,
                                             size_t plane, int ld, int cell, const ZvOpts &o,
                                             int lane)
{
    const int S = gm.S, R = gm.R;
    const size_t offT = (size_t)S * ld + cell;
    double e[NMAX], s5[NMAX];
    double YcT, eT, s5T, solT;
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) {
            m.Z[k * 64 + lane] = v[k];
            vn[k] = 0.0;
            e[k] = 0.0;
            s5[k] = 0.0;
        }
    YcT = vT;
    solT = eT = s5T = 0.0;
#pragma unroll 1
    for (int st = 0; st < 5; ++st) {
        // nodes c = (0, 1/2, 1/2, 1, 3/4); b = (1/6, 1/3, 1/3, 1/6, 0);
        // d = b - bhat = (2/3, -2, -2, -2, 16/3); stage-5 row (5/32, 7/32, 13/32, -1/32)
        const double cs = (st == 0) ? 0.0 : ((st == 3) ? 1.0 : ((st == 4) ? 0.75 : 0.5));
        const double b = (st == 0 || st == 3) ? (1.0 / 6.0) : (1.0 / 3.0);
        const double d = (st == 0) ? (2.0 / 3.0) : ((st == 4) ? (16.0 / 3.0) : -2.0);
        const double r = (st == 0) ? (5.0 / 32.0)
                                   : ((st == 1) ? (7.0 / 32.0)
                                                : ((st == 2) ? (13.0 / 32.0) : (-1.0 / 32.0)));
        const double a = (st == 2) ? 1.0 : 0.5;
        const double tau = (t + cs * h) * invL;
        const double Tdot = gen_rhs<NMAX>(m, S, R, gm.T_ref, YcT, lane);
        const double kT = Tdot + gen_forcing<NP>(rho, plane, offT, tau);
        if (st < 4) {
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < S) {
                    const double kc = m.Wd[k * 64 + lane] +
                                      gen_forcing<NP>(rho, plane, (size_t)k * ld + cell, tau);
                    vn[k] = fma(b, kc, vn[k]);
                    e[k] = fma(d, kc, e[k]);
                    s5[k] = fma(r, kc, s5[k]);
                    m.Z[k * 64 + lane] = (st < 3) ? fma(a * h, kc, v[k]) : fma(h, s5[k], v[k]);
                }
            solT = fma(b, kT, solT);
            eT = fma(d, kT, eT);
            s5T = fma(r, kT, s5T);
            YcT = (st < 3) ? fma(a * h, kT, vT) : fma(h, s5T, vT);
        } else {
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < S) {
                    const double kc = m.Wd[k * 64 + lane] +
                                      gen_forcing<NP>(rho, plane, (size_t)k * ld + cell, tau);
                    e[k] = fma(d, kc, e[k]);
                }
            eT = fma(d, kT, eT);
        }
    }
    double ssq = 0.0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) {
            const double w = (h * e[k]) / (o.atol_Y + o.rtol * fabs(v[k]));
            ssq = fma(w, w, ssq);
            vn[k] = fma(h, vn[k], v[k]);
        }
    {
        const double w = (h * eT) / (o.atol_T + o.rtol * fabs(vT));
        ssq = fma(w, w, ssq);
        vnT = fma(h, solT, vT);
    }
    return sqrt(ssq / (S + 1));
}

template <int NMAX, int NP>
__global__ void __launch_bounds__(256)
    k_gen_zv(GenMech gm, int n_cells, int ld, const double *__restrict__ yin, double *yout,
             const double *__restrict__ rho, double L, ZvOpts o, int *status, int *steps,
             int accumulate, const unsigned int *n_live)
{
    const LdsView m = stage_mechanism(gm);
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells || (n_live && (unsigned int)cell >= *n_live)) return;
    const int S = gm.S, lane = threadIdx.x & 63;
    const size_t plane = (size_t)(S + 1) * ld;
    const size_t offT = (size_t)S * ld + cell;
    double v[NMAX], vn[NMAX];
    double vT = yin[offT], vnT = 0.0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) v[k] = yin[(size_t)k * ld + cell];
    const double hmax = L / 10.0, invL = 1.0 / L;
    double h = hmax, t = 0.0;
    int acc = 0, rej = 0, fl = 0;
    const int max_attempts = 4 * o.max_steps;
    while (true) {
        if (acc >= o.max_steps || acc + rej >= max_attempts) {
            fl |= 2;
            break;
        }
        double hs = fmin(h, hmax);
        bool last = false;
        if (t + hs >= L - 1e-12 * L) {
            hs = L - t;
            last = true;
        }
        double err = gen_zv_try<NMAX, NP>(m, gm, v, vT, vn, vnT, t, hs, invL, rho, plane, ld,
                                          cell, o, lane);
        if (!isfinite(err)) err = HUGE_VAL;
        if (fabs(err - 1.0) < 1e-12) fl |= 8;
        double fac = (err == 0.0) ? 5.0 : 0.9 * pow(err, -0.25);
        fac = fmin(5.0, fmax(0.2, fac));
        if (err <= 1.0) {
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < S) v[k] = vn[k];
            vT = vnT;
            t = last ? L : t + hs;
            ++acc;
            if (last) break;
        } else {
            ++rej;
        }
        h = hs * fac;
    }
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < S) yout[(size_t)k * ld + cell] = v[k];
    yout[offT] = vT;
    fl |= gen_flags<NMAX>(v, vT, S);
    if (status) status[cell] = accumulate ? (status[cell] | fl) : fl;
    if (steps) steps[cell] = accumulate ? (steps[cell] + acc) : acc;
}

// ---------------------------------------------------------------------------
// Linear test mode f = A v (n <= 16): RK4 with the same stage structure.
// ---------------------------------------------------------------------------
// Linear test mode with a general tableau (n <= 16 components), organised
// like k_gen_erk.
template <int NP>
__global__ void __launch_bounds__(256)
    k_lin_erk(int n, const double *__restrict__ A, ErkFull e, int n_cells, int ld,
              const double *__restrict__ yin, double *yout, const double *__restrict__ rho,
              double L, int n_sub, int *status, int *steps, int accumulate)
{
    constexpr int NM = 16, NK = ERK_SMAX - 1;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells) return;
    const size_t plane = (size_t)n * ld;
    double y0[NM], acc[NM], Yc[NM], kst[NK][NM];
#pragma unroll
    for (int c = 0; c < NM; ++c) {
        if (c < n) y0[c] = yin[(size_t)c * ld + cell];
#pragma unroll
        for (int j = 0; j < NK; ++j) kst[j][c] = 0.0;
    }
    const double h = L / n_sub, inv_nsub = 1.0 / n_sub;
    for (int it = 0; it < n_sub; ++it) {
#pragma unroll
        for (int c = 0; c < NM; ++c) acc[c] = 0.0;
#pragma unroll 1
        for (int st = 0; st < e.s; ++st) {
            double ah[NK];
#pragma unroll
            for (int j = 0; j < NK; ++j) ah[j] = h * e.a[st][j];
#pragma unroll
            for (int c = 0; c < NM; ++c)
                if (c < n) {
                    double v = y0[c];
#pragma unroll
                    for (int j = 0; j < NK; ++j) v = fma(ah[j], kst[j][c], v);
                    Yc[c] = v;
                }
            const double bw = e.b[st];
            const double tau = (it + e.c[st]) * inv_nsub;
#pragma unroll
            for (int r = 0; r < NM; ++r)
                if (r < n) {
                    double s = 0.0;
#pragma unroll
                    for (int c = 0; c < NM; ++c)
                        if (c < n) s = fma(A[r * n + c], Yc[c], s);
                    const double kc = s + gen_forcing<NP>(rho, plane, (size_t)r * ld + cell, tau);
                    acc[r] = fma(bw, kc, acc[r]);
#pragma unroll
                    for (int j = 0; j < NK; ++j) kst[j][r] = (j == st) ? kc : kst[j][r];
                }
        }
#pragma unroll
        for (int c = 0; c < NM; ++c)
            if (c < n) y0[c] = fma(h, acc[c], y0[c]);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NM; ++c)
        if (c < n) {
            yout[(size_t)c * ld + cell] = y0[c];
            s += y0[c];
        }
    const int fl = isfinite(s) ? 0 : 1;
    if (status) status[cell] = accumulate ? (status[cell] | fl) : fl;
    if (steps) steps[cell] = accumulate ? (steps[cell] + n_sub) : n_sub;
}

template <int NP>
__global__ void __launch_bounds__(256)
    k_lin_rk4(int n, const double *__restrict__ A, ErkCoef e, int n_cells, int ld,
              const double *__restrict__ yin, double *yout, const double *__restrict__ rho,
              double L, int n_sub, int *status, int *steps, int accumulate)
{
    constexpr int NM = 16;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells) return;
    const size_t plane = (size_t)n * ld;
    double y0[NM], acc[NM], Yc[NM], f[NM];
#pragma unroll
    for (int c = 0; c < NM; ++c)
        if (c < n) y0[c] = yin[(size_t)c * ld + cell];
    const double h = L / n_sub, inv_nsub = 1.0 / n_sub;
    for (int it = 0; it < n_sub; ++it) {
#pragma unroll
        for (int c = 0; c < NM; ++c)
            if (c < n) {
                acc[c] = 0.0;
                Yc[c] = y0[c];
            }
#pragma unroll 1
        for (int st = 0; st < e.s; ++st) {
            const double cn = e.c[st], bw = e.b[st], ah = e.a[st] * h;
            const double tau = (it + cn) * inv_nsub;
#pragma unroll
            for (int r = 0; r < NM; ++r)
                if (r < n) {
                    double s = 0.0;
#pragma unroll
                    for (int c = 0; c < NM; ++c)
                        if (c < n) s = fma(A[r * n + c], Yc[c], s);
                    f[r] = s;
                }
#pragma unroll
            for (int c = 0; c < NM; ++c)
                if (c < n) {
                    const double kc = f[c] + gen_forcing<NP>(rho, plane, (size_t)c * ld + cell, tau);
                    acc[c] = fma(bw, kc, acc[c]);
                    Yc[c] = fma(ah, kc, y0[c]);
                }
        }
#pragma unroll
        for (int c = 0; c < NM; ++c)
            if (c < n) y0[c] = fma(h, acc[c], y0[c]);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NM; ++c)
        if (c < n) {
            yout[(size_t)c * ld + cell] = y0[c];
            s += y0[c];
        }
    const int fl = isfinite(s) ? 0 : 1;
    if (status) status[cell] = accumulate ? (status[cell] | fl) : fl;
    if (steps) steps[cell] = accumulate ? (steps[cell] + n_sub) : n_sub;
}

// Stiffness monitor: B = max_k sum_j |nu_kj| w_j with w_j = kf (C_a + C_b) +
// kr (C_c + C_d), an upper bound of the spectral radius of the species block of
// the chemistry Jacobian at fixed T (Gershgorin in concentration variables, a
// similarity transform of the mass-fraction variables).  With E_k = e^(g_k/RT)
// and Z_k = C_k E_k: kf = kappa E_a E_b and kr = kappa E_c E_d, so
// w_j = kappa (Z_a E_b + Z_b E_a + Z_c E_d + Z_d E_c).  Per lane three LDS
// columns (Z, E, B) after the block's copy of the mechanism.
__global__ void __launch_bounds__(64)
    k_gen_stiff(GenMech gm, int n_cells, int ld, const double *__restrict__ y, double h,
                double limit, double *__restrict__ bound, int *__restrict__ status,
                int *__restrict__ steps, int accumulate, int flag)
{
    const LdsView m = stage_mechanism(gm);
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n_cells) return;     // no barrier below this point
    const int S = gm.S, R = gm.R, lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    double *Z = m.Z, *E = m.Wd;
    // the third column set follows the two of every wave
    double *B = m.Z + (size_t)(n_waves - wave) * 2 * S * 64 + (size_t)wave * S * 64;
    const double T = y[(size_t)S * ld + cell];
    const double invT = 1.0 / T;
    const double l2T = log2(T);
    for (int k = 0; k < S; ++k) {
        const double *p = m.sp + k * GEN_SP_STRIDE;
        const double e = mri_exp2(fma(p[2], invT, p[3]));
        E[k * 64 + lane] = e;
        Z[k * 64 + lane] = (y[(size_t)k * ld + cell] * p[0]) * e;
        B[k * 64 + lane] = 0.0;
    }
    for (int j = 0; j < R; ++j) {
        const double lna = m.rx[3 * j], be = m.rx[3 * j + 1], th = m.rx[3 * j + 2];
        const uint32_t id = m.rxi[j];
        const int a = (id & 255u) * 64 + lane, b = ((id >> 8) & 255u) * 64 + lane;
        const int c = ((id >> 16) & 255u) * 64 + lane, d = (id >> 24) * 64 + lane;
        const double kap = mri_exp2(fma(-th, invT, fma(be, l2T, lna)));
        const double w = kap * (fma(Z[a], E[b], Z[b] * E[a]) + fma(Z[c], E[d], Z[d] * E[c]));
        B[a] += w;
        B[b] += w;
        B[c] += w;
        B[d] += w;
    }
    double bmax = 0.0;
    for (int k = 0; k < S; ++k) bmax = fmax(bmax, B[k * 64 + lane]);
    if (bound) bound[cell] = bmax;
    const int st = (h * bmax <= limit) ? 0 : flag;
    if (status) status[cell] = accumulate ? (status[cell] | st) : st;
    if (steps && !accumulate) steps[cell] = 0;
}

}  // namespace

size_t gen_lds_bytes(int S, int R, int block)
{
    const size_t mech = sizeof(double) * (GEN_SP_STRIDE * S + 3 * R + (R + 1) / 2);
    const size_t per_wave = sizeof(double) * 2 * S * 64;
    return mech + per_wave * ((block + 63) / 64);
}

#define GEN_DISPATCH_NP(KERNEL, NMAX, ...)                                                   \
    switch (n_poly) {                                                                      \
    case 0: hipLaunchKernelGGL((KERNEL<NMAX, 0>), grid, dim3(block), lds, s, __VA_ARGS__); \
        break;                                                                             \
    case 1: hipLaunchKernelGGL((KERNEL<NMAX, 1>), grid, dim3(block), lds, s, __VA_ARGS__); \
        break;                                                                             \
    case 2: hipLaunchKernelGGL((KERNEL<NMAX, 2>), grid, dim3(block), lds, s, __VA_ARGS__); \
        break;                                                                             \
    case 3: hipLaunchKernelGGL((KERNEL<NMAX, 3>), grid, dim3(block), lds, s, __VA_ARGS__); \
        break;                                                                             \
    default: hipLaunchKernelGGL((KERNEL<NMAX, 4>), grid, dim3(block), lds, s, __VA_ARGS__); \
        break;                                                                             \
    }

hipError_t launch_gen_rk4(const GenMech &gm, const ErkCoef &e, int block, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          const unsigned int *n_live, hipStream_t s)
{
    const dim3 grid((unsigned)(((long long)n_cells + block - 1) / block));
    const size_t lds = gen_lds_bytes(gm.S, gm.R, block);
    if (gm.S <= GEN_NMAX_SMALL) {
        GEN_DISPATCH_NP(k_gen_rk4, GEN_NMAX_SMALL, gm, e, n_cells, ld, yin, yout, rho, L, n_sub,
                        status, steps, accumulate, n_live)
    } else {
        GEN_DISPATCH_NP(k_gen_rk4, GEN_NMAX_LARGE, gm, e, n_cells, ld, yin, yout, rho, L, n_sub,
                        status, steps, accumulate, n_live)
    }
    return hipGetLastError();
}

hipError_t launch_gen_zv(const GenMech &gm, int block, int n_cells, int ld, const double *yin,
                         double *yout, int n_poly, const double *rho, double L, ZvOpts o,
                         int *status, int *steps, int accumulate, const unsigned int *n_live,
                         hipStream_t s)
{
    const dim3 grid((unsigned)(((long long)n_cells + block - 1) / block));
    const size_t lds = gen_lds_bytes(gm.S, gm.R, block);
    if (gm.S <= GEN_NMAX_SMALL) {
        GEN_DISPATCH_NP(k_gen_zv, GEN_NMAX_SMALL, gm, n_cells, ld, yin, yout, rho, L, o, status,
                        steps, accumulate, n_live)
    } else {
        GEN_DISPATCH_NP(k_gen_zv, GEN_NMAX_LARGE, gm, n_cells, ld, yin, yout, rho, L, o, status,
                        steps, accumulate, n_live)
    }
    return hipGetLastError();
}

hipError_t launch_gen_erk(const GenMech &gm, const ErkFull &e, int block, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          const unsigned int *n_live, hipStream_t s)
{
    const dim3 grid((unsigned)(((long long)n_cells + block - 1) / block));
    if (gm.S > GEN_NMAX_SMALL || e.s < 1 || e.s > ERK_SMAX) return hipErrorInvalidValue;
    const size_t lds = gen_lds_bytes(gm.S, gm.R, block);
    GEN_DISPATCH_NP(k_gen_erk, GEN_NMAX_SMALL, gm, e, n_cells, ld, yin, yout, rho, L, n_sub,
                    status, steps, accumulate, n_live)
    return hipGetLastError();
}

hipError_t launch_lin_erk(int n, const double *A, const ErkFull &e, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          hipStream_t s)
{
    if (n > 16 || e.s < 1 || e.s > ERK_SMAX) return hipErrorInvalidValue;
    const int block = 256;
    const dim3 grid((unsigned)(((long long)n_cells + block - 1) / block));
    switch (n_poly) {
    case 0:
        hipLaunchKernelGGL(k_lin_erk<0>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    case 1:
        hipLaunchKernelGGL(k_lin_erk<1>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    case 2:
        hipLaunchKernelGGL(k_lin_erk<2>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    case 3:
        hipLaunchKernelGGL(k_lin_erk<3>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    default:
        hipLaunchKernelGGL(k_lin_erk<4>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_lin_rk4(int n, const double *A, const ErkCoef &e, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          hipStream_t s)
{
    const int block = 256;
    const dim3 grid((unsigned)(((long long)n_cells + block - 1) / block));
    switch (n_poly) {
    case 0:
        hipLaunchKernelGGL(k_lin_rk4<0>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    case 1:
        hipLaunchKernelGGL(k_lin_rk4<1>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    case 2:
        hipLaunchKernelGGL(k_lin_rk4<2>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    case 3:
        hipLaunchKernelGGL(k_lin_rk4<3>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    default:
        hipLaunchKernelGGL(k_lin_rk4<4>, grid, dim3(block), 0, s, n, A, e, n_cells, ld, yin, yout,
                           rho, L, n_sub, status, steps, accumulate);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_gen_stiff(const GenMech &gm, int n_cells, int ld, const double *y, double h,
                            double limit, double *bound, int *status, int *steps, int accumulate,
                            int flag, hipStream_t s)
{
    const int block = 64;
    const dim3 grid((unsigned)(((long long)n_cells + block - 1) / block));
    const size_t lds = gen_lds_bytes(gm.S, gm.R, block) + sizeof(double) * gm.S * 64;
    hipLaunchKernelGGL(k_gen_stiff, grid, dim3(block), lds, s, gm, n_cells, ld, y, h, limit,
                       bound, status, steps, accumulate, flag);
    return hipGetLastError();
}
