/*
 * mlp_oracle.c -- plain CPU reference of the surrogate MLP (forward, MSE loss
 * gradient, backward).  TEST INFRASTRUCTURE ONLY; shares nothing with the GPU
 * path.
 *
 * Network: x -> z_1 = W_1 x + b_1 -> a_1 = silu(z_1) -> ... -> z_L = W_L a_(L-1) + b_L
 * (no activation on the last layer), silu(z) = z / (1 + exp(-z)).  W_l is stored
 * [out][in] row-major; params are packed W_1, b_1, W_2, b_2, ...
 *
 * Precision modes: `mode` is a set of rounding points (ORA_R_* bits below).
 *   mode = 0: everything in FP64.
 *   mode = ORA_R_ALL: the GPU's rounding points -- the network input, every
 *             weight and every hidden activation are rounded to bfloat16 (round
 *             to nearest even), each pre-activation is accumulated (here in
 *             FP64) and rounded to FP32, the bias is rounded to FP32 and added in
 *             FP32; the backward pass rounds the output-error signal and every
 *             propagated error to bfloat16 before it enters a product, with FP32
 *             results.
 * Single bits switch single rounding points off, which the tests use to show
 * that each of them is visible in a hand-computed case.
 *
 * The surrogate functions further down (features, inference, gate) restate
 * the learned fast-stage surrogate: an MLP that predicts the correction of a
 * coarse FP64 fast-stage solve (the stage solve of the MRI algorithm, Sec. 2.1
 * step 2b), checked by the disagreement of two independently trained networks
 * and the mass-sum invariant, with the plain FP64 stage as fallback.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Round a float to the nearest bfloat16 (ties to even), returned as float. */
float ora_bf16_round(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) { /* inf / nan: keep, quiet nan */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

void ora_bf16_round_array(const float *x, float *y, int n)
{
    for (int i = 0; i < n; ++i) y[i] = ora_bf16_round(x[i]);
}

static double silu(double z) { return z / (1.0 + exp(-z)); }

static double silu_grad(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

static size_t param_count(int n_layers, const int *w)
{
    size_t n = 0;
    for (int l = 0; l < n_layers; ++l) n += (size_t)w[l + 1] * w[l] + w[l + 1];
    return n;
}

#define ORA_R_INPUT 1   /* network input to bfloat16 */
#define ORA_R_WEIGHT 2  /* weights to bfloat16 */
#define ORA_R_ACC 4     /* accumulated products to FP32 (forward and backward) */
#define ORA_R_BIAS 8    /* bias to FP32 */
#define ORA_R_SUM 16    /* accumulator + bias to FP32 */
#define ORA_R_ACT 32    /* SiLU (and its derivative) to FP32, activations to bfloat16 */
#define ORA_R_GRAD 64   /* backward error signals to bfloat16 */
#define ORA_R_ALL 127

static double q(double v, int on) { return on ? (double)ora_bf16_round((float)v) : v; }
static double f32(double v, int on) { return on ? (double)(float)v : v; }

/*
 * Forward pass for a batch.  X [batch][w_0], Y [batch][w_L].  Z (nullable)
 * receives all pre-activations [l][batch][w_(l+1)] concatenated, A (nullable)
 * all hidden activations after rounding [l][batch][w_(l+1)] for l < L-1.
 */
void ora_mlp_forward(int n_layers, const int *w, const double *params, int batch,
                     const double *X, double *Y, double *Z, double *A, int mode)
{
    const int rin = mode & ORA_R_INPUT, rw = mode & ORA_R_WEIGHT, racc = mode & ORA_R_ACC;
    const int rb = mode & ORA_R_BIAS, rs = mode & ORA_R_SUM, ract = mode & ORA_R_ACT;
    int wmax = 0;
    for (int l = 0; l <= n_layers; ++l)
        if (w[l] > wmax) wmax = w[l];
    double *in = (double *)malloc(sizeof(double) * wmax);
    double *out = (double *)malloc(sizeof(double) * wmax);
    for (int r = 0; r < batch; ++r) {
        for (int i = 0; i < w[0]; ++i) in[i] = q(X[(size_t)r * w[0] + i], rin);
        const double *p = params;
        size_t zoff = 0, aoff = 0;
        for (int l = 0; l < n_layers; ++l) {
            const int ni = w[l], no = w[l + 1];
            const double *W = p, *b = p + (size_t)no * ni;
            for (int o = 0; o < no; ++o) {
                double acc = 0.0;
                for (int i = 0; i < ni; ++i) acc += q(W[(size_t)o * ni + i], rw) * in[i];
                double z = f32(f32(acc, racc) + f32(b[o], rb), rs);
                if (Z) Z[zoff + (size_t)r * no + o] = z;
                if (l < n_layers - 1) {
                    out[o] = q(f32(silu(z), ract), ract);
                    if (A) A[aoff + (size_t)r * no + o] = out[o];
                } else {
                    Y[(size_t)r * no + o] = z;
                }
            }
            zoff += (size_t)batch * no;
            if (l < n_layers - 1) aoff += (size_t)batch * no;
            memcpy(in, out, sizeof(double) * no);
            p += (size_t)no * ni + no;
        }
    }
    free(in);
    free(out);
}

/*
 * Loss = (1 / (batch * w_L)) sum (Y - T)^2 and its gradient with respect to
 * every parameter (packed like params).  Returns the loss.
 */
double ora_mlp_loss_grad(int n_layers, const int *w, const double *params, int batch,
                         const double *X, const double *T, double *grad, int mode)
{
    const int rin = mode & ORA_R_INPUT, rw = mode & ORA_R_WEIGHT, racc = mode & ORA_R_ACC;
    const int ract = mode & ORA_R_ACT, rg = mode & ORA_R_GRAD;
    const int L = n_layers, wo = w[L];
    size_t zsize = 0, asize = 0;
    for (int l = 0; l < L; ++l) {
        zsize += (size_t)batch * w[l + 1];
        if (l < L - 1) asize += (size_t)batch * w[l + 1];
    }
    double *Z = (double *)malloc(sizeof(double) * zsize);
    double *A = (double *)malloc(sizeof(double) * (asize ? asize : 1));
    double *Y = (double *)malloc(sizeof(double) * (size_t)batch * wo);
    ora_mlp_forward(L, w, params, batch, X, Y, Z, A, mode);
    size_t np = param_count(L, w);
    memset(grad, 0, sizeof(double) * np);
    double loss = 0.0;
    const double scale = 1.0 / ((double)batch * wo);
    /* offsets of each layer's parameters, pre-activations and activations */
    size_t *poff = (size_t *)malloc(sizeof(size_t) * L);
    size_t *zoff = (size_t *)malloc(sizeof(size_t) * L);
    size_t *aoff = (size_t *)malloc(sizeof(size_t) * L);
    size_t pp = 0, zz = 0, aa = 0;
    for (int l = 0; l < L; ++l) {
        poff[l] = pp;
        zoff[l] = zz;
        aoff[l] = aa;
        pp += (size_t)w[l + 1] * w[l] + w[l + 1];
        zz += (size_t)batch * w[l + 1];
        if (l < L - 1) aa += (size_t)batch * w[l + 1];
    }
    int wmax = 0;
    for (int l = 0; l <= L; ++l)
        if (w[l] > wmax) wmax = w[l];
    double *dz = (double *)malloc(sizeof(double) * wmax);
    double *dzq = (double *)malloc(sizeof(double) * wmax);
    double *da = (double *)malloc(sizeof(double) * wmax);
    double *xin = (double *)malloc(sizeof(double) * wmax);
    for (int r = 0; r < batch; ++r) {
        for (int o = 0; o < wo; ++o) {
            double e = Y[(size_t)r * wo + o] - T[(size_t)r * wo + o];
            loss += e * e * scale;
            dz[o] = f32(2.0 * e * scale, racc);
        }
        for (int l = L - 1; l >= 0; --l) {
            const int ni = w[l], no = w[l + 1];
            const double *W = params + poff[l];
            double *gW = grad + poff[l], *gb = grad + poff[l] + (size_t)no * ni;
            /* input of this layer */
            for (int i = 0; i < ni; ++i)
                xin[i] = (l == 0) ? q(X[(size_t)r * ni + i], rin) : A[aoff[l - 1] + (size_t)r * ni + i];
            for (int o = 0; o < no; ++o) dzq[o] = q(dz[o], rg);
            for (int o = 0; o < no; ++o) {
                gb[o] += dz[o];
                for (int i = 0; i < ni; ++i) gW[(size_t)o * ni + i] += dzq[o] * xin[i];
            }
            if (l > 0) {
                for (int i = 0; i < ni; ++i) {
                    double acc = 0.0;
                    for (int o = 0; o < no; ++o) acc += dzq[o] * q(W[(size_t)o * ni + i], rw);
                    da[i] = f32(acc, racc);
                }
                for (int i = 0; i < ni; ++i)
                    dz[i] = f32(da[i] * f32(silu_grad(Z[zoff[l - 1] + (size_t)r * ni + i]), ract),
                                racc);
            }
        }
    }
    free(Z);
    free(A);
    free(Y);
    free(poff);
    free(zoff);
    free(aoff);
    free(dz);
    free(dzq);
    free(da);
    free(xin);
    return loss;
}

double ora_silu(double z) { return silu(z); }
double ora_silu_grad(double z) { return silu_grad(z); }

/* ------------------------------------------------------------------------- */
/* Learned fast-stage surrogate.  State of a cell: n = S + 1 components, the  */
/* mass fractions Y_0..Y_(S-1) then T.  Arrays are SoA with leading dimension */
/* ld: Y[c*ld + i]; forcing RHO[(p*n + c)*ld + i], p < n_poly <= 3, the       */
/* coefficients of r(tau) = sum_p tau^p rho_p on the normalized stage time.   */
/* ------------------------------------------------------------------------- */
#define SUR_YFLOOR 1e-30   /* floor of the logarithm of a mass fraction feature */
#define SUR_EPS 1e-8       /* offset of the logarithmic targets (the error floor) */

/* Number of raw features: S log mass fractions, T, 3 n forcing coefficients
   (zero-padded beyond n_poly), log L. */
int ora_sur_n_features(int S) { return S + 1 + 3 * (S + 1) + 1; }

/* Raw features of cell i: log max(Y_k, 1e-30), T, rho_(p,c), log L. */
static void sur_raw_features(int S, long ld, long i, const double *Y, int n_poly,
                             const double *RHO, double L, double *f)
{
    const int n = S + 1;
    for (int k = 0; k < S; ++k) {
        const double y = Y[(size_t)k * ld + i];
        f[k] = log(y > SUR_YFLOOR ? y : SUR_YFLOOR);
    }
    f[S] = Y[(size_t)S * ld + i];
    for (int p = 0; p < 3; ++p)
        for (int c = 0; c < n; ++c)
            f[S + 1 + p * n + c] = (p < n_poly) ? RHO[((size_t)p * n + c) * ld + i] : 0.0;
    f[S + 1 + 3 * n] = log(L);
}

/* Raw target of component c: the correction from the base state yb to the
   state y1, in log(Y + 1e-8) for a mass fraction (negative values clamped to
   0) and plain for T. */
static double sur_raw_target(int S, int c, double yb, double y1)
{
    if (c == S) return y1 - yb;
    return log((y1 > 0.0 ? y1 : 0.0) + SUR_EPS) - log((yb > 0.0 ? yb : 0.0) + SUR_EPS);
}

/* Inverse of sur_raw_target: the state from the base state and a correction. */
static double sur_apply(int S, int c, double yb, double d)
{
    if (c == S) return yb + d;
    return ((yb > 0.0 ? yb : 0.0) + SUR_EPS) * exp(d) - SUR_EPS;
}

/* Mean and standard deviation of N values (two passes); the inverse standard
   deviation is 1 for a feature that is constant (sd <= 1e-30 max(1, |mean|)). */
static void sur_moments(const double *x, long N, double *mean, double *sd)
{
    double s = 0.0;
    for (long i = 0; i < N; ++i) s += x[i];
    const double m = s / (double)N;
    double v = 0.0;
    for (long i = 0; i < N; ++i) v += (x[i] - m) * (x[i] - m);
    *mean = m;
    *sd = sqrt(v / (double)N);
}

/*
 * Standardization statistics of N samples: stats = [x_mean (F), x_inv_std (F),
 * y_mean (n), y_inv_std (n), y_std (n)] with F = ora_sur_n_features(S); the
 * targets are the corrections from Yb (NULL: Y0) to Y1; Lv[i] is sample i's
 * stage length.
 */
void ora_sur_stats(int S, long N, long ld, const double *Y0, int n_poly, const double *RHO,
                   const double *Lv, const double *Yb, const double *Y1, double *stats)
{
    const int n = S + 1, F = ora_sur_n_features(S);
    double *col = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *f = (double *)malloc(sizeof(double) * (size_t)F);
    if (!Yb) Yb = Y0;
    for (int k = 0; k < F; ++k) {
        for (long i = 0; i < N; ++i) {
            sur_raw_features(S, ld, i, Y0, n_poly, RHO, Lv[i], f);
            col[i] = f[k];
        }
        double m, sd;
        sur_moments(col, N, &m, &sd);
        stats[k] = m;
        stats[F + k] = (sd > 1e-30 * (fabs(m) > 1.0 ? fabs(m) : 1.0)) ? 1.0 / sd : 1.0;
    }
    for (int c = 0; c < n; ++c) {
        for (long i = 0; i < N; ++i)
            col[i] = sur_raw_target(S, c, Yb[(size_t)c * ld + i], Y1[(size_t)c * ld + i]);
        double m, sd;
        sur_moments(col, N, &m, &sd);
        stats[2 * F + c] = m;
        stats[2 * F + n + c] = (sd > 1e-30 * (fabs(m) > 1.0 ? fabs(m) : 1.0)) ? 1.0 / sd : 1.0;
        stats[2 * F + 2 * n + c] = (sd > 0.0) ? sd : 1.0;
    }
    free(col);
    free(f);
}

/* Standardized feature rows X [N][kpad] (columns beyond F are zero) and, when
   T is not NULL, standardized targets T [N][n] (corrections from Yb, NULL: Y0,
   to Y1). */
void ora_sur_featurize(int S, long N, long ld, const double *Y0, int n_poly, const double *RHO,
                       const double *Lv, const double *Yb, const double *Y1,
                       const double *stats, int kpad, double *X, double *T)
{
    const int n = S + 1, F = ora_sur_n_features(S);
    double *f = (double *)malloc(sizeof(double) * (size_t)F);
    if (!Yb) Yb = Y0;
    for (long i = 0; i < N; ++i) {
        sur_raw_features(S, ld, i, Y0, n_poly, RHO, Lv[i], f);
        for (int k = 0; k < kpad; ++k)
            X[(size_t)i * kpad + k] = (k < F) ? (f[k] - stats[k]) * stats[F + k] : 0.0;
        if (T)
            for (int c = 0; c < n; ++c)
                T[(size_t)i * n + c] =
                    (sur_raw_target(S, c, Yb[(size_t)c * ld + i], Y1[(size_t)c * ld + i]) -
                     stats[2 * F + c]) * stats[2 * F + n + c];
    }
    free(f);
}

/*
 * Inference on N cells: the network (widths[0] >= F inputs, the padding
 * columns zero; widths[n_layers] = n outputs) maps the standardized features
 * of (Y, RHO, L) to a standardized correction z; d = y_mean + y_std z is
 * applied to the base state B (NULL: Y): OUT[c*ld + i] = apply(B, d).  `mode`
 * selects the rounding points of the network (ORA_R_*); the features are
 * rounded to FP32 before the network's own input rounding, as the device
 * does.  Z (nullable) receives z [N][n].
 */
void ora_sur_infer(int S, long N, long ld, const double *Y, int n_poly, const double *RHO,
                   double L, const double *B, int n_layers, const int *widths,
                   const double *params, const double *stats, int mode, double *OUT, double *Z)
{
    const int n = S + 1, F = ora_sur_n_features(S), kin = widths[0];
    if (!B) B = Y;
    /* cells are independent; the threads only shorten the CPU timing */
#pragma omp parallel
    {
        double *f = (double *)malloc(sizeof(double) * (size_t)F);
        double *x = (double *)malloc(sizeof(double) * (size_t)kin);
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic, 64)
        for (long i = 0; i < N; ++i) {
            sur_raw_features(S, ld, i, Y, n_poly, RHO, L, f);
            for (int k = 0; k < kin; ++k)
                x[k] = (k < F) ? f32((f[k] - stats[k]) * stats[F + k], mode & ORA_R_INPUT) : 0.0;
            ora_mlp_forward(n_layers, widths, params, 1, x, z, NULL, NULL, mode);
            for (int c = 0; c < n; ++c) {
                const double d = stats[2 * F + c] + stats[2 * F + 2 * n + c] * z[c];
                OUT[(size_t)c * ld + i] = sur_apply(S, c, B[(size_t)c * ld + i], d);
                if (Z) Z[(size_t)i * n + c] = z[c];
            }
        }
        free(f);
        free(x);
        free(z);
    }
}

/*
 * The surrogate's residual check on N cells.  Vc: the coarse FP64 stage
 * (n_sub substeps), Vh: the same with half the substeps, Vn: the network's
 * correction of Vc.  The Richardson extrapolation Ve = Vc + rich (Vc - Vh),
 * rich = 1 / (2^p - 1) for a fast method of order p, estimates the fine stage
 * from FP64 work alone; the check is
 *   G = max(D, I),  D = max_c |Vn_c - Ve_c| / max(|Ve_c|, floor_c)
 * (floor 1e-8 for mass fractions, 0 for T), I = the residual of the mass-sum
 * invariant of Vn: |sum_k (Vn_k - Y0_k) - L sum_p sum_k rho_(p,k) / (p + 1)|
 * / sum_k |Y0_k| (the chemistry conserves sum_k Y_k, so over the stage the sum
 * changes only by the integral of the forcing).  A cell is accepted when
 * G <= tol (a NaN never is) and its coarse status (nullable) is 0.
 */
void ora_sur_gate(int S, long N, long ld, const double *Y0, int n_poly, const double *RHO,
                  double L, const double *Vc, const double *Vh, const double *Vn,
                  const int *status_c, double rich, double tol, double *G, int *accept)
{
    const int n = S + 1;
    for (long i = 0; i < N; ++i) {
        double D = 0.0;
        int nan = 0;
        for (int c = 0; c < n; ++c) {
            const double vc = Vc[(size_t)c * ld + i], vh = Vh[(size_t)c * ld + i];
            const double ve = vc + rich * (vc - vh);
            const double fl = (c < S) ? 1e-8 : 0.0;
            const double den = fabs(ve) > fl ? fabs(ve) : fl;
            const double e = fabs(Vn[(size_t)c * ld + i] - ve) / den;
            if (e != e) nan = 1;
            else if (e > D) D = e;
        }
        double dsum = 0.0, y0sum = 0.0, fsum = 0.0;
        for (int k = 0; k < S; ++k) {
            dsum += Vn[(size_t)k * ld + i] - Y0[(size_t)k * ld + i];
            y0sum += fabs(Y0[(size_t)k * ld + i]);
            for (int p = 0; p < n_poly; ++p) fsum += RHO[((size_t)p * n + k) * ld + i] / (p + 1);
        }
        const double I = fabs(dsum - L * fsum) / (y0sum > 1e-300 ? y0sum : 1e-300);
        if (I != I) nan = 1;
        const double g = nan ? NAN : (I > D ? I : D);
        G[i] = g;
        accept[i] = (!nan && g <= tol && !(status_c && status_c[i])) ? 1 : 0;
    }
}
