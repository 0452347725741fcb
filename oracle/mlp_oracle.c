/*
 * mlp_oracle.c -- plain CPU reference of the surrogate MLP (forward, MSE loss
 * gradient, backward).  TEST INFRASTRUCTURE ONLY; shares nothing with the GPU
 * path.
 *
 * Network: x -> z_1 = W_1 x + b_1 -> a_1 = silu(z_1) -> ... -> z_L = W_L a_(L-1) + b_L
 * (no activation on the last layer), silu(z) = z / (1 + exp(-z)).  W_l is stored
 * [out][in] row-major; params are packed W_1, b_1, W_2, b_2, ...
 *
 * Two modes:
 *   bf16 = 0: everything in FP64.
 *   bf16 = 1: the GPU's rounding points -- the network input, every weight and
 *             every hidden activation are rounded to bfloat16 (round to nearest
 *             even), each pre-activation is accumulated (here in FP64) and rounded
 *             to FP32 before the bias is added in FP32; the backward pass rounds
 *             the output-error signal and every propagated error to bfloat16
 *             before it enters a product, with FP32 results.
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

static double q(double v, int bf16) { return bf16 ? (double)ora_bf16_round((float)v) : v; }
static double f32(double v, int bf16) { return bf16 ? (double)(float)v : v; }

/*
 * Forward pass for a batch.  X [batch][w_0], Y [batch][w_L].  Z (nullable)
 * receives all pre-activations [l][batch][w_(l+1)] concatenated, A (nullable)
 * all hidden activations after rounding [l][batch][w_(l+1)] for l < L-1.
 */
void ora_mlp_forward(int n_layers, const int *w, const double *params, int batch,
                     const double *X, double *Y, double *Z, double *A, int bf16)
{
    int wmax = 0;
    for (int l = 0; l <= n_layers; ++l)
        if (w[l] > wmax) wmax = w[l];
    double *in = (double *)malloc(sizeof(double) * wmax);
    double *out = (double *)malloc(sizeof(double) * wmax);
    for (int r = 0; r < batch; ++r) {
        for (int i = 0; i < w[0]; ++i) in[i] = q(X[(size_t)r * w[0] + i], bf16);
        const double *p = params;
        size_t zoff = 0, aoff = 0;
        for (int l = 0; l < n_layers; ++l) {
            const int ni = w[l], no = w[l + 1];
            const double *W = p, *b = p + (size_t)no * ni;
            for (int o = 0; o < no; ++o) {
                double acc = 0.0;
                for (int i = 0; i < ni; ++i) acc += q(W[(size_t)o * ni + i], bf16) * in[i];
                double z = f32(f32(acc, bf16) + f32(b[o], bf16), bf16);
                if (Z) Z[zoff + (size_t)r * no + o] = z;
                if (l < n_layers - 1) {
                    out[o] = q(f32(silu(z), bf16), bf16);
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
                         const double *X, const double *T, double *grad, int bf16)
{
    const int L = n_layers, wo = w[L];
    size_t zsize = 0, asize = 0;
    for (int l = 0; l < L; ++l) {
        zsize += (size_t)batch * w[l + 1];
        if (l < L - 1) asize += (size_t)batch * w[l + 1];
    }
    double *Z = (double *)malloc(sizeof(double) * zsize);
    double *A = (double *)malloc(sizeof(double) * (asize ? asize : 1));
    double *Y = (double *)malloc(sizeof(double) * (size_t)batch * wo);
    ora_mlp_forward(L, w, params, batch, X, Y, Z, A, bf16);
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
            dz[o] = f32(2.0 * e * scale, bf16);
        }
        for (int l = L - 1; l >= 0; --l) {
            const int ni = w[l], no = w[l + 1];
            const double *W = params + poff[l];
            double *gW = grad + poff[l], *gb = grad + poff[l] + (size_t)no * ni;
            /* input of this layer */
            for (int i = 0; i < ni; ++i)
                xin[i] = (l == 0) ? q(X[(size_t)r * ni + i], bf16) : A[aoff[l - 1] + (size_t)r * ni + i];
            for (int o = 0; o < no; ++o) dzq[o] = q(dz[o], bf16);
            for (int o = 0; o < no; ++o) {
                gb[o] += dz[o];
                for (int i = 0; i < ni; ++i) gW[(size_t)o * ni + i] += dzq[o] * xin[i];
            }
            if (l > 0) {
                for (int i = 0; i < ni; ++i) {
                    double acc = 0.0;
                    for (int o = 0; o < no; ++o) acc += dzq[o] * q(W[(size_t)o * ni + i], bf16);
                    da[i] = f32(acc, bf16);
                }
                for (int i = 0; i < ni; ++i)
                    dz[i] = f32(da[i] * f32(silu_grad(Z[zoff[l - 1] + (size_t)r * ni + i]), bf16),
                                bf16);
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
