// surrogate_api.cpp -- host side of the MLP surrogate: trainable network
// (forward, backward, Adam on device buffers), training-data features, the
// packed inference network and the gated surrogate stage with FP64 fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "mlp_dev.h"
#include "mri_internal.h"
#include "mri_surrogate.h"

#define fail mri_fail
#define HIP_TRY MRI_HIP_TRY

namespace {

template <class T>
hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, sizeof(T) * std::max<size_t>(n, 1));
}

}  // namespace

struct mri_mlp {
    int L = 0;
    std::vector<int> w;
    int max_batch = 0;
    int64_t n_params = 0;
    std::vector<size_t> woff, boff;       // offsets of W_l, b_l in the packed arrays
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;   // packed f32
    uint16_t *pq = nullptr;                // packed bf16 copy of params
    // activations of the last forward: Z_l f32 [B][w_(l+1)], A_l bf16 (hidden)
    std::vector<float *> Z;
    std::vector<uint16_t *> A;
    const uint16_t *X = nullptr;           // input of the last forward (caller-owned)
    float *dZ = nullptr, *dA = nullptr;
    uint16_t *dZq = nullptr;
    float *part = nullptr;                 // split-K / split-row partial sums
    size_t part_elems = 0;
    int step = 0;
    int last_batch = 0;
    // releases whatever a partial creation allocated
    ~mri_mlp()
    {
        for (void *q : {(void *)p, (void *)g, (void *)m1, (void *)m2, (void *)pq, (void *)dZ,
                        (void *)dA, (void *)dZq, (void *)part})
            if (q) (void)hipFree(q);
        for (auto *z : Z)
            if (z) (void)hipFree(z);
        for (auto *a : A)
            if (a) (void)hipFree(a);
    }
};

struct mri_surrogate {
    uint16_t *W[4] = {};
    float *b[4] = {};
    double *stats = nullptr;
    ~mri_surrogate()
    {
        for (int l = 0; l < 4; ++l) {
            if (W[l]) (void)hipFree(W[l]);
            if (b[l]) (void)hipFree(b[l]);
        }
        if (stats) (void)hipFree(stats);
    }
};

extern "C" {

mri_status mri_mlp_create(int n_layers, const int *widths, const float *params, int max_batch,
                          mri_mlp **out)
{
    if (!out) return fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_layers < 1 || n_layers > 8 || !widths || !params || max_batch < 1)
        return fail(MRI_EINVAL, "need 1 <= n_layers <= 8, widths, params, max_batch >= 1");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 4096) return fail(MRI_EINVAL, "bad width %d", widths[l]);
    std::unique_ptr<mri_mlp> m(new mri_mlp);
    m->L = n_layers;
    m->w.assign(widths, widths + n_layers + 1);
    m->max_batch = max_batch;
    size_t off = 0;
    int wmax = 0;
    for (int l = 0; l < n_layers; ++l) {
        m->woff.push_back(off);
        off += (size_t)widths[l + 1] * widths[l];
        m->boff.push_back(off);
        off += widths[l + 1];
        wmax = std::max(wmax, widths[l + 1]);
    }
    m->n_params = (int64_t)off;
    for (size_t i = 0; i < off; ++i)
        if (!std::isfinite(params[i])) return fail(MRI_EINVAL, "non-finite parameter %zu", i);
    HIP_TRY(dalloc(&m->p, off));
    HIP_TRY(dalloc(&m->g, off));
    HIP_TRY(dalloc(&m->m1, off));
    HIP_TRY(dalloc(&m->m2, off));
    HIP_TRY(dalloc(&m->pq, off));
    HIP_TRY(hipMemcpy(m->p, params, sizeof(float) * off, hipMemcpyHostToDevice));
    std::vector<float> zeros(off, 0.0f);
    HIP_TRY(hipMemcpy(m->m1, zeros.data(), sizeof(float) * off, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->m2, zeros.data(), sizeof(float) * off, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->g, zeros.data(), sizeof(float) * off, hipMemcpyHostToDevice));
    HIP_TRY(mlp_to_bf16((long long)off, m->p, m->pq, nullptr));
    for (int l = 0; l < n_layers; ++l) {
        float *z = nullptr;
        HIP_TRY(dalloc(&z, (size_t)max_batch * widths[l + 1]));
        m->Z.push_back(z);
        uint16_t *a = nullptr;
        if (l < n_layers - 1) HIP_TRY(dalloc(&a, (size_t)max_batch * widths[l + 1]));
        m->A.push_back(a);
    }
    int wall = 0;
    for (int l = 0; l <= n_layers; ++l) wall = std::max(wall, widths[l]);
    HIP_TRY(dalloc(&m->dZ, (size_t)max_batch * wall));
    HIP_TRY(dalloc(&m->dA, (size_t)max_batch * wall));
    HIP_TRY(dalloc(&m->dZq, (size_t)max_batch * wall));
    m->part_elems = (size_t)32 * wall * wall;
    HIP_TRY(dalloc(&m->part, m->part_elems));
    HIP_TRY(hipDeviceSynchronize());
    *out = m.release();
    return MRI_OK;
}

void mri_mlp_destroy(mri_mlp *m) { delete m; }

int64_t mri_mlp_param_count(const mri_mlp *m) { return m ? m->n_params : -1; }

mri_status mri_mlp_get_params(const mri_mlp *m, float *params)
{
    if (!m || !params) return fail(MRI_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpy(params, m->p, sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    return MRI_OK;
}

mri_status mri_mlp_get_grads(const mri_mlp *m, float *grads)
{
    if (!m || !grads) return fail(MRI_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpy(grads, m->g, sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    return MRI_OK;
}

mri_status mri_mlp_forward(mri_mlp *m, int batch, const uint16_t *X, float *Y,
                           mri_stream_t stream)
{
    if (!m || !X) return fail(MRI_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->max_batch) return fail(MRI_EINVAL, "batch outside [1, max_batch]");
    hipStream_t s = (hipStream_t)stream;
    const uint16_t *in = X;
    for (int l = 0; l < m->L; ++l) {
        const int ni = m->w[l], no = m->w[l + 1];
        // Z = in [B x ni] . W^T [ni x no]  (W stored [no][ni])
        HIP_TRY(mlp_gemm(batch, no, ni, in, ni, 0, m->pq + m->woff[l], ni, 1, m->Z[l], no, s));
        HIP_TRY(mlp_bias_act(batch, no, m->Z[l], m->p + m->boff[l], l < m->L - 1 ? 1 : 0, m->A[l],
                             s));
        in = m->A[l];
    }
    if (Y)
        HIP_TRY(hipMemcpyAsync(Y, m->Z[m->L - 1], sizeof(float) * batch * m->w[m->L],
                               hipMemcpyDeviceToDevice, s));
    m->X = X;
    m->last_batch = batch;
    return MRI_OK;
}

mri_status mri_mlp_backward(mri_mlp *m, int batch, const float *T, double *loss,
                            mri_stream_t stream)
{
    if (!m || !T) return fail(MRI_EINVAL, "NULL argument");
    if (batch != m->last_batch || !m->X)
        return fail(MRI_EINVAL, "backward needs the forward of the same batch first");
    hipStream_t s = (hipStream_t)stream;
    const int L = m->L;
    HIP_TRY(mlp_mse_grad(batch, m->w[L], m->Z[L - 1], T, m->dZ, m->dZq, loss, s));
    for (int l = L - 1; l >= 0; --l) {
        const int ni = m->w[l], no = m->w[l + 1];
        const uint16_t *in = (l == 0) ? m->X : m->A[l - 1];
        // dW [no x ni] = dZ^T [no x B] . in [B x ni]
        HIP_TRY(mlp_gemm(no, ni, batch, m->dZq, no, 1, in, ni, 0, m->g + m->woff[l], ni, s,
                         m->part, m->part_elems));
        HIP_TRY(mlp_colsum(batch, no, m->dZ, m->g + m->boff[l], s, m->part, m->part_elems));
        if (l > 0) {
            // dA [B x ni] = dZ [B x no] . W [no x ni]
            HIP_TRY(mlp_gemm(batch, ni, no, m->dZq, no, 0, m->pq + m->woff[l], ni, 0, m->dA, ni,
                             s));
            HIP_TRY(mlp_silu_bwd((long long)batch * ni, m->dA, m->Z[l - 1], m->dZ, m->dZq, s));
        }
    }
    return MRI_OK;
}

mri_status mri_adam_step(mri_mlp *m, float lr, float beta1, float beta2, float eps,
                         mri_stream_t stream)
{
    if (!m) return fail(MRI_EINVAL, "mlp is NULL");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(MRI_EINVAL, "bad Adam hyper-parameters");
    ++m->step;
    const float c1 = 1.0f / (1.0f - std::pow(beta1, (float)m->step));
    const float c2 = 1.0f / (1.0f - std::pow(beta2, (float)m->step));
    HIP_TRY(mlp_adam(m->n_params, m->p, m->g, m->m1, m->m2, m->pq, lr, beta1, beta2, eps, c1, c2,
                     (hipStream_t)stream));
    return MRI_OK;
}

mri_status mri_mlp_feature_stats(int64_t n, int64_t ld, const double *Y0, int n_poly,
                                 const double *RHO, const double *Lv, const double *Yb,
                                 const double *Y1, double *stats, mri_stream_t stream)
{
    if (n < 1 || ld < n || !Y0 || !Lv || !Y1 || !stats || n_poly < 0 || n_poly > 3 ||
        (n_poly > 0 && !RHO))
        return fail(MRI_EINVAL, "bad arguments");
    const int n_blocks = 512;
    double *part = nullptr;
    HIP_TRY(dalloc(&part, (size_t)n_blocks * 2 * (MLP_FEAT + MLP_NC)));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mlp_stats(n, ld, Y0, n_poly, RHO, Lv, Yb, Y1, part, n_blocks, stats, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(MRI_EHIP, "feature statistics: %s", hipGetErrorString(e));
    return MRI_OK;
}

mri_status mri_mlp_featurize(int batch, const int32_t *idx, int64_t ld, const double *Y0,
                             int n_poly, const double *RHO, const double *Lv, const double *Yb,
                             const double *Y1, const double *stats, uint16_t *X, float *T,
                             mri_stream_t stream)
{
    if (batch < 0 || !Y0 || !Lv || !stats || !X || n_poly < 0 || n_poly > 3 ||
        (n_poly > 0 && !RHO) || (T && !Y1))
        return fail(MRI_EINVAL, "bad arguments");
    if (batch == 0) return MRI_OK;
    HIP_TRY(mlp_featurize(batch, idx, ld, Y0, n_poly, RHO, Lv, Yb, Y1, stats, X, T,
                          (hipStream_t)stream));
    return MRI_OK;
}

// Layers 2-4 take their inputs in the order the fused kernel keeps the previous
// layer's outputs in registers: logical input 32 t + 8 g + e is output
// 32 t + (e < 4 ? 4 g + e : 16 + 4 g + e - 4).
static int perm_in(int k)
{
    const int t = k / 32, g = (k % 32) / 8, e = k % 8;
    return 32 * t + (e < 4 ? 4 * g + e : 16 + 4 * g + e - 4);
}

static uint16_t bf16_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

mri_status mri_surrogate_create(const int *widths, const float *params, const double *stats,
                                mri_surrogate **out)
{
    if (!out) return fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!widths || !params || !stats) return fail(MRI_EINVAL, "NULL argument");
    // the input width may be the 89 features or the 96 padded columns the
    // training path feeds (padding columns are ignored)
    int want[5] = {MLP_FEAT, MLP_HID, MLP_HID, MLP_HID, MLP_NC};
    if (widths[0] == MLP_KPAD) want[0] = MLP_KPAD;
    for (int l = 0; l < 5; ++l)
        if (widths[l] != want[l])
            return fail(MRI_EUNSUPPORTED,
                        "the fused kernel needs widths {89 or 96, 256, 256, 256, 22}");
    for (int i = 0; i < MLP_STATS; ++i)
        if (!std::isfinite(stats[i])) return fail(MRI_EINVAL, "non-finite statistics");
    std::unique_ptr<mri_surrogate> sg(new mri_surrogate);
    const int in_pad[4] = {MLP_K0_IN, MLP_HID, MLP_HID, MLP_HID};
    const int out_pad[4] = {MLP_HID, MLP_HID, MLP_HID, MLP_OUT_PAD};
    size_t off = 0;
    for (int l = 0; l < 4; ++l) {
        const int ni = want[l], no = want[l + 1];
        std::vector<uint16_t> W((size_t)out_pad[l] * in_pad[l], 0);
        std::vector<float> b(out_pad[l], 0.0f);
        for (int o = 0; o < no; ++o) {
            for (int k = 0; k < in_pad[l]; ++k) {
                const int src = (l == 0) ? k : perm_in(k);
                const int lim = (l == 0) ? MLP_FEAT : ni;
                if (src < lim) W[(size_t)o * in_pad[l] + k] = bf16_bits(params[off + (size_t)o * ni + src]);
            }
            b[o] = params[off + (size_t)no * ni + o];
        }
        off += (size_t)no * ni + no;
        HIP_TRY(dalloc(&sg->W[l], W.size()));
        HIP_TRY(dalloc(&sg->b[l], b.size()));
        HIP_TRY(hipMemcpy(sg->W[l], W.data(), sizeof(uint16_t) * W.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(sg->b[l], b.data(), sizeof(float) * b.size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(dalloc(&sg->stats, MLP_STATS));
    HIP_TRY(hipMemcpy(sg->stats, stats, sizeof(double) * MLP_STATS, hipMemcpyHostToDevice));
    *out = sg.release();
    return MRI_OK;
}

void mri_surrogate_destroy(mri_surrogate *s) { delete s; }

static mri_status check_cells(int n_cells, int ld, int n_poly, const double *rho, double L)
{
    if (n_cells < 0 || ld < n_cells) return fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > (1ll << 31) - 1024) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    if (n_poly < 0 || n_poly > 3 || (n_poly > 0 && !rho)) return fail(MRI_EINVAL, "bad n_poly");
    if (!(L > 0.0) || !std::isfinite(L)) return fail(MRI_EINVAL, "L must be positive");
    return MRI_OK;
}

mri_status mri_surrogate_infer(const mri_surrogate *s, int n_cells, int ld, const double *y_in,
                               const double *base, double *y_out, int n_poly, const double *rho,
                               double L, mri_stream_t stream)
{
    if (!s) return fail(MRI_EINVAL, "surrogate is NULL");
    mri_status st = check_cells(n_cells, ld, n_poly, rho, L);
    if (st != MRI_OK) return st;
    if (n_cells == 0) return MRI_OK;
    if (!y_in || !y_out || y_in == y_out || base == y_out)
        return fail(MRI_EINVAL, "need y_in and y_out, y_out distinct from y_in and base");
    HIP_TRY(mlp_infer(y_in, base, y_out, rho, s->W, s->b, s->stats, ld, n_cells, n_poly, L,
                      (hipStream_t)stream));
    return MRI_OK;
}

mri_status mri_surrogate_gate(int n_cells, int ld, const double *y_in, int n_poly,
                              const double *rho, double L, const double *v_coarse,
                              const double *v_half, const double *v_net,
                              const int32_t *status_coarse, double richardson, double gate_tol,
                              double *y_out, int32_t *used_fallback, double *gate_value,
                              int32_t *fallback_list, uint32_t *n_fallback, mri_stream_t stream)
{
    mri_status st = check_cells(n_cells, ld, n_poly, rho, L);
    if (st != MRI_OK) return st;
    if (!(gate_tol >= 0.0)) return fail(MRI_EINVAL, "gate_tol must be >= 0");
    if (!(richardson >= 0.0) || !std::isfinite(richardson))
        return fail(MRI_EINVAL, "richardson must be finite and >= 0");
    if (!fallback_list || !n_fallback) return fail(MRI_EINVAL, "fallback list or count is NULL");
    if (n_cells == 0) {
        HIP_TRY(mlp_zero_u32(n_fallback, (hipStream_t)stream));
        return MRI_OK;
    }
    if (!y_in || !v_coarse || !v_half || !v_net || !y_out)
        return fail(MRI_EINVAL, "NULL state array");
    HIP_TRY(mlp_gate(n_cells, ld, y_in, rho, n_poly, L, v_coarse, v_half, v_net, status_coarse,
                     richardson, gate_tol, y_out, used_fallback, gate_value, nullptr,
                     fallback_list, n_fallback, (hipStream_t)stream));
    return MRI_OK;
}

// Workspace of the gated stage (all [22][ld] planes FP64): coarse, half and
// network states, the compacted forcing; int32 coarse status, fallback list and
// compacted status [ld]; the device fallback count.
static size_t stage_ws_bytes(int ld, int n_poly)
{
    const size_t plane = sizeof(double) * (size_t)ld * MLP_NC;
    return plane * (3 + (size_t)n_poly) + 3 * sizeof(int) * (size_t)ld + 256;
}

mri_status mri_surrogate_workspace_bytes(int n_cells, int ld, int n_poly, size_t *bytes)
{
    if (!bytes || n_cells < 0 || ld < n_cells || n_poly < 0 || n_poly > 3)
        return fail(MRI_EINVAL, "bad arguments");
    *bytes = stage_ws_bytes(ld, n_poly);
    return MRI_OK;
}

static int method_order(int method)
{
    switch (method) {
    case MRI_FAST_HEUN: return 2;
    case MRI_FAST_BS3: return 3;
    case MRI_FAST_CK5: return 5;
    default: return 4;
    }
}

mri_status mri_surrogate_stage(const mri_surrogate *s, const mri_mech *mech,
                               const mri_fast_opts *coarse, const mri_fast_opts *fallback,
                               double gate_tol, int n_cells, int ld, const double *y_in,
                               double *y_out, int n_poly, const double *rho, double L,
                               int32_t *used_fallback, double *gate_value, int32_t *status_out,
                               uint32_t *n_fallback, void *ws, size_t ws_bytes,
                               mri_stream_t stream)
{
    if (!s || !mech || !coarse || !fallback) return fail(MRI_EINVAL, "NULL argument");
    if (!mri_internal_is_chem(mech) || mri_internal_state_width(mech) != MLP_NC)
        return fail(MRI_EUNSUPPORTED, "the surrogate is built for 21-species mechanisms");
    if (!(gate_tol >= 0.0)) return fail(MRI_EINVAL, "gate_tol must be >= 0");
    mri_status st = check_cells(n_cells, ld, n_poly, rho, L);
    if (st != MRI_OK) return st;
    if (coarse->method == MRI_FAST_ZONNEVELD43)
        return fail(MRI_EINVAL, "the coarse stage needs a fixed-step method");
    if (coarse->n_sub < 2 || coarse->n_sub % 2)
        return fail(MRI_EINVAL, "the coarse stage needs an even n_sub >= 2 (got %d)",
                    coarse->n_sub);
    const size_t need = stage_ws_bytes(ld, n_poly);
    if (n_cells == 0) {
        if (n_fallback) HIP_TRY(mlp_zero_u32(n_fallback, (hipStream_t)stream));
        return MRI_OK;
    }
    if (!y_in || !y_out) return fail(MRI_EINVAL, "y_in or y_out is NULL");
    if (!ws || ws_bytes < need)
        return fail(MRI_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, need);
    hipStream_t hs = (hipStream_t)stream;
    const size_t plane = (size_t)ld * MLP_NC;
    double *vc = (double *)ws, *vh = vc + plane, *vn = vh + plane;
    double *rho_c = vn + plane;
    int *st_c = (int *)(rho_c + (size_t)n_poly * plane);
    int *list = st_c + ld, *st_f = list + ld;
    unsigned int *count = (unsigned int *)(st_f + ld);
    mri_mech *m = const_cast<mri_mech *>(mech);
    // coarse FP64 stage and the same with half the substeps (statuses OR-ed)
    mri_fast_opts half = *coarse;
    half.n_sub = coarse->n_sub / 2;
    half.stiff_limit = 0.0;   // the coarse solve's stiffness monitor flags the cell for both
    st = mri_internal_fast_stage(m, coarse, n_cells, ld, y_in, vc, n_poly, rho, L, st_c, nullptr,
                                 hs);
    if (st != MRI_OK) return st;
    st = mri_internal_fast_stage(m, &half, n_cells, ld, y_in, vh, n_poly, rho, L, st_c, nullptr,
                                 hs, nullptr, 1);
    if (st != MRI_OK) return st;
    // the network's correction of the coarse result and, in the same launch,
    // the residual check against the Richardson extrapolation; accepted cells
    // take the corrected state, the others go to the fallback list
    const double rich = 1.0 / (std::ldexp(1.0, method_order(coarse->method)) - 1.0);
    HIP_TRY(mlp_infer_gate(y_in, vc, vh, rho, s->W, s->b, s->stats, ld, n_cells, n_poly, L, st_c,
                           rich, gate_tol, y_out, used_fallback, gate_value, status_out, list,
                           count, hs));
    // plain FP64 stage of the rejected cells: compacted (state into vh, forcing
    // into rho_c), integrated into vn with a launch sized for every cell whose
    // kernels stop at the device count, scattered back; no host synchronization
    HIP_TRY(mlp_gather(MLP_NC, count, list, n_cells, y_in, ld, vh, ld, hs));
    if (n_poly > 0)
        HIP_TRY(mlp_gather(n_poly * MLP_NC, count, list, n_cells, rho, ld, rho_c, ld, hs));
    st = mri_internal_fast_stage(m, fallback, n_cells, ld, vh, vn, n_poly, rho_c, L,
                                 status_out ? st_f : nullptr, nullptr, hs, count);
    if (st != MRI_OK) return st;
    HIP_TRY(mlp_scatter(MLP_NC, count, list, n_cells, vn, ld, y_out, ld, hs));
    if (status_out) HIP_TRY(mlp_scatter_i32(count, list, n_cells, st_f, status_out, hs));
    if (n_fallback)
        HIP_TRY(hipMemcpyAsync(n_fallback, count, sizeof(uint32_t), hipMemcpyDeviceToDevice, hs));
    return MRI_OK;
}

}  // extern "C"
