// imex.cpp -- IMEX-MRI-GARK slow steps (Sec. 2.1 with the slow operator split
// as f^S = f^I + f^E; the implicit part is taken on solve-decoupled stages,
// Delta c_i = 0) and the built-in split of the advection-diffusion operator
// with a conjugate-gradient diffusion solve (Sec. 3.2 and Sec. 6 put the
// diffusion into f^I and the advection into f^E).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "imex_dev.h"
#include "mri_dev.h"
#include "mri_internal.h"

struct mri_imex_table {
    int s = 0, ng = 0;
    std::vector<double> c, gamma, omega;   // gamma / omega [ng][s][s]
    double g(int k, int i, int j) const { return gamma[((size_t)k * s + i) * s + j]; }
    double w(int k, int i, int j) const { return omega[((size_t)k * s + i) * s + j]; }
    // integral weights of the forcing polynomial over a stage
    double gbar(int i, int j) const
    {
        double a = 0.0;
        for (int k = 0; k < ng; ++k) a += g(k, i, j) / (k + 1.0);
        return a;
    }
    double wbar(int i, int j) const
    {
        double a = 0.0;
        for (int k = 0; k < ng; ++k) a += w(k, i, j) / (k + 1.0);
        return a;
    }
};

namespace {

constexpr long long kMaxCells = (1ll << 31) - 1024;

#define IMEX_TRY(expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return mri_fail(MRI_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// Conjugate-gradient workspace layout for n_comp components of ld cells.
struct CgLayout {
    size_t r, p, q, part_a, part_b, sc, done, total;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

CgLayout cg_layout(const mri_advdiff_params *g, int ld)
{
    CgLayout L{};
    const size_t plane = sizeof(double) * (size_t)g->n_comp * (size_t)ld;
    const int ncells = g->nx * g->ny * g->nz;
    const size_t nb = (size_t)std::max(cg_apply_blocks(g->nx, g->ny, g->nz), cg_vec_blocks(ncells));
    size_t off = 0;
    L.r = off, off += align256(plane);
    L.p = off, off += align256(plane);
    L.q = off, off += align256(plane);
    L.part_a = off, off += align256(sizeof(double) * nb * g->n_comp);
    L.part_b = off, off += align256(sizeof(double) * nb * g->n_comp);
    L.sc = off, off += align256(sizeof(CgScalars) * g->n_comp);
    L.done = off, off += align256(sizeof(int) * g->n_comp);
    L.total = off;
    return L;
}

int check_grid(const mri_advdiff_params *p, int n_cells, int ld)
{
    if (!p) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->n_comp < 1) return -2;
    if ((long long)p->nx * p->ny * p->nz != n_cells || ld < n_cells) return -3;
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return -4;
    if (p->ny > 65535 || p->nz > 65535) return -6;
    return 0;
}

}  // namespace

extern "C" {

mri_status mri_imex_table_create(const mri_imex_table_desc *d, mri_imex_table **out)
{
    if (!out) return mri_fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d || !d->c || !d->gamma || !d->omega) return mri_fail(MRI_EINVAL, "NULL table field");
    const int s = d->s, ng = d->n_gamma;
    if (s < 2 || s > IMEX_JMAX + 1) return mri_fail(MRI_EINVAL, "s must be in [2, %d]", IMEX_JMAX + 1);
    if (ng < 1 || ng > IMEX_KMAX) return mri_fail(MRI_EINVAL, "n_gamma must be in [1, %d]", IMEX_KMAX);
    mri_imex_table *t = new mri_imex_table;
    t->s = s;
    t->ng = ng;
    t->c.assign(d->c, d->c + s);
    t->gamma.assign(d->gamma, d->gamma + (size_t)ng * s * s);
    t->omega.assign(d->omega, d->omega + (size_t)ng * s * s);
    auto bad = [&](const char *fmt, int a, int b) {
        delete t;
        return mri_fail(MRI_EINVAL, fmt, a, b);
    };
    for (double v : t->c)
        if (!std::isfinite(v)) return bad("non-finite c (%d, %d)", 0, 0);
    for (double v : t->gamma)
        if (!std::isfinite(v)) return bad("non-finite gamma (%d, %d)", 0, 0);
    for (double v : t->omega)
        if (!std::isfinite(v)) return bad("non-finite omega (%d, %d)", 0, 0);
    if (t->c[0] != 0.0 || std::fabs(t->c[s - 1] - 1.0) > 1e-12)
        return bad("need c_1 = 0 and c_s = 1 (%d, %d)", 0, s);
    int n_fast = 0;
    for (int i = 1; i < s; ++i) {
        const double dc = t->c[i] - t->c[i - 1];
        if (dc < 0.0) return bad("c decreases at stage %d (%d)", i + 1, 0);
        if (dc > 0.0) ++n_fast;
        for (int k = 0; k < ng; ++k) {
            for (int j = i; j < s; ++j)
                if (t->w(k, i, j) != 0.0) return bad("omega not strictly lower at row %d col %d", i + 1, j + 1);
            for (int j = i + 1; j < s; ++j)
                if (t->g(k, i, j) != 0.0) return bad("gamma above the diagonal at row %d col %d", i + 1, j + 1);
            if (dc > 0.0 && t->g(k, i, i) != 0.0)
                return bad("gamma diagonal on fast stage %d (%d)", i + 1, 0);
        }
        double gs = 0.0, ws = 0.0;
        for (int j = 0; j <= i; ++j) {
            gs += t->gbar(i, j);
            ws += t->wbar(i, j);
        }
        if (std::fabs(gs - dc) > 1e-12 || std::fabs(ws - dc) > 1e-12)
            return bad("row %d integral weights do not sum to Delta c (%d)", i + 1, 0);
    }
    for (int k = 0; k < ng; ++k)
        for (int j = 0; j < s; ++j)
            if (t->g(k, 0, j) != 0.0 || t->w(k, 0, j) != 0.0)
                return bad("first row must be zero (col %d, term %d)", j + 1, k);
    if (n_fast == 0) return bad("no fast stage (%d, %d)", 0, 0);
    *out = t;
    return MRI_OK;
}

void mri_imex_table_destroy(mri_imex_table *t) { delete t; }

mri_status mri_imex_workspace_bytes(const mri_mech *m, const mri_imex_table *t, int n_cells,
                                    int ld, size_t *bytes)
{
    if (!m || !t || !bytes) return mri_fail(MRI_EINVAL, "NULL argument");
    if (n_cells < 0 || ld < n_cells) return mri_fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return mri_fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    const int n = mri_internal_state_width(m);
    *bytes = sizeof(double) * (size_t)n * (size_t)ld * (size_t)(2 * (t->s - 1) + t->ng);
    return MRI_OK;
}

mri_status mri_imex_slow_step(const mri_mech *mc, const mri_imex_table *t,
                              const mri_fast_opts *opts, mri_slow_rhs f_expl,
                              mri_slow_rhs f_impl, mri_implicit_solve solve_impl, void *user,
                              double t0, double H, int n_cells, int ld, double *y, void *ws,
                              size_t ws_bytes, int32_t *status_out, int32_t *steps_out,
                              mri_stream_t stream)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    if (!m || !t || !opts) return mri_fail(MRI_EINVAL, "mech, table or options is NULL");
    if (!f_expl || !f_impl || !solve_impl) return mri_fail(MRI_EINVAL, "callback is NULL");
    if (n_cells < 0 || ld < n_cells) return mri_fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return mri_fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    const int n = mri_internal_state_width(m);
    if ((long long)ld * n > (1ll << 31) - 1)
        return mri_fail(MRI_EINVAL, "n * ld exceeds 2^31 - 1 elements");
    if (!(H > 0.0) || !std::isfinite(H) || !std::isfinite(t0))
        return mri_fail(MRI_EINVAL, "H must be positive and finite");
    size_t need = 0;
    mri_imex_workspace_bytes(m, t, n_cells, ld, &need);
    if (n_cells == 0) return MRI_OK;
    if (!y) return mri_fail(MRI_EINVAL, "y is NULL");
    if (!ws || ws_bytes < need)
        return mri_fail(MRI_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, need);
    const hipStream_t s = (hipStream_t)stream;
    const int S = t->s, ng = t->ng;
    const size_t vec = (size_t)n * ld;
    double *FE = (double *)ws;                       // [s-1][n][ld]
    double *FI = FE + (size_t)(S - 1) * vec;         // [s-1][n][ld]
    double *rho = FI + (size_t)(S - 1) * vec;        // [ng][n][ld]
    // step 1: Y_1 = y_n, both slow evaluations at (t_n, Y_1)
    int rc = f_expl(t0, y, FE, n_cells, ld, user, stream);
    if (rc != 0) return mri_fail(MRI_EINVAL, "explicit slow RHS callback returned %d", rc);
    rc = f_impl(t0, y, FI, n_cells, ld, user, stream);
    if (rc != 0) return mri_fail(MRI_EINVAL, "implicit slow RHS callback returned %d", rc);
    bool first_fast = true;
    for (int i = 1; i < S; ++i) {
        const double dc = t->c[i] - t->c[i - 1];
        const double Ti = t0 + t->c[i] * H;
        ImexCoef coef{};
        if (dc > 0.0) {
            // step 2a: forcing polynomial from FE_j, FI_j, j < i
            for (int k = 0; k < ng; ++k)
                for (int j = 0; j < i; ++j) {
                    coef.e[k][j] = t->w(k, i, j) / dc;
                    coef.i[k][j] = t->g(k, i, j) / dc;
                }
            IMEX_TRY(launch_imex_combine(n, n_cells, ld, ng, i, FE, FI, coef, nullptr, rho, s));
            // steps 2b-2c: the modified fast IVP over the stage, in place
            mri_status st = mri_internal_fast_stage(m, opts, n_cells, ld, y, y, ng, rho, dc * H,
                                                    status_out, steps_out, s, nullptr,
                                                    first_fast ? 0 : 1);
            if (st != MRI_OK) return st;
            first_fast = false;
        } else {
            // solve-decoupled stage: right-hand side from the integral weights,
            // then y - H gbar_ii f^I(T_i, y) = rhs
            for (int j = 0; j < i; ++j) {
                coef.e[0][j] = H * t->wbar(i, j);
                coef.i[0][j] = H * t->gbar(i, j);
            }
            IMEX_TRY(launch_imex_combine(n, n_cells, ld, 1, i, FE, FI, coef, y, rho, s));
            const double a = H * t->gbar(i, i);
            if (a != 0.0) {
                rc = solve_impl(Ti, a, rho, y, n_cells, ld, user, stream);
                if (rc != 0)
                    return mri_fail(MRI_ENOCONV, "implicit solve callback returned %d at stage %d",
                                    rc, i + 1);
            } else {
                IMEX_TRY(launch_copy_planes(n, n_cells, ld, rho, y, s));
            }
        }
        if (i < S - 1) {
            rc = f_expl(Ti, y, FE + (size_t)i * vec, n_cells, ld, user, stream);
            if (rc != 0) return mri_fail(MRI_EINVAL, "explicit slow RHS callback returned %d", rc);
            rc = f_impl(Ti, y, FI + (size_t)i * vec, n_cells, ld, user, stream);
            if (rc != 0) return mri_fail(MRI_EINVAL, "implicit slow RHS callback returned %d", rc);
        }
    }
    // step 3: y_(n+1) = Y_s (already in y)
    return MRI_OK;
}

mri_status mri_diffusion_solve_workspace_bytes(const mri_advdiff_params *grid, int ld,
                                               size_t *bytes)
{
    if (!grid || !bytes) return mri_fail(MRI_EINVAL, "NULL argument");
    const int ncells = grid->nx * grid->ny * grid->nz;
    if (check_grid(grid, ncells, ld) != 0) return mri_fail(MRI_EINVAL, "bad grid or ld");
    *bytes = cg_layout(grid, ld).total;
    return MRI_OK;
}

int mri_advection_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                      mri_stream_t stream)
{
    (void)t;
    const mri_imex_advdiff *a = (const mri_imex_advdiff *)user;
    if (!a || !y || !fy) return -1;
    const int rc = check_grid(&a->grid, n_cells, ld);
    if (rc != 0) return rc;
    if (launch_advdiff(a->grid.nx, a->grid.ny, a->grid.nz, a->grid.n_comp, ld, a->grid.u, 0.0,
                       a->grid.dx, y, fy, (hipStream_t)stream) != hipSuccess)
        return -5;
    return 0;
}

int mri_diffusion_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                      mri_stream_t stream)
{
    (void)t;
    const mri_imex_advdiff *a = (const mri_imex_advdiff *)user;
    if (!a || !y || !fy) return -1;
    const int rc = check_grid(&a->grid, n_cells, ld);
    if (rc != 0) return rc;
    const double u0[3] = {0.0, 0.0, 0.0};
    if (launch_advdiff(a->grid.nx, a->grid.ny, a->grid.nz, a->grid.n_comp, ld, u0, a->grid.D,
                       a->grid.dx, y, fy, (hipStream_t)stream) != hipSuccess)
        return -5;
    return 0;
}

// Conjugate gradients on (I - a D lap) y = r, one CG per component, started
// from y = r; convergence checked on the host every 8 iterations.
int mri_diffusion_solve(double t, double a, const double *r, double *y, int n_cells, int ld,
                        void *user, mri_stream_t stream)
{
    (void)t;
    mri_imex_advdiff *A = (mri_imex_advdiff *)user;
    if (!A || !r || !y) return -1;
    const mri_advdiff_params *g = &A->grid;
    int rc = check_grid(g, n_cells, ld);
    if (rc != 0) return rc;
    if (!(a >= 0.0) || !std::isfinite(a) || !std::isfinite(g->D) || g->D < 0.0) return -7;
    if (!(A->cg_rtol > 0.0) || A->cg_max_iter < 1) return -8;
    const CgLayout L = cg_layout(g, ld);
    if (!A->cg_ws || A->cg_ws_bytes < L.total) return -9;
    if (r == y) return -10;
    const hipStream_t s = (hipStream_t)stream;
    char *base = (char *)A->cg_ws;
    double *R = (double *)(base + L.r), *P = (double *)(base + L.p), *Q = (double *)(base + L.q);
    double *pa = (double *)(base + L.part_a), *pb = (double *)(base + L.part_b);
    CgScalars *sc = (CgScalars *)(base + L.sc);
    int *done = (int *)(base + L.done);
    const int nc = g->n_comp;
    const double aD = a * g->D, tol2 = A->cg_rtol * A->cg_rtol;
    const int nb_apply = cg_apply_blocks(g->nx, g->ny, g->nz), nb_vec = cg_vec_blocks(n_cells);
    A->cg_iters = 0;
    ++A->cg_solves;
    auto ok = [](hipError_t e) { return e == hipSuccess; };
    // y = r; q = A y; r0 = r - q; p = r0; scalars and convergence flags
    if (!ok(launch_fill_i32(done, nc, 0, s)) || !ok(launch_copy_planes(nc, n_cells, ld, r, y, s)) ||
        !ok(launch_cg_apply(g->nx, g->ny, g->nz, nc, ld, aD, g->dx, y, Q, done, pa, s)) ||
        !ok(launch_cg_init(nc, n_cells, ld, r, Q, R, P, pa, pb, s)) ||
        !ok(launch_cg_reduce(0, nc, nb_vec, pa, pb, tol2, sc, done, s)))
        return -5;
    std::vector<int> h_done(nc);
    for (int it = 0; it < A->cg_max_iter;) {
        if (it % 8 == 0) {
            if (hipMemcpyAsync(h_done.data(), done, sizeof(int) * nc, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return -5;
            if (std::all_of(h_done.begin(), h_done.end(), [](int v) { return v != 0; })) {
                A->cg_iters = it;
                return 0;
            }
        }
        if (!ok(launch_cg_apply(g->nx, g->ny, g->nz, nc, ld, aD, g->dx, P, Q, done, pa, s)) ||
            !ok(launch_cg_reduce(1, nc, nb_apply, pa, nullptr, tol2, sc, done, s)) ||
            !ok(launch_cg_update(nc, n_cells, ld, sc, done, y, R, P, Q, pa, s)) ||
            !ok(launch_cg_reduce(2, nc, nb_vec, pa, nullptr, tol2, sc, done, s)) ||
            !ok(launch_cg_dir(nc, n_cells, ld, sc, done, R, P, s)))
            return -5;
        ++it;
        A->cg_iters = it;
    }
    if (hipMemcpyAsync(h_done.data(), done, sizeof(int) * nc, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -5;
    return std::all_of(h_done.begin(), h_done.end(), [](int v) { return v != 0; }) ? 0 : -11;
}

}  // extern "C"
