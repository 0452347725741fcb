/*
 * mri.h -- C ABI of libmri, a batched multirate-infinitesimal (MRI) fast-stage
 * solver for AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Loffeld et al., "Performance of explicit and IMEX MRI
 * multirate methods ...", Sec. 1, eq. IVP_fastslow2): y' = f^F(t,y) + f^S(t,y),
 * slow step H, fast step h << H.  One explicit MRI-GARK slow step follows the
 * three-step stage algorithm of Sec. 2.1: Y_1 = y_n; for i = 2..s solve the
 * modified fast IVP v' = f^F(v) + r_i(theta) over [T_(i-1), T_i] from
 * Y_(i-1) and set Y_i = v(T_i); y_(n+1) = Y_s.  The forcing r_i is built from
 * slow evaluations f^S(T_j, Y_j), j < i, with a user-supplied coupling table
 * (Sec. 4.2: users may supply their own coupling tables).
 *
 * f^F here is per-cell mass-action chemistry (the fast partition of Sec. 3.2,
 * f^F = omega_k W_k / rho for the species, plus a constant-volume energy
 * equation for T).  Cells are independent in the fast stage, so every call
 * processes a batch of cells.
 *
 * Conventions
 *   - Every function returns mri_status; 0 (MRI_OK) is success.  Invalid
 *     arguments return MRI_EINVAL before any device work is enqueued, and
 *     mri_last_error() (thread-local) describes the failure.
 *   - Device arrays are caller-owned device pointers (e.g. torch CUDA tensors'
 *     data_ptr()).  Host arrays passed to *_create are copied; the caller keeps
 *     ownership.  Handles are immutable after creation and may be shared by
 *     threads and streams; destroy them once, after the last use has
 *     completed on every stream.
 *   - State layout is structure-of-arrays (SoA): y[comp * ld + cell], with
 *     comp 0..S-1 the mass fractions Y_k and comp S the temperature T [K];
 *     ld >= n_cells is the leading dimension.  Forcing coefficients are
 *     rho_poly[k * n * ld + comp * ld + cell], k = 0..n_poly-1, n = S + 1.
 *     Size limits (MRI_EINVAL beyond them): n * ld <= 2^31 - 1 elements per
 *     array and ld <= 2^31 - 1024 cells.
 *   - All compute calls are asynchronous on the given stream (a hipStream_t
 *     passed as void*; NULL = the legacy default stream).  Per-cell errors
 *     detected on the device are written to the optional status array as the
 *     MRI_CELL_* bits below; mri_status_count() summarizes them.
 */
#ifndef MRI_H
#define MRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRI_ABI_VERSION 3

typedef enum {
    MRI_OK = 0,
    MRI_EINVAL = -1,        /* invalid argument (checked on the host)           */
    MRI_EHIP = -2,          /* a HIP runtime call failed                         */
    MRI_ENONFINITE = -3,    /* reserved for synchronous non-finite reports      */
    MRI_EMAXSTEPS = -4,     /* reserved for synchronous step-cap reports        */
    MRI_ENOMEM = -5,        /* host or device allocation failed                 */
    MRI_EUNSUPPORTED = -6,  /* valid request outside what this build supports   */
    MRI_ECOMPILE = -7,      /* run-time specialization of a kernel failed        */
    MRI_ENOCONV = -8        /* an iterative solve missed its tolerance           */
} mri_status;

/* Per-cell status bits written to status_out arrays. */
#define MRI_CELL_NONFINITE 1   /* a non-finite value in the result              */
#define MRI_CELL_MAXSTEPS 2    /* adaptive: accepted-step cap reached           */
#define MRI_CELL_TRANGE 4      /* T left [200, 6000] K                          */
#define MRI_CELL_NEARTIE 8     /* adaptive: an accept/reject had |err - 1| < 1e-12 */
#define MRI_CELL_STIFF 16      /* stiffness monitor: h B above the limit at a    */
                               /* stage start (stability not guaranteed)         */

typedef void *mri_stream_t;     /* hipStream_t */

typedef struct mri_mech mri_mech;
typedef struct mri_table mri_table;
typedef struct mri_batch_plan mri_batch_plan;
typedef struct mri_surrogate mri_surrogate;

int mri_abi_version(void);
/* Text for the last non-OK status returned on this thread ("" if none). */
const char *mri_last_error(void);

/* ------------------------------------------------------------------------- */
/* Fast partition f^F: mass-action Arrhenius chemistry (Sec. 3, eq. problem2  */
/* reaction term; the rate law is the standard one behind omega_k of Sec. 3). */
/* Every reaction is 2 -> 2: reactants {a, b} <-> products {c, d} (a == b is   */
/* allowed).  Per cell, with C_k = rho Y_k / W_k [mol/cm^3]:                   */
/*   k_f = exp(lnA) T^beta exp(-theta / T)            [cm^3 mol^-1 s^-1]      */
/*   K_c = exp(-(g_c + g_d - g_a - g_b) / (R T)),  g_k = g_a[k] + g_b[k] T      */
/*   q   = k_f C_a C_b - (k_f / K_c) C_c C_d                                   */
/*   dY_k/dt = W_k omega_k / rho,   omega = sum_j nu_kj q_j                    */
/*   dT/dt = -sum_k e_k(T) dY_k/dt / sum_k Y_k cv_k,                           */
/*           e_k = g_a[k] / W_k + cv_k (T - T_ref)  (J/kg)                     */
/* Units: lnA = ln(A) in CGS; theta = Ea/R in K; g_a J/mol; g_b J/(mol K);     */
/* W kg/mol; cv J/(kg K); rho kg/m^3 (used as 1e-3 rho g/cm^3 in C_k).          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n_species;                      /* S, 1..255                        */
    int n_reactions;                    /* R, >= 1                          */
    const int32_t *reactants;           /* host [R][2], indices in [0, S)   */
    const int32_t *products;            /* host [R][2]                      */
    const double *lnA, *beta, *theta;   /* host [R]                         */
    const double *g_a, *g_b;            /* host [S]                         */
    const double *W, *cv;               /* host [S]                         */
    double rho, T_ref;
} mri_mech_desc;

/* Copies the mechanism to the device.  Fails with MRI_EINVAL on bad indices
   or non-finite/non-positive coefficients, MRI_EUNSUPPORTED when
   |g_k|/(R T) could overflow the factorized rate evaluation for T >= 200 K. */
mri_status mri_mech_create(const mri_mech_desc *desc, mri_mech **out);
/* Test mode: f^F(v) = A v with a dense host A[n][n] (row-major), n <= 16.
   Used to check the MRI driver against closed-form linear solutions. */
mri_status mri_mech_create_linear(int n, const double *A, mri_mech **out);
void mri_mech_destroy(mri_mech *m);
/* State width n (S + 1 for chemistry, n for linear); -1 for NULL. */
int mri_mech_state_width(const mri_mech *m);
/* Compile the mechanism-specialized kernels (hipRTC) for a block size of 64,
   128 or 256 threads ahead of first use.  load = 0 only compiles (no GPU is
   needed) and reports the code-object size; load = 1 also loads the module on
   the current device.  Returns MRI_ECOMPILE with the compiler log in
   mri_last_error() on failure. */
mri_status mri_mech_specialize(mri_mech *m, int block_size, int load, size_t *code_bytes);
/* The same for the kernel of one fast method (MRI_FAST_*) with n_poly forcing
   terms (0..4); mri_mech_specialize is the RK4 kernel with one term. */
mri_status mri_mech_specialize_method(mri_mech *m, int method, int n_poly, int block_size,
                                      int load, size_t *code_bytes);
/* The same for the stiffness monitor the fixed-step stages run when
   opts.stiff_limit > 0 (see mri_stiffness_check): with the specialized
   kernels the monitor is specialized too (128 threads per block), else the
   generic one runs. */
mri_status mri_mech_specialize_monitor(mri_mech *m, int load, size_t *code_bytes);
/* 64-bit FNV-1a hash of that kernel's machine code and constant data (the
   .text and .rodata sections of its code object; compiled, not loaded, no GPU
   needed): identifies the exact code the GPU runs, e.g. to tell whether
   profiler counters taken earlier still describe the kernel. */
mri_status mri_mech_code_hash(mri_mech *m, int method, int n_poly, int block_size,
                              uint64_t *hash);

/* ------------------------------------------------------------------------- */
/* MRI-GARK coupling table (Sec. 2.1; MIS and MRI-GARK families of Sec. 2.1).  */
/* c[s] stage times (c_1 = 0, strictly increasing: explicit, Delta c_i > 0);   */
/* gamma[k][i][j], k < n_gamma, strictly lower triangular.  Stage i's forcing  */
/* is r_i(tau) = (1/Delta c_i) sum_k tau^k sum_(j<i) gamma[k][i][j] F_j,       */
/* tau in [0,1] the normalized time in the stage, F_j = f^S(T_j, Y_j).          */
/* Creation checks sum_j sum_k gamma[k][i][j]/(k+1) = Delta c_i (1e-12).       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int s;                              /* number of stages, 2..8           */
    int n_gamma;                        /* forcing polynomial terms, 1..4   */
    const double *c;                    /* host [s]                         */
    const double *gamma;                /* host [n_gamma][s][s]             */
} mri_table_desc;

mri_status mri_table_create(const mri_table_desc *desc, mri_table **out);
void mri_table_destroy(mri_table *t);

/* ------------------------------------------------------------------------- */
/* Fast-stage options.                                                        */
/* ------------------------------------------------------------------------- */
/* Fast methods (Sec. 3.2 pairs the slow MRI method with fast explicit RK
   methods of orders 2 to 5, the MRI-P(k) family of Sec. 5.1):
     MRI_FAST_RK4          classic RK4, n_sub uniform substeps per stage
     MRI_FAST_ZONNEVELD43  Zonneveld 4(3), adaptive (tolerances below)
     MRI_FAST_HEUN         Heun's 2nd-order method, n_sub uniform substeps
     MRI_FAST_BS3          Bogacki-Shampine 3rd-order solution, n_sub uniform
                           substeps (the embedded estimate is not used)
     MRI_FAST_CK5          Cash-Karp 5th-order solution, n_sub uniform
                           substeps (the embedded estimate is not used);
                           chemistry with at most 24 species, else
                           MRI_EUNSUPPORTED                                */
enum {
    MRI_FAST_RK4 = 0,
    MRI_FAST_ZONNEVELD43 = 1,
    MRI_FAST_HEUN = 2,
    MRI_FAST_BS3 = 3,
    MRI_FAST_CK5 = 4
};
enum {
    MRI_KERNEL_AUTO = 0,        /* specialized if available, else generic       */
    MRI_KERNEL_GENERIC = 1,     /* one binary for every mechanism; coefficients  */
                                /* staged in LDS                                 */
    MRI_KERNEL_SPECIALIZED = 2  /* compiled at run time (hipRTC) for the         */
                                /* mechanism, coefficients folded into the code  */
};

typedef struct {
    int method;                 /* MRI_FAST_*                                     */
    int n_sub;                  /* fixed-step methods: substeps per stage, >= 1   */
    double rtol, atol_Y, atol_T;/* Zonneveld: WRMS weights 1/(atol + rtol |y|)    */
    int max_steps;              /* Zonneveld: accepted-step cap per cell-stage    */
    int kernel;                 /* MRI_KERNEL_*                                   */
    int block_size;             /* threads per block, 0 = tuned default           */
    double stiff_limit;         /* fixed-step methods: > 0 runs the stiffness     */
                                /* monitor at the stage start state and sets      */
                                /* MRI_CELL_STIFF where h B > stiff_limit (B: see */
                                /* mri_stiffness_check); 0 = off                  */
} mri_fast_opts;

/* ------------------------------------------------------------------------- */
/* HOT PATH.  One fast stage for a batch of cells (Sec. 2.1 step 2b):          */
/*   v' = f^F(v) + sum_k tau^k rho_k,  tau = theta / L in [0, 1],              */
/*   v(0) = y_in, y_out = v(L).                                                */
/* RK4: h = L / n_sub; the forcing is evaluated at tau = (m + c_r)/n_sub.       */
/* Zonneveld 4(3): adaptive h, h_0 = h_max = L/10, accept when WRMS err <= 1,  */
/* h <- h min(5, max(0.2, 0.9 err^(-1/4))), last step clipped to land on L.    */
/* y_in, y_out: device [n][ld] (y_out may alias y_in).  rho_poly: device        */
/* [n_poly][n][ld], may be NULL when n_poly == 0.  status_out, steps_out:       */
/* optional device int32 [n_cells] (accepted steps; RK4 writes n_sub).          */
/* ------------------------------------------------------------------------- */
mri_status mri_fast_stage(const mri_mech *m, const mri_fast_opts *opts, int n_cells, int ld,
                          const double *y_in, double *y_out, int n_poly, const double *rho_poly,
                          double L, int32_t *status_out, int32_t *steps_out, mri_stream_t stream);

/* ------------------------------------------------------------------------- */
/* One explicit MRI-GARK slow step y_n -> y_(n+1) in place (Sec. 2.1, steps   */
/* 1-3).  The slow right-hand side is a callback that enqueues device work on  */
/* `stream` computing fy = f^S(t, y) for the SoA arrays; it returns 0 on        */
/* success.  s-1 slow evaluations are made per step (F_s is never needed).       */
/* ws: device workspace of at least mri_workspace_bytes(); caller-owned.        */
/* status_out/steps_out (optional, device [n_cells]) accumulate over stages.    */
/* ------------------------------------------------------------------------- */
typedef int (*mri_slow_rhs)(double t, const double *y, double *fy, int n_cells, int ld,
                            void *user, mri_stream_t stream);

mri_status mri_workspace_bytes(const mri_mech *m, const mri_table *t, int n_cells, int ld,
                               size_t *bytes);
mri_status mri_slow_step(const mri_mech *m, const mri_table *t, const mri_fast_opts *opts,
                         mri_slow_rhs f_slow, void *user, double t0, double H, int n_cells,
                         int ld, double *y, void *ws, size_t ws_bytes, int32_t *status_out,
                         int32_t *steps_out, mri_stream_t stream);

/* ------------------------------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph        */
/* capture, tight serving loops, harnesses that forbid hipMalloc): the slow    */
/* step of mri_slow_step with no workspace argument.  The slow evaluations and */
/* forcing planes live in a device array inside the library of                 */
/* MRI_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends); a step     */
/* needs 8 n ld (s - 1 + n_gamma) bytes of it (MRI_EINVAL beyond, e.g. n = 22  */
/* with MIS-KW3 up to ld = 381,300 cells).  The call allocates nothing: the    */
/* fast-stage kernel must already be set up on the device by one earlier       */
/* mri_fast_stage or mri_slow_step with the same options and number of forcing */
/* terms (MRI_EINVAL otherwise).  Every call on a GPU shares that GPU's array: */
/* calls that overlap on one GPU (other streams or threads) race.  Each plane  */
/* is written before it is read, so no content carries over between calls.    */
/* The slow RHS callback receives pointers into the array.                     */
/* ------------------------------------------------------------------------- */
#define MRI_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
size_t mri_noalloc_scratch_bytes(void);
mri_status mri_slow_step_noalloc(const mri_mech *m, const mri_table *t,
                                 const mri_fast_opts *opts, mri_slow_rhs f_slow, void *user,
                                 double t0, double H, int n_cells, int ld, double *y,
                                 int32_t *status_out, int32_t *steps_out, mri_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Adaptive slow steps (Sec. 7 names adaptive step control as the way to spare */
/* users the manual choice of fast and slow step sizes).  Integrates y in place */
/* from t0 to t_end with mri_slow_step, choosing H by step doubling: an attempt */
/* takes one step of H and two of H/2 from the same state; the error estimate   */
/* is e = (y_half - y_full) / (2^order - 1) in the WRMS norm over every cell and */
/* component, sqrt(mean (e / (atol_c + rtol |y_half|))^2), atol_c = atol_T for  */
/* the temperature of chemistry states and atol_Y otherwise.  ||e|| <= 1 accepts */
/* (y <- y_half, t <- t + H); either way H <- H min(fac_max, max(fac_min,        */
/* safety ||e||^(-1/(order+1)))) (fac_max if ||e|| = 0, fac_min if not finite),  */
/* bounded by H_max; the last step is shortened to end exactly at t_end.         */
/* Fast side: the adaptive fast method uses opts as given; a fixed-step method   */
/* keeps the fast step of the first step, opts->n_sub substeps per stage at H0:  */
/* a step of size h uses max(1, ceil(n_sub h / H0 - 1e-9)) substeps per stage.  */
/* Fails with MRI_EMAXSTEPS when max_attempts attempts do not reach t_end or a  */
/* rejected step falls below H_min (stats then describe the state reached; y    */
/* holds the last accepted state).  status_out (optional, device [n_cells]) is  */
/* the OR of the cell flags of every accepted step.  Synchronizes the stream    */
/* once per attempt (the accept decision is taken on the host).                */
/* ------------------------------------------------------------------------- */
typedef struct {
    double rtol, atol_Y, atol_T;  /* error weights (rtol >= 0, atol > 0)          */
    double H0;                    /* first step size (> 0)                          */
    double H_min, H_max;          /* bounds; H_max = 0 means unbounded             */
    int order;                    /* order p of the slow table, 1..8               */
    int max_attempts;             /* cap on attempted steps (>= 1)                 */
    double safety, fac_min, fac_max; /* 0 selects 0.9, 0.2, 5                      */
} mri_adapt_opts;

typedef struct {
    int accepted, rejected;       /* slow steps                                     */
    double t;                     /* time reached                                   */
    double H_last;                /* last accepted step size                        */
    double H_next;                /* proposed next step size                        */
    double err_last;              /* WRMS error estimate of the last attempt       */
    int64_t fast_steps;           /* fast substeps of the accepted steps' half     */
                                  /* steps, summed over cells                       */
} mri_adapt_stats;

/* Workspace of mri_adaptive_run: mri_workspace_bytes plus two state copies,
   four per-cell counters and the per-block error partials. */
mri_status mri_adaptive_workspace_bytes(const mri_mech *m, const mri_table *t, int n_cells,
                                        int ld, size_t *bytes);
mri_status mri_adaptive_run(const mri_mech *m, const mri_table *t, const mri_fast_opts *opts,
                            const mri_adapt_opts *a, mri_slow_rhs f_slow, void *user, double t0,
                            double t_end, int n_cells, int ld, double *y, void *ws,
                            size_t ws_bytes, int32_t *status_out, mri_adapt_stats *stats,
                            mri_stream_t stream);

/* Built-in slow RHS: 2nd-order centred advection-diffusion on a periodic grid
   (Sec. 3, eq. problem2 transport terms; Sec. 3.1 second-order stencils) for
   every component: f = -u . grad(phi) + D lap(phi).  Cell index
   (z*ny + y)*nx + x; n_cells must equal nx*ny*nz, ny and nz at most 65535
   (the callback returns nonzero otherwise).  Pass a pointer to this
   struct as `user` with mri_advdiff_slow_rhs as the callback. */
typedef struct {
    int nx, ny, nz;
    int n_comp;
    double u[3];
    double D, dx;
} mri_advdiff_params;
int mri_advdiff_slow_rhs(double t, const double *y, double *fy, int n_cells, int ld,
                         void *user, mri_stream_t stream);

/* Built-in slow RHS for tests: f^S = A y per cell, A a linear mechanism handle
   (mri_mech_create_linear) passed as `user`. */
int mri_linear_slow_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                        mri_stream_t stream);

/* ------------------------------------------------------------------------- */
/* IMEX-MRI-GARK slow step (Sec. 2.1: the slow operator split as              */
/* f^S = f^I + f^E, f^I treated implicitly on solve-decoupled stages; Sec. 3.2 */
/* and Sec. 6 take the diffusion implicitly and the advection explicitly).     */
/* Table: c[s] nondecreasing with c_1 = 0 and c_s = 1; gamma[k][i][j] weighs   */
/* the implicit evaluations FI_j = f^I(T_j, Y_j), omega[k][i][j] the explicit  */
/* ones FE_j = f^E(T_j, Y_j).  A stage with Delta c_i > 0 is a fast stage       */
/* with forcing r_i(tau) = (1/Delta c_i) sum_k tau^k sum_(j<i) (gamma[k][i][j] */
/* FI_j + omega[k][i][j] FE_j); a stage with Delta c_i = 0 is solve-decoupled:  */
/* Y_i = Y_(i-1) + H sum_(j<i) (gbar_ij FI_j + obar_ij FE_j) + H gbar_ii FI_i,  */
/* gbar_ij = sum_k gamma[k][i][j] / (k + 1) (obar likewise), solved for Y_i.    */
/* Creation checks: omega strictly lower triangular; gamma lower triangular    */
/* with its diagonal zero on fast stages; both rows' integral weights sum to   */
/* Delta c_i (1e-12); at least one fast stage; s <= 13, n_gamma <= 4.          */
/* ------------------------------------------------------------------------- */
typedef struct mri_imex_table mri_imex_table;
typedef struct {
    int s;                              /* number of stages, 2..13          */
    int n_gamma;                        /* forcing polynomial terms, 1..4   */
    const double *c;                    /* host [s]                         */
    const double *gamma;                /* host [n_gamma][s][s], f^I        */
    const double *omega;                /* host [n_gamma][s][s], f^E        */
} mri_imex_table_desc;
mri_status mri_imex_table_create(const mri_imex_table_desc *desc, mri_imex_table **out);
void mri_imex_table_destroy(mri_imex_table *t);

/* Implicit solve callback: enqueue on `stream` the solution y of
   y - a f^I(t, y) = r for the SoA arrays (device [n][ld], cells below
   n_cells); returns 0 on success, nonzero on failure (the step then returns
   MRI_ENOCONV). */
typedef int (*mri_implicit_solve)(double t, double a, const double *r, double *y, int n_cells,
                                  int ld, void *user, mri_stream_t stream);

/* Workspace: 8 n ld (2 (s - 1) + n_gamma) bytes (the slow evaluations of both
   partitions and the forcing planes, the first of which also holds the
   right-hand side of a solve-decoupled stage). */
mri_status mri_imex_workspace_bytes(const mri_mech *m, const mri_imex_table *t, int n_cells,
                                    int ld, size_t *bytes);
/* One IMEX-MRI-GARK step y_n -> y_(n+1) in place.  f_expl, f_impl: slow RHS
   callbacks as for mri_slow_step; solve_impl: the implicit solve; all three
   get `user`.  Evaluations per step: s - 1 of each partition; one solve per
   solve-decoupled stage with gbar_ii != 0.  status_out / steps_out (optional,
   device [n_cells]) accumulate over the fast stages.  The solve callback may
   synchronize the stream (the built-in one does). */
mri_status mri_imex_slow_step(const mri_mech *m, const mri_imex_table *t,
                              const mri_fast_opts *opts, mri_slow_rhs f_expl,
                              mri_slow_rhs f_impl, mri_implicit_solve solve_impl, void *user,
                              double t0, double H, int n_cells, int ld, double *y, void *ws,
                              size_t ws_bytes, int32_t *status_out, int32_t *steps_out,
                              mri_stream_t stream);

/* Built-in split of the advection-diffusion operator for the IMEX step (pass
   a pointer to this struct as `user`): f^E = -u . grad(phi) and f^I =
   D lap(phi), the two halves of mri_advdiff_slow_rhs's stencil, and the
   implicit diffusion solve (I - a D lap) y = r by conjugate gradients, one
   independent CG per component (the operator is symmetric positive definite
   on the periodic grid, with eigenvalues in [1, 1 + 12 a D / dx^2]), started
   from y = r and stopped when ||r_c - A y_c||_2 <= cg_rtol ||r_c||_2 for
   every component c (recursive residual).  Because ||A^-1|| <= 1, the error
   of every element of y_c is then at most cg_rtol ||r_c||_2.  The solve
   checks convergence on the host every 8 iterations (synchronizing the
   stream) and fails after cg_max_iter iterations. */
typedef struct {
    mri_advdiff_params grid;            /* grid, n_comp, u, D, dx                */
    double cg_rtol;                     /* > 0, e.g. 1e-13                       */
    int cg_max_iter;                    /* >= 1                                  */
    void *cg_ws;                        /* device, mri_diffusion_solve_workspace */
    size_t cg_ws_bytes;
    int cg_iters;                       /* out: iterations of the last solve     */
    int cg_solves;                      /* out: incremented by every solve       */
} mri_imex_advdiff;
mri_status mri_diffusion_solve_workspace_bytes(const mri_advdiff_params *grid, int ld,
                                               size_t *bytes);
int mri_advection_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                      mri_stream_t stream);
int mri_diffusion_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                      mri_stream_t stream);
int mri_diffusion_solve(double t, double a, const double *r, double *y, int n_cells, int ld,
                        void *user, mri_stream_t stream);

/* Diagnostic: y[i] = 2^x[i] (device arrays, n elements) with the polynomial
   exponential of the generic kernels and of the specialized kernels that run
   one wave per SIMD, for accuracy tests. */
mri_status mri_selftest_exp2(const double *x, double *y, int n, mri_stream_t stream);
/* The same with the table-driven exponential of the specialized kernels that
   run two waves per SIMD (2^(j/256) table plus a degree-4 polynomial;
   |x| < 1022). */
mri_status mri_selftest_exp2_t256(const double *x, double *y, int n, mri_stream_t stream);

/* Stiffness monitor (the stability statements of Sec. 5.2 compare h times the
   fastest chemical rate with a method's stability interval, 2.785 on the
   negative real axis for RK4).  For the chemistry mechanism m and the states
   y (device [n][ld]): B = max_k sum_j |nu_kj| (kf_j (C_a + C_b) + kr_j (C_c +
   C_d)), an upper bound (Gershgorin, in concentration variables, which have
   the same eigenvalues) of the spectral radius of the species block of the
   Jacobian of f^F at fixed T, in 1/s.  bound_out (nullable, device FP64
   [n_cells]) receives B; status (nullable, device int32 [n_cells]) gets
   MRI_CELL_STIFF OR-ed in where h B > limit.  MRI_EUNSUPPORTED for linear
   mechanisms. */
mri_status mri_stiffness_check(const mri_mech *m, int n_cells, int ld, const double *y, double h,
                               double limit, double *bound_out, int32_t *status,
                               mri_stream_t stream);

/* Counts cells with (status & mask) != 0; synchronizes the stream.  Uses one
   device counter per GPU, allocated on the first call there and kept until the
   process ends; concurrent calls take turns. */
mri_status mri_status_count(const int32_t *status, int n_cells, int32_t mask, int64_t *n_bad,
                            mri_stream_t stream);

/* Cumulative counters since load (or the last reset): slow RHS evaluations made
   by mri_slow_step, fast-stage launches and cell-stages integrated. */
typedef struct {
    int64_t slow_evals;
    int64_t fast_stages;
    int64_t cell_stages;
    int64_t specializations;   /* run-time kernel compilations performed */
} mri_counters;
void mri_get_counters(mri_counters *out);
void mri_reset_counters(void);

/* Kernel timing: while enabled, every fast-stage launch is bracketed by two
   hipEvents on its own stream.  mri_timing_read() waits for the recorded
   events, returns the summed kernel time [ms] and the number of timed launches,
   and (reset != 0) starts a new accumulation.  Host thread-safe; meant for
   benchmarking, adds a few microseconds per launch. */
mri_status mri_timing_enable(int enable);
mri_status mri_timing_read(double *fast_ms, int64_t *n_launches, int reset);

/* ------------------------------------------------------------------------- */
/* Batched uneven reactor sets.  Cells of set i are [set_offsets[i],          */
/* set_offsets[i+1]) of one SoA array; set i integrates one fast stage of     */
/* length L_per_set[i].  The plan stores the set layout, picks tiles with an   */
/* autotuner (timed on first run) and runs one persistent work-queue kernel    */
/* in which each lane pulls the next cell when its cell finishes; the launch   */
/* is captured in a hipGraph and replayed on later runs.                       */
/* ------------------------------------------------------------------------- */
mri_status mri_batch_plan_create(const mri_mech *m, const mri_fast_opts *opts, int n_sets,
                                 const int64_t *set_offsets /* host [n_sets+1] */,
                                 mri_batch_plan **out);
/* y_in/y_out device [n][ld], distinct (the first run times tile candidates on
   a prefix of the sets, writing y_out); rho_poly device [n_poly][n][ld] or
   NULL; L_per_set host [n_sets], copied to the device on the stream;
   status_out/steps_out/rejects_out optional device [n_total]: status bits,
   accepted and rejected steps of each cell (written once, when its lane
   finishes it; with mri_batch_lane_stats, sum(accepted + rejected) equals the
   useful lane-steps exactly when every cell was integrated by one lane). */
mri_status mri_batch_run(mri_batch_plan *p, const double *y_in, double *y_out, int64_t ld,
                         int n_poly, const double *rho_poly, const double *L_per_set,
                         int32_t *status_out, int32_t *steps_out, int32_t *rejects_out,
                         mri_stream_t stream);
/* Tile chosen by the autotuner (threads per block, persistent blocks); valid
   after the first run. */
mri_status mri_batch_plan_tile(const mri_batch_plan *p, int *block_size, int *n_blocks);
/* The autotuner's trials of the first run (none when the choice came from the
   tuning cache, *from_cache then 1) and its choice.  Tiling fields: threads
   per block, persistent blocks, waves per SIMD the register allocation allows
   (0 = built-in rule), exponential (1 = 2^(j/256) table in LDS, 0 =
   polynomial, -1 = built-in rule), scheduling window in rate evaluations (0 =
   built-in), and the trial's time on the tuning prefix.  The tuner times 64 /
   128 / 256 threads at 1x and 2x the resident grid, then at the best block
   size the other waves-per-SIMD setting, the other exponential and windows of
   1 and 4; it caches the choice per mechanism, fast method, forcing terms,
   tolerances, size class (floor(log2(n_total))) and device architecture in
   memory and in the file MRI_TUNE_CACHE names ("off": memory only; default
   $XDG_CACHE_HOME or $HOME/.cache + /libmri/batch_tune.txt).  The choice's ms
   is its time on the tuning prefix (also when it came from the cache).  The
   variants with the other exponential round differently: results are bitwise
   independent of the tile for one variant, not across exponentials. */
typedef struct {
    int block_size, n_blocks, waves_per_simd, exp_table, sched_window;
    float ms;
} mri_tune_trial;
mri_status mri_batch_plan_tune_log(const mri_batch_plan *p, int max_entries,
                                   mri_tune_trial *trials, int *n_entries, int *from_cache,
                                   mri_tune_trial *choice);
/* Hash of the machine code of the plan's work-queue kernel (the tile chosen by
   the first run, else the requested or default block size) for n_poly forcing
   terms; the same hash as mri_mech_code_hash gives for the other kernels. */
mri_status mri_batch_plan_code_hash(const mri_batch_plan *p, int n_poly, uint64_t *hash);
/* Lane utilization of the last run: useful lane-steps (a lane advancing a
   cell) and issued lane-steps (lanes x loop trips).  Synchronizes the stream. */
mri_status mri_batch_lane_stats(const mri_batch_plan *p, uint64_t *useful, uint64_t *issued,
                                mri_stream_t stream);
void mri_batch_plan_destroy(mri_batch_plan *p);

#ifdef __cplusplus
}
#endif
#endif /* MRI_H */
