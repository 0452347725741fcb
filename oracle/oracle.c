/*
 * oracle.c -- plain, slow, FP64 CPU reference for the MRI fast-stage solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may link, load or call this file; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no code,
 * header or constant with the GPU path.
 *
 * Every function follows the definition it cites, written out with plain loops
 * in the order the definition states it.  Build: gcc -O2 -fopenmp
 * -ffp-contract=off -fno-fast-math (no FMA contraction, libm exp/log/pow).
 *
 * Contents
 *   chemistry RHS f^F (mass action, Arrhenius forward rates, reverse rates
 *     through K_c = exp(-dG/RT), species production, constant-volume energy)
 *   linear fast RHS (f^F = A v) for order tests
 *   classic RK4 over one fast stage with a polynomial forcing
 *   a general explicit Runge-Kutta stage (Heun, Bogacki-Shampine, Cash-Karp)
 *   Zonneveld 4(3) adaptive integration over one fast stage
 *   the explicit MRI-GARK slow step (Sec. 2.1 algorithm, steps 1-3)
 *   the 2nd-order centred periodic advection-diffusion slow RHS (Sec. 3.1)
 *   a finite-difference Jacobian of f^F (stiffness calibration) and a
 *     Gershgorin bound of its species block (stiffness monitor)
 *   an MLP forward/backward in FP64 and in a BF16-emulating mode
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_R_GAS 8.314462618        /* J/(mol K) */
#define ORA_ST_NONFINITE 1
#define ORA_ST_MAXSTEPS 2
#define ORA_ST_TRANGE 4
#define ORA_ST_NEARTIE 8

typedef struct {
    int S, R;
    const int32_t *reac, *prod;          /* [R][2] species indices            */
    const double *lnA, *beta, *theta;    /* [R] ln(s*A) CGS, beta, Ea/R_cal K */
    const double *g_a, *g_b;             /* [S] g_k(T) = a_k + b_k T, J/mol   */
    const double *W, *cv;                /* [S] kg/mol, J/(kg K)              */
    double rho, T_ref;                   /* kg/m^3, K                         */
} ora_mech;

/* Fast partition: kind 0 = chemistry (n = S+1), kind 1 = linear f = A v. */
typedef struct {
    int kind;
    int n;
    const ora_mech *mech;
    const double *A;                     /* [n][n] row-major (kind 1)         */
} ora_fast;

typedef struct {
    int s, n_gamma;
    const double *c;                     /* [s]                               */
    const double *gamma;                 /* [n_gamma][s][s]                   */
} ora_table;

typedef struct {
    int method;                          /* 0 = classic RK4, 1 = Zonneveld 4(3),
                                            2 = Heun (2nd order), 3 = Bogacki-
                                            Shampine (3rd order), 4 = Cash-Karp
                                            (5th order), fixed steps            */
    int n_sub;                           /* RK4 substeps per stage            */
    double rtol, atol_Y, atol_T;         /* Zonneveld tolerances              */
    int max_steps;                       /* Zonneveld accepted-step cap       */
} ora_fast_opts;

/* ------------------------------------------------------------------------ */
/* Chemistry right-hand side (one cell).                                     */
/* Production rates omega_k enter the species equation as omega_k W_k / rho  */
/* (Sec. 3, eq. problem2, and the fast partition of Sec. 3.2); temperature    */
/* follows from constant-volume energy conservation (Sec. 3, eq. problem1,    */
/* energy equation, with the transport terms in the slow partition).          */
/* Optional outputs kf, kr, q ([R]) and wdot ([S]) may be NULL.              */
/* ------------------------------------------------------------------------ */
void ora_chem_rhs_parts(const ora_mech *m, const double *y, double *ydot,
                        double *kf_out, double *kr_out, double *q_out, double *wdot_out)
{
    const int S = m->S, R = m->R;
    const double T = y[S];
    const double rho_cgs = m->rho * 1e-3;          /* g/cm^3 */
    double *C = (double *)malloc(sizeof(double) * S);
    double *wdot = (double *)malloc(sizeof(double) * S);
    for (int k = 0; k < S; ++k) {
        double W_g = m->W[k] * 1e3;                /* g/mol */
        C[k] = rho_cgs * y[k] / W_g;               /* mol/cm^3 */
        wdot[k] = 0.0;
    }
    for (int j = 0; j < R; ++j) {
        int a = m->reac[2 * j], b = m->reac[2 * j + 1];
        int c = m->prod[2 * j], d = m->prod[2 * j + 1];
        /* forward rate constant: A T^beta exp(-Ea/(R_cal T)) (A with s folded in) */
        double kf = exp(m->lnA[j]) * pow(T, m->beta[j]) * exp(-m->theta[j] / T);
        /* equilibrium constant from the Gibbs energy change of the reaction */
        double g_c = m->g_a[c] + m->g_b[c] * T, g_d = m->g_a[d] + m->g_b[d] * T;
        double g_ra = m->g_a[a] + m->g_b[a] * T, g_rb = m->g_a[b] + m->g_b[b] * T;
        double dG = (g_c + g_d) - (g_ra + g_rb);
        double Kc = exp(-dG / (ORA_R_GAS * T));
        double kr = kf / Kc;
        double q = kf * C[a] * C[b] - kr * C[c] * C[d];
        wdot[a] -= q;
        wdot[b] -= q;
        wdot[c] += q;
        wdot[d] += q;
        if (kf_out) kf_out[j] = kf;
        if (kr_out) kr_out[j] = kr;
        if (q_out) q_out[j] = q;
    }
    double num = 0.0, den = 0.0;
    for (int k = 0; k < S; ++k) {
        double W_g = m->W[k] * 1e3;
        ydot[k] = wdot[k] * W_g / rho_cgs;         /* 1/s */
        double e_k = m->g_a[k] / m->W[k] + m->cv[k] * (T - m->T_ref);   /* J/kg */
        num += e_k * ydot[k];
        den += y[k] * m->cv[k];
    }
    ydot[S] = -num / den;
    if (wdot_out) memcpy(wdot_out, wdot, sizeof(double) * S);
    free(C);
    free(wdot);
}

/* ------------------------------------------------------------------------ */
/* Stiffness monitor: an upper bound of the spectral radius of the species    */
/* block of the chemistry Jacobian at fixed T (the stability statements of    */
/* the fast methods, Sec. 5.2, compare h times the fastest rate with the      */
/* method's stability interval).  In concentration variables -- a similarity */
/* transform of the mass-fraction variables (Y_k = C_k W_k / rho), so the     */
/* same eigenvalues -- d(omega_k)/d(C_l) = sum_j nu_kj dq_j/dC_l with          */
/* dq_j/dC_a = kf C_b, dq_j/dC_b = kf C_a, dq_j/dC_c = -kr C_d,               */
/* dq_j/dC_d = -kr C_c; by the triangle inequality every absolute row sum is  */
/* at most B_k = sum_j |nu_kj| w_j, w_j = kf (C_a + C_b) + kr (C_c + C_d),     */
/* and the spectral radius is at most max_k B_k (Gershgorin).                 */
/* ------------------------------------------------------------------------ */
double ora_stiff_bound(const ora_mech *m, const double *y)
{
    const int S = m->S, R = m->R;
    double *kf = (double *)malloc(sizeof(double) * R);
    double *kr = (double *)malloc(sizeof(double) * R);
    double *C = (double *)malloc(sizeof(double) * S);
    double *B = (double *)malloc(sizeof(double) * S);
    double *ydot = (double *)malloc(sizeof(double) * (S + 1));
    ora_chem_rhs_parts(m, y, ydot, kf, kr, NULL, NULL);
    const double rho_cgs = m->rho * 1e-3;
    for (int k = 0; k < S; ++k) {
        C[k] = rho_cgs * y[k] / (m->W[k] * 1e3);
        B[k] = 0.0;
    }
    for (int j = 0; j < R; ++j) {
        int a = m->reac[2 * j], b = m->reac[2 * j + 1];
        int c = m->prod[2 * j], d = m->prod[2 * j + 1];
        double w = kf[j] * (C[a] + C[b]) + kr[j] * (C[c] + C[d]);
        B[a] += w;          /* one term per occurrence: |nu| = 2 when a = b */
        B[b] += w;
        B[c] += w;
        B[d] += w;
    }
    double bmax = 0.0;
    for (int k = 0; k < S; ++k)
        if (B[k] > bmax) bmax = B[k];
    free(kf);
    free(kr);
    free(C);
    free(B);
    free(ydot);
    return bmax;
}

void ora_stiff_bound_soa(const ora_mech *m, int n_cells, int ld, const double *y, double *out)
{
    const int n = m->S + 1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n_cells; ++i) {
        double *v = (double *)malloc(sizeof(double) * n);
        for (int c = 0; c < n; ++c) v[c] = y[(size_t)c * ld + i];
        out[i] = ora_stiff_bound(m, v);
        free(v);
    }
}

void ora_chem_rhs(const ora_mech *m, const double *y, double *ydot)
{
    ora_chem_rhs_parts(m, y, ydot, NULL, NULL, NULL, NULL);
}

/* Specific internal energy of the mixture, E = sum_k Y_k e_k(T) (J/kg). */
double ora_energy(const ora_mech *m, const double *y)
{
    double E = 0.0, T = y[m->S];
    for (int k = 0; k < m->S; ++k)
        E += y[k] * (m->g_a[k] / m->W[k] + m->cv[k] * (T - m->T_ref));
    return E;
}

void ora_fast_rhs(const ora_fast *f, const double *y, double *ydot)
{
    if (f->kind == 0) {
        ora_chem_rhs(f->mech, y, ydot);
    } else {
        for (int i = 0; i < f->n; ++i) {
            double s = 0.0;
            for (int j = 0; j < f->n; ++j) s += f->A[i * f->n + j] * y[j];
            ydot[i] = s;
        }
    }
}

/* Batched RHS over SoA arrays y[comp*ld + cell]. */
void ora_fast_rhs_soa(const ora_fast *f, int n_cells, int ld, const double *y, double *ydot)
{
    const int n = f->n;
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * n);
        double *dv = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (int i = 0; i < n_cells; ++i) {
            for (int c = 0; c < n; ++c) v[c] = y[(size_t)c * ld + i];
            ora_fast_rhs(f, v, dv);
            for (int c = 0; c < n; ++c) ydot[(size_t)c * ld + i] = dv[c];
        }
        free(v);
        free(dv);
    }
}

/* Forcing polynomial r(tau) = sum_k tau^k rho_k, rho given as [n_poly][n]. */
static void forcing_eval(int n, int n_poly, const double *rho, double tau, double *r)
{
    for (int c = 0; c < n; ++c) {
        double acc = 0.0, tk = 1.0;
        for (int k = 0; k < n_poly; ++k) {
            acc += tk * rho[k * n + c];
            tk *= tau;
        }
        r[c] = acc;
    }
}

static int finite_vec(int n, const double *v)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int check_state(const ora_fast *f, const double *v)
{
    int st = 0;
    if (!finite_vec(f->n, v)) st |= ORA_ST_NONFINITE;
    if (f->kind == 0) {
        double T = v[f->n - 1];
        if (!(T >= 200.0 && T <= 6000.0)) st |= ORA_ST_TRANGE;
    }
    return st;
}

/* ------------------------------------------------------------------------ */
/* Classic RK4 over one fast stage of length L (the modified fast IVP of     */
/* Sec. 2.1, step 2b), n_sub uniform substeps h = L/n_sub; the forcing is    */
/* evaluated at tau = (m + c_r)/n_sub for RK node c_r of substep m.          */
/* ------------------------------------------------------------------------ */
int ora_rk4_stage(const ora_fast *f, const double *y_in, int n_poly, const double *rho,
                  double L, int n_sub, double *y_out)
{
    const int n = f->n;
    const double h = L / n_sub;
    double *v = (double *)malloc(sizeof(double) * n * 7);
    double *k1 = v + n, *k2 = v + 2 * n, *k3 = v + 3 * n, *k4 = v + 4 * n;
    double *tmp = v + 5 * n, *r = v + 6 * n;
    memcpy(v, y_in, sizeof(double) * n);
    for (int m = 0; m < n_sub; ++m) {
        double t0 = (double)m / n_sub, th = (m + 0.5) / n_sub, t1 = (double)(m + 1) / n_sub;
        ora_fast_rhs(f, v, k1);
        forcing_eval(n, n_poly, rho, t0, r);
        for (int c = 0; c < n; ++c) k1[c] += r[c];
        for (int c = 0; c < n; ++c) tmp[c] = v[c] + 0.5 * h * k1[c];
        ora_fast_rhs(f, tmp, k2);
        forcing_eval(n, n_poly, rho, th, r);
        for (int c = 0; c < n; ++c) k2[c] += r[c];
        for (int c = 0; c < n; ++c) tmp[c] = v[c] + 0.5 * h * k2[c];
        ora_fast_rhs(f, tmp, k3);
        for (int c = 0; c < n; ++c) k3[c] += r[c];
        for (int c = 0; c < n; ++c) tmp[c] = v[c] + h * k3[c];
        ora_fast_rhs(f, tmp, k4);
        forcing_eval(n, n_poly, rho, t1, r);
        for (int c = 0; c < n; ++c) k4[c] += r[c];
        for (int c = 0; c < n; ++c)
            v[c] = v[c] + (h / 6.0) * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    }
    memcpy(y_out, v, sizeof(double) * n);
    int st = check_state(f, v);
    free(v);
    return st;
}

/* ------------------------------------------------------------------------ */
/* General explicit Runge-Kutta method over one fast stage: s stages,        */
/* strictly lower-triangular A (row-major [s][s]), weights b, nodes c.  Each  */
/* substep stores every stage derivative and forms                           */
/*   Y_i = v + h sum_(j<i) a_ij k_j,  k_i = f(Y_i) + r((m + c_i)/n_sub),      */
/*   v <- v + h sum_i b_i k_i.                                                */
/* The fast methods of Sec. 3.2 of orders 2, 3 and 5 (the MRI-P(k) family):   */
/* Heun's method, the Bogacki-Shampine 3rd-order and the Cash-Karp 5th-order  */
/* solutions.                                                                  */
/* ------------------------------------------------------------------------ */
static const double HEUN_A[4] = {0.0, 0.0, 1.0, 0.0};
static const double HEUN_B[2] = {0.5, 0.5};
static const double HEUN_C[2] = {0.0, 1.0};
static const double BS3_A[9] = {0.0, 0.0, 0.0, 0.5, 0.0, 0.0, 0.0, 0.75, 0.0};
static const double BS3_B[3] = {2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0};
static const double BS3_C[3] = {0.0, 0.5, 0.75};
/* Cash-Karp: the 5th-order solution of the 5(4) pair (the order-5 fast method
   of Sec. 3.2). */
static const double CK5_A[36] = {
    0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
    1.0 / 5.0, 0.0, 0.0, 0.0, 0.0, 0.0,
    3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0, 0.0,
    3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0, 0.0,
    -11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0, 0.0,
    1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0, 0.0};
static const double CK5_B[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0,
                                512.0 / 1771.0};
static const double CK5_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};

/* The tableau of fixed-step method 2 (Heun), 3 (Bogacki-Shampine) or 4
   (Cash-Karp); returns the stage count (0 for other methods).  A is [s][s],
   b and c are [s]. */
int ora_erk_tableau(int method, double *A, double *b, double *c)
{
    const double *a0, *b0, *c0;
    int s;
    if (method == 2) {
        s = 2, a0 = HEUN_A, b0 = HEUN_B, c0 = HEUN_C;
    } else if (method == 3) {
        s = 3, a0 = BS3_A, b0 = BS3_B, c0 = BS3_C;
    } else if (method == 4) {
        s = 6, a0 = CK5_A, b0 = CK5_B, c0 = CK5_C;
    } else {
        return 0;
    }
    if (A) memcpy(A, a0, sizeof(double) * s * s);
    if (b) memcpy(b, b0, sizeof(double) * s);
    if (c) memcpy(c, c0, sizeof(double) * s);
    return s;
}

int ora_erk_stage(const ora_fast *f, const double *y_in, int n_poly, const double *rho,
                  double L, int n_sub, int s, const double *A, const double *b, const double *c,
                  double *y_out)
{
    const int n = f->n;
    const double h = L / n_sub;
    double *v = (double *)malloc(sizeof(double) * n * (s + 3));
    double *k = v + n, *tmp = v + (size_t)(s + 1) * n, *r = v + (size_t)(s + 2) * n;
    memcpy(v, y_in, sizeof(double) * n);
    for (int m = 0; m < n_sub; ++m) {
        for (int i = 0; i < s; ++i) {
            for (int e = 0; e < n; ++e) {
                double sum = 0.0;
                for (int j = 0; j < i; ++j) sum += A[i * s + j] * k[(size_t)j * n + e];
                tmp[e] = v[e] + h * sum;
            }
            ora_fast_rhs(f, tmp, k + (size_t)i * n);
            forcing_eval(n, n_poly, rho, (m + c[i]) / n_sub, r);
            for (int e = 0; e < n; ++e) k[(size_t)i * n + e] += r[e];
        }
        for (int e = 0; e < n; ++e) {
            double sum = 0.0;
            for (int i = 0; i < s; ++i) sum += b[i] * k[(size_t)i * n + e];
            v[e] = v[e] + h * sum;
        }
    }
    memcpy(y_out, v, sizeof(double) * n);
    int st = check_state(f, v);
    free(v);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Zonneveld 4(3) embedded pair (the 4th-order fast method of Sec. 3.2).     */
/* Stages 1-4 are classic RK4; stage 5 sits at c = 3/4.  The propagated      */
/* solution is the RK4 combination; the embedded 3rd-order combination gives */
/* the local error estimate.                                                  */
/* ------------------------------------------------------------------------ */
static const double ZV_C[5] = {0.0, 0.5, 0.5, 1.0, 0.75};
static const double ZV_A[5][4] = {
    {0.0, 0.0, 0.0, 0.0},
    {0.5, 0.0, 0.0, 0.0},
    {0.0, 0.5, 0.0, 0.0},
    {0.0, 0.0, 1.0, 0.0},
    {5.0 / 32.0, 7.0 / 32.0, 13.0 / 32.0, -1.0 / 32.0},
};
static const double ZV_B[5] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0, 0.0};
static const double ZV_BHAT[5] = {-0.5, 7.0 / 3.0, 7.0 / 3.0, 13.0 / 6.0, -16.0 / 3.0};

void ora_zonneveld_tableau(double *c5, double *a5x4, double *b5, double *bhat5)
{
    for (int i = 0; i < 5; ++i) {
        c5[i] = ZV_C[i];
        b5[i] = ZV_B[i];
        bhat5[i] = ZV_BHAT[i];
        for (int j = 0; j < 4; ++j) a5x4[i * 4 + j] = ZV_A[i][j];
    }
}

/*
 * One attempted Zonneveld step of size h from (t, v) within a stage of length
 * L.  Writes the propagated solution to v_new and returns the WRMS norm of
 * the error estimate with weights 1/(atol_c + rtol |v_c|) taken at the step
 * start.
 */
double ora_zonneveld_try(const ora_fast *f, const double *v, double t, double h, double L,
                         int n_poly, const double *rho, const ora_fast_opts *o, double *v_new)
{
    const int n = f->n;
    double *K = (double *)malloc(sizeof(double) * n * 5);
    double *tmp = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < 5; ++i) {
        for (int c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int j = 0; j < i && j < 4; ++j) acc += ZV_A[i][j] * K[j * n + c];
            tmp[c] = v[c] + h * acc;
        }
        ora_fast_rhs(f, tmp, K + i * n);
        forcing_eval(n, n_poly, rho, (t + ZV_C[i] * h) / L, r);
        for (int c = 0; c < n; ++c) K[i * n + c] += r[c];
    }
    double ssq = 0.0;
    for (int c = 0; c < n; ++c) {
        double sol = 0.0, err = 0.0;
        for (int i = 0; i < 5; ++i) {
            sol += ZV_B[i] * K[i * n + c];
            err += (ZV_B[i] - ZV_BHAT[i]) * K[i * n + c];
        }
        v_new[c] = v[c] + h * sol;
        double atol = (f->kind == 0 && c == n - 1) ? o->atol_T : o->atol_Y;
        double w = 1.0 / (atol + o->rtol * fabs(v[c]));
        double e = h * err * w;
        ssq += e * e;
    }
    free(K);
    free(tmp);
    free(r);
    return sqrt(ssq / n);
}

/*
 * Adaptive Zonneveld integration over one stage.  h_0 = h_max = L/10;
 * accept if err <= 1; h <- h * min(5, max(0.2, 0.9 err^(-1/4))); the last
 * step is clipped to land on L.  Decisions with |err - 1| < 1e-12 set the
 * near-tie flag.  `forced` (nullable) replays a decision sequence (1 accept,
 * 0 reject) instead of the err <= 1 test, for cells whose decisions tie.
 */
int ora_zonneveld_stage(const ora_fast *f, const double *y_in, int n_poly, const double *rho,
                        double L, const ora_fast_opts *o, double *y_out,
                        int32_t *n_accept, int32_t *n_reject,
                        const int8_t *forced, int n_forced)
{
    const int n = f->n;
    double *v = (double *)malloc(sizeof(double) * n);
    double *vn = (double *)malloc(sizeof(double) * n);
    memcpy(v, y_in, sizeof(double) * n);
    const double h_max = L / 10.0;
    double h = h_max, t = 0.0;
    int acc = 0, rej = 0, st = 0, done = 0, dec = 0;
    const int max_attempts = 4 * o->max_steps;
    while (!done) {
        if (acc >= o->max_steps || acc + rej >= max_attempts) {
            st |= ORA_ST_MAXSTEPS;
            break;
        }
        double hs = h < h_max ? h : h_max;
        int last = 0;
        if (t + hs >= L - 1e-12 * L) {
            hs = L - t;
            last = 1;
        }
        double err = ora_zonneveld_try(f, v, t, hs, L, n_poly, rho, o, vn);
        /* a non-finite estimate (overflow in a too-large step) is a rejection */
        if (!isfinite(err)) err = HUGE_VAL;
        if (fabs(err - 1.0) < 1e-12) st |= ORA_ST_NEARTIE;
        int accept = (err <= 1.0);
        if (forced && dec < n_forced) accept = forced[dec];
        ++dec;
        double fac = (err == 0.0) ? 5.0 : 0.9 * pow(err, -0.25);
        if (fac > 5.0) fac = 5.0;
        if (fac < 0.2) fac = 0.2;
        if (accept) {
            memcpy(v, vn, sizeof(double) * n);
            t = last ? L : t + hs;
            ++acc;
            if (last) done = 1;
        } else {
            ++rej;
        }
        h = hs * fac;
    }
    memcpy(y_out, v, sizeof(double) * n);
    st |= check_state(f, v);
    if (n_accept) *n_accept = acc;
    if (n_reject) *n_reject = rej;
    free(v);
    free(vn);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Batched fast stage over SoA arrays: rho_poly[k*n*ld + c*ld + cell].       */
/* ------------------------------------------------------------------------ */
void ora_fast_stage_soa(const ora_fast *f, const ora_fast_opts *o, int n_cells, int ld,
                        const double *y_in, double *y_out, int n_poly, const double *rho_poly,
                        double L, int32_t *status, int32_t *steps, int32_t *rejects)
{
    const int n = f->n;
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * n);
        double *w = (double *)malloc(sizeof(double) * n);
        double *rho = (double *)malloc(sizeof(double) * n * (n_poly > 0 ? n_poly : 1));
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < n_cells; ++i) {
            for (int c = 0; c < n; ++c) v[c] = y_in[(size_t)c * ld + i];
            for (int k = 0; k < n_poly; ++k)
                for (int c = 0; c < n; ++c)
                    rho[k * n + c] = rho_poly[(size_t)k * n * ld + (size_t)c * ld + i];
            int st;
            int32_t acc = 0, rej = 0;
            if (o->method == 0) {
                st = ora_rk4_stage(f, v, n_poly, rho, L, o->n_sub, w);
                acc = o->n_sub;
            } else if (o->method >= 2 && o->method <= 4) {
                double A[36], b[6], c[6];
                const int s = ora_erk_tableau(o->method, A, b, c);
                st = ora_erk_stage(f, v, n_poly, rho, L, o->n_sub, s, A, b, c, w);
                acc = o->n_sub;
            } else {
                st = ora_zonneveld_stage(f, v, n_poly, rho, L, o, w, &acc, &rej, NULL, 0);
            }
            for (int c = 0; c < n; ++c) y_out[(size_t)c * ld + i] = w[c];
            if (status) status[i] = st;
            if (steps) steps[i] = acc;
            if (rejects) rejects[i] = rej;
        }
        free(v);
        free(w);
        free(rho);
    }
}

/* ------------------------------------------------------------------------ */
/* Slow right-hand sides.                                                     */
/* ------------------------------------------------------------------------ */
/* Slow RHS callback: f^S evaluated at (t, Y) for the stage with index j.    */
typedef void (*ora_slow_fn)(void *ctx, int j, double t, const double *y, double *fy,
                            int n_comp, int n_cells, int ld);

/* Given slow evaluations: fy = F[j] (tests feed fixed tendencies). */
typedef struct {
    const double *F;                     /* [s-1][n][ld] */
} ora_slow_given_ctx;

void ora_slow_given(void *ctx, int j, double t, const double *y, double *fy,
                    int n_comp, int n_cells, int ld)
{
    (void)t;
    (void)y;
    (void)n_cells;
    const ora_slow_given_ctx *g = (const ora_slow_given_ctx *)ctx;
    memcpy(fy, g->F + (size_t)j * n_comp * ld, sizeof(double) * (size_t)n_comp * ld);
}

/* Linear slow RHS: f^S = A y with a dense [n][n] A, cell by cell. */
typedef struct {
    const double *A;
} ora_slow_linear_ctx;

void ora_slow_linear(void *ctx, int j, double t, const double *y, double *fy,
                     int n_comp, int n_cells, int ld)
{
    (void)j;
    (void)t;
    const ora_slow_linear_ctx *g = (const ora_slow_linear_ctx *)ctx;
    for (int i = 0; i < n_cells; ++i)
        for (int r = 0; r < n_comp; ++r) {
            double s = 0.0;
            for (int c = 0; c < n_comp; ++c) s += g->A[r * n_comp + c] * y[(size_t)c * ld + i];
            fy[(size_t)r * ld + i] = s;
        }
}

/*
 * Advection-diffusion slow RHS for every field phi (Sec. 3, eq. problem2,
 * transport terms, discretized with 2nd-order centred stencils on a periodic
 * grid as in Sec. 3.1):  f = -u . grad(phi) + D lap(phi).  Cell index
 * (z*ny + y)*nx + x.
 */
typedef struct {
    int nx, ny, nz;
    double u[3], D, dx;
} ora_advdiff_ctx;

void ora_advdiff(const ora_advdiff_ctx *g, int n_comp, int ld, const double *y, double *fy)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const double dx = g->dx;
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < n_comp; ++c)
        for (int z = 0; z < nz; ++z)
            for (int yy = 0; yy < ny; ++yy)
                for (int x = 0; x < nx; ++x) {
                    const double *p = y + (size_t)c * ld;
                    int xm = (x + nx - 1) % nx, xp = (x + 1) % nx;
                    int ym = (yy + ny - 1) % ny, yp = (yy + 1) % ny;
                    int zm = (z + nz - 1) % nz, zp = (z + 1) % nz;
#define IDX(X, Y, Z) (((size_t)(Z) * ny + (Y)) * nx + (X))
                    double ctr = p[IDX(x, yy, z)];
                    double pxm = p[IDX(xm, yy, z)], pxp = p[IDX(xp, yy, z)];
                    double pym = p[IDX(x, ym, z)], pyp = p[IDX(x, yp, z)];
                    double pzm = p[IDX(x, yy, zm)], pzp = p[IDX(x, yy, zp)];
                    double adv = g->u[0] * (pxp - pxm) / (2.0 * dx) +
                                 g->u[1] * (pyp - pym) / (2.0 * dx) +
                                 g->u[2] * (pzp - pzm) / (2.0 * dx);
                    double lap = (pxp + pxm + pyp + pym + pzp + pzm - 6.0 * ctr) / (dx * dx);
                    fy[(size_t)c * ld + IDX(x, yy, z)] = -adv + g->D * lap;
#undef IDX
                }
}

void ora_slow_advdiff(void *ctx, int j, double t, const double *y, double *fy,
                      int n_comp, int n_cells, int ld)
{
    (void)j;
    (void)t;
    (void)n_cells;
    ora_advdiff((const ora_advdiff_ctx *)ctx, n_comp, ld, y, fy);
}

/* ------------------------------------------------------------------------ */
/* Explicit MRI-GARK slow step (Sec. 2.1, steps 1-3):                        */
/*   Y_1 = y_n;  for i = 2..s: forcing from f^S(T_j, Y_j), j < i, solve the   */
/*   modified fast IVP over [T_(i-1), T_i] from Y_(i-1), Y_i = v(T_i);        */
/*   y_(n+1) = Y_s.                                                           */
/* The forcing of stage i is r_i(tau) = (1/dc_i) sum_k tau^k sum_j           */
/* Gamma^(k)_ij F_j with tau in [0, 1] the normalized time within the stage.  */
/* Returns the number of slow RHS evaluations performed.                      */
/* ------------------------------------------------------------------------ */
int ora_mri_step(const ora_fast *f, const ora_table *tb, const ora_fast_opts *o,
                 ora_slow_fn fS, void *ctx, double t, double H, int n_cells, int ld,
                 double *y, int32_t *status, int32_t *steps)
{
    const int n = f->n, s = tb->s, ng = tb->n_gamma;
    const size_t vec = (size_t)n * ld;
    double *F = (double *)calloc((size_t)s * vec, sizeof(double));
    double *rho = (double *)calloc((size_t)ng * vec, sizeof(double));
    double *ynew = (double *)calloc(vec, sizeof(double));
    int32_t *st = (int32_t *)calloc((size_t)ld, sizeof(int32_t));
    int32_t *stp = (int32_t *)calloc((size_t)ld, sizeof(int32_t));
    int n_slow = 0;
    if (status) memset(status, 0, sizeof(int32_t) * ld);
    if (steps) memset(steps, 0, sizeof(int32_t) * ld);
    /* step 1: Y_1 = y_n, T_1 = t_n */
    fS(ctx, 0, t, y, F, n, n_cells, ld);
    ++n_slow;
    for (int i = 1; i < s; ++i) {
        double dc = tb->c[i] - tb->c[i - 1];
        double L = dc * H;
        /* step 2a: forcing coefficients from the slow evaluations F_j, j < i */
        for (int k = 0; k < ng; ++k)
            for (size_t e = 0; e < vec; ++e) {
                double acc = 0.0;
                for (int j = 0; j < i; ++j)
                    acc += tb->gamma[((size_t)k * s + i) * s + j] * F[(size_t)j * vec + e];
                rho[(size_t)k * vec + e] = acc / dc;
            }
        /* steps 2b-2c: modified fast IVP from Y_(i-1) over the stage */
        ora_fast_stage_soa(f, o, n_cells, ld, y, ynew, ng, rho, L, st, stp, NULL);
        memcpy(y, ynew, sizeof(double) * vec);
        for (int c = 0; c < n_cells; ++c) {
            if (status) status[c] |= st[c];
            if (steps) steps[c] += stp[c];
        }
        if (i < s - 1) {
            fS(ctx, i, t + tb->c[i] * H, y, F + (size_t)i * vec, n, n_cells, ld);
            ++n_slow;
        }
    }
    /* step 3: y_(n+1) = Y_s (already in y) */
    free(F);
    free(rho);
    free(ynew);
    free(st);
    free(stp);
    return n_slow;
}

/* Convenience wrappers with the built-in slow right-hand sides. */
int ora_mri_step_given(const ora_fast *f, const ora_table *tb, const ora_fast_opts *o,
                       const double *Fgiven, double t, double H, int n_cells, int ld,
                       double *y, int32_t *status, int32_t *steps)
{
    ora_slow_given_ctx g = {Fgiven};
    return ora_mri_step(f, tb, o, ora_slow_given, &g, t, H, n_cells, ld, y, status, steps);
}

int ora_mri_step_linear(const ora_fast *f, const ora_table *tb, const ora_fast_opts *o,
                        const double *AS, double t, double H, int n_cells, int ld,
                        double *y, int32_t *status, int32_t *steps)
{
    ora_slow_linear_ctx g = {AS};
    return ora_mri_step(f, tb, o, ora_slow_linear, &g, t, H, n_cells, ld, y, status, steps);
}

int ora_mri_step_advdiff(const ora_fast *f, const ora_table *tb, const ora_fast_opts *o,
                         const ora_advdiff_ctx *g, double t, double H, int n_cells, int ld,
                         double *y, int32_t *status, int32_t *steps)
{
    return ora_mri_step(f, tb, o, ora_slow_advdiff, (void *)g, t, H, n_cells, ld, y, status,
                        steps);
}

/* ------------------------------------------------------------------------ */
/* Central-difference Jacobian of f^F at y: J[i*n + j] = d f_i / d y_j.      */
/* ------------------------------------------------------------------------ */
void ora_jacobian_fd(const ora_fast *f, const double *y, double *J)
{
    const int n = f->n;
    double *yp = (double *)malloc(sizeof(double) * n);
    double *fp = (double *)malloc(sizeof(double) * n);
    double *fm = (double *)malloc(sizeof(double) * n);
    for (int j = 0; j < n; ++j) {
        memcpy(yp, y, sizeof(double) * n);
        double scale = fabs(y[j]);
        double floor_ = (f->kind == 0 && j == n - 1) ? 1.0 : 1e-6;
        if (scale < floor_) scale = floor_;
        double eps = 1e-6 * scale;
        yp[j] = y[j] + eps;
        ora_fast_rhs(f, yp, fp);
        yp[j] = y[j] - eps;
        ora_fast_rhs(f, yp, fm);
        for (int i = 0; i < n; ++i) J[i * n + j] = (fp[i] - fm[i]) / (2.0 * eps);
    }
    free(yp);
    free(fp);
    free(fm);
}

/* Jacobians of many cells (SoA input), output J[cell][n][n]. */
void ora_jacobian_fd_soa(const ora_fast *f, int n_cells, int ld, const double *y, double *J)
{
    const int n = f->n;
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (int i = 0; i < n_cells; ++i) {
            for (int c = 0; c < n; ++c) v[c] = y[(size_t)c * ld + i];
            ora_jacobian_fd(f, v, J + (size_t)i * n * n);
        }
        free(v);
    }
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
