// mri_dev.h -- device-side data structures and launchers of the ahead-of-time
// compiled kernels of libmri (generic fast-stage kernels and helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spec_abi.h"

// Mechanism in the packed form the kernels use.  Species block sp[k*6 + i]:
//   0 CF = rho_cgs / W_g         (C_k = CF * Y_k, mol/cm^3)
//   1 WF = W_g / rho_cgs         (dY_k/dt = WF * omega_k)
//   2 AR = g_a / R,  3 BR = g_b / R   (g_k/(R T) = AR/T + BR)
//   4 EA = g_a / W (J/kg),  5 CV
// Reaction block rx[j*3 + i]: 0 ln A' = ln A - BR_a - BR_b, 1 beta,
//   2 theta' = theta + AR_a + AR_b, so that
//   kappa_j = exp(ln A' + beta ln T - theta'/T) = k_f exp(-(g_a + g_b)/(R T)).
// rxi[j] = a | b << 8 | c << 16 | d << 24.  The device copy the generic
// kernels read holds AR, BR, ln A' and theta' multiplied by log2(e) (base-2
// exponentials; beta then multiplies log2 T).
struct GenMech {
    int S, R;
    const double *sp;
    const double *rx;
    const uint32_t *rxi;
    double T_ref;
};

constexpr int GEN_SP_STRIDE = 6;

// Largest species count of each generic-kernel instantiation.
constexpr int GEN_NMAX_SMALL = 24;
constexpr int GEN_NMAX_LARGE = 56;

size_t gen_lds_bytes(int S, int R, int block);

// Fixed-step explicit RK method whose stage inputs use only the previous
// stage derivative (classic RK4, Heun, Bogacki-Shampine): per stage i the node
// c[i], the weight b[i] and a[i] = a_(i+1,i), the coefficient of k_i in the
// next stage input (a[s-1] unused).
struct ErkCoef {
    int s;
    double c[4], b[4], a[4];
};

// Fixed-step explicit RK method with a general strictly lower-triangular
// tableau of at most ERK_SMAX stages (Cash-Karp's 5th-order solution).  The
// kernels keep the stage derivatives in registers, so mechanisms are limited
// to GEN_NMAX_SMALL species.
constexpr int ERK_SMAX = 6;
struct ErkFull {
    int s;
    double c[ERK_SMAX], b[ERK_SMAX], a[ERK_SMAX][ERK_SMAX];
};

// n_live (nullable, device): cells at or beyond *n_live are skipped, so a
// launch sized for n_cells can serve a count known only on the device.
hipError_t launch_gen_erk(const GenMech &gm, const ErkFull &e, int block, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          const unsigned int *n_live, hipStream_t s);
hipError_t launch_lin_erk(int n, const double *A, const ErkFull &e, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          hipStream_t s);

hipError_t launch_gen_rk4(const GenMech &gm, const ErkCoef &e, int block, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          const unsigned int *n_live, hipStream_t s);
// Stiffness monitor: bound[i] = B (1/s; nullable), B an upper bound of the
// spectral radius of the species block of the chemistry Jacobian at fixed T;
// status[i] (nullable) gets `flag` where h B > limit, OR-ed in when accumulate
// is set, written otherwise (steps[i], nullable, then set to 0, so that a
// stage launched after it with accumulate set counts from zero).
hipError_t launch_gen_stiff(const GenMech &gm, int n_cells, int ld, const double *y, double h,
                            double limit, double *bound, int *status, int *steps, int accumulate,
                            int flag, hipStream_t s);
hipError_t launch_gen_zv(const GenMech &gm, int block, int n_cells, int ld, const double *yin,
                         double *yout, int n_poly, const double *rho, double L, ZvOpts o,
                         int *status, int *steps, int accumulate, const unsigned int *n_live,
                         hipStream_t s);

// Linear test mode: f = A v, n <= 16, A row-major on the device.
hipError_t launch_lin_rk4(int n, const double *A, const ErkCoef &e, int n_cells, int ld,
                          const double *yin, double *yout, int n_poly, const double *rho,
                          double L, int n_sub, int *status, int *steps, int accumulate,
                          hipStream_t s);

// rho[k][e] = sum_{j < nj} coef[k*8 + j] * F[j][e], e < n_elem, k < n_gamma.
struct ForcingCoef {
    double c[4 * 8];
};
hipError_t launch_forcing(long long n_elem, int n_gamma, int nj, const double *F,
                          long long F_stride, ForcingCoef coef, double *rho, hipStream_t s);

hipError_t launch_advdiff(int nx, int ny, int nz, int n_comp, int ld, const double *u,
                          double D, double dx, const double *y, double *fy, hipStream_t s);
hipError_t launch_lin_apply(int n, const double *A, int n_cells, int ld, const double *y,
                            double *fy, hipStream_t s);
hipError_t launch_status_count(const int32_t *status, int n_cells, int32_t mask,
                               unsigned long long *count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s);
// adaptive slow steps: partial reductions of the step-doubling error (one
// partial per 256-cell block) and the status merge of an accepted step
inline int step_err_blocks(int n_cells) { return (n_cells + 255) / 256; }
hipError_t launch_step_err(int n, int t_comp, int n_cells, int ld, const double *y_half,
                           const double *y_full, double scale, double rtol, double atol,
                           double atol_t, const int32_t *sp_a, const int32_t *sp_b,
                           double *part_w2, long long *part_steps, hipStream_t s);
hipError_t launch_status_merge(int n_cells, const int32_t *st_a, const int32_t *st_b,
                               int32_t *status_out, hipStream_t s);
hipError_t launch_exp2_t256(const double *x, double *y, int n, hipStream_t s);
hipError_t launch_exp2(const double *x, double *y, int n, hipStream_t s);
