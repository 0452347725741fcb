// mri_internal.h -- functions shared between libmri's host translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "mri.h"

// Records the thread-local error text and returns st.
mri_status mri_fail(mri_status st, const char *fmt, ...);

// One fast stage (options validated here), used by the surrogate.  n_live
// (nullable, device): only cells below *n_live are integrated (a launch sized
// for n_cells serving a count the device computed); accumulate ORs status and
// adds steps.
mri_status mri_internal_fast_stage(mri_mech *m, const mri_fast_opts *o, int n_cells, int ld,
                                   const double *yin, double *yout, int n_poly, const double *rho,
                                   double L, int32_t *status, int32_t *steps, hipStream_t s,
                                   const unsigned int *n_live = nullptr, int accumulate = 0);
int mri_internal_state_width(const mri_mech *m);
// Argument checks of mri_slow_step (everything but y and the workspace).
mri_status mri_internal_check_slow_step(const mri_mech *m, const mri_table *t,
                                        const mri_fast_opts *opts, mri_slow_rhs f_slow,
                                        double t0, double H, int n_cells, int ld);
// One slow step (Sec. 2.1) on validated arguments with caller-provided slow
// evaluations F [s-1][n][ld] and forcing rho [n_gamma][n][ld]; timed = 0 records
// no events.
mri_status mri_internal_slow_step(mri_mech *m, const mri_table *t, const mri_fast_opts *opts,
                                  mri_slow_rhs f_slow, void *user, double t0, double H,
                                  int n_cells, int ld, double *y, double *F, double *rho,
                                  int32_t *status_out, int32_t *steps_out, int timed,
                                  hipStream_t s);
// True when a fast stage with these options would first copy the mechanism to
// the device or compile / load a specialized kernel.
bool mri_internal_stage_needs_setup(mri_mech *m, const mri_fast_opts *o, int n_poly);
int mri_internal_table_stages(const mri_table *t);
int mri_internal_table_terms(const mri_table *t);
int mri_internal_is_chem(const mri_mech *m);

#define MRI_HIP_TRY(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return mri_fail(MRI_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)
