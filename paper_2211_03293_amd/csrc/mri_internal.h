// mri_internal.h -- functions shared between libmri's host translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "mri.h"

// Records the thread-local error text and returns st.
mri_status mri_fail(mri_status st, const char *fmt, ...);

// One fast stage (validated options), used by the surrogate's fallback path.
mri_status mri_internal_fast_stage(mri_mech *m, const mri_fast_opts *o, int n_cells, int ld,
                                   const double *yin, double *yout, int n_poly, const double *rho,
                                   double L, int32_t *status, int32_t *steps, hipStream_t s);
int mri_internal_state_width(const mri_mech *m);
int mri_internal_is_chem(const mri_mech *m);

#define MRI_HIP_TRY(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return mri_fail(MRI_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)
