// noalloc.hip -- the slow step for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Its slow evaluations and forcing planes live in a file-scope
// device array instead of a caller workspace.
//
// The array is a device symbol: host code never uses its name as an address.
// Its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and kept per device; kernels receive that
// address, exactly as they receive the workspace in mri_slow_step.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mri.h"
#include "mri_internal.h"

namespace {

constexpr size_t kScratchBytes = MRI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Slow evaluations F [s-1][n][ld] followed by the forcing planes rho [n_gamma][n][ld].
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device.
mri_status scratch_ptr(double **out)
{
    int dev = -1;
    MRI_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return mri_fail(MRI_EUNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        MRI_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return mri_fail(MRI_EHIP, "hipGetSymbolAddress returned NULL");
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return MRI_OK;
}

}  // namespace

extern "C" {

size_t mri_noalloc_scratch_bytes(void) { return kScratchBytes; }

mri_status mri_slow_step_noalloc(const mri_mech *mc, const mri_table *t,
                                 const mri_fast_opts *opts, mri_slow_rhs f_slow, void *user,
                                 double t0, double H, int n_cells, int ld, double *y,
                                 int32_t *status_out, int32_t *steps_out, mri_stream_t stream)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    mri_status st = mri_internal_check_slow_step(m, t, opts, f_slow, t0, H, n_cells, ld);
    if (st != MRI_OK) return st;
    const int n = mri_internal_state_width(m);
    const int s = mri_internal_table_stages(t), ng = mri_internal_table_terms(t);
    const size_t vec = (size_t)n * (size_t)ld;
    const size_t need = sizeof(double) * vec * (size_t)(s - 1 + ng);
    if (need > kScratchBytes)
        return mri_fail(MRI_EINVAL,
                        "slow step needs %zu bytes of scratch, more than the %zu this entry "
                        "point holds (n * ld * (s - 1 + n_gamma) doubles); use mri_slow_step",
                        need, kScratchBytes);
    if (n_cells == 0) return MRI_OK;
    if (!y) return mri_fail(MRI_EINVAL, "y is NULL");
    if (mri_internal_stage_needs_setup(m, opts, ng))
        return mri_fail(MRI_EINVAL,
                        "the fast-stage kernel is not set up on the device yet: run one "
                        "mri_fast_stage or mri_slow_step with the same options and number of "
                        "forcing terms first");
    double *base = nullptr;
    st = scratch_ptr(&base);
    if (st != MRI_OK) return st;
    double *F = base;
    double *rho = base + (size_t)(s - 1) * vec;
    return mri_internal_slow_step(m, t, opts, f_slow, user, t0, H, n_cells, ld, y, F, rho,
                                  status_out, steps_out, 0, (hipStream_t)stream);
}

}  // extern "C"
