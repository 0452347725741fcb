"""ctypes binding of libmri (include/mri.h): argument marshalling only.

Every computation runs in libmri's HIP kernels.  Device arrays are torch CUDA
tensors (float64 / int32, contiguous); streams are torch streams.  Importing
this module loads libmri.so and fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MRI_LIB_PATH") or os.path.join(_HERE, "libmri.so")

MRI_OK, MRI_EINVAL, MRI_EHIP, MRI_ENONFINITE, MRI_EMAXSTEPS, MRI_ENOMEM, MRI_EUNSUPPORTED, \
    MRI_ECOMPILE, MRI_ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7, -8
CELL_NONFINITE, CELL_MAXSTEPS, CELL_TRANGE, CELL_NEARTIE, CELL_STIFF = 1, 2, 4, 8, 16
FAST_RK4, FAST_ZONNEVELD43, FAST_HEUN, FAST_BS3, FAST_CK5 = 0, 1, 2, 3, 4
KERNEL_AUTO, KERNEL_GENERIC, KERNEL_SPECIALIZED = 0, 1, 2


class MriError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmri status {status}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2211_03293_amd.build.build()")

# torch ships its own HIP runtime under the same soname as the system one that
# libmri links.  Loaded first, it is the one libmri binds to, so the process
# holds a single HIP runtime whichever module the caller imports first (with
# libmri loaded first, the two runtimes do not see the same devices).
try:
    import torch  # noqa: F401
except ImportError:
    pass

lib = C.CDLL(LIB_PATH)


class mri_mech_desc(C.Structure):
    _fields_ = [("n_species", C.c_int), ("n_reactions", C.c_int),
                ("reactants", C.POINTER(C.c_int32)), ("products", C.POINTER(C.c_int32)),
                ("lnA", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("theta", C.POINTER(C.c_double)), ("g_a", C.POINTER(C.c_double)),
                ("g_b", C.POINTER(C.c_double)), ("W", C.POINTER(C.c_double)),
                ("cv", C.POINTER(C.c_double)), ("rho", C.c_double), ("T_ref", C.c_double)]


class mri_table_desc(C.Structure):
    _fields_ = [("s", C.c_int), ("n_gamma", C.c_int), ("c", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double))]


class mri_fast_opts(C.Structure):
    _fields_ = [("method", C.c_int), ("n_sub", C.c_int), ("rtol", C.c_double),
                ("atol_Y", C.c_double), ("atol_T", C.c_double), ("max_steps", C.c_int),
                ("kernel", C.c_int), ("block_size", C.c_int), ("stiff_limit", C.c_double)]


class mri_imex_table_desc(C.Structure):
    _fields_ = [("s", C.c_int), ("n_gamma", C.c_int), ("c", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double))]


class mri_tune_trial(C.Structure):
    _fields_ = [("block_size", C.c_int), ("n_blocks", C.c_int), ("waves_per_simd", C.c_int),
                ("exp_table", C.c_int), ("sched_window", C.c_int), ("ms", C.c_float)]


class mri_advdiff_params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("n_comp", C.c_int),
                ("u", C.c_double * 3), ("D", C.c_double), ("dx", C.c_double)]


class mri_imex_advdiff(C.Structure):
    _fields_ = [("grid", mri_advdiff_params), ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int),
                ("cg_ws", C.c_void_p), ("cg_ws_bytes", C.c_size_t), ("cg_iters", C.c_int),
                ("cg_solves", C.c_int)]


class mri_adapt_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("H0", C.c_double), ("H_min", C.c_double), ("H_max", C.c_double),
                ("order", C.c_int), ("max_attempts", C.c_int), ("safety", C.c_double),
                ("fac_min", C.c_double), ("fac_max", C.c_double)]


class mri_adapt_stats(C.Structure):
    _fields_ = [("accepted", C.c_int), ("rejected", C.c_int), ("t", C.c_double),
                ("H_last", C.c_double), ("H_next", C.c_double), ("err_last", C.c_double),
                ("fast_steps", C.c_int64)]


class mri_counters(C.Structure):
    _fields_ = [("slow_evals", C.c_int64), ("fast_stages", C.c_int64),
                ("cell_stages", C.c_int64), ("specializations", C.c_int64)]


_vp, _i, _d, _sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_SIGS = {
    "mri_abi_version": (_i, []),
    "mri_last_error": (C.c_char_p, []),
    "mri_mech_create": (_i, [C.POINTER(mri_mech_desc), C.POINTER(_vp)]),
    "mri_mech_create_linear": (_i, [_i, C.POINTER(C.c_double), C.POINTER(_vp)]),
    "mri_mech_destroy": (None, [_vp]),
    "mri_mech_state_width": (_i, [_vp]),
    "mri_mech_specialize": (_i, [_vp, _i, _i, C.POINTER(_sz)]),
    "mri_mech_specialize_method": (_i, [_vp, _i, _i, _i, _i, C.POINTER(_sz)]),
    "mri_mech_code_hash": (_i, [_vp, _i, _i, _i, C.POINTER(C.c_uint64)]),
    "mri_mech_specialize_monitor": (_i, [_vp, _i, C.POINTER(_sz)]),
    "mri_table_create": (_i, [C.POINTER(mri_table_desc), C.POINTER(_vp)]),
    "mri_table_destroy": (None, [_vp]),
    "mri_fast_stage": (_i, [_vp, C.POINTER(mri_fast_opts), _i, _i, _vp, _vp, _i, _vp, _d, _vp,
                            _vp, _vp]),
    "mri_workspace_bytes": (_i, [_vp, _vp, _i, _i, C.POINTER(_sz)]),
    "mri_slow_step": (_i, [_vp, _vp, C.POINTER(mri_fast_opts), _vp, _vp, _d, _d, _i, _i, _vp,
                           _vp, _sz, _vp, _vp, _vp]),
    "mri_slow_step_noalloc": (_i, [_vp, _vp, C.POINTER(mri_fast_opts), _vp, _vp, _d, _d, _i, _i,
                                   _vp, _vp, _vp, _vp]),
    "mri_noalloc_scratch_bytes": (_sz, []),
    "mri_adaptive_workspace_bytes": (_i, [_vp, _vp, _i, _i, C.POINTER(_sz)]),
    "mri_adaptive_run": (_i, [_vp, _vp, C.POINTER(mri_fast_opts), C.POINTER(mri_adapt_opts), _vp,
                              _vp, _d, _d, _i, _i, _vp, _vp, _sz, _vp,
                              C.POINTER(mri_adapt_stats), _vp]),
    "mri_advdiff_slow_rhs": (_i, [_d, _vp, _vp, _i, _i, _vp, _vp]),
    "mri_linear_slow_rhs": (_i, [_d, _vp, _vp, _i, _i, _vp, _vp]),
    "mri_imex_table_create": (_i, [C.POINTER(mri_imex_table_desc), C.POINTER(_vp)]),
    "mri_imex_table_destroy": (None, [_vp]),
    "mri_imex_workspace_bytes": (_i, [_vp, _vp, _i, _i, C.POINTER(_sz)]),
    "mri_imex_slow_step": (_i, [_vp, _vp, C.POINTER(mri_fast_opts), _vp, _vp, _vp, _vp, _d, _d,
                                _i, _i, _vp, _vp, _sz, _vp, _vp, _vp]),
    "mri_diffusion_solve_workspace_bytes": (_i, [C.POINTER(mri_advdiff_params), _i,
                                                 C.POINTER(_sz)]),
    "mri_advection_rhs": (_i, [_d, _vp, _vp, _i, _i, _vp, _vp]),
    "mri_diffusion_rhs": (_i, [_d, _vp, _vp, _i, _i, _vp, _vp]),
    "mri_diffusion_solve": (_i, [_d, _d, _vp, _vp, _i, _i, _vp, _vp]),
    "mri_selftest_exp2": (_i, [_vp, _vp, _i, _vp]),
    "mri_selftest_exp2_t256": (_i, [_vp, _vp, _i, _vp]),
    "mri_status_count": (_i, [_vp, _i, C.c_int32, C.POINTER(C.c_int64), _vp]),
    "mri_stiffness_check": (_i, [_vp, _i, _i, _vp, _d, _d, _vp, _vp, _vp]),
    "mri_get_counters": (None, [C.POINTER(mri_counters)]),
    "mri_reset_counters": (None, []),
    "mri_timing_enable": (_i, [_i]),
    "mri_timing_read": (_i, [C.POINTER(C.c_double), C.POINTER(C.c_int64), _i]),
    "mri_batch_plan_code_hash": (_i, [_vp, _i, C.POINTER(C.c_uint64)]),
    "mri_batch_plan_tune_log": (_i, [_vp, _i, C.POINTER(mri_tune_trial), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(mri_tune_trial)]),
    "mri_batch_plan_create": (_i, [_vp, C.POINTER(mri_fast_opts), _i, C.POINTER(C.c_int64),
                                   C.POINTER(_vp)]),
    "mri_batch_run": (_i, [_vp, _vp, _vp, C.c_int64, _i, _vp, C.POINTER(C.c_double), _vp, _vp,
                           _vp, _vp]),
    "mri_batch_plan_tile": (_i, [_vp, C.POINTER(_i), C.POINTER(_i)]),
    "mri_batch_lane_stats": (_i, [_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), _vp]),
    "mri_batch_plan_destroy": (None, [_vp]),
    "mri_forcing_assemble": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "mri_mlp_create": (_i, [_i, C.POINTER(C.c_int), C.POINTER(C.c_float), _i, C.POINTER(_vp)]),
    "mri_mlp_destroy": (None, [_vp]),
    "mri_mlp_param_count": (C.c_int64, [_vp]),
    "mri_mlp_get_params": (_i, [_vp, C.POINTER(C.c_float)]),
    "mri_mlp_get_grads": (_i, [_vp, C.POINTER(C.c_float)]),
    "mri_mlp_forward": (_i, [_vp, _i, _vp, _vp, _vp]),
    "mri_mlp_backward": (_i, [_vp, _i, _vp, _vp, _vp]),
    "mri_adam_step": (_i, [_vp, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    "mri_mlp_feature_stats": (_i, [C.c_int64, C.c_int64, _vp, _i, _vp, _vp, _vp, _vp, _vp,
                                   _vp]),
    "mri_mlp_featurize": (_i, [_i, _vp, C.c_int64, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp]),
    "mri_surrogate_create": (_i, [C.POINTER(C.c_int), C.POINTER(C.c_float),
                                  C.POINTER(C.c_double), C.POINTER(_vp)]),
    "mri_surrogate_destroy": (None, [_vp]),
    "mri_surrogate_infer": (_i, [_vp, _i, _i, _vp, _vp, _vp, _i, _vp, _d, _vp]),
    "mri_surrogate_gate": (_i, [_i, _i, _vp, _i, _vp, _d, _vp, _vp, _vp, _vp, _d, _d, _vp, _vp,
                                _vp, _vp, _vp, _vp]),
    "mri_surrogate_workspace_bytes": (_i, [_i, _i, _i, C.POINTER(_sz)]),
    "mri_surrogate_stage": (_i, [_vp, _vp, C.POINTER(mri_fast_opts), C.POINTER(mri_fast_opts), _d,
                                 _i, _i, _vp, _vp, _i, _vp, _d, _vp, _vp, _vp, _vp, _vp, _sz,
                                 _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(st):
    if st != MRI_OK:
        raise MriError(st, lib.mri_last_error().decode())


def last_error() -> str:
    return lib.mri_last_error().decode()


def _ptr(t, dtype=None):
    """Device address of a tensor, None for None.  Every array these entry
    points take through here is device memory: a host array or a tensor of
    another element type would be read or written out of bounds by a kernel,
    so both are refused here (ValueError / TypeError)."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"expected a device tensor, got {type(t).__name__}"
                         + (f" on {t.device}" if hasattr(t, "device") else ""))
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise TypeError(f"expected a {dtype} tensor, got {t.dtype}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Mech:
    """Owns an mri_mech handle (chemistry or linear test mode)."""

    def __init__(self, mech=None, A_linear=None):
        self.h = C.c_void_p()
        if mech is not None:
            self._keep = dict(
                reac=np.ascontiguousarray(mech.reactants, dtype=np.int32),
                prod=np.ascontiguousarray(mech.products, dtype=np.int32),
                lnA=_f64(mech.lnA), beta=_f64(mech.beta), theta=_f64(mech.theta),
                g_a=_f64(mech.g_a), g_b=_f64(mech.g_b), W=_f64(mech.W), cv=_f64(mech.cv))
            k = self._keep
            P = lambda a, t=C.c_double: a.ctypes.data_as(C.POINTER(t))  # noqa: E731
            d = mri_mech_desc(mech.n_species, mech.n_reactions, P(k["reac"], C.c_int32),
                              P(k["prod"], C.c_int32), P(k["lnA"]), P(k["beta"]), P(k["theta"]),
                              P(k["g_a"]), P(k["g_b"]), P(k["W"]), P(k["cv"]), float(mech.rho),
                              float(mech.T_ref))
            _check(lib.mri_mech_create(C.byref(d), C.byref(self.h)))
        else:
            A = _f64(A_linear)
            _check(lib.mri_mech_create_linear(A.shape[0], A.ctypes.data_as(C.POINTER(C.c_double)),
                                              C.byref(self.h)))
        self.n = lib.mri_mech_state_width(self.h)

    def specialize(self, block_size=128, load=True, method=None, n_poly=1):
        """Compile (and with load, load) the run-time specialized kernel: the
        RK4 kernel with one forcing term by default, else that of `method`."""
        nb = C.c_size_t(0)
        if method is None:
            _check(lib.mri_mech_specialize(self.h, block_size, int(load), C.byref(nb)))
        else:
            _check(lib.mri_mech_specialize_method(self.h, int(method), int(n_poly), block_size,
                                                  int(load), C.byref(nb)))
        return nb.value

    def specialize_monitor(self, load=True):
        """Compile (and with load, load) the specialized stiffness monitor."""
        nb = C.c_size_t(0)
        _check(lib.mri_mech_specialize_monitor(self.h, int(load), C.byref(nb)))
        return nb.value

    def code_hash(self, method=0, n_poly=1, block_size=128):
        """Hex FNV-1a hash of the specialized kernel's code object (no GPU needed)."""
        h = C.c_uint64(0)
        _check(lib.mri_mech_code_hash(self.h, int(method), int(n_poly), block_size, C.byref(h)))
        return f"{h.value:016x}"

    def __del__(self, _destroy=lib.mri_mech_destroy, _null=C.c_void_p):
        if getattr(self, "h", None) and self.h.value:
            _destroy(self.h)
            self.h = _null()


class Table:
    def __init__(self, table):
        self.c = _f64(table.c)
        self.gamma = _f64(table.gamma)
        self.s, self.n_gamma = self.c.size, self.gamma.shape[0]
        self.h = C.c_void_p()
        d = mri_table_desc(self.s, self.n_gamma, self.c.ctypes.data_as(C.POINTER(C.c_double)),
                           self.gamma.ctypes.data_as(C.POINTER(C.c_double)))
        _check(lib.mri_table_create(C.byref(d), C.byref(self.h)))

    def __del__(self, _destroy=lib.mri_table_destroy, _null=C.c_void_p):
        if getattr(self, "h", None) and self.h.value:
            _destroy(self.h)
            self.h = _null()


class ImexTable:
    """IMEX-MRI-GARK coupling table (include/mri.h: mri_imex_table_create)."""

    def __init__(self, table):
        self.c = _f64(table.c)
        self.gamma = _f64(table.gamma)
        self.omega = _f64(table.omega)
        self.s, self.n_gamma = self.c.size, self.gamma.shape[0]
        self.h = C.c_void_p()
        dp = C.POINTER(C.c_double)
        d = mri_imex_table_desc(self.s, self.n_gamma, self.c.ctypes.data_as(dp),
                                self.gamma.ctypes.data_as(dp), self.omega.ctypes.data_as(dp))
        _check(lib.mri_imex_table_create(C.byref(d), C.byref(self.h)))

    def __del__(self, _destroy=lib.mri_imex_table_destroy, _null=C.c_void_p):
        if getattr(self, "h", None) and self.h.value:
            _destroy(self.h)
            self.h = _null()


def fast_opts(method=FAST_RK4, n_sub=1, rtol=1e-8, atol_Y=1e-8, atol_T=1e-5, max_steps=2000,
              kernel=KERNEL_AUTO, block_size=0, stiff_limit=0.0):
    return mri_fast_opts(method, n_sub, rtol, atol_Y, atol_T, max_steps, kernel, block_size,
                         stiff_limit)


def mri_stiffness_check(mech: Mech, n_cells, ld, y, h, limit, bound_out=None, status=None,
                        stream=None):
    _check(lib.mri_stiffness_check(mech.h, n_cells, ld, _ptr(y, "float64"), float(h),
                                   float(limit), _ptr(bound_out, "float64"),
                                   _ptr(status, "int32"), _stream(stream)))


def mri_fast_stage(mech: Mech, opts, n_cells, ld, y_in, y_out, n_poly, rho_poly, L,
                   status_out=None, steps_out=None, stream=None):
    _check(lib.mri_fast_stage(mech.h, C.byref(opts), n_cells, ld, _ptr(y_in, "float64"),
                              _ptr(y_out, "float64"), n_poly, _ptr(rho_poly, "float64"), float(L),
                              _ptr(status_out, "int32"), _ptr(steps_out, "int32"),
                              _stream(stream)))


def mri_workspace_bytes(mech: Mech, table: Table, n_cells, ld):
    b = C.c_size_t(0)
    _check(lib.mri_workspace_bytes(mech.h, table.h, n_cells, ld, C.byref(b)))
    return b.value


ADVDIFF_RHS = C.cast(lib.mri_advdiff_slow_rhs, C.c_void_p).value
LINEAR_RHS = C.cast(lib.mri_linear_slow_rhs, C.c_void_p).value


def advdiff_params(grid, n_comp, u=(10.0, 10.0, 10.0), D=1e-5, dx=1e-4):
    return mri_advdiff_params(grid[0], grid[1], grid[2], n_comp, (C.c_double * 3)(*u), D, dx)


ADVECTION_RHS = C.cast(lib.mri_advection_rhs, C.c_void_p).value
DIFFUSION_RHS = C.cast(lib.mri_diffusion_rhs, C.c_void_p).value
DIFFUSION_SOLVE = C.cast(lib.mri_diffusion_solve, C.c_void_p).value


def diffusion_solve_workspace_bytes(params, ld):
    b = C.c_size_t(0)
    _check(lib.mri_diffusion_solve_workspace_bytes(C.byref(params), ld, C.byref(b)))
    return b.value


def imex_advdiff(params, cg_ws, cg_rtol=1e-13, cg_max_iter=500):
    """The built-in advection (explicit) / diffusion (implicit) split for
    mri_imex_slow_step; cg_ws: a device tensor of at least
    diffusion_solve_workspace_bytes(params, ld) bytes (kept alive by the caller)."""
    return mri_imex_advdiff(params, float(cg_rtol), int(cg_max_iter), _ptr(cg_ws),
                            cg_ws.numel() * cg_ws.element_size(), 0, 0)


def _user_ptr(user):
    if isinstance(user, C.Structure):
        return C.cast(C.pointer(user), C.c_void_p).value
    if isinstance(user, Mech):
        return user.h.value
    return user


def mri_diffusion_solve(ctx, a, r, y, n_cells, ld, t=0.0, stream=None):
    """(I - a D lap) y = r by the built-in CG (ctx: imex_advdiff); raises on a
    nonzero return (no convergence, bad arguments)."""
    rc = lib.mri_diffusion_solve(float(t), float(a), _ptr(r, "float64"), _ptr(y, "float64"),
                                 n_cells, ld, _user_ptr(ctx), _stream(stream))
    if rc != 0:
        raise MriError(MRI_ENOCONV, f"mri_diffusion_solve returned {rc}")


def mri_imex_workspace_bytes(mech: Mech, table: ImexTable, n_cells, ld):
    b = C.c_size_t(0)
    _check(lib.mri_imex_workspace_bytes(mech.h, table.h, n_cells, ld, C.byref(b)))
    return b.value


def mri_imex_slow_step(mech: Mech, table: ImexTable, opts, ctx, t0, H, n_cells, ld, y, ws,
                       status_out=None, steps_out=None, stream=None, f_expl=None, f_impl=None,
                       solve_impl=None):
    """One IMEX-MRI-GARK step with the built-in advection / diffusion split
    (or other C callbacks by address) and ctx as `user`."""
    nbytes = ws.numel() * ws.element_size()
    _check(lib.mri_imex_slow_step(mech.h, table.h, C.byref(opts), f_expl or ADVECTION_RHS,
                                  f_impl or DIFFUSION_RHS, solve_impl or DIFFUSION_SOLVE,
                                  _user_ptr(ctx), float(t0), float(H), n_cells, ld,
                                  _ptr(y, "float64"), _ptr(ws), nbytes, _ptr(status_out, "int32"),
                                  _ptr(steps_out, "int32"), _stream(stream)))


def mri_slow_step(mech: Mech, table: Table, opts, f_slow, user, t0, H, n_cells, ld, y, ws,
                  status_out=None, steps_out=None, stream=None):
    """f_slow: a C function address (ADVDIFF_RHS, LINEAR_RHS); user: ctypes object or
    address passed through to it."""
    if isinstance(user, C.Structure):
        user_p = C.cast(C.pointer(user), C.c_void_p).value
    elif isinstance(user, Mech):
        user_p = user.h.value
    else:
        user_p = user
    nbytes = ws.numel() * ws.element_size()
    _check(lib.mri_slow_step(mech.h, table.h, C.byref(opts), f_slow, user_p, float(t0), float(H),
                             n_cells, ld, _ptr(y, "float64"), _ptr(ws), nbytes,
                             _ptr(status_out, "int32"), _ptr(steps_out, "int32"),
                             _stream(stream)))


def mri_slow_step_noalloc(mech: Mech, table: Table, opts, f_slow, user, t0, H, n_cells, ld, y,
                          status_out=None, steps_out=None, stream=None):
    """mri_slow_step without a workspace (the library's own device array)."""
    if isinstance(user, C.Structure):
        user_p = C.cast(C.pointer(user), C.c_void_p).value
    elif isinstance(user, Mech):
        user_p = user.h.value
    else:
        user_p = user
    _check(lib.mri_slow_step_noalloc(mech.h, table.h, C.byref(opts), f_slow, user_p, float(t0),
                                     float(H), n_cells, ld, _ptr(y, "float64"),
                                     _ptr(status_out, "int32"), _ptr(steps_out, "int32"),
                                     _stream(stream)))


def mri_noalloc_scratch_bytes():
    return int(lib.mri_noalloc_scratch_bytes())


def adapt_opts(rtol, atol_Y, atol_T, H0, order, H_min=0.0, H_max=0.0, max_attempts=10000,
               safety=0.0, fac_min=0.0, fac_max=0.0):
    return mri_adapt_opts(rtol, atol_Y, atol_T, H0, H_min, H_max, order, max_attempts, safety,
                          fac_min, fac_max)


def mri_adaptive_workspace_bytes(mech: Mech, table: Table, n_cells, ld):
    b = C.c_size_t()
    _check(lib.mri_adaptive_workspace_bytes(mech.h, table.h, n_cells, ld, C.byref(b)))
    return b.value


def mri_adaptive_run(mech: Mech, table: Table, opts, aopts, f_slow, user, t0, t_end, n_cells, ld,
                     y, ws, status_out=None, stream=None):
    """Adaptive slow steps from t0 to t_end (step doubling); returns the statistics
    as a dict.  f_slow and user as for mri_slow_step."""
    if isinstance(user, C.Structure):
        user_p = C.cast(C.pointer(user), C.c_void_p).value
    elif isinstance(user, Mech):
        user_p = user.h.value
    else:
        user_p = user
    st = mri_adapt_stats()
    nbytes = ws.numel() * ws.element_size()
    _check(lib.mri_adaptive_run(mech.h, table.h, C.byref(opts), C.byref(aopts), f_slow, user_p,
                                float(t0), float(t_end), n_cells, ld, _ptr(y, "float64"), _ptr(ws),
                                nbytes, _ptr(status_out, "int32"), C.byref(st), _stream(stream)))
    return {f: getattr(st, f) for f, _ in mri_adapt_stats._fields_}


def mri_selftest_exp2(x, y, stream=None):
    _check(lib.mri_selftest_exp2(_ptr(x), _ptr(y), x.numel(), _stream(stream)))


def mri_selftest_exp2_t256(x, y, stream=None):
    _check(lib.mri_selftest_exp2_t256(_ptr(x), _ptr(y), x.numel(), _stream(stream)))


def mri_status_count(status, n_cells, mask=0xFF, stream=None):
    n = C.c_int64(0)
    _check(lib.mri_status_count(_ptr(status), n_cells, mask, C.byref(n), _stream(stream)))
    return n.value


def counters():
    c = mri_counters()
    lib.mri_get_counters(C.byref(c))
    return dict(slow_evals=c.slow_evals, fast_stages=c.fast_stages, cell_stages=c.cell_stages,
                specializations=c.specializations)


def reset_counters():
    lib.mri_reset_counters()


def timing_enable(on=True):
    _check(lib.mri_timing_enable(int(on)))


def timing_read(reset=True):
    """(summed fast-stage kernel time in ms, number of timed launches)."""
    ms, n = C.c_double(0.0), C.c_int64(0)
    _check(lib.mri_timing_read(C.byref(ms), C.byref(n), int(reset)))
    return ms.value, n.value


class BatchPlan:
    def __init__(self, mech: Mech, opts, set_offsets):
        off = np.ascontiguousarray(set_offsets, dtype=np.int64)
        self.n_sets = off.size - 1
        self.n_total = int(off[-1])
        self.mech = mech
        self.h = C.c_void_p()
        _check(lib.mri_batch_plan_create(mech.h, C.byref(opts), self.n_sets,
                                         off.ctypes.data_as(C.POINTER(C.c_int64)),
                                         C.byref(self.h)))

    def run(self, y_in, y_out, ld, n_poly, rho_poly, L_per_set, status_out=None, steps_out=None,
            rejects_out=None, stream=None):
        L = _f64(L_per_set)
        _check(lib.mri_batch_run(self.h, _ptr(y_in, "float64"), _ptr(y_out, "float64"), int(ld),
                                 n_poly, _ptr(rho_poly, "float64"),
                                 L.ctypes.data_as(C.POINTER(C.c_double)),
                                 _ptr(status_out, "int32"), _ptr(steps_out, "int32"),
                                 _ptr(rejects_out, "int32"), _stream(stream)))

    def tile(self):
        b, n = C.c_int(0), C.c_int(0)
        _check(lib.mri_batch_plan_tile(self.h, C.byref(b), C.byref(n)))
        return b.value, n.value

    def tune_log(self):
        """(trials, from_cache, choice): the autotuner's timed candidates of the
        first run and its choice, as dicts."""
        n, fc, ch = C.c_int(0), C.c_int(0), mri_tune_trial()
        _check(lib.mri_batch_plan_tune_log(self.h, 0, None, C.byref(n), C.byref(fc),
                                           C.byref(ch)))
        buf = (mri_tune_trial * max(1, n.value))()
        _check(lib.mri_batch_plan_tune_log(self.h, n.value, buf, C.byref(n), None, None))

        def d(t):
            return {k: getattr(t, k) for k, _ in mri_tune_trial._fields_}
        return [d(buf[i]) for i in range(n.value)], bool(fc.value), d(ch)

    def code_hash(self, n_poly=0):
        h = C.c_uint64(0)
        _check(lib.mri_batch_plan_code_hash(self.h, n_poly, C.byref(h)))
        return f"{h.value:016x}"

    def lane_stats(self, stream=None):
        u, i = C.c_uint64(0), C.c_uint64(0)
        _check(lib.mri_batch_lane_stats(self.h, C.byref(u), C.byref(i), _stream(stream)))
        return u.value, i.value

    def __del__(self, _destroy=lib.mri_batch_plan_destroy, _null=C.c_void_p):
        if getattr(self, "h", None) and self.h.value:
            _destroy(self.h)
            self.h = _null()


# ---------------------------------------------------------------------------
# Surrogate (include/mri_surrogate.h)
# ---------------------------------------------------------------------------
MLP_FEATURES, MLP_KPAD, MLP_OUTPUTS = 89, 96, 22
MLP_STATS = 2 * 89 + 3 * 22


def mri_forcing_assemble(table: Table, stage, n, ld, F, rho, stream=None):
    _check(lib.mri_forcing_assemble(table.h, stage, n, ld, _ptr(F), _ptr(rho), _stream(stream)))


class MLP:
    """Trainable MLP handle (FP32 master weights, bf16 MFMA arithmetic)."""

    def __init__(self, widths, params, max_batch):
        self.widths = [int(w) for w in widths]
        w = (C.c_int * len(self.widths))(*self.widths)
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.h = C.c_void_p()
        _check(lib.mri_mlp_create(len(self.widths) - 1, w, p.ctypes.data_as(C.POINTER(C.c_float)),
                                  int(max_batch), C.byref(self.h)))
        self.n_params = lib.mri_mlp_param_count(self.h)

    def params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib.mri_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def grads(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib.mri_mlp_get_grads(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def forward(self, X, Y=None, stream=None):
        _check(lib.mri_mlp_forward(self.h, X.shape[0], _ptr(X), _ptr(Y), _stream(stream)))

    def backward(self, T, loss=None, stream=None):
        _check(lib.mri_mlp_backward(self.h, T.shape[0], _ptr(T), _ptr(loss), _stream(stream)))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib.mri_adam_step(self.h, lr, beta1, beta2, eps, _stream(stream)))

    def __del__(self, _destroy=lib.mri_mlp_destroy, _null=C.c_void_p):
        if getattr(self, "h", None) and self.h.value:
            _destroy(self.h)
            self.h = _null()


def mri_mlp_feature_stats(n, ld, Y0, n_poly, RHO, Lv, Y1, stats, Yb=None, stream=None):
    _check(lib.mri_mlp_feature_stats(int(n), int(ld), _ptr(Y0, "float64"), n_poly,
                                     _ptr(RHO, "float64"), _ptr(Lv, "float64"),
                                     _ptr(Yb, "float64"), _ptr(Y1, "float64"),
                                     _ptr(stats, "float64"), _stream(stream)))


def mri_mlp_featurize(batch, idx, ld, Y0, n_poly, RHO, Lv, Y1, stats, X, T=None, Yb=None,
                      stream=None):
    _check(lib.mri_mlp_featurize(int(batch), _ptr(idx, "int32"), int(ld), _ptr(Y0, "float64"),
                                 n_poly, _ptr(RHO, "float64"), _ptr(Lv, "float64"),
                                 _ptr(Yb, "float64"), _ptr(Y1, "float64"),
                                 _ptr(stats, "float64"), _ptr(X, "bfloat16"),
                                 _ptr(T, "float32"), _stream(stream)))


def mri_surrogate_gate(n_cells, ld, y_in, n_poly, rho, L, v_coarse, v_half, v_net, richardson,
                       gate_tol, y_out, fallback_list, n_fallback, status_coarse=None,
                       used_fallback=None, gate_value=None, stream=None):
    _check(lib.mri_surrogate_gate(n_cells, ld, _ptr(y_in, "float64"), n_poly,
                                  _ptr(rho, "float64"), float(L), _ptr(v_coarse, "float64"),
                                  _ptr(v_half, "float64"), _ptr(v_net, "float64"),
                                  _ptr(status_coarse, "int32"), float(richardson),
                                  float(gate_tol), _ptr(y_out, "float64"),
                                  _ptr(used_fallback, "int32"), _ptr(gate_value, "float64"),
                                  _ptr(fallback_list, "int32"), _ptr(n_fallback, "int32"),
                                  _stream(stream)))


class Surrogate:
    def __init__(self, widths, params, stats):
        w = (C.c_int * len(widths))(*[int(x) for x in widths])
        p = np.ascontiguousarray(params, dtype=np.float32)
        st = np.ascontiguousarray(stats, dtype=np.float64)
        self.h = C.c_void_p()
        _check(lib.mri_surrogate_create(w, p.ctypes.data_as(C.POINTER(C.c_float)),
                                        st.ctypes.data_as(C.POINTER(C.c_double)), C.byref(self.h)))

    def infer(self, n_cells, ld, y_in, y_out, n_poly, rho, L, base=None, stream=None):
        _check(lib.mri_surrogate_infer(self.h, n_cells, ld, _ptr(y_in, "float64"),
                                       _ptr(base, "float64"), _ptr(y_out, "float64"), n_poly,
                                       _ptr(rho, "float64"), float(L), _stream(stream)))

    @staticmethod
    def workspace_bytes(n_cells, ld, n_poly):
        b = C.c_size_t(0)
        _check(lib.mri_surrogate_workspace_bytes(n_cells, ld, n_poly, C.byref(b)))
        return b.value

    def stage(self, mech: Mech, coarse_opts, fallback_opts, gate_tol, n_cells, ld, y_in, y_out,
              n_poly, rho, L, ws, used_fallback=None, gate_value=None, status_out=None,
              n_fallback=None, stream=None):
        """Gated stage; n_fallback: an optional device int32 tensor of one element
        that receives the fallback count (nothing synchronizes)."""
        nbytes = ws.numel() * ws.element_size()
        _check(lib.mri_surrogate_stage(self.h, mech.h, C.byref(coarse_opts),
                                       C.byref(fallback_opts), float(gate_tol), n_cells, ld,
                                       _ptr(y_in, "float64"), _ptr(y_out, "float64"), n_poly,
                                       _ptr(rho, "float64"), float(L),
                                       _ptr(used_fallback, "int32"),
                                       _ptr(gate_value, "float64"), _ptr(status_out, "int32"),
                                       _ptr(n_fallback, "int32"), _ptr(ws), nbytes,
                                       _stream(stream)))

    def __del__(self, _destroy=lib.mri_surrogate_destroy, _null=C.c_void_p):
        if getattr(self, "h", None) and self.h.value:
            _destroy(self.h)
            self.h = _null()
