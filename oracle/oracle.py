"""ctypes loader for the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports this module.

Arrays are numpy float64 / int32, C-contiguous.  State layout is SoA:
y[comp, cell] with comp 0..S-1 the mass fractions Y_k and comp S the
temperature T; the leading dimension `ld` is y.shape[1].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "mlp_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
             "-std=c11", "-Wall"]

ST_NONFINITE, ST_MAXSTEPS, ST_TRANGE, ST_NEARTIE = 1, 2, 4, 8


# MRI_ORACLE_SANITIZE=1 builds and loads a separate copy instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer (run Python with
# LD_PRELOAD=$(gcc -print-file-name=libasan.so) ASAN_OPTIONS=detect_leaks=0).
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build(force: bool = False) -> str:
    srcs = [s for s in _SRC if os.path.exists(s)]
    san = os.environ.get("MRI_ORACLE_SANITIZE") == "1"
    path = _LIB.replace(".so", "_san.so") if san else _LIB
    stale = force or not os.path.exists(path) or any(
        os.path.getmtime(s) > os.path.getmtime(path) for s in srcs)
    if stale:
        tmp = path + f".tmp{os.getpid()}"
        flags = GCC_FLAGS + (SAN_FLAGS if san else [])
        subprocess.check_call(["gcc", *flags, "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, path)
    return path


class Mech(C.Structure):
    _fields_ = [("S", C.c_int), ("R", C.c_int),
                ("reac", C.POINTER(C.c_int32)), ("prod", C.POINTER(C.c_int32)),
                ("lnA", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("theta", C.POINTER(C.c_double)), ("g_a", C.POINTER(C.c_double)),
                ("g_b", C.POINTER(C.c_double)), ("W", C.POINTER(C.c_double)),
                ("cv", C.POINTER(C.c_double)), ("rho", C.c_double), ("T_ref", C.c_double)]


class Fast(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("mech", C.POINTER(Mech)),
                ("A", C.POINTER(C.c_double))]


class Table(C.Structure):
    _fields_ = [("s", C.c_int), ("n_gamma", C.c_int), ("c", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double))]


class FastOpts(C.Structure):
    _fields_ = [("method", C.c_int), ("n_sub", C.c_int), ("rtol", C.c_double),
                ("atol_Y", C.c_double), ("atol_T", C.c_double), ("max_steps", C.c_int)]


class AdvDiff(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("u", C.c_double * 3), ("D", C.c_double), ("dx", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.ora_energy.restype = C.c_double
        _lib.ora_zonneveld_try.restype = C.c_double
        _lib.ora_num_threads.restype = C.c_int
    return _lib


def _p(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Holds a mechanism (or a linear fast RHS) and the ctypes structures."""

    def __init__(self, mech=None, A_fast=None):
        self._keep = []
        if mech is not None:
            d = dict(reac=np.ascontiguousarray(mech.reactants, dtype=np.int32),
                     prod=np.ascontiguousarray(mech.products, dtype=np.int32),
                     lnA=_f64(mech.lnA), beta=_f64(mech.beta), theta=_f64(mech.theta),
                     g_a=_f64(mech.g_a), g_b=_f64(mech.g_b), W=_f64(mech.W), cv=_f64(mech.cv))
            self._keep.append(d)
            self.m = Mech(mech.n_species, mech.n_reactions, _p(d["reac"], C.c_int32),
                          _p(d["prod"], C.c_int32), _p(d["lnA"]), _p(d["beta"]),
                          _p(d["theta"]), _p(d["g_a"]), _p(d["g_b"]), _p(d["W"]), _p(d["cv"]),
                          float(mech.rho), float(mech.T_ref))
            self.n = mech.n_species + 1
            self.f = Fast(0, self.n, C.pointer(self.m), None)
        else:
            A = _f64(A_fast)
            self._keep.append(A)
            self.n = A.shape[0]
            self.f = Fast(1, self.n, None, _p(A))
        self.L = lib()

    # ---- single-cell chemistry -------------------------------------------
    def rhs(self, y):
        y = _f64(y)
        out = np.zeros(self.n)
        self.L.ora_fast_rhs(C.byref(self.f), _p(y), _p(out))
        return out

    def rhs_parts(self, y):
        y = _f64(y)
        S, R = self.m.S, self.m.R
        out, kf, kr, q, wd = np.zeros(self.n), np.zeros(R), np.zeros(R), np.zeros(R), np.zeros(S)
        self.L.ora_chem_rhs_parts(C.byref(self.m), _p(y), _p(out), _p(kf), _p(kr), _p(q), _p(wd))
        return dict(ydot=out, kf=kf, kr=kr, q=q, wdot=wd)

    def energy(self, y):
        return self.L.ora_energy(C.byref(self.m), _p(_f64(y)))

    def rhs_soa(self, y):
        y = _f64(y)
        out = np.zeros_like(y)
        self.L.ora_fast_rhs_soa(C.byref(self.f), y.shape[1], y.shape[1], _p(y), _p(out))
        return out

    def jacobian(self, y):
        y = _f64(y)
        J = np.zeros((self.n, self.n))
        self.L.ora_jacobian_fd(C.byref(self.f), _p(y), _p(J))
        return J

    def jacobians_soa(self, y, n_cells=None):
        y = _f64(y)
        n_cells = n_cells or y.shape[1]
        J = np.zeros((n_cells, self.n, self.n))
        self.L.ora_jacobian_fd_soa(C.byref(self.f), n_cells, y.shape[1], _p(y), _p(J))
        return J

    # ---- one fast stage ----------------------------------------------------
    def stiff_bound(self, y):
        """Upper bound of the spectral radius of the species Jacobian (1/s) of one
        cell (state y) or of every column of an SoA array."""
        y = _f64(y)
        self.L.ora_stiff_bound.restype = C.c_double
        if y.ndim == 1:
            return self.L.ora_stiff_bound(C.byref(self.m), _p(y))
        out = np.zeros(y.shape[1])
        self.L.ora_stiff_bound_soa(C.byref(self.m), y.shape[1], y.shape[1], _p(y), _p(out))
        return out

    def rk4_stage(self, y, rho_poly, L, n_sub):
        """Single cell; rho_poly [n_poly][n]."""
        y = _f64(y)
        rho = _f64(np.atleast_2d(rho_poly))
        out = np.zeros(self.n)
        st = self.L.ora_rk4_stage(C.byref(self.f), _p(y), rho.shape[0], _p(rho), C.c_double(L),
                                  int(n_sub), _p(out))
        return out, st

    def erk_stage(self, y, rho_poly, L, n_sub, A, b, c):
        """Single cell, general explicit RK tableau (A [s][s], b [s], c [s])."""
        y = _f64(y)
        rho = _f64(np.atleast_2d(rho_poly))
        A, b, c = _f64(A), _f64(b), _f64(c)
        out = np.zeros(self.n)
        st = self.L.ora_erk_stage(C.byref(self.f), _p(y), rho.shape[0], _p(rho), C.c_double(L),
                                  int(n_sub), b.size, _p(A), _p(b), _p(c), _p(out))
        return out, st

    def zonneveld_try(self, y, t, h, L, rho_poly, opts):
        y = _f64(y)
        rho = _f64(np.atleast_2d(rho_poly))
        out = np.zeros(self.n)
        err = self.L.ora_zonneveld_try(C.byref(self.f), _p(y), C.c_double(t), C.c_double(h),
                                       C.c_double(L), rho.shape[0], _p(rho), C.byref(opts), _p(out))
        return out, err

    def zonneveld_stage(self, y, rho_poly, L, opts, forced=None):
        y = _f64(y)
        rho = _f64(np.atleast_2d(rho_poly))
        out = np.zeros(self.n)
        acc, rej = C.c_int32(0), C.c_int32(0)
        if forced is not None:
            fz = np.ascontiguousarray(forced, dtype=np.int8)
            fp, nf = _p(fz, C.c_int8), fz.size
        else:
            fp, nf = None, 0
        st = self.L.ora_zonneveld_stage(C.byref(self.f), _p(y), rho.shape[0], _p(rho),
                                        C.c_double(L), C.byref(opts), _p(out), C.byref(acc),
                                        C.byref(rej), fp, nf)
        return out, st, acc.value, rej.value

    def fast_stage_soa(self, y, rho_poly, L, opts, n_cells=None):
        y = _f64(y)
        ld = y.shape[1]
        n_cells = n_cells or ld
        rho = _f64(rho_poly)
        n_poly = rho.shape[0] if rho.ndim == 3 else 0
        out = np.zeros_like(y)
        st = np.zeros(ld, dtype=np.int32)
        steps = np.zeros(ld, dtype=np.int32)
        rej = np.zeros(ld, dtype=np.int32)
        self.L.ora_fast_stage_soa(C.byref(self.f), C.byref(opts), n_cells, ld, _p(y), _p(out),
                                  n_poly, _p(rho), C.c_double(L), _p(st, C.c_int32),
                                  _p(steps, C.c_int32), _p(rej, C.c_int32))
        return out, st, steps, rej

    # ---- MRI slow step -------------------------------------------------------
    @staticmethod
    def table(tb):
        c = _f64(tb.c)
        g = _f64(tb.gamma)
        t = Table(c.size, g.shape[0], _p(c), _p(g))
        t._keep = (c, g)
        return t

    def mri_step_given(self, tb, opts, F, y, H, t=0.0, n_cells=None):
        y = _f64(y).copy()
        ld = y.shape[1]
        n_cells = n_cells or ld
        F = _f64(F)
        T = self.table(tb)
        st = np.zeros(ld, dtype=np.int32)
        steps = np.zeros(ld, dtype=np.int32)
        ns = self.L.ora_mri_step_given(C.byref(self.f), C.byref(T), C.byref(opts), _p(F),
                                       C.c_double(t), C.c_double(H), n_cells, ld, _p(y),
                                       _p(st, C.c_int32), _p(steps, C.c_int32))
        return y, st, steps, ns

    def mri_step_linear(self, tb, opts, AS, y, H, t=0.0):
        y = _f64(y).copy()
        if y.ndim == 1:
            y = y[:, None]
        ld = y.shape[1]
        AS = _f64(AS)
        T = self.table(tb)
        st = np.zeros(ld, dtype=np.int32)
        steps = np.zeros(ld, dtype=np.int32)
        ns = self.L.ora_mri_step_linear(C.byref(self.f), C.byref(T), C.byref(opts), _p(AS),
                                        C.c_double(t), C.c_double(H), ld, ld, _p(y),
                                        _p(st, C.c_int32), _p(steps, C.c_int32))
        return y, st, steps, ns

    def mri_step_advdiff(self, tb, opts, grid, y, H, u=(10.0, 10.0, 10.0), D=1e-5, dx=1e-4,
                         t=0.0):
        y = _f64(y).copy()
        ld = y.shape[1]
        n_cells = int(np.prod(grid))
        T = self.table(tb)
        g = AdvDiff(grid[0], grid[1], grid[2], (C.c_double * 3)(*u), D, dx)
        st = np.zeros(ld, dtype=np.int32)
        steps = np.zeros(ld, dtype=np.int32)
        ns = self.L.ora_mri_step_advdiff(C.byref(self.f), C.byref(T), C.byref(opts), C.byref(g),
                                         C.c_double(t), C.c_double(H), n_cells, ld, _p(y),
                                         _p(st, C.c_int32), _p(steps, C.c_int32))
        return y, st, steps, ns


def advdiff(y, grid, u=(10.0, 10.0, 10.0), D=1e-5, dx=1e-4):
    y = _f64(y)
    out = np.zeros_like(y)
    g = AdvDiff(grid[0], grid[1], grid[2], (C.c_double * 3)(*u), D, dx)
    lib().ora_advdiff(C.byref(g), y.shape[0], y.shape[1], _p(y), _p(out))
    return out


def rk4_opts(n_sub):
    return FastOpts(0, int(n_sub), 0.0, 0.0, 0.0, 0)


def zonneveld_opts(rtol=1e-8, atol_Y=1e-8, atol_T=1e-5, max_steps=2000):
    return FastOpts(1, 0, rtol, atol_Y, atol_T, max_steps)


ERK_HEUN, ERK_BS3, ERK_CK5 = 2, 3, 4


def erk_opts(method, n_sub):
    """Fixed-step Heun (method 2), Bogacki-Shampine (3) or Cash-Karp (4)."""
    return FastOpts(int(method), int(n_sub), 0.0, 0.0, 0.0, 0)


def erk_tableau(method):
    A, b, c = np.zeros(36), np.zeros(6), np.zeros(6)
    s = lib().ora_erk_tableau(int(method), _p(A), _p(b), _p(c))
    return A[:s * s].reshape(s, s), b[:s], c[:s]


def zonneveld_tableau():
    c, a, b, bh = np.zeros(5), np.zeros(20), np.zeros(5), np.zeros(5)
    lib().ora_zonneveld_tableau(_p(c), _p(a), _p(b), _p(bh))
    return c, a.reshape(5, 4), b, bh


def adaptive_run(step, y0, t0, t_end, order, rtol, atol_Y, atol_T, H0, t_comp=None,
                 n_cells=None, H_min=0.0, H_max=0.0, max_attempts=10000, safety=0.9,
                 fac_min=0.2, fac_max=5.0):
    """Adaptive slow steps by step doubling (the adaptive step control Sec. 7
    proposes for multirate methods), written out plainly.

    step(y, t, H) -> (y_new, status): one MRI step.  Each attempt takes one step
    of H and two of H/2 from the same state; the error estimate of the half-step
    result is (y_half - y_full) / (2^order - 1) (Richardson: the two results
    differ by (2^order - 1) times the half-step error to leading order).  Its
    WRMS norm over the first n_cells columns and every component, with weights
    1 / (atol + rtol |y_half|) (atol_T on row t_comp, atol_Y elsewhere), accepts
    at <= 1.  Step-size factor safety err^(-1/(order+1)), clipped to
    [fac_min, fac_max]; the last step ends exactly at t_end.
    Returns (y, stats, history) with history = [(t, H, err, accepted), ...]."""
    y = np.array(y0, dtype=np.float64, copy=True)
    n_cells = y.shape[1] if n_cells is None else n_cells
    atol = np.full((y.shape[0], 1), float(atol_Y))
    if t_comp is not None:
        atol[t_comp] = atol_T
    t = t0
    H = min(H0, H_max) if H_max > 0 else H0
    stats = dict(accepted=0, rejected=0, H_last=0.0)
    hist = []
    attempts = 0
    while t < t_end:
        if attempts >= max_attempts:
            raise RuntimeError("attempt cap reached")
        attempts += 1
        Hs, last = H, False
        if t + Hs >= t_end - 1e-12 * (t_end - t0):
            Hs, last = t_end - t, True
        y_full, _ = step(y, t, Hs)
        y_mid, st1 = step(y, t, 0.5 * Hs)
        y_half, st2 = step(y_mid, t + 0.5 * Hs, 0.5 * Hs)
        e = (y_half[:, :n_cells] - y_full[:, :n_cells]) / (2.0 ** order - 1.0)
        w = e / (atol + rtol * np.abs(y_half[:, :n_cells]))
        err = float(np.sqrt(np.mean(w * w)))
        if not np.isfinite(err):
            err = np.inf
        if err == 0.0:
            fac = fac_max
        elif err == np.inf:
            fac = fac_min
        else:
            fac = safety * err ** (-1.0 / (order + 1))
        fac = min(fac_max, max(fac_min, fac))
        hist.append((t, Hs, err, err <= 1.0))
        if err <= 1.0:
            y = y_half
            t = t_end if last else t + Hs
            stats["accepted"] += 1
            stats["H_last"] = Hs
        else:
            stats["rejected"] += 1
        H = Hs * fac
        if H_max > 0:
            H = min(H, H_max)
        if err > 1.0 and H < H_min:
            raise RuntimeError("step size fell below H_min")
    stats["t"] = t
    stats["H_next"] = H
    return y, stats, hist


def fixed_substeps(n_sub, H, H0):
    """Substeps per stage of a fixed-step fast method for a slow step H when the
    fast step of the first step (n_sub at H0) is kept."""
    import math
    return max(1, math.ceil(n_sub * (H / H0) - 1e-9))


def set_threads(n):
    lib().ora_set_num_threads(int(n))


def num_threads():
    return lib().ora_num_threads()


# ---------------------------------------------------------------------------
# Surrogate MLP (mlp_oracle.c)
# ---------------------------------------------------------------------------
def _mlp_setup():
    L = lib()
    L.ora_mlp_loss_grad.restype = C.c_double
    L.ora_bf16_round.restype = C.c_float
    L.ora_bf16_round.argtypes = [C.c_float]
    L.ora_silu.restype = C.c_double
    L.ora_silu.argtypes = [C.c_double]
    L.ora_silu_grad.restype = C.c_double
    L.ora_silu_grad.argtypes = [C.c_double]
    return L


# rounding points of the bfloat16-emulating mode (mlp_oracle.c ORA_R_*)
R_INPUT, R_WEIGHT, R_ACC, R_BIAS, R_SUM, R_ACT, R_GRAD = 1, 2, 4, 8, 16, 32, 64
R_ALL = 127


def _mode(bf16):
    """True: every rounding point of the GPU; False: FP64; an int: that set."""
    if bf16 is True:
        return R_ALL
    return int(bf16 or 0)


def mlp_param_count(widths):
    return sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))


def mlp_pack(Ws, bs):
    """Pack per-layer W [out][in] and b [out] as the oracle expects."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float64).ravel(),
                                           np.asarray(b, np.float64).ravel()])
                           for W, b in zip(Ws, bs)])


def mlp_forward(widths, params, X, bf16=False, cache=False):
    L = _mlp_setup()
    w = np.ascontiguousarray(widths, dtype=np.int32)
    p = _f64(params)
    X = _f64(X)
    batch = X.shape[0]
    Y = np.zeros((batch, widths[-1]))
    nz = sum(batch * widths[l + 1] for l in range(len(widths) - 1))
    na = sum(batch * widths[l + 1] for l in range(len(widths) - 2))
    Z = np.zeros(nz) if cache else None
    A = np.zeros(max(na, 1)) if cache else None
    L.ora_mlp_forward(len(widths) - 1, _p(w, C.c_int32), _p(p), batch, _p(X), _p(Y),
                      _p(Z) if cache else None, _p(A) if cache else None, _mode(bf16))
    return (Y, Z, A) if cache else Y


def mlp_loss_grad(widths, params, X, T, bf16=False):
    L = _mlp_setup()
    w = np.ascontiguousarray(widths, dtype=np.int32)
    p = _f64(params)
    X, T = _f64(X), _f64(T)
    g = np.zeros(p.size)
    loss = L.ora_mlp_loss_grad(len(widths) - 1, _p(w, C.c_int32), _p(p), X.shape[0], _p(X),
                               _p(T), _p(g), _mode(bf16))
    return loss, g


def bf16_round(x):
    L = _mlp_setup()
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros_like(x)
    L.ora_bf16_round_array(x.ctypes.data_as(C.POINTER(C.c_float)),
                           y.ctypes.data_as(C.POINTER(C.c_float)), x.size)
    return y


def silu(z):
    return _mlp_setup().ora_silu(float(z))


def silu_grad(z):
    return _mlp_setup().ora_silu_grad(float(z))


# ---------------------------------------------------------------------------
# Learned fast-stage surrogate (mlp_oracle.c ora_sur_*)
# ---------------------------------------------------------------------------
def sur_n_features(S):
    return int(lib().ora_sur_n_features(int(S)))


def _soa(a):
    return _f64(a)


def sur_stats(S, Y0, RHO, Lv, Y1, Yb=None):
    """Standardization statistics [x_mean, x_inv_std, y_mean, y_inv_std, y_std]
    of the samples (columns of the SoA arrays; RHO [n_poly][n][ld])."""
    Y0, Y1, Lv = _soa(Y0), _soa(Y1), _soa(Lv)
    RHO = _soa(RHO)
    N, ld = Lv.size, Y0.shape[1]
    F, n = sur_n_features(S), S + 1
    stats = np.zeros(2 * F + 3 * n)
    lib().ora_sur_stats(int(S), C.c_long(N), C.c_long(ld), _p(Y0), RHO.shape[0], _p(RHO), _p(Lv),
                        _p(_soa(Yb)) if Yb is not None else None, _p(Y1), _p(stats))
    return stats


def sur_featurize(S, Y0, RHO, Lv, stats, kpad=96, Yb=None, Y1=None):
    """Standardized feature rows [N][kpad] (FP64) and, given Y1, standardized
    targets [N][n] (corrections from Yb, default Y0)."""
    Y0, Lv, RHO = _soa(Y0), _soa(Lv), _soa(RHO)
    N, ld = Lv.size, Y0.shape[1]
    X = np.zeros((N, kpad))
    T = np.zeros((N, S + 1)) if Y1 is not None else None
    lib().ora_sur_featurize(int(S), C.c_long(N), C.c_long(ld), _p(Y0), RHO.shape[0], _p(RHO),
                            _p(Lv), _p(_soa(Yb)) if Yb is not None else None,
                            _p(_soa(Y1)) if Y1 is not None else None, _p(_f64(stats)), int(kpad),
                            _p(X), _p(T) if T is not None else None)
    return (X, T) if Y1 is not None else X


def sur_infer(S, widths, params, stats, Y, RHO, L, N=None, base=None, bf16=True, want_z=False):
    """The surrogate's prediction on the first N cells of Y [n][ld] (forcing
    RHO [n_poly][n][ld], stage length L), applied to `base` (default Y)."""
    Y, RHO = _soa(Y), _soa(RHO)
    n, ld = Y.shape
    N = ld if N is None else N
    w = np.ascontiguousarray(widths, dtype=np.int32)
    out = np.zeros_like(Y)
    Z = np.zeros((N, n)) if want_z else None
    lib().ora_sur_infer(int(S), C.c_long(N), C.c_long(ld), _p(Y), RHO.shape[0], _p(RHO),
                        C.c_double(L), _p(_soa(base)) if base is not None else None,
                        len(widths) - 1, _p(w, C.c_int32), _p(_f64(params)), _p(_f64(stats)),
                        _mode(bf16), _p(out), _p(Z) if want_z else None)
    return (out, Z) if want_z else out


def sur_gate(S, Y0, RHO, L, Vc, Vh, Vn, rich, tol, N=None, status_c=None):
    """Residual check of the surrogate: (G [N], accept [N] as bool)."""
    Y0, RHO, Vc, Vh, Vn = _soa(Y0), _soa(RHO), _soa(Vc), _soa(Vh), _soa(Vn)
    ld = Y0.shape[1]
    N = ld if N is None else N
    G = np.zeros(N)
    acc = np.zeros(N, dtype=np.int32)
    st = np.ascontiguousarray(status_c, dtype=np.int32) if status_c is not None else None
    lib().ora_sur_gate(int(S), C.c_long(N), C.c_long(ld), _p(Y0), RHO.shape[0], _p(RHO),
                       C.c_double(L), _p(Vc), _p(Vh), _p(Vn),
                       _p(st, C.c_int32) if st is not None else None, C.c_double(rich),
                       C.c_double(tol), _p(G), _p(acc, C.c_int32))
    return G, acc.astype(bool)


def sur_stage(orc, widths, params, stats, y, rho, L, n_coarse, n_fine, tol, N=None, bf16=True,
              stiff_limit=0.0):
    """The gated surrogate stage composed from the oracle's steps: RK4 stages
    with n_coarse and n_coarse/2 substeps, the network's correction of the
    first, the residual check against their Richardson extrapolation (RK4:
    1/15), and the plain RK4 stage with n_fine substeps for every rejected
    cell.  With stiff_limit > 0 a cell whose coarse step times the stiffness
    bound of its start state (stiff_bound, the Gershgorin bound of the
    species Jacobian) exceeds the limit counts as flagged by the coarse solve
    (the stability statements of Sec. 5.2 compare h times the fastest rate
    with a method's stability interval) and is rejected.  Returns (out [n][N],
    accept [N], G [N], status of the plain stage [N])."""
    y, rho = _f64(y), _f64(rho)
    N = y.shape[1] if N is None else N
    S = y.shape[0] - 1
    vc, sc, _, _ = orc.fast_stage_soa(y, rho, L, rk4_opts(n_coarse), N)
    vh, sh, _, _ = orc.fast_stage_soa(y, rho, L, rk4_opts(n_coarse // 2), N)
    if stiff_limit > 0.0:
        B = orc.stiff_bound(np.ascontiguousarray(y[:, :N]))
        sc = sc.copy()
        sc[:N] |= np.where((L / n_coarse) * B > stiff_limit, 16, 0).astype(sc.dtype)
    vn = sur_infer(S, widths, params, stats, y, rho, L, N=N, base=vc, bf16=bf16)
    G, acc = sur_gate(S, y, rho, L, vc, vh, vn, 1.0 / 15.0, tol, N=N, status_c=(sc | sh)[:N])
    out = vn[:, :N].copy()
    sf = np.zeros(N, dtype=np.int32)
    rej = np.nonzero(~acc)[0]
    if rej.size:
        yr = np.ascontiguousarray(y[:, rej])
        rr = np.ascontiguousarray(rho[:, :, rej])
        fine, s_f, _, _ = orc.fast_stage_soa(yr, rr, L, rk4_opts(n_fine))
        out[:, rej] = fine
        sf[rej] = s_f
    return out, acc, G, sf
