"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, rejects invalid arguments before touching the device, and its
run-time specialized kernels compile for gfx950."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2211_03293_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mri():
    from paper_2211_03293_amd import mri as M
    return M


def _declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w \*]*?\b(mri_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(mri):
    names = _declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(mri.lib, n)]
    assert not missing, missing


def test_abi_version(mri):
    assert mri.lib.mri_abi_version() == 3


def test_mech_validation(mri):
    m = I.make_mechanism(I.SMALL)
    bad = I.Mechanism(**{**m.__dict__})
    bad.reactants = m.reactants.copy()
    bad.reactants[3, 1] = m.n_species          # index out of range
    with pytest.raises(mri.MriError) as e:
        mri.Mech(bad)
    assert e.value.status == mri.MRI_EINVAL and "out of range" in str(e.value)
    bad = I.Mechanism(**{**m.__dict__})
    bad.W = m.W.copy()
    bad.W[0] = -1.0
    with pytest.raises(mri.MriError) as e:
        mri.Mech(bad)
    assert e.value.status == mri.MRI_EINVAL
    bad = I.Mechanism(**{**m.__dict__})
    bad.g_a = m.g_a * 100.0                    # exp(g/RT) would overflow at 200 K
    with pytest.raises(mri.MriError) as e:
        mri.Mech(bad)
    assert e.value.status == mri.MRI_EUNSUPPORTED


def test_table_validation(mri):
    mri.Table(I.table_mis_kw3())
    mri.Table(I.table_erk33a())
    t = I.table_mis_kw3()
    t.gamma = t.gamma.copy()
    t.gamma[0, 3, 2] += 1e-3                    # breaks the row-sum consistency
    with pytest.raises(mri.MriError) as e:
        mri.Table(t)
    assert "violates" in str(e.value)
    t = I.table_mis_kw3()
    t.gamma = t.gamma.copy()
    t.gamma[0, 1, 1] = 0.1                      # not explicit
    with pytest.raises(mri.MriError):
        mri.Table(t)
    t = I.table_mis_kw3()
    t.c = np.array([0.0, 0.5, 0.5, 1.0])        # dc = 0 stage (implicit form)
    with pytest.raises(mri.MriError):
        mri.Table(t)


def test_imex_table_and_callback_validation(mri):
    """IMEX-MRI-GARK tables: the 2nd-order table is accepted; a diagonal
    implicit coefficient on a fast stage, an explicit coefficient on the
    diagonal, rows whose integral weights miss Delta c, decreasing c and a
    table without a fast stage are refused on the host.  The built-in
    callbacks refuse a grid that does not match n_cells without touching the
    device, and the IMEX step refuses NULL callbacks and a short workspace."""
    import copy
    good = I.table_imex_trap2()
    mri.ImexTable(good)

    def refused(edit):
        t = copy.deepcopy(good)
        edit(t)
        with pytest.raises(mri.MriError):
            mri.ImexTable(t)

    refused(lambda t: t.gamma.__setitem__((0, 1, 1), 0.5))
    refused(lambda t: t.omega.__setitem__((0, 2, 2), 0.5))
    refused(lambda t: t.omega.__setitem__((0, 2, 1), 0.6))
    refused(lambda t: setattr(t, "c", np.array([0.0, 1.0, 0.5])))
    z = I.ImexTable("no fast stage", np.array([0.0, 0.0, 1.0]), np.zeros((1, 3, 3)),
                    np.zeros((1, 3, 3)))
    with pytest.raises(mri.MriError):
        mri.ImexTable(z)
    p = mri.advdiff_params((4, 4, 4), 22)
    nb = mri.diffusion_solve_workspace_bytes(p, 64)
    assert nb >= 3 * 8 * 22 * 64
    ctx = mri.mri_imex_advdiff(p, 1e-13, 10, None, 0, 0, 0)
    user = mri.C.cast(mri.C.pointer(ctx), mri.C.c_void_p).value
    assert mri.lib.mri_advection_rhs(0.0, 1, 1, 63, 64, user, 0) != 0      # 63 != 4^3
    assert mri.lib.mri_diffusion_rhs(0.0, 1, 1, 64, 32, user, 0) != 0      # ld < n_cells
    assert mri.lib.mri_diffusion_solve(0.0, 1.0, 1, 2, 64, 64, user, 0) != 0  # no workspace
    m = mri.Mech(I.make_mechanism(I.FIELD64))
    t = mri.ImexTable(good)
    b = mri.C.c_size_t(0)
    assert mri.lib.mri_imex_workspace_bytes(m.h, t.h, 64, 64, mri.C.byref(b)) == 0
    assert b.value == 8 * 22 * 64 * (2 * 2 + 1)
    o = mri.fast_opts(n_sub=4)
    rc = mri.lib.mri_imex_slow_step(m.h, t.h, mri.C.byref(o), None, mri.DIFFUSION_RHS,
                                    mri.DIFFUSION_SOLVE, user, 0.0, 1e-7, 64, 64, 1, 1, b.value,
                                    None, None, 0)
    assert rc == mri.MRI_EINVAL
    rc = mri.lib.mri_imex_slow_step(m.h, t.h, mri.C.byref(o), mri.ADVECTION_RHS,
                                    mri.DIFFUSION_RHS, mri.DIFFUSION_SOLVE, user, 0.0, 1e-7, 64,
                                    64, 1, 1, b.value - 8, None, None, 0)
    assert rc == mri.MRI_EINVAL and "workspace" in mri.last_error()


def test_fast_stage_rejects_bad_arguments_without_device(mri):
    m = mri.Mech(I.make_mechanism(I.SMALL))
    ok = mri.fast_opts(n_sub=4)
    L = mri.lib

    def call(opts=ok, n_cells=64, ld=64, yin=1, yout=1, n_poly=0, rho=None, Lval=1e-7):
        return L.mri_fast_stage(m.h, C.byref(opts), n_cells, ld, yin, yout, n_poly, rho, Lval,
                                None, None, None)

    assert call(n_cells=65, ld=64) == mri.MRI_EINVAL
    assert call(n_cells=-1) == mri.MRI_EINVAL
    assert call(Lval=0.0) == mri.MRI_EINVAL
    assert call(Lval=float("nan")) == mri.MRI_EINVAL
    assert call(n_poly=2, rho=None) == mri.MRI_EINVAL
    assert call(n_poly=5, rho=1) == mri.MRI_EINVAL
    assert call(opts=mri.fast_opts(n_sub=0)) == mri.MRI_EINVAL
    assert call(opts=mri.fast_opts(method=7)) == mri.MRI_EINVAL
    for meth in (mri.FAST_HEUN, mri.FAST_BS3, mri.FAST_CK5):
        assert call(opts=mri.fast_opts(method=meth, n_sub=0)) == mri.MRI_EINVAL
        assert call(opts=mri.fast_opts(method=meth, n_sub=4), n_cells=0, ld=0, yin=None,
                    yout=None) == mri.MRI_OK
    assert call(opts=mri.fast_opts(n_sub=4, block_size=96)) == mri.MRI_EINVAL
    assert call(opts=mri.fast_opts(method=mri.FAST_ZONNEVELD43, atol_Y=0.0)) == mri.MRI_EINVAL
    assert call(yin=None) == mri.MRI_EINVAL
    # an empty batch is a no-op and needs no device
    assert call(n_cells=0, ld=0, yin=None, yout=None) == mri.MRI_OK
    assert L.mri_fast_stage(None, C.byref(ok), 1, 1, 1, 1, 0, None, 1.0, None, None,
                            None) == mri.MRI_EINVAL


def test_slow_step_and_batch_validation(mri):
    m = mri.Mech(I.make_mechanism(I.SMALL))
    t = mri.Table(I.table_mis_kw3())
    L = mri.lib
    opts = mri.fast_opts(n_sub=4)
    assert mri.mri_workspace_bytes(m, t, 512, 512) == 8 * 10 * 512 * (3 + 1)
    rc = L.mri_slow_step(m.h, t.h, C.byref(opts), None, None, 0.0, 1e-6, 512, 512, 1, 1,
                         10 ** 9, None, None, None)
    assert rc == mri.MRI_EINVAL                  # NULL callback
    rc = L.mri_slow_step(m.h, t.h, C.byref(opts), mri.ADVDIFF_RHS, None, 0.0, 1e-6, 512, 512, 1,
                         1, 16, None, None, None)
    assert rc == mri.MRI_EINVAL and "workspace" in mri.last_error()
    rk4 = mri.fast_opts(n_sub=4)
    off = np.array([0, 10, 20], dtype=np.int64)
    h = C.c_void_p()
    rc = L.mri_batch_plan_create(m.h, C.byref(rk4), 2, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                 C.byref(h))
    assert rc == mri.MRI_EINVAL                  # batches are adaptive
    bad = np.array([0, 10, 5], dtype=np.int64)
    zv = mri.fast_opts(method=mri.FAST_ZONNEVELD43)
    rc = L.mri_batch_plan_create(m.h, C.byref(zv), 2, bad.ctypes.data_as(C.POINTER(C.c_int64)),
                                 C.byref(h))
    assert rc == mri.MRI_EINVAL


def test_linear_mode_validation(mri):
    with pytest.raises(mri.MriError):
        mri.Mech(A_linear=np.zeros((17, 17)))
    m = mri.Mech(A_linear=np.eye(2))
    assert m.n == 2
    zv = mri.fast_opts(method=mri.FAST_ZONNEVELD43)
    rc = mri.lib.mri_fast_stage(m.h, C.byref(zv), 1, 1, 1, 1, 0, None, 1.0, None, None, None)
    assert rc == mri.MRI_EUNSUPPORTED


def test_size_limits(mri):
    """A one-component state may use ld up to 2^31 - 1024 cells (n * ld <=
    2^31 - 1 elements is not the binding limit there): beyond it the block
    index arithmetic of the kernels would leave the int range, so the call is
    refused before any device work; so is a status count of that size."""
    L = mri.lib
    m = mri.Mech(A_linear=np.eye(1))
    rk4 = mri.fast_opts(n_sub=1)
    big = (1 << 31) - 1000
    assert L.mri_fast_stage(m.h, C.byref(rk4), big, big, 1, 1, 0, None, 1.0, None, None,
                            None) == mri.MRI_EINVAL
    assert "2^31 - 1024" in mri.last_error()
    n = C.c_int64(0)
    assert L.mri_status_count(1, big, 0xFF, C.byref(n), None) == mri.MRI_EINVAL
    chem = mri.Mech(I.make_mechanism(I.SMALL))         # n = 10: n * ld is the limit
    ld = (1 << 31) // 10 + 1
    assert L.mri_fast_stage(chem.h, C.byref(rk4), ld, ld, 1, 1, 0, None, 1.0, None, None,
                            None) == mri.MRI_EINVAL
    assert "n * ld" in mri.last_error()


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64])
def test_specialized_kernels_compile_for_gfx950(mri, workload):
    m = mri.Mech(I.make_mechanism(workload))
    nbytes = m.specialize(128, load=False)
    assert nbytes > 1000


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64, I.LARGE128])
def test_specialized_stiffness_monitor_compiles(mri, workload):
    m = mri.Mech(I.make_mechanism(workload))
    assert m.specialize_monitor(load=False) > 0


def test_specialized_kernels_compile_for_every_fast_method(mri):
    m = mri.Mech(I.make_mechanism(I.SMALL))
    for meth in (mri.FAST_RK4, mri.FAST_ZONNEVELD43, mri.FAST_HEUN, mri.FAST_BS3,
                 mri.FAST_CK5):
        for n_poly in (0, 2):
            assert m.specialize(64, load=False, method=meth, n_poly=n_poly) > 1000
    with pytest.raises(mri.MriError):
        m.specialize(64, load=False, method=9)
    with pytest.raises(mri.MriError, match="24 species"):
        mri.Mech(I.make_mechanism(I.LARGE128)).specialize(64, load=False, method=mri.FAST_CK5)
    with pytest.raises(mri.MriError):
        m.specialize(64, load=False, method=mri.FAST_HEUN, n_poly=5)


def test_cash_karp_limits(mri):
    """Cash-Karp 5 runs chemistry of up to 24 species; larger mechanisms are
    refused before any device work."""
    L = mri.lib

    def call(m, **kw):
        o = mri.fast_opts(method=mri.FAST_CK5, n_sub=4, **kw)
        return L.mri_fast_stage(m.h, C.byref(o), 0, 0, None, None, 0, None, 1e-7, None, None,
                                None)

    small = mri.Mech(I.make_mechanism(I.SMALL))
    assert call(small) == mri.MRI_OK
    assert call(small, kernel=mri.KERNEL_GENERIC) == mri.MRI_OK
    assert call(small, kernel=mri.KERNEL_SPECIALIZED) == mri.MRI_OK
    large = mri.Mech(I.make_mechanism(I.LARGE128))
    assert large.n - 1 > 24
    assert call(large) == mri.MRI_EUNSUPPORTED
    assert "24 species" in mri.last_error()
    lin = mri.Mech(A_linear=np.eye(3))
    assert call(lin, kernel=mri.KERNEL_SPECIALIZED) == mri.MRI_OK


def test_adaptive_run_validation(mri):
    """Invalid adaptive options fail before any device work; an empty batch
    reaches t_end without a device."""
    m = mri.Mech(I.make_mechanism(I.SMALL))
    t = mri.Table(I.table_mis_kw3())
    L = mri.lib
    fo = mri.fast_opts(n_sub=4)
    good = mri.adapt_opts(1e-6, 1e-8, 1e-5, 1e-7, 3)

    def call(a=good, fo=fo, t0=0.0, t1=1e-6, n_cells=64, ld=64, ws_bytes=1 << 40, cb=None):
        st = mri.mri_adapt_stats()
        rc = L.mri_adaptive_run(m.h, t.h, C.byref(fo), C.byref(a) if a is not None else None,
                                cb if cb is not None else mri.ADVDIFF_RHS, None, t0, t1, n_cells,
                                ld, 1, 1, ws_bytes, None, C.byref(st), None)
        return rc, st

    assert call(a=None)[0] == mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(-1.0, 1e-8, 1e-5, 1e-7, 3))[0] == mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(1e-6, 0.0, 1e-5, 1e-7, 3))[0] == mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(1e-6, 1e-8, 1e-5, 0.0, 3))[0] == mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(1e-6, 1e-8, 1e-5, 1e-7, 0))[0] == mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(1e-6, 1e-8, 1e-5, 1e-7, 3, max_attempts=0))[0] == mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(1e-6, 1e-8, 1e-5, 1e-7, 3, H_min=1e-6, H_max=1e-7))[0] == \
        mri.MRI_EINVAL
    assert call(a=mri.adapt_opts(1e-6, 1e-8, 1e-5, 1e-7, 3, fac_max=0.5))[0] == mri.MRI_EINVAL
    assert call(t0=1e-6, t1=1e-6)[0] == mri.MRI_EINVAL
    assert call(t1=float("nan"))[0] == mri.MRI_EINVAL
    assert call(fo=mri.fast_opts(n_sub=0))[0] == mri.MRI_EINVAL
    assert call(ws_bytes=8)[0] == mri.MRI_EINVAL and "workspace" in mri.last_error()
    rc, st = call(n_cells=0, ld=0)
    assert rc == mri.MRI_OK and st.t == 1e-6 and st.accepted == 0
    need = mri.mri_adaptive_workspace_bytes(m, t, 512, 512)
    assert need >= mri.mri_workspace_bytes(m, t, 512, 512) + 2 * 8 * 10 * 512


def test_code_hash_identifies_the_compiled_kernel(mri):
    m = mri.Mech(I.make_mechanism(I.SMALL))
    h1 = m.code_hash(mri.FAST_RK4, 1, 128)
    assert h1 == m.code_hash(mri.FAST_RK4, 1, 128)            # deterministic
    assert h1 != m.code_hash(mri.FAST_RK4, 2, 128)
    assert h1 != m.code_hash(mri.FAST_HEUN, 1, 128)
    assert h1 != mri.Mech(I.make_mechanism(I.FIELD64)).code_hash(mri.FAST_RK4, 1, 128)


def test_binding_refuses_host_and_mistyped_arrays(mri):
    """The binding passes device addresses only: a host tensor or array, or a
    device tensor of another element type, is refused before the library is
    called (a kernel would read it out of bounds)."""
    import torch

    m = mri.Mech(I.make_mechanism(I.SMALL))
    opts = mri.fast_opts(n_sub=1)
    y = torch.zeros((10, 8), dtype=torch.float64)
    with pytest.raises(ValueError, match="device tensor"):
        mri.mri_fast_stage(m, opts, 8, 8, y, y, 0, None, 1e-9)
    with pytest.raises(ValueError, match="device tensor"):
        mri.mri_fast_stage(m, opts, 8, 8, y.numpy(), y.numpy(), 0, None, 1e-9)

    class DeviceF32:                     # stands in for a float32 device tensor
        is_cuda = True
        dtype = torch.float32

        def data_ptr(self):
            return 0

    with pytest.raises(TypeError, match="float64"):
        mri._ptr(DeviceF32(), "float64")
    assert mri._ptr(None, "float64") is None


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises ImportError at import: there
    is no CPU fallback for any entry point."""
    import subprocess
    import sys

    env = dict(os.environ, MRI_LIB_PATH=str(tmp_path / "absent" / "libmri.so"))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", "import paper_2211_03293_amd.mri"], cwd=root,
                       env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "is missing" in r.stderr


def test_product_package_does_not_use_the_oracle():
    """The oracle is test infrastructure: no module of the package imports it."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2211_03293_amd")
    pat = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b|from\s+\.\.?oracle\b)", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                with open(os.path.join(dirpath, f)) as fh:
                    assert not pat.search(fh.read()), f


def test_concurrent_specialization_of_one_handle(mri):
    """A handle may be shared by threads: concurrent run-time compilations of
    one mechanism (serialized inside the library) all succeed and produce the
    same code object."""
    import threading

    m = mri.Mech(I.make_mechanism(I.SMALL))
    out, errs = [], []

    def work(method):
        try:
            out.append((method, m.code_hash(method, 1, 64)))
        except Exception as e:           # noqa: BLE001 - reported below
            errs.append(e)

    threads = [threading.Thread(target=work, args=(meth,))
               for meth in (mri.FAST_RK4, mri.FAST_HEUN, mri.FAST_RK4, mri.FAST_HEUN)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=600)
    assert not errs, errs
    assert len(out) == 4
    by_method = {}
    for meth, h in out:
        by_method.setdefault(meth, set()).add(h)
    assert all(len(v) == 1 for v in by_method.values()), by_method
    assert by_method[mri.FAST_RK4] != by_method[mri.FAST_HEUN]


def test_stiffness_check_validation(mri):
    """Argument errors of the stiffness monitor come back before device work."""
    m = mri.Mech(I.make_mechanism(I.SMALL))
    lin = mri.Mech(A_linear=np.eye(3))
    for args, status in (((m, -1, 64, None, 1e-8, 2.785), mri.MRI_EINVAL),
                         ((m, 64, 32, None, 1e-8, 2.785), mri.MRI_EINVAL),
                         ((m, 8, 64, None, -1e-8, 2.785), mri.MRI_EINVAL),
                         ((m, 8, 64, None, 1e-8, float("nan")), mri.MRI_EINVAL),
                         ((lin, 8, 64, None, 1e-8, 2.785), mri.MRI_EUNSUPPORTED)):
        with pytest.raises(mri.MriError) as e:
            mri.mri_stiffness_check(*args, stream=0)
        assert e.value.status == status
    mri.mri_stiffness_check(m, 0, 64, None, 1e-8, 2.785, stream=0)      # nothing to do
    with pytest.raises(mri.MriError) as e:
        mri.mri_fast_stage(m, mri.fast_opts(n_sub=4, stiff_limit=-1.0), 0, 64, None, None, 0,
                           None, 1e-8, stream=0)
    assert e.value.status == mri.MRI_EINVAL


def test_exp2_coefficient_generators_reproduce_the_header():
    """The constants of both device exponentials in mri_math.h are what their
    committed generators compute (polynomial: interpolation at the Chebyshev
    nodes in 50-digit arithmetic; table: 2^(j/256) and Taylor terms in 60)."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2211_03293_amd", "csrc")
    text = open(os.path.join(here, "mri_math.h")).read()
    for name in ("gen_exp2_poly", "gen_exp2_table"):
        spec = importlib.util.spec_from_file_location(name, os.path.join(here, name + ".py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        a = text.index(mod.BEGIN) + len(mod.BEGIN)
        assert text[a:text.index(mod.END)] == mod.body(), name
