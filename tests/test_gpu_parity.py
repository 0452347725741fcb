"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element (small sizes spanning several blocks and
a ragged tail) and on sampled cells at the full benchmark size."""
import ctypes as C

import numpy as np
import pytest

from paper_2211_03293_amd import inputs as I
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu

KERNELS = ["specialized", "generic"]


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def mri(torch):
    from paper_2211_03293_amd import mri as M
    return M


@pytest.fixture(scope="module")
def O(oracle_mod):
    oracle_mod.set_threads(16)
    return oracle_mod


def _kernel(mri, name):
    return mri.KERNEL_SPECIALIZED if name == "specialized" else mri.KERNEL_GENERIC


def _dev(torch, a, dtype=None):
    import torch as T
    return T.as_tensor(np.ascontiguousarray(a), dtype=dtype or T.float64, device="cuda")


def _small_forcing(O, orc, y0, n_stages=3):
    """Slow tendencies of the 512-cell workload, r_j = 1e-3 |f^F(y0)| xi_j (the
    oracle supplies |f^F|)."""
    fF = orc.rhs_soa(y0)
    xi = I.gaussian_xi(I.SMALL, n_stages, y0.shape[0], y0.shape[1])
    return 1e-3 * np.abs(fF)[None] * xi


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("n_poly", [1, 2, 3])
def test_rk4_stage_small(torch, mri, O, kernel, n_poly):
    mech = I.make_mechanism(I.SMALL)
    orc = O.Oracle(mech)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    F = _small_forcing(O, orc, y0)
    rho = np.stack([F[k] / (k + 1) for k in range(n_poly)])     # polynomial forcing terms
    L, n_sub = (5.0 / 12.0) * 1e-6, 20
    ref, st_o, _, _ = orc.fast_stage_soa(y0, rho, L, O.rk4_opts(n_sub))
    assert np.all(st_o[:512] == 0)
    m = mri.Mech(mech)
    yd = _dev(torch, y0)
    out = torch.empty_like(yd)
    st = torch.full((ld,), -1, dtype=torch.int32, device="cuda")
    steps = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    opts = mri.fast_opts(n_sub=n_sub, kernel=_kernel(mri, kernel))
    mri.mri_fast_stage(m, opts, 512, ld, yd, out, n_poly, _dev(torch, rho), L, st, steps)
    torch.cuda.synchronize()
    e = assert_parity(out.cpu().numpy(), ref, mech.n_species, what=f"{kernel} np={n_poly}")
    print(f"rk4 small {kernel} n_poly={n_poly}: max rel err {e:.2e}")
    assert np.all(st.cpu().numpy()[:512] == 0)
    assert np.all(steps.cpu().numpy()[:512] == n_sub)


@pytest.mark.parametrize("kernel", KERNELS)
def test_ragged_tail_and_in_place(torch, mri, O, kernel):
    """517 cells in ld = 576: the padding stays untouched; y_out may alias y_in."""
    mech = I.make_mechanism(I.FIELD64)
    orc = O.Oracle(mech)
    rng = np.random.Generator(np.random.PCG64(77))
    y0 = I.independent_cells(517, mech.n_species, rng, ld=576)
    y0[:, 517:] = 12345.0
    rho = rng.normal(size=(1, *y0.shape)) * 10.0
    L, n_sub = 3e-8, 7
    ref, _, _, _ = orc.fast_stage_soa(y0, rho, L, O.rk4_opts(n_sub), n_cells=517)
    m = mri.Mech(mech)
    yd = _dev(torch, y0)
    mri.mri_fast_stage(m, mri.fast_opts(n_sub=n_sub, kernel=_kernel(mri, kernel)), 517, 576, yd,
                       yd, 1, _dev(torch, rho), L)
    got = yd.cpu().numpy()
    assert_parity(got[:, :517], ref[:, :517], mech.n_species, what=kernel)
    assert np.all(got[:, 517:] == 12345.0)
    # empty batch: no launch, nothing written
    mri.mri_fast_stage(m, mri.fast_opts(n_sub=n_sub), 0, 576, yd, yd, 1, _dev(torch, rho), L)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), got)


@pytest.mark.parametrize("method", ["rk4", "zonneveld"])
def test_stage_result_is_independent_of_the_block_size(torch, mri, method):
    """One lane integrates one cell with the same arithmetic whatever the block
    size the kernel is compiled for: blocks of 64, 128 and 256 lanes give
    bitwise equal states, status bits and step counts (specialized kernels)."""
    mech = I.make_mechanism(I.SMALL)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    m = mri.Mech(mech)
    yd = _dev(torch, y0)
    rho = torch.zeros((1, n, ld), dtype=torch.float64, device="cuda")
    res = []
    for block in (64, 128, 256):
        if method == "rk4":
            opts = mri.fast_opts(n_sub=20, kernel=mri.KERNEL_SPECIALIZED, block_size=block)
        else:
            opts = mri.fast_opts(method=mri.FAST_ZONNEVELD43, rtol=1e-8, atol_Y=1e-8,
                                 atol_T=1e-5, kernel=mri.KERNEL_SPECIALIZED, block_size=block)
        out = torch.empty_like(yd)
        st = torch.zeros((ld,), dtype=torch.int32, device="cuda")
        steps = torch.zeros((ld,), dtype=torch.int32, device="cuda")
        mri.mri_fast_stage(m, opts, 512, ld, yd, out, 1, rho, (5.0 / 12.0) * 1e-6, st, steps)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy()[:, :512], st.cpu().numpy()[:512],
                    steps.cpu().numpy()[:512]))
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0])
        assert np.array_equal(r[1], res[0][1]) and np.array_equal(r[2], res[0][2])


@pytest.mark.parametrize("kernel", KERNELS)
def test_stage_on_a_side_stream(torch, mri, kernel):
    """Every call runs on the stream it is given: a stage enqueued on a side
    stream (default priority) behind a copy into its input on that stream sees
    the copied input, and equals bitwise the same stage on the current stream."""
    mech = I.make_mechanism(I.SMALL)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    m = mri.Mech(mech)
    src = _dev(torch, y0)
    rho = torch.zeros((1, n, ld), dtype=torch.float64, device="cuda")
    opts = mri.fast_opts(n_sub=20, kernel=_kernel(mri, kernel))
    L = (5.0 / 12.0) * 1e-6
    ref = torch.empty_like(src)
    mri.mri_fast_stage(m, opts, 512, ld, src, ref, 1, rho, L)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    yin = torch.zeros_like(src)
    out = torch.full_like(src, -1.0)
    side.wait_stream(torch.cuda.current_stream())     # the two fills above come first
    with torch.cuda.stream(side):
        yin.copy_(src)                       # ordered before the stage on `side`
        mri.mri_fast_stage(m, opts, 512, ld, yin, out, 1, rho, L, stream=side)
    side.synchronize()
    assert torch.equal(out[:, :512], ref[:, :512])


@pytest.mark.parametrize("kernel", KERNELS)
def test_zonneveld_stage_small(torch, mri, O, kernel):
    mech = I.make_mechanism(I.SMALL)
    orc = O.Oracle(mech)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    F = _small_forcing(O, orc, y0)
    rho = F[:1]
    L = (5.0 / 12.0) * 1e-6
    zo = O.zonneveld_opts(rtol=1e-8, atol_Y=1e-8, atol_T=1e-5, max_steps=2000)
    ref, st_o, acc_o, _ = orc.fast_stage_soa(y0, rho, L, zo)
    m = mri.Mech(mech)
    yd = _dev(torch, y0)
    out = torch.empty_like(yd)
    st = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    steps = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    opts = mri.fast_opts(method=mri.FAST_ZONNEVELD43, rtol=1e-8, atol_Y=1e-8, atol_T=1e-5,
                         max_steps=2000, kernel=_kernel(mri, kernel))
    mri.mri_fast_stage(m, opts, 512, ld, yd, out, 1, _dev(torch, rho), L, st, steps)
    torch.cuda.synchronize()
    st_g, acc_g = st.cpu().numpy()[:512], steps.cpu().numpy()[:512]
    tie = ((st_g | st_o[:512]) & mri.CELL_NEARTIE) != 0
    ok = ~tie
    assert ok.sum() >= 500
    np.testing.assert_array_equal(acc_g[ok], acc_o[:512][ok])
    assert_parity(out.cpu().numpy(), ref, mech.n_species, cells=np.nonzero(ok)[0], what=kernel)
    print(f"zonneveld {kernel}: steps {acc_g.min()}..{acc_g.max()}, near ties {tie.sum()}")


def _given_callback(torch, mri, ws, F_dev, vec):
    CB = C.CFUNCTYPE(C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                     C.c_void_p)
    base = ws.data_ptr()

    def cb(t, y, fy, n_cells, ld, user, stream):
        j = (fy - base) // (8 * vec)
        ws[j * vec:(j + 1) * vec].copy_(F_dev[j].reshape(-1))
        return 0

    return CB(cb)


TABLES = {"MIS-KW3": I.table_mis_kw3, "ERK33a": I.table_erk33a, "ERK45a": I.table_erk45a}


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("table_name", list(TABLES))
def test_mri_slow_step_small(torch, mri, O, kernel, table_name):
    """One explicit MRI-GARK step of the 512-cell workload (H = 1e-6, RK4 with 20
    substeps per stage), slow evaluations given as its Gaussian tendencies (one per
    new slow stage: 3 for the 4-stage tables, 5 for ERK45a)."""
    tb = TABLES[table_name]()
    ns = tb.s - 1
    mech = I.make_mechanism(I.SMALL)
    orc = O.Oracle(mech)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    F = _small_forcing(O, orc, y0, n_stages=ns)
    ref, st_o, steps_o, n_slow = orc.mri_step_given(tb, O.rk4_opts(20), F, y0, 1e-6)
    assert n_slow == ns and np.all(st_o[:512] == 0)
    m, t = mri.Mech(mech), mri.Table(tb)
    yd = _dev(torch, y0)
    ws = torch.empty(mri.mri_workspace_bytes(m, t, 512, ld) // 8, dtype=torch.float64,
                     device="cuda")
    cb = _given_callback(torch, mri, ws, _dev(torch, F), n * ld)
    st = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    steps = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    mri.reset_counters()
    mri.mri_slow_step(m, t, mri.fast_opts(n_sub=20, kernel=_kernel(mri, kernel)),
                      C.cast(cb, C.c_void_p).value, None, 0.0, 1e-6, 512, ld, yd, ws, st, steps)
    torch.cuda.synchronize()
    c = mri.counters()
    assert c["slow_evals"] == ns and c["fast_stages"] == ns and c["cell_stages"] == ns * 512
    assert_parity(yd.cpu().numpy(), ref, mech.n_species, what=f"{kernel} {table_name}")
    assert np.all(steps.cpu().numpy()[:512] == 20 * ns)
    assert mri.mri_status_count(st, 512) == 0


@pytest.mark.parametrize("kernel", KERNELS)
def test_mri_slow_steps_advdiff_small_grid(torch, mri, O, kernel):
    """The 64^3 workload's physics on a 12 x 10 x 8 periodic grid: two MRI steps with the
    advection-diffusion slow RHS, H = 1e-7, RK4 with 50 substeps per stage."""
    grid = (12, 10, 8)
    mech = I.make_mechanism(I.FIELD64)
    orc = O.Oracle(mech)
    y0 = I.field_state(I.FIELD64, grid=grid)
    n, ld = y0.shape
    N = int(np.prod(grid))
    tb = I.table_mis_kw3()
    ref = y0.copy()
    for step in range(2):
        ref, st_o, _, _ = orc.mri_step_advdiff(tb, O.rk4_opts(50), grid, ref, 1e-7, t=step * 1e-7)
        assert np.all(st_o[:N] == 0)
    m, t = mri.Mech(mech), mri.Table(tb)
    yd = _dev(torch, y0)
    ws = torch.empty(mri.mri_workspace_bytes(m, t, N, ld) // 8, dtype=torch.float64,
                     device="cuda")
    params = mri.advdiff_params(grid, n)
    for step in range(2):
        mri.mri_slow_step(m, t, mri.fast_opts(n_sub=50, kernel=_kernel(mri, kernel)),
                          mri.ADVDIFF_RHS, params, step * 1e-7, 1e-7, N, ld, yd, ws)
    torch.cuda.synchronize()
    assert_parity(yd.cpu().numpy(), ref, mech.n_species, what=kernel)


def test_linear_mode_matches_oracle_and_converges_at_table_order(torch, mri, O):
    """Linear two-rate problem through the device path: every step matches the
    oracle; MIS-KW3 and ERK33a converge at order 3, ERK45a at order 4."""
    from scipy.linalg import expm
    A_F = np.array([[-6.0, 5.0], [-5.0, -4.0]])
    A_S = np.array([[0.3, 1.0], [-1.2, 0.2]])
    orc = O.Oracle(A_fast=A_F)
    mF, mS = mri.Mech(A_linear=A_F), mri.Mech(A_linear=A_S)
    errs = []
    for tb in (I.table_mis_kw3(), I.table_erk33a(), I.table_erk45a()):
        t = mri.Table(tb)
        errs = []
        for n_steps in (8, 16, 32):
            H = 1.0 / n_steps
            y = np.array([[1.0] * 64, [0.5] * 64])
            yd = _dev(torch, y)
            ws = torch.empty(mri.mri_workspace_bytes(mF, t, 64, 64) // 8, dtype=torch.float64,
                             device="cuda")
            yo = y[:, :1].copy()
            for k in range(n_steps):
                mri.mri_slow_step(mF, t, mri.fast_opts(n_sub=64), mri.LINEAR_RHS, mS, k * H, H, 64,
                                  64, yd, ws)
                yo, _, _, _ = orc.mri_step_linear(tb, O.rk4_opts(64), A_S, yo[:, 0], H)
            got = yd.cpu().numpy()
            np.testing.assert_allclose(got[:, 0], yo[:, 0], rtol=1e-12)
            assert np.all(got == got[:, :1])
            errs.append(np.abs(got[:, 0] - expm(A_F + A_S) @ np.array([1.0, 0.5])).max())
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        order = 4 if tb.s == 6 else 3
        print(f"{tb.name}: rates {np.round(rates, 2)}")
        assert np.all(rates > order - 0.3), (tb.name, rates)


def _erk_methods(O, mri, method):
    return {"heun": (O.ERK_HEUN, mri.FAST_HEUN), "bs3": (O.ERK_BS3, mri.FAST_BS3),
            "ck5": (O.ERK_CK5, mri.FAST_CK5)}[method]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("method", ["heun", "bs3", "ck5"])
def test_fixed_step_methods_stage_small(torch, mri, O, kernel, method):
    """Heun, Bogacki-Shampine and Cash-Karp fast stages (the order-2, 3 and 5
    fast methods of the MRI-P(k) family) against the oracle's general explicit
    RK stage with its own tableaus."""
    mech = I.make_mechanism(I.SMALL)
    orc = O.Oracle(mech)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    F = _small_forcing(O, orc, y0)
    rho = np.stack([F[k] / (k + 1) for k in range(2)])
    L, n_sub = (5.0 / 12.0) * 1e-6, 20
    om, gm = _erk_methods(O, mri, method)
    m = mri.Mech(mech)
    yd = _dev(torch, y0)
    out = torch.empty_like(yd)
    steps = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    opts = mri.fast_opts(method=gm, n_sub=n_sub, kernel=_kernel(mri, kernel))
    ref, st_o, _, _ = orc.fast_stage_soa(y0, rho, L, O.erk_opts(om, n_sub))
    assert np.all(st_o[:512] == 0)
    mri.mri_fast_stage(m, opts, 512, ld, yd, out, 2, _dev(torch, rho), L, None, steps)
    torch.cuda.synchronize()
    e = assert_parity(out.cpu().numpy(), ref, mech.n_species, what=f"{method} {kernel}")
    print(f"{method} small {kernel}: max rel err {e:.2e}")
    assert np.all(steps.cpu().numpy()[:512] == n_sub)


@pytest.mark.parametrize("method,order", [("heun", 2), ("bs3", 3), ("ck5", 5)])
def test_mri_order_with_low_order_fast_methods(torch, mri, O, method, order):
    """MRI-P(k) on the linear two-rate problem: MIS-KW3 with k fixed fast
    substeps per stage and a fast method of order P converges at order
    min(3, P) in H; every step matches the oracle."""
    from scipy.linalg import expm
    A_F = np.array([[-6.0, 5.0], [-5.0, -4.0]])
    A_S = np.array([[0.3, 1.0], [-1.2, 0.2]])
    orc = O.Oracle(A_fast=A_F)
    mF, mS = mri.Mech(A_linear=A_F), mri.Mech(A_linear=A_S)
    tb = I.table_mis_kw3()
    t = mri.Table(tb)
    om, gm = _erk_methods(O, mri, method)
    k = 4
    errs = []
    for n_steps in (16, 32, 64, 128):
        H = 1.0 / n_steps
        y = np.array([[1.0] * 64, [0.5] * 64])
        yd = _dev(torch, y)
        ws = torch.empty(mri.mri_workspace_bytes(mF, t, 64, 64) // 8, dtype=torch.float64,
                         device="cuda")
        yo = y[:, :1].copy()
        for step in range(n_steps):
            mri.mri_slow_step(mF, t, mri.fast_opts(method=gm, n_sub=k), mri.LINEAR_RHS, mS,
                              step * H, H, 64, 64, yd, ws)
            yo, _, _, _ = orc.mri_step_linear(tb, O.erk_opts(om, k), A_S, yo[:, 0], H)
        got = yd.cpu().numpy()
        np.testing.assert_allclose(got[:, 0], yo[:, 0], rtol=1e-12)
        errs.append(np.abs(got[:, 0] - expm(A_F + A_S) @ np.array([1.0, 0.5])).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print(f"MRI-{order}({k}) rates {np.round(rates, 2)}")
    assert np.all(np.abs(rates[1:] - min(3, order)) < 0.3), rates


@pytest.mark.parametrize("kernel", KERNELS)
def test_determinism_and_fault_isolation(torch, mri, O, kernel):
    mech = I.make_mechanism(I.SMALL)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    m = mri.Mech(mech)
    opts = mri.fast_opts(n_sub=20, kernel=_kernel(mri, kernel))
    L = 1e-7

    def run(y):
        yd = _dev(torch, y)
        out = torch.empty_like(yd)
        st = torch.zeros((ld,), dtype=torch.int32, device="cuda")
        mri.mri_fast_stage(m, opts, 512, ld, yd, out, 0, None, L, st)
        torch.cuda.synchronize()
        return out.cpu().numpy(), st.cpu().numpy()

    a, sa = run(y0)
    b, sb = run(y0)
    assert np.array_equal(a, b) and np.all(sa[:512] == 0)
    bad = y0.copy()
    bad[3, 17] = np.nan            # NaN mass fraction in cell 17
    bad[n - 1, 200] = 100.0        # cell 200 starts far below 200 K
    c, sc = run(bad)
    assert sc[17] & mri.CELL_NONFINITE
    assert sc[200] & (mri.CELL_TRANGE | mri.CELL_NONFINITE)
    others = np.setdiff1d(np.arange(512), [17, 200])
    assert np.all(sc[others] == 0)
    assert np.array_equal(c[:, others], a[:, others])
    assert mri.mri_status_count(torch.as_tensor(sc, device="cuda"), 512) == 2


@pytest.mark.parametrize("variant", ["polynomial", "table"])
def test_device_exp2_accuracy(torch, mri, variant):
    """The kernels' two 2^t against numpy's exp2 over the exponent range the
    kernels use: the degree-11 polynomial on [-1/2, 1/2] (generic kernels and
    specialized kernels at one wave per SIMD) and the 2^(j/256) table with a
    degree-4 polynomial (specialized kernels at two waves per SIMD)."""
    fn = mri.mri_selftest_exp2 if variant == "polynomial" else mri.mri_selftest_exp2_t256
    rng = np.random.Generator(np.random.PCG64(8))
    # grid of step 1/16384 on [-4, 4]: every table entry and every rounding
    # tie of the table index (x an odd multiple of 1/512) in both signs
    x = np.concatenate([rng.uniform(-1000, 1000, 200000), rng.uniform(-1, 1, 100000),
                        np.arange(-60, 61, 0.5), np.arange(-65536, 65537) / 16384.0,
                        [0.0, -0.0, 1e-300, 0.49999999999999994, -0.5, 0.5, 1021.9]])
    xd = torch.as_tensor(x, device="cuda")
    yd = torch.empty_like(xd)
    fn(xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    ref = np.exp2(x)
    ulp = np.spacing(np.abs(ref))
    err = np.abs(y - ref) / ulp
    print(f"exp2 {variant}: max {err.max():.2f} ulp, mean {err.mean():.3f}")
    assert err.max() <= 2.0, (err.max(), x[np.argmax(err)])
    # NaN propagates; results beyond the double range saturate
    xs = torch.tensor([np.nan, 1100.0, 5000.0, -1100.0, -5000.0], dtype=torch.float64,
                      device="cuda")
    ys = torch.empty_like(xs)
    fn(xs, ys)
    torch.cuda.synchronize()
    ys = ys.cpu().numpy()
    assert np.isnan(ys[0])
    assert np.all(ys[1:3] == np.inf) and np.all(ys[3:] == 0.0), ys


@pytest.mark.parametrize("kernel", KERNELS)
def test_zonneveld_step_cap_flags_cells(torch, mri, O, kernel):
    """A cap of 12 accepted steps per cell-stage (every cell needs at least 10,
    the first step being L/10): every cell that needs more is flagged MAXSTEPS
    (173 of 512 cells), cells within the cap are not, and the accepted-step
    counts equal the oracle's.  Cells that finish end at t = L and meet the
    1e-10 bar.  A capped cell stops at the time its 12 accepted steps reach;
    those steps come from the embedded error estimate, a difference of
    near-equal terms on which the device and the oracle agree only to about
    1e-16 / tol = 1e-8 relative, so the stopping times and hence the capped
    states agree to about that (checked at 1e-6)."""
    mech = I.make_mechanism(I.SMALL)
    orc = O.Oracle(mech)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    rho = _small_forcing(O, orc, y0)[:1]
    L = (5.0 / 12.0) * 1e-6
    zo = O.zonneveld_opts(rtol=1e-8, atol_Y=1e-8, atol_T=1e-5, max_steps=12)
    ref, st_o, acc_o, _ = orc.fast_stage_soa(y0, rho, L, zo)
    capped = (st_o[:512] & O.ST_MAXSTEPS) != 0
    assert 0 < capped.sum() < 512
    m = mri.Mech(mech)
    yd = _dev(torch, y0)
    out = torch.empty_like(yd)
    st = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    steps = torch.zeros((ld,), dtype=torch.int32, device="cuda")
    opts = mri.fast_opts(method=mri.FAST_ZONNEVELD43, rtol=1e-8, atol_Y=1e-8, atol_T=1e-5,
                         max_steps=12, kernel=_kernel(mri, kernel))
    mri.mri_fast_stage(m, opts, 512, ld, yd, out, 1, _dev(torch, rho), L, st, steps)
    torch.cuda.synchronize()
    st_g = st.cpu().numpy()[:512]
    tie = ((st_g | st_o[:512]) & mri.CELL_NEARTIE) != 0
    ok = ~tie
    np.testing.assert_array_equal((st_g[ok] & mri.CELL_MAXSTEPS) != 0, capped[ok])
    np.testing.assert_array_equal(steps.cpu().numpy()[:512][ok], acc_o[:512][ok])
    got = out.cpu().numpy()
    assert_parity(got, ref, mech.n_species, cells=np.nonzero(ok & ~capped)[0],
                  what=f"finished cells {kernel}")
    e = assert_parity(got, ref, mech.n_species, cells=np.nonzero(ok & capped)[0], tol=1e-6,
                      what=f"capped cells {kernel}")
    print(f"capped cells: max rel difference {e:.2e}")
    print(f"step cap {kernel}: {capped.sum()} of 512 cells capped, near ties {tie.sum()}")


def test_checkpoint_resume_is_bitwise(torch, mri, tmp_path):
    """The whole integration state is the SoA array and the time: six MRI steps
    straight through equal three steps, a save to disk, a load into fresh
    device memory and three more steps, bit for bit."""
    grid = (12, 10, 8)
    mech = I.make_mechanism(I.FIELD64)
    y0 = I.field_state(I.FIELD64, grid=grid)
    n, ld = y0.shape
    N = int(np.prod(grid))
    m, t = mri.Mech(mech), mri.Table(I.table_mis_kw3())
    ws = torch.empty(mri.mri_workspace_bytes(m, t, N, ld) // 8, dtype=torch.float64,
                     device="cuda")
    params = mri.advdiff_params(grid, n)
    opts = mri.fast_opts(n_sub=50)
    H = 1e-7

    def steps(y, k0, k1):
        for k in range(k0, k1):
            mri.mri_slow_step(m, t, opts, mri.ADVDIFF_RHS, params, k * H, H, N, ld, y, ws)
        torch.cuda.synchronize()

    a = _dev(torch, y0)
    steps(a, 0, 6)
    b = _dev(torch, y0)
    steps(b, 0, 3)
    path = tmp_path / "state.npz"
    np.savez(path, y=b.cpu().numpy(), t=3 * H, step=3)
    del b
    ck = np.load(path)
    c = _dev(torch, ck["y"])
    steps(c, int(ck["step"]), 6)
    assert float(ck["t"]) == 3 * H
    assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())


def test_stiffness_bound_matches_oracle(torch, mri, O):
    """The device's stiffness bound (Gershgorin bound of the species Jacobian)
    against the oracle's on 1000 cells of the 21- and 53-species mechanisms, and
    the MRI_CELL_STIFF bit exactly where h B exceeds the limit (cells within
    1e-10 of the threshold excluded)."""
    for wl in (I.FIELD64, I.LARGE128):
        mech = I.make_mechanism(wl)
        rng = np.random.Generator(np.random.PCG64(71))
        y = I.independent_cells(1000, mech.n_species, rng)
        n, ld = y.shape
        ref = O.Oracle(mech).stiff_bound(np.ascontiguousarray(y[:, :1000]))
        m = mri.Mech(mech)
        b = torch.zeros(ld, dtype=torch.float64, device="cuda")
        st = torch.full((ld,), 4, dtype=torch.int32, device="cuda")
        h = 2.785 / float(np.median(ref))
        mri.mri_stiffness_check(m, 1000, ld, _dev(torch, y), h, 2.785, b, st)
        torch.cuda.synchronize()
        got = b.cpu().numpy()[:1000]
        rel = np.abs(got - ref) / ref
        flag = (st.cpu().numpy()[:1000] & mri.CELL_STIFF) != 0
        want = h * ref > 2.785
        near = np.abs(h * ref / 2.785 - 1.0) < 1e-10
        print(f"{wl}: bound max rel diff {rel.max():.1e}, {flag.sum()} of 1000 flagged")
        assert rel.max() <= 1e-12
        assert np.array_equal(flag[~near], want[~near]) and 300 < flag.sum() < 700
        # OR-ed into the existing words
        assert np.all((st.cpu().numpy()[:1000] & 4) == 4)


@pytest.mark.parametrize("kernel", KERNELS)
def test_stage_stiffness_monitor(torch, mri, O, kernel):
    """A fixed-step stage with the monitor on: the state is bitwise the stage
    without it, the step counts are n_sub, and MRI_CELL_STIFF marks exactly the
    cells whose stage start state has h B above the limit (h = L / n_sub)."""
    mech = I.make_mechanism(I.SMALL)
    orc = O.Oracle(mech)
    y0 = I.initial_state(I.SMALL)
    n, ld = y0.shape
    rho = _small_forcing(O, orc, y0, 1)
    L, n_sub = 3e-7, 5
    bound = orc.stiff_bound(np.ascontiguousarray(y0[:, :512]))
    limit = float(np.median(bound)) * L / n_sub
    m = mri.Mech(mech)
    yd, rd = _dev(torch, y0), _dev(torch, rho)
    outs = []
    for lim in (0.0, limit):
        out = torch.zeros_like(yd)
        st = torch.full((ld,), 99, dtype=torch.int32, device="cuda")
        steps = torch.full((ld,), 99, dtype=torch.int32, device="cuda")
        opts = mri.fast_opts(n_sub=n_sub, kernel=_kernel(mri, kernel), stiff_limit=lim)
        mri.mri_fast_stage(m, opts, 512, ld, yd, out, 1, rd, L, st, steps)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), st.cpu().numpy()[:512], steps.cpu().numpy()[:512]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.all(outs[1][2] == n_sub)
    want = (L / n_sub) * bound > limit
    near = np.abs((L / n_sub) * bound / limit - 1.0) < 1e-10
    got = (outs[1][1] & mri.CELL_STIFF) != 0
    assert np.array_equal(got[~near], want[~near]) and 100 < got.sum() < 400
    assert np.array_equal(outs[1][1] & ~mri.CELL_STIFF, outs[0][1])
