"""Pins of the IMEX-MRI-GARK oracle (Sec. 2.1 with f^S = f^I + f^E, solve-
decoupled implicit stages) and of its two tables: internal consistency; for
the 2nd-order table the three limits that reduce the method to textbook
schemes (trapezoidal rule for f^I alone, Heun's method for f^E alone, the
exact fast flow for f^F alone), order 2 on a non-commuting linear three-rate
problem with a closed-form solution (local error O(H^3), global O(H^2)) and in
self-convergence on nonlinear chemistry with advection and diffusion; for the
3rd-order table the exact fast flow, order 3 on the same two problems, the
order conditions through H^3 on random three-way split quadratic fields by
power series (an implementation independent of the oracle), and the
L-stability of its implicit part; stability of both past the explicit tables'
diffusion limit; and the exact periodic diffusion solve against the stencil
it inverts and against a single Fourier mode."""
import numpy as np
import pytest
import scipy.linalg

from paper_2211_03293_amd import inputs as I


@pytest.fixture(scope="module")
def X(oracle_mod):
    from oracle import imex_oracle
    return imex_oracle


def _mats(seed, n=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    AF = rng.normal(size=(n, n)) - 3.0 * np.eye(n)
    AE = 0.5 * rng.normal(size=(n, n))
    AI = rng.normal(size=(n, n))
    AI = -(AI @ AI.T) - np.eye(n)          # symmetric negative definite, like diffusion
    return AF, AE, AI, rng.normal(size=n)


@pytest.mark.parametrize("make", [I.table_imex_trap2, I.table_imex_mri3])
def test_table_is_internally_consistent(X, make):
    """sum_j of each row's integral weights equals dc_i for both partitions (a
    constant slow tendency is integrated exactly), the explicit part is
    strictly lower triangular, and the implicit diagonal sits only on stages
    with dc_i = 0."""
    tb = make()
    for i in range(1, tb.s):
        dc = tb.c[i] - tb.c[i - 1]
        gsum = sum(X._bar(tb.gamma, i, j) for j in range(i + 1))
        wsum = sum(X._bar(tb.omega, i, j) for j in range(i + 1))
        assert gsum == pytest.approx(dc, abs=1e-15) and wsum == pytest.approx(dc, abs=1e-15)
        assert np.all(tb.omega[:, i, i:] == 0.0)
        assert np.all(tb.gamma[:, i, i + 1:] == 0.0)
        if dc > 0.0:
            assert np.all(tb.gamma[:, i, i] == 0.0)


def test_limits_reduce_to_textbook_schemes(X):
    """f^F = f^E = 0: the trapezoidal rule; f^F = f^I = 0: Heun's method
    (I + H A + H^2 A^2 / 2 on a linear problem); f^E = f^I = 0: the exact flow."""
    tb = I.table_imex_trap2()
    AF, AE, AI, y = _mats(3)
    Z = np.zeros_like(AF)
    n = AF.shape[0]
    H = 0.3
    trap = np.linalg.solve(np.eye(n) - 0.5 * H * AI, (np.eye(n) + 0.5 * H * AI) @ y)
    np.testing.assert_allclose(X.imex_mri_step_linear(tb, Z, Z, AI, y, H), trap, rtol=1e-13)
    heun = (np.eye(n) + H * AE + 0.5 * H * H * AE @ AE) @ y
    np.testing.assert_allclose(X.imex_mri_step_linear(tb, Z, AE, Z, y, H), heun, rtol=1e-13)
    flow = scipy.linalg.expm(H * AF) @ y
    np.testing.assert_allclose(X.imex_mri_step_linear(tb, AF, Z, Z, y, H), flow, rtol=1e-12)


def test_solve_decoupled_rows_use_the_integral_weights(X):
    """On a stage with dc_i = 0 only the integral of the forcing polynomial
    matters, gbar_ij = sum_k gamma[k][i][j] / (k + 1): moving part of the last
    row's coefficients into a linear-in-tau term of equal integral (Gamma^0 -=
    x, Gamma^1 += 2x) leaves the step unchanged to rounding, and changes it
    when the same move is made on the fast stage's row (whose forcing is then
    no longer constant in time)."""
    import copy
    tb = I.table_imex_trap2()
    AF, AE, AI, y = _mats(7)
    H = 0.02
    ref = X.imex_mri_step_linear(tb, AF, AE, AI, y, H)
    t2 = copy.deepcopy(tb)
    t2.gamma = np.concatenate([tb.gamma, np.zeros_like(tb.gamma)])
    t2.omega = np.concatenate([tb.omega, np.zeros_like(tb.omega)])
    x = 0.3
    for c in (t2.gamma, t2.omega):
        c[0, 2, 0] -= x
        c[1, 2, 0] += 2 * x
    np.testing.assert_allclose(X.imex_mri_step_linear(t2, AF, AE, AI, y, H), ref, rtol=1e-13)
    t3 = copy.deepcopy(t2)
    t3.gamma[0, 1, 0] -= x
    t3.gamma[1, 1, 0] += 2 * x
    assert np.abs(X.imex_mri_step_linear(t3, AF, AE, AI, y, H) - ref).max() > 1e-8


def test_order_two_on_the_linear_three_rate_problem(X):
    """Non-commuting A_F, A_E, A_I with the closed-form solution
    expm(t (A_F + A_E + A_I)) y0: the local error falls by 8 and the global
    error by 4 per halving of H; a wrong sign or a dropped coefficient in any
    row of the table breaks one of the two."""
    tb = I.table_imex_trap2()
    AF, AE, AI, y0 = _mats(5)
    A = AF + AE + AI
    loc = []
    for H in (0.01, 0.005, 0.0025, 0.00125):
        loc.append(np.linalg.norm(X.imex_mri_step_linear(tb, AF, AE, AI, y0, H)
                                  - scipy.linalg.expm(H * A) @ y0))
    lr = np.log2(np.array(loc[:-1]) / np.array(loc[1:]))
    assert np.all(np.abs(lr - 3.0) < 0.15), (loc, lr)
    T = 0.5
    glob = []
    for n in (32, 64, 128, 256):
        y = y0.copy()
        for _ in range(n):
            y = X.imex_mri_step_linear(tb, AF, AE, AI, y, T / n)
        glob.append(np.linalg.norm(y - scipy.linalg.expm(T * A) @ y0))
    gr = np.log2(np.array(glob[:-1]) / np.array(glob[1:]))
    assert np.all(np.abs(gr - 2.0) < 0.1), (glob, gr)


def test_mri3_exact_fast_flow_and_order_three_on_the_linear_three_rate_problem(X):
    """3rd-order table: with f^E = f^I = 0 the step is the exact fast flow;
    on the non-commuting problem of the 2nd-order pin the local error falls by
    16 and the global error by 8 per halving of H."""
    tb = I.table_imex_mri3()
    AF, AE, AI, y0 = _mats(5)
    Z = np.zeros_like(AF)
    np.testing.assert_allclose(X.imex_mri_step_linear(tb, AF, Z, Z, y0, 0.3),
                               scipy.linalg.expm(0.3 * AF) @ y0, rtol=1e-12)
    A = AF + AE + AI
    loc = [np.linalg.norm(X.imex_mri_step_linear(tb, AF, AE, AI, y0, H)
                          - scipy.linalg.expm(H * A) @ y0) for H in (0.02, 0.01, 0.005)]
    lr = np.log2(np.array(loc[:-1]) / np.array(loc[1:]))
    assert np.all(np.abs(lr - 4.0) < 0.2), (loc, lr)
    T = 0.5
    glob = []
    for n in (16, 32, 64):
        y = y0.copy()
        for _ in range(n):
            y = X.imex_mri_step_linear(tb, AF, AE, AI, y, T / n)
        glob.append(np.linalg.norm(y - scipy.linalg.expm(T * A) @ y0))
    gr = np.log2(np.array(glob[:-1]) / np.array(glob[1:]))
    assert np.all(np.abs(gr - 3.0) < 0.15), (glob, gr)


def test_mri3_order_conditions_by_power_series():
    """The 3rd-order table against the exact flow through H^3 on 20 random
    three-way split quadratic vector fields, one step expanded as truncated
    power series (fast stages by Picard iteration in the stage-internal time,
    implicit stages by fixed-point iteration): every coefficient through H^3
    vanishes to rounding, while H^4 does not; a 2nd-order table fails at H^3."""
    from paper_2211_03293_amd import derive_imex3_table as D
    tb = I.table_imex_mri3()
    probs = D.problems(4242, 20)
    assert np.abs(D.order_residual(tb.gamma, tb.omega, probs)).max() < 1e-12
    n_keep = D.N
    D.N = 4                                  # expand one order further
    try:
        e4 = max(np.abs(D.local_error(tb.gamma, tb.omega, p, y0)[:, 4]).max()
                 for p, y0 in probs[:3])
    finally:
        D.N = n_keep
    assert e4 > 1e-3
    bad = tb.gamma.copy()
    bad[0, 6, 6] += 1e-3
    bad[0, 6, 5] -= 1e-3
    assert np.abs(D.order_residual(bad, tb.omega, probs)).max() > 1e-5


def test_mri3_implicit_part_is_L_stable(X):
    """With f^F = f^E = 0 and f^I = lambda y the step multiplies by R(z),
    z = H lambda: |R(z)| <= 1 along the negative real axis (the diffusion
    operator's spectrum) and R(z) -> 0 as z -> -inf."""
    tb = I.table_imex_mri3()
    Z = np.zeros((1, 1))
    R = lambda z: float(X.imex_mri_step_linear(tb, Z, Z, np.array([[z]]), np.ones(1), 1.0)[0])
    vals = np.array([R(-z) for z in np.logspace(-3, 4, 120)])
    assert np.all(np.abs(vals) <= 1.0 + 1e-12)
    assert abs(R(-1e4)) < 1e-2 and abs(R(-1e3)) < 5e-2
    assert R(-1.0) == pytest.approx(np.exp(-1.0), abs=3e-3)


def test_diffusion_solve_inverts_the_stencil(X, oracle_mod):
    """The FFT solve returns Y with Y - a D lap(Y) = r for the C oracle's
    7-point stencil, on an odd non-cubic grid with several components and
    padding columns left untouched; a = 0 is the identity."""
    grid = (6, 4, 5)
    N = int(np.prod(grid))
    rng = np.random.Generator(np.random.PCG64(11))
    r = rng.normal(size=(3, N + 7))
    D, dx, a = 0.3, 0.1, 0.02
    Y = X.diffusion_solve(a, r, grid, D, dx)
    res = Y - a * X.diffusion(Y, grid, D, dx) - r
    assert np.abs(res[:, :N]).max() <= 1e-12 * np.abs(r).max()
    np.testing.assert_array_equal(Y[:, N:], r[:, N:])
    np.testing.assert_array_equal(X.diffusion_solve(0.0, r, grid, D, dx)[:, :N],
                                  np.real(np.fft.ifftn(np.fft.fftn(
                                      r[:, :N].reshape(3, 5, 4, 6), axes=(1, 2, 3)),
                                      axes=(1, 2, 3))).reshape(3, N))


def test_diffusion_of_a_fourier_mode(X):
    """On phi = cos(2 pi (m_x x / n_x + m_z z / n_z)) the stencil returns
    sigma phi with sigma = sum_axes (2 cos(2 pi m / n) - 2) / dx^2, and the
    solve divides by 1 - a D sigma."""
    grid = (8, 6, 10)
    nx, ny, nz = grid
    z, yy, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mx, mz = 3, 2
    phi = np.cos(2 * np.pi * (mx * x / nx + mz * z / nz)).ravel()[None, :]
    dx, D, a = 0.5, 0.7, 0.3
    sigma = ((2 * np.cos(2 * np.pi * mx / nx) - 2) + (2 * np.cos(2 * np.pi * mz / nz) - 2)) / dx ** 2
    np.testing.assert_allclose(X.diffusion(phi, grid, D, dx), D * sigma * phi, atol=1e-12)
    np.testing.assert_allclose(X.diffusion_solve(a, phi, grid, D, dx), phi / (1 - a * D * sigma),
                               atol=1e-13)


def _chem_setup(oracle_mod, grid, scale=1e-3):
    mech = I.make_mechanism(I.FIELD64)
    mech = mech.with_scale(mech.rate_scale * scale)
    return oracle_mod.Oracle(mech), I.field_state(I.FIELD64, grid)


@pytest.mark.parametrize("make,order", [(I.table_imex_trap2, 2.0), (I.table_imex_mri3, 3.0)])
def test_order_on_nonlinear_chemistry_with_advection_and_diffusion(X, oracle_mod, make, order):
    """21-species chemistry (rates scaled by 1e-3, as for the 4th-order explicit
    table's pin) as the fast part, advection explicit and diffusion implicit
    on a 4^3 periodic grid with a diffusion number H D / dx^2 between 1.25 and
    0.3; self-convergence against 64 steps with the fast stages resolved by
    64 RK4 substeps: observed order 2 for the 2nd-order table, 3 for the
    3rd-order one."""
    grid = (4, 4, 4)
    orc, y0 = _chem_setup(oracle_mod, grid)
    tb = make()
    u, dx = (10.0, 10.0, 10.0), 1e-4
    T_end = 2e-6
    D = 2.5e-3

    def run(n):
        y = y0.copy()
        H = T_end / n
        for s in range(n):
            y, st = X.imex_mri_step_advdiff(orc, tb, oracle_mod.rk4_opts(64), grid, y, H, u, D, dx,
                                            t0=s * H)
            assert np.all(st[:64] == 0)
        return y[:, :64]

    ref = run(64)
    errs = [np.abs(run(n) - ref).max() for n in (4, 8, 16)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.3), (errs, rates)


@pytest.mark.parametrize("make", [I.table_imex_trap2, I.table_imex_mri3])
def test_stable_past_the_explicit_diffusion_limit(X, oracle_mod, make):
    """At the diffusion number H D / dx^2 = 1 (the stiff-diffusion constants
    of the 64^3 fields, H = 1e-7 s), on an 8^3 grid holding a smooth state (one
    long-wave temperature mode) plus a grid-scale checkerboard of 1e-6 K: the
    checkerboard grows under the explicit 3rd-order table (its stability
    polynomial at the checkerboard's eigenvalue H D sigma = -12 has modulus
    227) until the state leaves the physical range, and decays under the IMEX
    steps (factors R(-12): (1 - 6) / (1 + 6) for the 2nd-order table, 0.44 for
    the 3rd-order one), with the mass fractions in [0, 1] and their sum
    preserved."""
    grid = (8, 8, 8)
    N = 512
    orc, yf = _chem_setup(oracle_mod, (4, 4, 4), scale=1.0)
    z, yy, x = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    chk = ((-1.0) ** (x + yy + z)).ravel()
    y0 = np.repeat(yf[:, :1], N, axis=1)
    y0[-1] += 50.0 * np.cos(2.0 * np.pi * x.ravel() / 8.0) + 1e-6 * chk

    def amplitude(y):
        return abs(float(np.dot(y[-1, :N], chk))) / N

    P = I.ADVDIFF_STIFF
    H = 1e-7
    ye, yi = y0.copy(), y0.copy()
    a0 = amplitude(y0)
    bad_e = False
    for s in range(10):
        if not bad_e:
            ye, st, _, _ = orc.mri_step_advdiff(I.table_mis_kw3(), oracle_mod.rk4_opts(50), grid,
                                               ye, H, u=P["u"], D=P["D"], dx=P["dx"], t=s * H)
            bad_e = bool(np.any(st[:N] != 0)) or not np.all(np.isfinite(ye[:, :N])) \
                or amplitude(ye) > 1e2
        yi, sti = X.imex_mri_step_advdiff(orc, make(), oracle_mod.rk4_opts(50), grid,
                                          yi, H, P["u"], P["D"], P["dx"], t0=s * H)
        assert np.all(sti[:N] == 0)
    assert bad_e
    assert amplitude(yi) < 0.1 * a0
    Yi = yi[:-1, :N]
    assert Yi.min() > -1e-9 and Yi.max() < 1.0 + 1e-9
    np.testing.assert_allclose(Yi.sum(axis=0), 1.0, atol=1e-9)
