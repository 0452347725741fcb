"""Pins for the oracle's chemistry right-hand side f^F.

Each test checks the oracle against something other than itself: conservation
laws that any correct mass-action RHS obeys, a constructed detailed-balance
state, degenerate rate laws that reduce to plain arithmetic, and the closed
form of an isothermal single reversible reaction.
"""
import math

import numpy as np
import pytest

from paper_2211_03293_amd import inputs as I

R_GAS = 8.314462618


def _states(mech, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return I.independent_cells(n, mech.n_species, rng, ld=n)


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64, I.LARGE128])
def test_mass_fraction_sum_and_elements_conserved(oracle_mod, workload):
    mech = I.make_mechanism(workload)
    orc = oracle_mod.Oracle(mech)
    y = _states(mech, 64, 11)
    comp = mech.composition.astype(np.float64)
    for i in range(y.shape[1]):
        d = orc.rhs_parts(y[:, i])
        Yd = d["ydot"][:-1]
        scale = np.abs(Yd).max()
        assert abs(Yd.sum()) <= 1e-13 * scale
        # element e: sum_k n_ke Y_k / W_k is constant
        el = (comp * (Yd / mech.W)[:, None]).sum(0)
        el_scale = (comp * (np.abs(Yd) / mech.W)[:, None]).sum(0)
        assert np.all(np.abs(el) <= 1e-13 * el_scale)


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64])
def test_energy_rate_vanishes(oracle_mod, workload):
    """dE/dt = grad E . f^F = 0 for the constant-volume adiabatic cell."""
    mech = I.make_mechanism(workload)
    orc = oracle_mod.Oracle(mech)
    y = _states(mech, 16, 12)
    for i in range(y.shape[1]):
        v = y[:, i]
        f = orc.rhs(v)
        # E is a quadratic polynomial in y, so the central difference is exact up to
        # rounding for any step; a large step keeps the rounding small.
        eps = 1.0 / np.abs(f[:-1]).max()
        dE = (orc.energy(v + eps * f) - orc.energy(v - eps * f)) / (2 * eps)
        ref = sum(abs(mech.g_a[k] / mech.W[k] * f[k]) for k in range(mech.n_species))
        assert abs(dE) <= 1e-12 * ref


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64, I.LARGE128])
def test_detailed_balance_state_is_stationary(oracle_mod, workload):
    """C_k = c0 exp(-g_k/RT + lambda . n_k) balances every element-conserving reaction."""
    mech = I.make_mechanism(workload)
    orc = oracle_mod.Oracle(mech)
    rng = np.random.Generator(np.random.PCG64(5))
    for T in (900.0, 1500.0, 2300.0):
        lam = rng.normal(size=mech.composition.shape[1])
        mu = -(mech.g_a + mech.g_b * T) / (R_GAS * T) + mech.composition @ lam
        mu -= mu.max()
        C = 1e-6 * np.exp(mu)                        # mol/cm^3
        Y = C * mech.W * 1e3 / (mech.rho * 1e-3)
        v = np.concatenate([Y, [T]])
        d = orc.rhs_parts(v)
        reac, prod = mech.reactants, mech.products
        fwd = d["kf"] * C[reac[:, 0]] * C[reac[:, 1]]
        assert np.all(np.abs(d["q"]) <= 1e-11 * fwd)


def _one_reaction_mech(lnA, beta, theta, g_a, g_b, W, cv, T_ref=298.15):
    m = I.Mechanism(
        n_species=4, n_reactions=1,
        reactants=np.array([[0, 1]], dtype=np.int32), products=np.array([[2, 3]], dtype=np.int32),
        lnA=np.array([lnA]), beta=np.array([beta]), theta=np.array([theta]),
        g_a=np.asarray(g_a, float), g_b=np.asarray(g_b, float), W=np.asarray(W, float),
        cv=np.asarray(cv, float), composition=np.array([[1, 0], [1, 2], [2, 1], [0, 1]]),
        rho=1.0, T_ref=T_ref)
    return m


def test_degenerate_rate_laws(oracle_mod):
    """beta = theta = 0 and Delta G = 0 give k_f = k_r = A; then beta = 1 gives A T,
    theta > 0 gives A exp(-theta/T); a Delta G offset gives K_c = exp(-dG/RT)."""
    W = [0.012, 0.044, 0.040, 0.016]          # A=(1,0), B=(1,2), C=(2,1), D=(0,1) with m=(12,16)
    Y = np.array([0.1, 0.2, 0.3, 0.4])
    T = 1234.0
    C = 1e-3 * Y / (np.array(W) * 1e3)        # mol/cm^3 at rho = 1 kg/m^3
    v = np.concatenate([Y, [T]])
    A = 3.0e9
    # (i) K_c = 1, k = A
    m = _one_reaction_mech(math.log(A), 0.0, 0.0, [0] * 4, [0] * 4, W, [1000.0] * 4)
    d = oracle_mod.Oracle(m).rhs_parts(v)
    q = A * (C[0] * C[1] - C[2] * C[3])
    assert d["kf"][0] == pytest.approx(A, rel=1e-14)
    assert d["kr"][0] == pytest.approx(A, rel=1e-14)
    assert d["q"][0] == pytest.approx(q, rel=1e-12)
    assert d["ydot"][0] == pytest.approx(-q * W[0] * 1e3 / 1e-3, rel=1e-12)
    assert d["ydot"][2] == pytest.approx(q * W[2] * 1e3 / 1e-3, rel=1e-12)
    # (ii) beta = 1
    m = _one_reaction_mech(math.log(A), 1.0, 0.0, [0] * 4, [0] * 4, W, [1000.0] * 4)
    assert oracle_mod.Oracle(m).rhs_parts(v)["kf"][0] == pytest.approx(A * T, rel=1e-13)
    # (iii) activation temperature
    m = _one_reaction_mech(math.log(A), 0.0, 5000.0, [0] * 4, [0] * 4, W, [1000.0] * 4)
    assert oracle_mod.Oracle(m).rhs_parts(v)["kf"][0] == pytest.approx(
        A * math.exp(-5000.0 / T), rel=1e-13)
    # (iv) products lower in Gibbs energy by 20 kJ/mol: K_c = exp(2e4/(R T)), k_r = k_f/K_c
    m = _one_reaction_mech(math.log(A), 0.0, 0.0, [0, 0, -2e4, 0], [0] * 4, W, [1000.0] * 4)
    d = oracle_mod.Oracle(m).rhs_parts(v)
    assert d["kr"][0] == pytest.approx(A * math.exp(-2e4 / (R_GAS * T)), rel=1e-13)
    # (v) temperature rate: only enthalpy-carrying species contribute
    g_a = [1e5, 0.0, 0.0, 0.0]
    cv = [700.0, 900.0, 1100.0, 1300.0]
    m = _one_reaction_mech(math.log(A), 0.0, 0.0, g_a, [0] * 4, W, cv, T_ref=T)
    d = oracle_mod.Oracle(m).rhs_parts(v)
    e0 = 1e5 / W[0]                            # J/kg, T = T_ref
    Tdot = -(e0 * d["ydot"][0]) / float(np.dot(Y, cv))
    assert d["ydot"][4] == pytest.approx(Tdot, rel=1e-12)


def test_isothermal_single_reaction_closed_form(oracle_mod):
    """A + B <-> C + D with C_A = C_B = a - x, C_C = C_D = c + x:
    dx/dt = (alpha - p x)(beta - q x), p = sqrt(kf) + sqrt(kr), q = sqrt(kf) - sqrt(kr),
    alpha = sqrt(kf) a - sqrt(kr) c, beta = sqrt(kf) a + sqrt(kr) c, so
    ln[(beta - q x)/(alpha - p x)] - ln(beta/alpha) = (p beta - q alpha) t.
    All g_a = 0 and T0 = T_ref keep T constant."""
    W = np.array([0.012, 0.044, 0.040, 0.016])
    T = 298.15
    kf, Kc = 2.0e10, 3.0
    g_b = np.array([0.0, 0.0, -R_GAS * math.log(Kc), 0.0])   # dG = -RT ln Kc
    m = _one_reaction_mech(math.log(kf), 0.0, 0.0, [0] * 4, g_b, W, [800.0, 900.0, 1e3, 1.1e3],
                           T_ref=T)
    orc = oracle_mod.Oracle(m)
    a, c = 4.0e-6, 1.0e-6                      # mol/cm^3
    Cv = np.array([a, a, c, c])
    Y = Cv * W * 1e3 / 1e-3
    v0 = np.concatenate([Y, [T]])
    kr = kf / Kc
    sf, sr = math.sqrt(kf), math.sqrt(kr)
    p, q = sf + sr, sf - sr
    al, be = sf * a - sr * c, sf * a + sr * c
    t_end = 2.0e-5
    E = (be / al) * math.exp((p * be - q * al) * t_end)
    x = (be - E * al) / (q - E * p)
    out, st = orc.rk4_stage(v0, np.zeros((1, 5)), t_end, 400)
    assert st == 0
    C_end = out[:4] * 1e-3 / (W * 1e3)
    np.testing.assert_allclose(C_end, [a - x, a - x, c + x, c + x], rtol=1e-9)
    assert out[4] == T


def test_fd_jacobian_of_a_linear_rhs_is_its_matrix(oracle_mod):
    """Central differences are exact for f = A v (up to rounding): the oracle's
    Jacobian returns A itself, row i = d f_i / d y_j (A is not symmetric, so a
    transposed layout fails)."""
    rng = np.random.Generator(np.random.PCG64(41))
    A = rng.normal(size=(5, 5))
    orc = oracle_mod.Oracle(A_fast=A)
    J = orc.jacobian(rng.uniform(0.5, 2.0, 5))
    np.testing.assert_allclose(J, A, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64])
def test_fd_jacobian_matches_directional_derivative(oracle_mod, workload):
    """J delta equals (f(y + e delta) - f(y - e delta)) / (2 e) for a random
    direction delta (the chemistry Jacobian's columns and their scaling)."""
    mech = I.make_mechanism(workload)
    orc = oracle_mod.Oracle(mech)
    rng = np.random.Generator(np.random.PCG64(43))
    y = I.independent_cells(1, mech.n_species, rng, ld=1)[:, 0]
    n = y.size
    J = orc.jacobian(y)
    d = rng.normal(size=n) * np.abs(y) * 1e-2
    d[-1] = 1.0                                   # a temperature component in K
    for e in (1e-4, 1e-5):
        fd = (orc.rhs(y + e * d) - orc.rhs(y - e * d)) / (2 * e)
        scale = np.abs(J) @ np.abs(d) + 1e-300
        assert np.all(np.abs(J @ d - fd) <= 1e-4 * scale + 1e-12 * np.abs(fd).max())


def test_stiffness_bound_single_reaction_is_the_spectral_radius(oracle_mod):
    """One reversible reaction A + B <=> C + D: the species Jacobian (at fixed T)
    is the rank-one nu (grad q)^T, whose only nonzero eigenvalue is nu . grad q
    = -(kf C_b + kf C_a + kr C_d + kr C_c); the Gershgorin bound equals its
    magnitude, and so does the finite-difference Jacobian's leading eigenvalue."""
    W = [0.012, 0.044, 0.040, 0.016]
    mech = _one_reaction_mech(math.log(3e12), 0.5, 4000.0, [-1e4, 2e4, -5e4, 1e4],
                              [-20.0, 10.0, 5.0, -30.0], W, [1000.0, 1500.0, 800.0, 2000.0])
    orc = oracle_mod.Oracle(mech)
    y = np.array([0.3, 0.2, 0.4, 0.1, 1500.0])
    d = orc.rhs_parts(y)
    C = 1e-3 * y[:4] / (np.array(W) * 1e3)
    kf, kr = d["kf"][0], d["kr"][0]
    w = kf * (C[0] + C[1]) + kr * (C[2] + C[3])
    assert orc.stiff_bound(y) == pytest.approx(w, rel=1e-14)
    J = orc.jacobian(y)[:4, :4]
    ev = np.linalg.eigvals(J)
    lead = ev[np.argmax(np.abs(ev))]
    assert lead.real == pytest.approx(-w, rel=1e-5) and abs(lead.imag) <= 1e-6 * w


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64])
def test_stiffness_bound_dominates_the_spectral_radius(oracle_mod, workload):
    """On random cells of the workload mechanisms the bound is at least the
    spectral radius of the species block of the finite-difference Jacobian."""
    mech = I.make_mechanism(workload)
    orc = oracle_mod.Oracle(mech)
    y = _states(mech, 24, 44)
    S = mech.n_species
    b = orc.stiff_bound(y)
    ratios = []
    for i in range(y.shape[1]):
        assert b[i] == orc.stiff_bound(y[:, i])
        J = orc.jacobian(y[:, i])[:S, :S]
        rho = np.abs(np.linalg.eigvals(J)).max()
        assert b[i] >= rho * (1 - 1e-5), (i, b[i], rho)
        ratios.append(b[i] / rho)
    print(f"{workload}: bound / spectral radius in [{min(ratios):.2f}, {max(ratios):.2f}]")
