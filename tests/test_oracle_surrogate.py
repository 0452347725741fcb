"""Pins for the oracle's surrogate functions (features, statistics, targets,
inference, residual check), each against values worked out by hand from the
definitions, limiting cases and exact identities."""
import math

import numpy as np
import pytest


def _soa(cols):
    """SoA [n][ld] from a list of per-cell state vectors."""
    return np.ascontiguousarray(np.array(cols, dtype=np.float64).T)


def test_feature_layout_and_values(oracle_mod):
    """S = 2 species (n = 3): features log max(Y, 1e-30), T, rho_(p,c) with
    zeros beyond n_poly, log L; 2 + 1 + 9 + 1 = 13 of them."""
    O = oracle_mod
    S = 2
    assert O.sur_n_features(S) == 13
    assert O.sur_n_features(21) == 89
    Y = _soa([[0.25, 0.0, 1500.0]])                    # Y_1 = 0 hits the 1e-30 floor
    RHO = np.zeros((2, 3, 1))
    RHO[0, :, 0] = [1.0, -2.0, 3.0]
    RHO[1, :, 0] = [4.0, 5.0, -6.0]
    stats = np.zeros(2 * 13 + 9)
    stats[13:26] = 1.0                                 # raw features: mean 0, inverse std 1
    X = O.sur_featurize(S, Y, RHO, np.array([2e-8]), stats, kpad=16)
    want = [math.log(0.25), math.log(1e-30), 1500.0, 1.0, -2.0, 3.0, 4.0, 5.0, -6.0,
            0.0, 0.0, 0.0, math.log(2e-8), 0.0, 0.0, 0.0]
    assert X.shape == (1, 16)
    assert X[0].tolist() == want


def test_standardization_and_constant_features(oracle_mod):
    """Three samples whose T is 1, 2, 3 (mean 2, std sqrt(2/3)); every other
    feature constant (inverse std 1); targets: log-correction of Y + 1e-8 and
    the plain T difference, standardized by their own moments."""
    O = oracle_mod
    S = 1
    Y0 = _soa([[0.5, 1.0], [0.5, 2.0], [0.5, 3.0]])
    Y1 = _soa([[0.5 * math.e - 1e-8 + 0.5e-8, 2.0], [0.5, 4.0], [0.5, 6.0]])
    RHO = np.zeros((1, 2, 3))
    Lv = np.full(3, 1e-7)
    st = O.sur_stats(S, Y0, RHO, Lv, Y1)
    F = O.sur_n_features(S)
    assert st[S] == 2.0 and st[F + S] == pytest.approx(1.0 / math.sqrt(2.0 / 3.0), rel=1e-15)
    for k in range(F):
        if k != S:
            assert st[F + k] == 1.0, k               # constant feature: inverse std 1
    # target of sample 0, species: log(0.5 e + 0.5e-8) - log(0.5 + 1e-8)
    t_sp = [math.log(0.5 * math.e + 0.5e-8) - math.log(0.5 + 1e-8), 0.0, 0.0]
    t_T = [1.0, 2.0, 3.0]
    for c, t in ((0, t_sp), (1, t_T)):
        m = sum(t) / 3
        sd = math.sqrt(sum((x - m) ** 2 for x in t) / 3)
        assert st[2 * F + c] == pytest.approx(m, rel=1e-14)
        assert st[2 * F + 2 * 2 + c] == pytest.approx(sd, rel=1e-12)
        assert st[2 * F + 2 + c] == pytest.approx(1.0 / sd, rel=1e-12)
    X, T = O.sur_featurize(S, Y0, RHO, Lv, st, kpad=F, Y1=Y1)
    np.testing.assert_allclose(X[:, S], [-math.sqrt(1.5), 0.0, math.sqrt(1.5)], rtol=1e-14,
                               atol=1e-15)
    assert np.all(X[:, :S] == 0.0)                    # (x - mean) * 1 with constant x
    # standardized targets have mean 0 and unit variance
    np.testing.assert_allclose(T.mean(axis=0), 0.0, atol=1e-14)
    np.testing.assert_allclose(T.std(axis=0), 1.0, rtol=1e-12)


def test_targets_relative_to_a_base_state(oracle_mod):
    """With a base state Yb the targets are the corrections from Yb to Y1."""
    O = oracle_mod
    S = 1
    Y0 = _soa([[0.3, 1000.0], [0.6, 1200.0]])
    Yb = _soa([[0.2, 1100.0], [0.4, 1300.0]])
    Y1 = _soa([[0.2 * math.exp(0.5) + 1e-8 * (math.exp(0.5) - 1), 1101.0],
               [0.4 * math.exp(-0.5) + 1e-8 * (math.exp(-0.5) - 1), 1299.0]])
    RHO = np.zeros((1, 2, 2))
    Lv = np.full(2, 1e-7)
    stats = O.sur_stats(S, Y0, RHO, Lv, Y1, Yb=Yb)
    F = O.sur_n_features(S)
    # species corrections are +-0.5 exactly (Y1 + 1e-8 = (Yb + 1e-8) e^(+-1/2)); T +1, -1
    assert stats[2 * F] == pytest.approx(0.0, abs=1e-15)
    assert stats[2 * F + 2 * 2] == pytest.approx(0.5, rel=1e-14)
    assert stats[2 * F + 1] == 0.0 and stats[2 * F + 2 * 2 + 1] == 1.0


def _linear_net(F, n, pick):
    """One affine layer [F] -> [n] whose output c copies feature pick[c]."""
    W = np.zeros((n, F))
    for c, k in enumerate(pick):
        if k is not None:
            W[c, k] = 1.0
    return np.concatenate([W.ravel(), np.zeros(n)])


def test_inference_applies_the_correction_to_the_base(oracle_mod):
    """A linear network that copies T's standardized feature into the T output
    and log Y_0's into the Y_0 output: with FP64 arithmetic the corrected state
    is base_T + y_mean + y_std z and (base_Y + 1e-8) e^d - 1e-8."""
    O = oracle_mod
    S = 1
    F = O.sur_n_features(S)
    Y = _soa([[0.25, 1500.0], [0.5, 1800.0]])
    B = _soa([[0.2, 1490.0], [0.1, 1790.0]])
    RHO = np.zeros((1, 2, 2))
    stats = np.zeros(2 * F + 6)
    stats[:F] = 0.0
    stats[F:2 * F] = 1.0
    stats[S] = 1600.0
    stats[F + S] = 0.01                       # T feature: (T - 1600) / 100
    stats[2 * F:2 * F + 2] = [0.1, 2.0]       # y_mean
    stats[2 * F + 4:2 * F + 6] = [0.5, 3.0]   # y_std
    p = _linear_net(F, 2, [0, S])
    out = O.sur_infer(S, [F, 2], p, stats, Y, RHO, 1e-7, base=B, bf16=False)
    for i in range(2):
        zT = (Y[1, i] - 1600.0) * 0.01
        assert out[1, i] == pytest.approx(B[1, i] + 2.0 + 3.0 * zT, rel=1e-15)
        d = 0.1 + 0.5 * math.log(Y[0, i])
        assert out[0, i] == pytest.approx((B[0, i] + 1e-8) * math.exp(d) - 1e-8, rel=1e-14)
    # without a base the correction applies to the start state itself
    out2 = O.sur_infer(S, [F, 2], p, stats, Y, RHO, 1e-7, bf16=False)
    assert out2[1, 0] == pytest.approx(Y[1, 0] + 2.0 + 3.0 * (Y[1, 0] - 1600.0) * 0.01,
                                       rel=1e-15)
    # a zero network leaves the base (negative mass fractions clamp to 0)
    z = np.zeros_like(p)
    st0 = stats.copy()
    st0[2 * F:2 * F + 2] = 0.0
    B2 = _soa([[-1e-9, 1490.0], [0.1, 1790.0]])
    out3 = O.sur_infer(S, [F, 2], z, st0, Y, RHO, 1e-7, base=B2, bf16=False)
    assert out3[0].tolist() == [0.0, 0.1 + 1e-8 - 1e-8] and out3[1].tolist() == [1490.0, 1790.0]


def test_gate_by_hand(oracle_mod):
    """Residual check on hand-made cells (S = 2, n = 3, tolerance 1e-4, Richardson
    factor 1/15, no forcing unless stated)."""
    O = oracle_mod
    S, tol, r = 2, 1e-4, 1.0 / 15.0
    y0 = [0.5, 0.5, 1000.0]
    cells = []
    # 0: Vc = Vh -> Ve = Vc; Vn = Ve: G = 0, accepted
    cells.append(([0.4, 0.6, 1010.0], [0.4, 0.6, 1010.0], [0.4, 0.6, 1010.0]))
    # 1: Vn differs from Ve in T by 0.101 K of 1010: D = 1e-4, accepted (G <= tol)
    cells.append(([0.4, 0.6, 1010.0], [0.4, 0.6, 1010.0], [0.4, 0.6, 1010.101]))
    # 2: Richardson: Vc - Vh = 1.5e-3 in T -> Ve = Vc + 1e-4; Vn = Vc: D = 1e-4/1010.0001
    cells.append(([0.4, 0.6, 1010.0], [0.4, 0.6, 1009.9985], [0.4, 0.6, 1010.0]))
    # 3: a species below the 1e-8 floor: |Vn - Ve| = 2e-12 over the floor -> D = 2e-4
    cells.append(([1e-12, 1.0 - 1e-12, 1010.0], [1e-12, 1.0 - 1e-12, 1010.0],
                  [3e-12, 1.0 - 1e-12, 1010.0]))
    # 4: Vn = Ve (D = 0) but the mass sum grew by 3e-4 of sum |y0| = 1: I = 3e-4, rejected
    cells.append(([0.4, 0.6003, 1010.0], [0.4, 0.6003, 1010.0], [0.4, 0.6003, 1010.0]))
    # 5: NaN in the prediction: rejected, G NaN
    cells.append(([0.4, 0.6, 1010.0], [0.4, 0.6, 1010.0], [0.4, float("nan"), 1010.0]))
    # 6: like 0 but flagged by the coarse solve: rejected
    cells.append(([0.4, 0.6, 1010.0], [0.4, 0.6, 1010.0], [0.4, 0.6, 1010.0]))
    Y0 = _soa([y0] * len(cells))
    Vc = _soa([c[0] for c in cells])
    Vh = _soa([c[1] for c in cells])
    Vn = _soa([c[2] for c in cells])
    RHO = np.zeros((1, 3, len(cells)))
    status = np.zeros(len(cells), dtype=np.int32)
    status[6] = 1
    G, acc = O.sur_gate(S, Y0, RHO, 1e-7, Vc, Vh, Vn, r, tol, status_c=status)
    assert G[0] == 0.0 and acc[0]
    assert G[1] == pytest.approx(0.101 / 1010.0, rel=1e-9) and acc[1] == (G[1] <= tol)
    assert G[2] == pytest.approx((1.5e-3 / 15.0) / (1010.0 + 1e-4), rel=1e-9) and acc[2]
    assert G[3] == pytest.approx(2e-4, rel=1e-6) and not acc[3]
    assert G[4] == pytest.approx(3e-4, rel=1e-9) and not acc[4]
    assert math.isnan(G[5]) and not acc[5]
    assert G[6] == 0.0 and not acc[6]
    # forcing: the mass sum may change by L sum_p sum_k rho_(p,k) / (p + 1)
    RHO2 = np.zeros((2, 3, 1))
    RHO2[0, :2, 0] = [1e3, 2e3]
    RHO2[1, :2, 0] = [3e3, -1e3]
    L = 1e-7
    gain = L * ((1e3 + 2e3) + (3e3 - 1e3) / 2.0)        # 4e-4
    Vf = _soa([[0.4 + gain, 0.6, 1010.0]])
    G2, acc2 = O.sur_gate(S, _soa([y0]), RHO2, L, Vf, Vf, Vf, r, tol)
    assert G2[0] == pytest.approx(0.0, abs=1e-15) and acc2[0]
    G3, acc3 = O.sur_gate(S, _soa([y0]), RHO2[:1], L, Vf, Vf, Vf, r, tol)   # one term only
    assert G3[0] == pytest.approx(L * 2e3 / 2.0, rel=1e-9) and not acc3[0]
