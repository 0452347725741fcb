"""Pins of the oracle's adaptive slow-step controller (step doubling, the
adaptive step control proposed in Sec. 7 for multirate methods) on the
non-commuting linear two-rate problem, whose exact flow is a matrix
exponential: the error estimate against the true error, tolerance
proportionality, the reject path and the end-time landing."""
import numpy as np
import pytest
from scipy.linalg import expm

from paper_2211_03293_amd import inputs as I

A_F = np.array([[-6.0, 5.0], [-5.0, -4.0]])
A_S = np.array([[0.3, 1.0], [-1.2, 0.2]])
Y0 = np.array([[1.0], [0.5]])


def _stepper(O, tb, n_sub=256):
    orc = O.Oracle(A_fast=A_F)

    def step(y, t, H):
        out, st, _, _ = orc.mri_step_linear(tb, O.rk4_opts(n_sub), A_S, y[:, 0], H, t=t)
        return out, st
    return step


@pytest.mark.parametrize("table,order", [(I.table_mis_kw3(), 3), (I.table_erk45a(), 4)])
def test_step_doubling_estimate_tracks_true_error(oracle_mod, table, order):
    """(y_half - y_full) / (2^p - 1) estimates the error of the half-step result;
    the ratio to the true error tends to 1 as H -> 0 (fast stages resolved)."""
    step = _stepper(oracle_mod, table)
    ratios = []
    for H in (0.25, 0.125, 0.0625):
        y_full, _ = step(Y0, 0.0, H)
        y_half, _ = step(step(Y0, 0.0, H / 2)[0], H / 2, H / 2)
        est = (y_half - y_full) / (2.0 ** order - 1.0)
        true = y_half[:, 0] - expm((A_F + A_S) * H) @ Y0[:, 0]
        ratios.append(np.linalg.norm(est[:, 0]) / np.linalg.norm(true))
    assert abs(ratios[-1] - 1.0) < 0.15 and abs(ratios[-1] - 1) < abs(ratios[0] - 1) + 0.05, \
        ratios


def test_controller_meets_tolerance_and_step_count_scales(oracle_mod):
    """The global error follows the tolerance; the number of accepted steps
    grows like tol^(-1/(p+1)) for the 3rd-order table."""
    step = _stepper(oracle_mod, I.table_mis_kw3())
    exact = expm(A_F + A_S) @ Y0[:, 0]
    res = {}
    for tol in (1e-5, 1e-7, 1e-9):
        y, st, hist = oracle_mod.adaptive_run(step, Y0, 0.0, 1.0, 3, 0.0, tol, tol, 0.05)
        assert st["t"] == 1.0
        err = np.abs(y[:, 0] - exact).max()
        res[tol] = (err, st["accepted"])
        assert 1e-3 * tol < err < 10 * tol, (tol, err)
    e = [res[t][0] for t in (1e-5, 1e-7, 1e-9)]
    assert e[0] > e[1] > e[2]
    growth = res[1e-9][1] / res[1e-5][1]
    assert 5.0 < growth < 20.0, res          # (1e4)^(1/4) = 10


def test_oversized_first_step_is_rejected_and_end_time_is_hit(oracle_mod):
    step = _stepper(oracle_mod, I.table_mis_kw3(), n_sub=64)
    y, st, hist = oracle_mod.adaptive_run(step, Y0, 0.0, 0.7, 3, 1e-8, 1e-8, 1e-8, 0.7)
    assert st["rejected"] >= 1 and not hist[0][3]
    assert all((e <= 1.0) == acc for _, _, e, acc in hist)
    for (t0, H0, e0, a0), (t1, H1, e1, a1) in zip(hist, hist[1:]):
        if not a0:
            assert t1 == t0 and H1 < H0        # retried from the same time, smaller step
    acc = [(t, H) for t, H, _, a in hist if a]
    assert sum(H for _, H in acc) == pytest.approx(0.7, rel=1e-14)
    assert st["t"] == 0.7
    assert np.abs(y[:, 0] - expm((A_F + A_S) * 0.7) @ Y0[:, 0]).max() < 1e-6


def test_fixed_substep_rule(oracle_mod):
    f = oracle_mod.fixed_substeps
    assert f(50, 0.5e-7, 1e-7) == 25
    assert f(50, 1e-7 / 3, 1e-7) == 17
    assert f(50, 2e-7, 1e-7) == 100
    assert f(50, 1e-7, 1e-7) == 50
    assert f(4, 1e-12, 1e-7) == 1
