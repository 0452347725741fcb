"""Properties of the seeded synthetic workloads (no method arithmetic here)."""
import numpy as np
import pytest

from paper_2211_03293_amd import inputs as I


@pytest.mark.parametrize("workload", [I.SMALL, I.FIELD64, I.LARGE128])
def test_mechanism_structure(workload):
    m = I.make_mechanism(workload)
    cfg = I.WORKLOADS[workload]
    assert (m.n_species, m.n_reactions) == (cfg.n_species, cfg.n_reactions)
    comp = m.composition
    assert len({tuple(r) for r in comp}) == m.n_species            # distinct species
    # every reaction conserves elements (hence mass)
    np.testing.assert_array_equal(comp[m.reactants].sum(1), comp[m.products].sum(1))
    # sides disjoint, no duplicate reactions in either direction
    keys = set()
    for r, p in zip(m.reactants, m.products):
        assert not (set(r) & set(p))
        k = (tuple(sorted(r)), tuple(sorted(p)))
        assert k not in keys and k[::-1] not in keys
        keys.add(k)
    # oriented: Delta G(1500 K) <= 0
    g = m.g_a + m.g_b * 1500.0
    assert np.all(g[m.products].sum(1) - g[m.reactants].sum(1) <= 0)
    Wg = m.W * 1e3
    assert Wg.max() == pytest.approx(50.0) and Wg.min() >= 2.0
    assert np.all((m.cv >= 500) & (m.cv <= 3000))
    assert np.all(np.abs(m.beta) <= 1)
    assert np.all((m.theta >= 0) & (m.theta <= 30e3 / I.R_CAL))


def test_seeded_reproducibility():
    a, b = I.make_mechanism(I.FIELD64), I.make_mechanism(I.FIELD64)
    np.testing.assert_array_equal(a.lnA, b.lnA)
    np.testing.assert_array_equal(I.initial_state(I.SMALL), I.initial_state(I.SMALL))


def test_independent_cells():
    y = I.initial_state(I.SMALL)
    S = I.WORKLOADS[I.SMALL].n_species
    np.testing.assert_allclose(y[:S].sum(0), 1.0, atol=1e-15)
    assert y[S].min() >= 1000 and y[S].max() <= 2000


def test_field_state_small_grid():
    y = I.field_state(I.FIELD64, grid=(8, 8, 8))
    S = I.WORKLOADS[I.FIELD64].n_species
    np.testing.assert_allclose(y[:S].sum(0), 1.0, atol=1e-14)
    assert y[S].min() >= 1000 - 1e-9 and y[S].max() <= 2000 + 1e-9


def test_set_sizes():
    s = I.set_sizes()
    assert s.size == 1000 and s.min() >= 64 and s.max() <= 65536
    off = I.set_offsets(s)
    assert off[-1] == s.sum()
