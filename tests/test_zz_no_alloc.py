"""The allocation-free slow step (mri_slow_step_noalloc) against mri_slow_step
with a caller workspace: two calls in a row, the second on a smaller grid, each
bitwise equal to the workspace path (same kernels, same order of operations) and
within the parity bound of the oracle."""
import numpy as np
import pytest

from paper_2211_03293_amd import inputs as I
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


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


def _step_pair(torch, mri, m, t, grid, H=1e-7, n_sub=50):
    y0 = I.field_state(I.FIELD64, grid=grid)
    n, ld = y0.shape
    N = int(np.prod(grid))
    params = mri.advdiff_params(grid, n)
    opts = mri.fast_opts(n_sub=n_sub)
    y_ws = torch.as_tensor(y0, device="cuda")
    ws = torch.empty(mri.mri_workspace_bytes(m, t, N, ld) // 8, dtype=torch.float64,
                     device="cuda")
    st_ws = torch.zeros(ld, dtype=torch.int32, device="cuda")
    mri.mri_slow_step(m, t, opts, mri.ADVDIFF_RHS, params, 0.0, H, N, ld, y_ws, ws, st_ws)
    y_na = torch.as_tensor(y0, device="cuda")
    st_na = torch.full((ld,), 7, dtype=torch.int32, device="cuda")
    mri.mri_slow_step_noalloc(m, t, opts, mri.ADVDIFF_RHS, params, 0.0, H, N, ld, y_na, st_na)
    torch.cuda.synchronize()
    return y0, y_ws.cpu().numpy(), y_na.cpu().numpy(), st_ws.cpu().numpy(), st_na.cpu().numpy()


def test_noalloc_slow_step_matches_workspace_path_twice(torch, mri, oracle_mod):
    mech = I.make_mechanism(I.FIELD64)
    tb = I.table_mis_kw3()
    m, t = mri.Mech(mech), mri.Table(tb)
    orc = oracle_mod.Oracle(mech)
    for grid in ((16, 12, 10), (8, 8, 6)):          # second call: smaller input
        print(f"noalloc slow step, grid {grid}", flush=True)
        y0, y_ws, y_na, st_ws, st_na = _step_pair(torch, mri, m, t, grid)
        N = int(np.prod(grid))
        assert np.array_equal(y_na, y_ws), f"grid {grid}: differs from the workspace path"
        assert np.array_equal(st_na[:N], st_ws[:N]) and not st_na[:N].any()
        ref, st_o, _, _ = orc.mri_step_advdiff(tb, oracle_mod.rk4_opts(50), grid, y0, 1e-7,
                                               t=0.0)
        assert not st_o[:N].any()
        assert_parity(y_na, ref, mech.n_species, what=f"noalloc {grid}")


def test_noalloc_refuses_oversize_and_unprepared_kernels(torch, mri):
    mech = I.make_mechanism(I.FIELD64)
    tb = I.table_mis_kw3()
    m, t = mri.Mech(mech), mri.Table(tb)
    n = mech.n_species + 1
    cap = mri.mri_noalloc_scratch_bytes()
    ld_max = cap // (8 * n * (tb.s - 1 + tb.n_gamma))
    y = torch.zeros((n, 64), dtype=torch.float64, device="cuda")
    params = mri.advdiff_params((4, 4, 4), n)
    # a fresh mechanism handle has no kernel on the device yet: refused, not set up
    with pytest.raises(mri.MriError, match="not set up"):
        mri.mri_slow_step_noalloc(m, t, mri.fast_opts(n_sub=5), mri.ADVDIFF_RHS, params, 0.0,
                                  1e-7, 64, 64, y)
    # more planes than the array holds: refused before any device work
    with pytest.raises(mri.MriError, match="scratch"):
        mri.mri_slow_step_noalloc(m, t, mri.fast_opts(n_sub=5), mri.ADVDIFF_RHS, params, 0.0,
                                  1e-7, 64, ld_max + 64, y)
