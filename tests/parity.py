"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

# Relative error bound between the HIP path and the oracle, per species and
# temperature: |x_gpu - x_ora| / max(|x_ora|, floor), floor 1e-12 for mass
# fractions (absolute noise below that level carries no information) and 0 for T.
REL_TOL = 1e-10
Y_FLOOR = 1e-12


def rel_err(gpu, ora, n_species, cells=None):
    gpu = np.asarray(gpu)
    ora = np.asarray(ora)
    if cells is not None:
        gpu = gpu[:, cells]
        ora = ora[:, cells]
    floor = np.zeros((gpu.shape[0], 1))
    floor[:n_species] = Y_FLOOR
    return np.abs(gpu - ora) / np.maximum(np.abs(ora), floor)


def assert_parity(gpu, ora, n_species, cells=None, tol=REL_TOL, what=""):
    e = rel_err(gpu, ora, n_species, cells)
    worst = np.unravel_index(np.argmax(e), e.shape)
    assert e.max() <= tol, f"{what}: max rel err {e.max():.3e} at comp {worst[0]} cell {worst[1]}"
    return float(e.max())
