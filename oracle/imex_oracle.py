"""IMEX-MRI-GARK slow step, plain numpy (Sec. 2.1 with the slow operator split
as f^S = f^I + f^E; Sec. 3.2 and Sec. 6 put the diffusion into f^I and the
advection into f^E).

TEST INFRASTRUCTURE ONLY: imported by tests/ (and by nothing on the product
path).  It shares no code with libmri: the fast stages of the chemistry come
from the C oracle (oracle.c), the implicit diffusion solve is an exact FFT
solve on the periodic grid (libmri iterates instead), and every step below is
written out in the order the algorithm states it.

Table convention (inputs.ImexTable): stage i (0-based, i >= 1) with
dc_i = c_i - c_(i-1)
  * dc_i > 0 (a fast stage): the modified fast IVP over [T_(i-1), T_i] from
    Y_(i-1) with forcing r_i(tau) = (1/dc_i) sum_k tau^k sum_(j<i)
    (gamma[k][i][j] f^I_j + omega[k][i][j] f^E_j), tau in [0, 1];
  * dc_i = 0 (a solve-decoupled stage): the fast IVP has zero length and the
    forcing integrates to a plain Runge-Kutta update,
    Y_i = Y_(i-1) + H sum_(j<i) (gbar_ij f^I_j + obar_ij f^E_j) + H gbar_ii f^I(T_i, Y_i),
    gbar_ij = sum_k gamma[k][i][j] / (k + 1) (likewise obar), solved for Y_i.
y_(n+1) = Y_s.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import oracle as O


def _bar(coef, i, j):
    """sum_k coef[k][i][j] / (k + 1): the forcing polynomial's integral weight."""
    return sum(coef[k, i, j] / (k + 1.0) for k in range(coef.shape[0]))


def imex_mri_step(tb, y, H, fast, f_expl, f_impl, solve_impl, t0=0.0):
    """One IMEX-MRI-GARK slow step y_n -> y_(n+1).

    fast(Y, rho, L): v(L) of v' = f^F(v) + sum_k tau^k rho[k], v(0) = Y;
    f_expl(t, Y), f_impl(t, Y): the slow parts f^E and f^I;
    solve_impl(t, a, r): the Y with Y - a f^I(t, Y) = r.
    Returns y_(n+1) and the number of implicit solves."""
    s, ng = tb.c.size, tb.gamma.shape[0]
    Y = np.array(y, dtype=np.float64, copy=True)
    FE = [f_expl(t0, Y)]
    FI = [f_impl(t0, Y)]
    n_solve = 0
    for i in range(1, s):
        dc = tb.c[i] - tb.c[i - 1]
        Ti = t0 + tb.c[i] * H
        if dc > 0.0:
            rho = np.zeros((ng,) + Y.shape)
            for k in range(ng):
                for j in range(i):
                    rho[k] += tb.gamma[k, i, j] * FI[j] + tb.omega[k, i, j] * FE[j]
                rho[k] /= dc
            Y = fast(Y, rho, dc * H)
        else:
            r = Y.copy()
            for j in range(i):
                r += H * (_bar(tb.gamma, i, j) * FI[j] + _bar(tb.omega, i, j) * FE[j])
            a = H * _bar(tb.gamma, i, i)
            if a != 0.0:
                Y = solve_impl(Ti, a, r)
                n_solve += 1
            else:
                Y = r
        if i < s - 1:
            FE.append(f_expl(Ti, Y))
            FI.append(f_impl(Ti, Y))
    return Y, n_solve


# ---------------------------------------------------------------------------
# Linear three-rate problem y' = A_F y + A_E y + A_I y with exact fast flows
# ---------------------------------------------------------------------------
def linear_fast_exact(AF, Y, rho, L):
    """Exact v(L) of v' = AF v + sum_k (theta/L)^k rho[k] by the matrix
    exponential of the system augmented with the monomials w_k = (theta/L)^k
    (w_0' = 0, w_k' = (k/L) w_(k-1))."""
    n = AF.shape[0]
    ng = rho.shape[0]
    M = np.zeros((n + ng, n + ng))
    M[:n, :n] = AF
    for k in range(ng):
        M[:n, n + k] = rho[k]
        if k > 0:
            M[n + k, n + k - 1] = k / L
    z0 = np.zeros(n + ng)
    z0[:n] = Y
    z0[n] = 1.0
    return (scipy.linalg.expm(L * M) @ z0)[:n]


def imex_mri_step_linear(tb, AF, AE, AI, y, H):
    """The IMEX-MRI-GARK step on the linear problem (one state vector y [n])
    with exact fast flows and a dense implicit solve."""
    n = AF.shape[0]

    def fast(Y, rho, L):
        return linear_fast_exact(AF, Y, rho, L)

    return imex_mri_step(tb, y, H, fast, lambda t, Y: AE @ Y, lambda t, Y: AI @ Y,
                         lambda t, a, r: np.linalg.solve(np.eye(n) - a * AI, r))[0]


# ---------------------------------------------------------------------------
# Advection (explicit) and diffusion (implicit) on the periodic grid
# ---------------------------------------------------------------------------
def advection(y, grid, u, dx):
    """f^E = -u . grad(phi), the 2nd-order centred stencil of the C oracle with D = 0."""
    return O.advdiff(y, grid, u=u, D=0.0, dx=dx)


def diffusion(y, grid, D, dx):
    """f^I = D lap(phi), the 7-point stencil of the C oracle with u = 0."""
    return O.advdiff(y, grid, u=(0.0, 0.0, 0.0), D=D, dx=dx)


def diffusion_symbol(grid, dx):
    """Eigenvalues of the periodic 7-point Laplacian on the FFT modes, shaped
    (nz, ny, nx): sum over the axes of (2 cos(2 pi m / n) - 2) / dx^2."""
    nx, ny, nz = grid
    sx = (2.0 * np.cos(2.0 * np.pi * np.arange(nx) / nx) - 2.0) / dx ** 2
    sy = (2.0 * np.cos(2.0 * np.pi * np.arange(ny) / ny) - 2.0) / dx ** 2
    sz = (2.0 * np.cos(2.0 * np.pi * np.arange(nz) / nz) - 2.0) / dx ** 2
    return sz[:, None, None] + sy[None, :, None] + sx[None, None, :]


def diffusion_solve(a, r, grid, D, dx):
    """Exact solution of Y - a D lap(Y) = r on the periodic grid, every
    component (rows of r [n][ld], cells (z*ny + y)*nx + x in the first
    nx*ny*nz columns), by diagonalizing the Laplacian with the FFT."""
    nx, ny, nz = grid
    N = nx * ny * nz
    r = np.asarray(r, dtype=np.float64)
    out = np.array(r, copy=True)
    denom = 1.0 - a * D * diffusion_symbol(grid, dx)
    for c in range(r.shape[0]):
        field = r[c, :N].reshape(nz, ny, nx)
        out[c, :N] = np.real(np.fft.ifftn(np.fft.fftn(field) / denom)).ravel()
    return out


def imex_mri_step_advdiff(orc, tb, opts, grid, y, H, u, D, dx, t0=0.0):
    """The IMEX-MRI-GARK step of the chemistry (fast, C oracle stages with the
    options opts) with advection explicit and diffusion implicit.  y [n][ld]
    SoA with the grid's cells in its first nx*ny*nz columns.  Returns
    (y_(n+1), status OR over the fast stages)."""
    n_cells = int(np.prod(grid))
    status = np.zeros(y.shape[1], dtype=np.int32)

    def fast(Y, rho, L):
        out, st, _, _ = orc.fast_stage_soa(Y, rho, L, opts, n_cells=n_cells)
        status[:] |= st
        return out

    yn, _ = imex_mri_step(tb, y, H, fast,
                          lambda t, Y: advection(Y, grid, u, dx),
                          lambda t, Y: diffusion(Y, grid, D, dx),
                          lambda t, a, r: diffusion_solve(a, r, grid, D, dx), t0=t0)
    return yn, status
