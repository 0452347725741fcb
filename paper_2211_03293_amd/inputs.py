"""Seeded synthetic workloads for the MRI fast-stage solver.

This module only draws random numbers and arranges them into arrays.  It holds
none of the method's arithmetic (no rate law, no RHS, no integrator), so both
the GPU path and the CPU oracle can be fed from it without sharing code.

Workload recipe (the paper's GRI-Mech 3.0 / PREMIX inputs, Sec. 5.1 and 5.2,
are not available and are not reproduced; these synthetic inputs stand in):

* Species are distinct element-composition vectors n_k on a small lattice, so
  that every drawn 2->2 reaction conserves elements and mass exactly.
  Molar masses W_k = n_k . m for atomic masses m scaled so max W = 50 g/mol.
* Reactions {a,b} <-> {c,d} are drawn uniformly from all element-balanced pairs
  with disjoint sides, then oriented so that Delta G(1500 K) <= 0.
* Arrhenius A log-uniform in [1e8, 1e14] (cm^3 mol^-1 s^-1), beta ~ U[-1, 1],
  Ea ~ U[0, 30] kcal/mol;  Gibbs g_k(T) = a_k + b_k T with a_k ~ U[-3e5, 3e5]
  J/mol, b_k ~ U[-200, 50] J/mol/K;  cv_k ~ U[500, 3000] J/kg/K;  rho = 1 kg/m^3.
* A global rate scale s multiplies every forward and reverse rate so that the
  longest fast substep satisfies h * rho(J_F) ~ 0.5 on the initial states.  The
  literal generators give rate constants up to 1e27 s^-1, which no explicit
  method can integrate at the stated step sizes.  s is stored in
  rate_scales.json (written by oracle/calibrate_scales.py).
* Seeds: numpy PCG64 with seed = 1000 * seed_base + purpose (seed_base is a
  fixed small integer per workload, below), purpose in
  {0 mechanism, 1 initial state, 2 forcing, 3 set sizes, 4 MLP init, 5 split}.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

R_GAS = 8.314462618        # J/(mol K)
R_CAL = 1.98720425864083   # cal/(mol K)

_HERE = os.path.dirname(os.path.abspath(__file__))
SCALES_PATH = os.path.join(_HERE, "rate_scales.json")


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    seed_base: int              # seeds are 1000 * seed_base + purpose
    n_species: int
    n_reactions: int
    n_elements: int
    n_max: int
    grid: tuple | None          # (nx, ny, nz) for field workloads, None for independent cells
    n_cells: int
    H: float                    # slow step [s]
    n_sub: int                  # RK4 substeps per fast stage
    n_slow_steps: int
    mech_of: str                # workload whose mechanism (seed) is used
    note: str = ""


# workload names: cell layout and size, then species count
SMALL = "cells512_s9"           # 512 independent cells, 9 species / 21 reactions
FIELD64 = "field64_s21"         # 64^3 periodic fields, 21 species / 84 reactions
SETS1000 = "sets1000_s21"       # 1000 uneven reactor sets, 21 species / 84 reactions
LARGE128 = "field128_s53"       # 128^3 periodic fields, 53 species / 325 reactions
FIELD128 = "field128_s21"       # 128^3 periodic fields, 21 species / 84 reactions

WORKLOADS = {
    SMALL: Workload(SMALL, 0, 9, 21, 2, 3, None, 512, 1e-6, 20, 1, SMALL,
                    "parity: 512 independent cells, Gaussian slow tendencies"),
    FIELD64: Workload(FIELD64, 1, 21, 84, 3, 2, (64, 64, 64), 64 ** 3, 1e-7, 50, 10, FIELD64,
                      "plain throughput: 64^3 periodic fields, advection-diffusion slow side"),
    SETS1000: Workload(SETS1000, 2, 21, 84, 3, 2, None, 0, 1e-7, 0, 1, FIELD64,
                       "batched uneven reactor sets, adaptive Zonneveld 4(3)"),
    LARGE128: Workload(LARGE128, 3, 53, 325, 3, 3, (128, 128, 128), 128 ** 3, 5e-8, 100, 1,
                       LARGE128, "large mechanism: 128^3 fields"),
    FIELD128: Workload(FIELD128, 4, 21, 84, 3, 2, (128, 128, 128), 128 ** 3, 1e-7, 50, 1, FIELD64,
                       "surrogate: 128^3 fields, mechanism of the 64^3 workload"),
}


def rng_for(workload: str, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * WORKLOADS[workload].seed_base + purpose))

# Slow-side constants for the field workloads (u in m/s, D in m^2/s, dx in m).
ADVDIFF = dict(u=(10.0, 10.0, 10.0), D=1e-5, dx=1e-4)


# ----------------------------------------------------------------------------
# MRI-GARK coupling tables
# ----------------------------------------------------------------------------
@dataclass
class Table:
    name: str
    c: np.ndarray               # [s]
    gamma: np.ndarray           # [n_gamma][s][s]

    @property
    def s(self):
        return self.c.shape[0]

    @property
    def n_gamma(self):
        return self.gamma.shape[0]


def table_mis_kw3() -> Table:
    """Knoth-Wolke 3rd-order explicit ERK written as an MIS / MRI-GARK table.

    ERK: A = [[0,0,0],[1/3,0,0],[-3/16,15/16,0]], b = (1/6, 3/10, 8/15);
    coupling rows Gamma_ij = a_ij - a_(i-1)j with a_(s+1)j = b_j.
    """
    c = np.array([0.0, 1.0 / 3.0, 3.0 / 4.0, 1.0])
    g = np.zeros((1, 4, 4))
    g[0, 1, 0] = 1.0 / 3.0
    g[0, 2, 0] = -25.0 / 48.0
    g[0, 2, 1] = 15.0 / 16.0
    g[0, 3, 0] = 17.0 / 48.0
    g[0, 3, 1] = -51.0 / 80.0
    g[0, 3, 2] = 8.0 / 15.0
    return Table("MIS-KW3", c, g)


def table_erk33a() -> Table:
    """3rd-order explicit MRI-GARK table with a linear-in-time forcing (n_gamma = 2)."""
    c = np.array([0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0])
    g = np.zeros((2, 4, 4))
    g[0, 1, 0] = 1.0 / 3.0
    g[0, 2, 0] = -1.0 / 3.0
    g[0, 2, 1] = 2.0 / 3.0
    g[0, 3, 1] = -2.0 / 3.0
    g[0, 3, 2] = 1.0
    g[1, 3, 0] = 0.5
    g[1, 3, 2] = -0.5
    return Table("MRI-GARK-ERK33a", c, g)


# 4th-order explicit MRI-GARK table with a linear-in-time forcing (Sandu's
# ERK45a, from the MRI-GARK family the paper builds on, Sec. 2.1): six stages at
# c = (0, 1/5, 2/5, 3/5, 4/5, 1); rows of Gamma^(0) and Gamma^(1) as exact
# rationals (numerator, denominator), column j = 0, 1, ...
ERK45A_GAMMA = (
    (((1, 5),),
     ((-53, 16), (281, 80)),
     ((-36562993, 71394880), (34903117, 17848720), (-88770499, 71394880)),
     ((-7631593, 71394880), (-166232021, 35697440), (6068517, 1519040), (8644289, 8924360)),
     ((277061, 303808), (-209323, 1139280), (-1360217, 1139280), (-148789, 56964),
      (147889, 45120))),
    (((0, 1),),
     ((503, 80), (-503, 80)),
     ((-1365537, 35697440), (4963773, 7139488), (-1465833, 2231090)),
     ((66974357, 35697440), (21445367, 7139488), (-3, 1), (-8388609, 4462180)),
     ((-18227, 7520), (2, 1), (1, 1), (5, 1), (-41933, 7520))),
)


def table_erk45a() -> Table:
    """4th-order explicit MRI-GARK table (n_gamma = 2, s = 6), ERK45A_GAMMA."""
    c = np.arange(6) / 5.0
    g = np.zeros((2, 6, 6))
    for k, rows in enumerate(ERK45A_GAMMA):
        for i, row in enumerate(rows, start=1):
            for j, (num, den) in enumerate(row):
                g[k, i, j] = num / den
    return Table("MRI-GARK-ERK45a", c, g)


@dataclass
class ImexTable:
    """Solve-decoupled IMEX-MRI-GARK coupling table (f^S = f^I + f^E).

    gamma[k][i][j] multiplies the implicit slow evaluation f^I(T_j, Y_j) and
    omega[k][i][j] the explicit one f^E(T_j, Y_j) in the k-th forcing term of
    stage i; gamma may be nonzero on its diagonal only on stages with
    c_i = c_(i-1) (the implicit, solve-decoupled stages)."""
    name: str
    c: np.ndarray               # [s]
    gamma: np.ndarray           # [n_gamma][s][s]
    omega: np.ndarray           # [n_gamma][s][s]

    @property
    def s(self):
        return self.c.shape[0]

    @property
    def n_gamma(self):
        return self.gamma.shape[0]


def table_imex_trap2() -> ImexTable:
    """2nd-order solve-decoupled IMEX-MRI-GARK table, s = 3, c = (0, 1, 1).

    Stage 2 integrates the fast IVP over the whole step forced by
    f^I(y_n) + f^E(y_n); stage 3 is the solve-decoupled implicit stage
    Y_3 = Y_2 + (H/2)(f^I(Y_3) - f^I(Y_1)) + (H/2)(f^E(Y_2) - f^E(Y_1)).
    With f^F = 0 this is the trapezoidal rule for f^I paired with Heun's
    method for f^E; with f^S = 0 the exact fast flow."""
    c = np.array([0.0, 1.0, 1.0])
    g = np.zeros((1, 3, 3))
    w = np.zeros((1, 3, 3))
    g[0, 1, 0] = 1.0
    g[0, 2, 0] = -0.5
    g[0, 2, 2] = 0.5
    w[0, 1, 0] = 1.0
    w[0, 2, 0] = -0.5
    w[0, 2, 1] = 0.5
    return ImexTable("IMEX-MRI-GARK-trap2", c, g, w)


def table_imex_mri3() -> ImexTable:
    """3rd-order solve-decoupled IMEX-MRI-GARK table, s = 7,
    c = (0, 1/3, 1/3, 2/3, 2/3, 1, 1): fast stages 2, 4, 6 of length H/3 with
    forcing linear in time, implicit stages 3, 5, 7 (dc = 0), y_(n+1) = Y_7.

    Derived here (derive_imex3_table.py) from the order-3 conditions of one
    step on three-way split quadratic vector fields against the exact flow,
    exact row sums (a constant slow tendency is integrated exactly) and an
    L-stable implicit part: with f^F = f^E = 0 the step is R(z) y_n with
    R = (1 + 0.5370 z + 0.1050 z^2) / (1 - 0.4630 z + 0.0681 z^2 - 0.0032 z^3),
    |R| <= 1 on the negative real axis and R(-inf) = 0.  The coefficients are
    FP64 values of a least-squares solution (order residuals about 1e-13)."""
    c = np.array([0.0, 1.0 / 3.0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 1.0, 1.0])
    g = np.zeros((2, 7, 7))
    w = np.zeros((2, 7, 7))
    g[0, 1, :1] = [0.3333333333333333]
    g[0, 2, :3] = [-0.14055348783455268, -0.08064985465503603, 0.22120334248958873]
    g[0, 3, :3] = [0.032213781813120144, 0.0015626135167343203, 0.2995569380034795]
    g[0, 4, :5] = [-0.619910360142106, 0.017227884821738967, 0.5851657760422352, -0.09702906068750315, 0.11454575996563497]
    g[0, 5, :5] = [0.21589011306261846, -0.08814942074251945, 0.06456399842107294, 0.07104135732634824, 0.06998728526581233]
    g[0, 6, :7] = [0.09710366871062757, 0.44053161781275346, -0.5815798475730799, -0.3142303216519329, 0.013992830250077448, 0.21690649560912834, 0.12727555684242597]
    g[1, 3, :3] = [-0.08683135001680223, -0.16789024616451798, 0.2547215961813189]
    g[1, 5, :5] = [0.06231314722761247, 0.21120795253535973, 0.008186915883229423, -0.14401739964512705, -0.13769061600107288]
    w[0, 1, :1] = [0.3333333333333333]
    w[0, 2, :2] = [-0.5400393337274775, 0.5400393337274775]
    w[0, 3, :3] = [0.1125779016953933, -0.007602694356648855, 0.2283581259945884]
    w[0, 4, :4] = [-0.22349883540104018, 0.14022454333535686, 0.6067439785945805, -0.5234696865288972]
    w[0, 5, :5] = [0.10237739523931555, -0.24906115031496037, 0.15697749920835516, -0.0674812442659541, 0.39052083346657673]
    w[0, 6, :6] = [0.15678040875694046, -0.2203952841190962, -0.23626446369293067, 0.14354728916280882, -0.23275118974956494, 0.38908323964184255]
    w[1, 3, :3] = [-0.2548569527854706, -0.021027114350733775, 0.2758840671362053]
    w[1, 5, :5] = [0.0936287337088565, -0.041147165330545056, 0.20274987364268302, -0.22879544909149913, -0.02643599292949447]
    return ImexTable("IMEX-MRI-GARK3 (derived)", c, g, w)


# The 64^3 fields with a diffusion coefficient raised so that the diffusion
# number H D / dx^2 is 1 at H = 1e-7 s: beyond the stability limit of the
# explicit slow tables (about 0.2 in 3-D for a 3rd-order explicit method), the
# regime in which the diffusion is taken implicitly.
ADVDIFF_STIFF = dict(u=(10.0, 10.0, 10.0), D=0.1, dx=1e-4)
# RK4 substeps of the one fast stage per step of table_imex_trap2 (it spans the
# whole step): H / 120 is the largest fast step of the explicit 64^3 workload
# (MIS-KW3's longest stage, 5H/12, over 50 substeps).
IMEX_N_SUB = 120
# RK4 substeps of each of table_imex_mri3's three fast stages (H/3 each): the
# same fast step H / 120.
IMEX3_N_SUB = 40


def table_zero_forcing(c) -> Table:
    """Coupling table with Gamma = 0 (pure fast integration over the stage grid)."""
    c = np.asarray(c, dtype=np.float64)
    return Table("zero-forcing", c, np.zeros((1, c.size, c.size)))


# ----------------------------------------------------------------------------
# Mechanism
# ----------------------------------------------------------------------------
@dataclass
class Mechanism:
    n_species: int
    n_reactions: int
    reactants: np.ndarray       # int32 [R][2]
    products: np.ndarray        # int32 [R][2]
    lnA: np.ndarray             # ln(s * A), A in cm^3 mol^-1 s^-1
    beta: np.ndarray
    theta: np.ndarray           # Ea / R_cal  [K]
    g_a: np.ndarray             # J/mol
    g_b: np.ndarray             # J/mol/K
    W: np.ndarray               # kg/mol
    cv: np.ndarray              # J/kg/K
    composition: np.ndarray     # int [S][E]
    rho: float = 1.0            # kg/m^3
    T_ref: float = 298.15
    rate_scale: float = 1.0
    meta: dict = field(default_factory=dict)

    def with_scale(self, s: float) -> "Mechanism":
        """Copy with the rate scale replaced (lnA is stored with s folded in)."""
        base = self.lnA - math.log(self.rate_scale)
        m = Mechanism(**{**self.__dict__})
        m.lnA = base + math.log(s)
        m.rate_scale = s
        return m


def _lattice_species(E: int, n_max: int, S: int, rng) -> np.ndarray:
    pts = [p for p in itertools.product(range(n_max + 1), repeat=E) if any(p)]
    pts = np.array(pts, dtype=np.int64)
    centre = np.full(E, n_max / 2.0)
    d = np.linalg.norm(pts - centre, axis=1)
    tie = rng.random(len(pts))
    order = np.lexsort((tie, d))
    if S > len(pts):
        raise ValueError("lattice too small for the requested species count")
    return pts[np.sort(order[:S])]


def _balanced_reactions(comp: np.ndarray):
    S = comp.shape[0]
    by_sum = {}
    for a in range(S):
        for b in range(a, S):
            key = tuple(comp[a] + comp[b])
            by_sum.setdefault(key, []).append((a, b))
    cands = []
    for pairs in by_sum.values():
        for i in range(len(pairs)):
            for j in range(i + 1, len(pairs)):
                l, r = pairs[i], pairs[j]
                if set(l) & set(r):
                    continue
                cands.append((l, r))
    return cands


def make_mechanism(workload: str, with_scale: bool = True) -> Mechanism:
    mc = WORKLOADS[workload].mech_of
    base = WORKLOADS[mc]
    rng = rng_for(mc, 0)
    S, R, E = base.n_species, base.n_reactions, base.n_elements
    comp = _lattice_species(E, base.n_max, S, rng)
    # atomic masses: uniform draw, scaled so that max W = 50 g/mol; redraw if min W < 2
    for _ in range(1000):
        m = rng.uniform(1.0, 16.0, size=E)
        W_g = comp @ m
        W_g = W_g * (50.0 / W_g.max())
        if W_g.min() >= 2.0:
            break
    else:
        raise RuntimeError("could not draw atomic masses")
    m = m * (50.0 / (comp @ m).max())
    W_g = comp @ m
    cands = _balanced_reactions(comp)
    if len(cands) < R:
        raise RuntimeError(f"only {len(cands)} balanced reactions for R={R}")
    pick = rng.choice(len(cands), size=R, replace=False)
    reac = np.array([cands[i][0] for i in pick], dtype=np.int32)
    prod = np.array([cands[i][1] for i in pick], dtype=np.int32)
    A = 10.0 ** rng.uniform(8.0, 14.0, size=R)
    beta = rng.uniform(-1.0, 1.0, size=R)
    Ea = rng.uniform(0.0, 30.0e3, size=R)          # cal/mol
    g_a = rng.uniform(-3.0e5, 3.0e5, size=S)
    g_b = rng.uniform(-200.0, 50.0, size=S)
    cv = rng.uniform(500.0, 3000.0, size=S)
    # orientation: Delta G(1500 K) <= 0, i.e. K_c >= 1 at 1500 K
    g1500 = g_a + g_b * 1500.0
    dG = g1500[prod].sum(1) - g1500[reac].sum(1)
    swap = dG > 0
    reac2 = np.where(swap[:, None], prod, reac)
    prod2 = np.where(swap[:, None], reac, prod)
    mech = Mechanism(
        n_species=S, n_reactions=R,
        reactants=np.ascontiguousarray(reac2, dtype=np.int32),
        products=np.ascontiguousarray(prod2, dtype=np.int32),
        lnA=np.log(A), beta=beta, theta=Ea / R_CAL,
        g_a=g_a, g_b=g_b, W=W_g * 1e-3, cv=cv,
        composition=comp.astype(np.int32), rho=1.0, T_ref=298.15, rate_scale=1.0,
        meta=dict(workload=mc, seed=1000 * base.seed_base + 0, atomic_masses_g=m.tolist(),
                  n_candidates=len(cands)),
    )
    if with_scale:
        s = load_rate_scale(mc)
        if s is not None:
            mech = mech.with_scale(s)
    return mech


def load_rate_scale(mech_of: str):
    if not os.path.exists(SCALES_PATH):
        return None
    with open(SCALES_PATH) as f:
        d = json.load(f)
    v = d.get("scales", {}).get(mech_of)
    return None if v is None else float(v["s"])


def longest_substep(workload: str, table: Table | None = None) -> float:
    cfg = WORKLOADS[workload]
    table = table or table_mis_kw3()
    dc = np.diff(table.c)
    return float(dc.max() * cfg.H / cfg.n_sub)


# ----------------------------------------------------------------------------
# Initial states (SoA: y[comp][ld], comp 0..S-1 = Y_k, comp S = T)
# ----------------------------------------------------------------------------
def pad_ld(n: int) -> int:
    return ((n + 63) // 64) * 64


def independent_cells(n_cells: int, S: int, rng, ld: int | None = None) -> np.ndarray:
    """T ~ U[1000, 2000] K, Y ~ Dirichlet(1), renormalized in FP64."""
    ld = ld or pad_ld(n_cells)
    y = np.zeros((S + 1, ld))
    Y = rng.dirichlet(np.ones(S), size=n_cells)
    Y = Y / Y.sum(axis=1, keepdims=True)
    y[:S, :n_cells] = Y.T
    y[S, :n_cells] = rng.uniform(1000.0, 2000.0, size=n_cells)
    if ld > n_cells:
        y[:S, n_cells:] = 1.0 / S
        y[S, n_cells:] = 1500.0
    return y


def _smooth_periodic_field(grid, rng, n_modes: int = 8, kmax: int = 4) -> np.ndarray:
    nx, ny, nz = grid
    x = np.arange(nx)[None, None, :] / nx
    yy = np.arange(ny)[None, :, None] / ny
    z = np.arange(nz)[:, None, None] / nz
    f = np.zeros((nz, ny, nx))
    for _ in range(n_modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if 0 < np.linalg.norm(k) <= kmax:
                break
        amp = rng.normal()
        ph = rng.uniform(0.0, 2.0 * np.pi)
        f += amp * np.cos(2.0 * np.pi * (k[0] * x + k[1] * yy + k[2] * z) + ph)
    f = f / np.abs(f).max()
    return f.reshape(-1)


def field_state(workload: str, grid=None) -> np.ndarray:
    """Smooth random periodic fields: Y = softmax of S fields, T = 1500 + 500 f."""
    cfg = WORKLOADS[workload]
    grid = grid or cfg.grid
    S = cfg.n_species
    rng = rng_for(workload, 1)
    N = int(np.prod(grid))
    ld = pad_ld(N)
    logits = np.stack([2.0 * _smooth_periodic_field(grid, rng) for _ in range(S)])
    logits -= logits.max(axis=0, keepdims=True)
    e = np.exp(logits)
    Y = e / e.sum(axis=0, keepdims=True)
    T = 1500.0 + 500.0 * _smooth_periodic_field(grid, rng)
    y = np.zeros((S + 1, ld))
    y[:S, :N] = Y
    y[S, :N] = T
    return y


def initial_state(workload: str) -> np.ndarray:
    cfg = WORKLOADS[workload]
    if cfg.grid is None:
        return independent_cells(cfg.n_cells, cfg.n_species, rng_for(workload, 1))
    return field_state(workload)


def gaussian_xi(workload: str, n_stages: int, n_comp: int, ld: int) -> np.ndarray:
    """Standard normal draws xi[j][comp][cell] for the 512-cell workload's slow
    tendencies.

    The tendencies are r_j = 1e-3 * |f^F(y0)| * xi_j; the magnitude |f^F(y0)|
    is evaluated by whichever side consumes these draws.
    """
    return rng_for(workload, 2).standard_normal((n_stages, n_comp, ld))


# ----------------------------------------------------------------------------
# Batched uneven reactor sets
# ----------------------------------------------------------------------------
def set_sizes(n_sets: int = 1000, lo: int = 64, hi: int = 65536,
              workload: str = SETS1000) -> np.ndarray:
    rng = rng_for(workload, 3)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_sets)
    return np.floor(np.exp(u)).astype(np.int64).clip(lo, hi)


def set_offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return off


def mechanism_arrays(m: Mechanism) -> dict:
    """Flat dictionary of contiguous arrays, in the boundary's units."""
    return dict(
        S=m.n_species, R=m.n_reactions,
        reactants=np.ascontiguousarray(m.reactants, dtype=np.int32),
        products=np.ascontiguousarray(m.products, dtype=np.int32),
        lnA=np.ascontiguousarray(m.lnA, dtype=np.float64),
        beta=np.ascontiguousarray(m.beta, dtype=np.float64),
        theta=np.ascontiguousarray(m.theta, dtype=np.float64),
        g_a=np.ascontiguousarray(m.g_a, dtype=np.float64),
        g_b=np.ascontiguousarray(m.g_b, dtype=np.float64),
        W=np.ascontiguousarray(m.W, dtype=np.float64),
        cv=np.ascontiguousarray(m.cv, dtype=np.float64),
        rho=float(m.rho), T_ref=float(m.T_ref),
    )


def batch_workload(n_sets: int = 1000, workload: str = SETS1000, divergent: bool = False):
    """Uneven reactor sets: sizes log-uniform in [64, 65536], every cell drawn
    like the independent-cell workload (T ~ U[1000, 2000] K, Y ~ Dirichlet(1)),
    and one fast stage per set whose length cycles through the three stage
    lengths dc_i H of the MIS-KW3 table (H = 1e-7 s).  No slow tendencies are
    stated for this workload: the stage is unforced (n_poly = 0).

    divergent: the same sets and cells with per-set stage lengths log-uniform
    in [1e-8, 1e-6] s (the stages of slow steps an adaptive slow controller
    takes up to about 2.4e-6 s), which spreads the adaptive fast method's
    accepted steps over 10 to 2,000 per cell."""
    cfg = WORKLOADS[workload]
    sizes = set_sizes(n_sets, workload=workload)
    off = set_offsets(sizes)
    y = independent_cells(int(off[-1]), WORKLOADS[cfg.mech_of].n_species, rng_for(workload, 1))
    if divergent:
        L = np.exp(rng_for(workload, 2).uniform(math.log(1e-8), math.log(1e-6), n_sets))
    else:
        dc = np.diff(table_mis_kw3().c)
        L = np.array([dc[i % dc.size] * cfg.H for i in range(n_sets)])
    return sizes, off, y, L
