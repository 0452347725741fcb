"""MRI-P(k) convergence and efficiency study on the synthetic reacting-flow
problem, run on the GPU through libmri (the analogue of the paper's Table 1
and Fig. 4, Sec. 5.1: a 3rd-order explicit MRI slow method paired with fast
explicit RK methods of order P, k fast steps per stage).

Problem: the 64^3 periodic fields, 21 species / 84 reactions, advection-
diffusion slow side, integrated to t = 1e-6 s.  For every fast method
(Heun P = 2, Bogacki-Shampine P = 3, classic RK4 P = 4, which is also the
propagated solution of Zonneveld's pair, Cash-Karp P = 5) and slow step H the
errors are taken over all cells against a reference run with H/8 of the finest
H and RK4 with 4 max(k) substeps: the max absolute mass-fraction error (the
paper reports max-norm errors, Table 1), the max relative temperature error
and the max relative state error with the mass-fraction floor 1e-8.  --k takes
one substep count for every method or one per method (Sec. 5.1 found
MRI-2(8), MRI-3(4), MRI-4(8) and MRI-5(4) the most efficient pairings).

--table erk45a replaces the 3rd-order MIS-KW3 slow table by the 4th-order
explicit MRI-GARK table (Sec. 2.1: explicit MRI-GARK methods reach order 4).
--adaptive TOL ... adds runs whose slow step is chosen by step doubling
(mri_adaptive_run, rtol = TOL, atol_Y = 1e-3 TOL, atol_T = 1e-3 TOL K) from
H0 = the largest H, each fast method keeping the fast step of H0.

    python -m paper_2211_03293_amd.study_mri_pk [--cells-per-side 32] [--k 16]
    python -m paper_2211_03293_amd.study_mri_pk --k 8 4 8 4 --H 2.5e-8 1.25e-8 6.25e-9
    python -m paper_2211_03293_amd.study_mri_pk --table erk45a
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as I
from . import mri

T_END = 1e-6
METHODS = (("Heun", 2), ("Bogacki-Shampine", 3), ("RK4", 4), ("Cash-Karp", 5))


def _fields(n_side):
    """The 64^3 workload's initial fields on an n_side^3 periodic grid."""
    grid = (n_side, n_side, n_side)
    return I.field_state(I.FIELD64, grid), grid


def run(torch, m, t, y_host, grid, method, k, H):
    n, ld = y_host.shape
    N = int(np.prod(grid))
    y = torch.as_tensor(y_host, device="cuda")
    ws = torch.empty(mri.mri_workspace_bytes(m, t, N, ld) // 8, dtype=torch.float64,
                     device="cuda")
    status = torch.zeros(ld, dtype=torch.int32, device="cuda")
    params = mri.advdiff_params(grid, n)
    opts = mri.fast_opts(method=method, n_sub=k)
    n_steps = int(round(T_END / H))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(n_steps):
        mri.mri_slow_step(m, t, opts, mri.ADVDIFF_RHS, params, s * H, H, N, ld, y, ws, status)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bad = mri.mri_status_count(status, N)
    return y.cpu().numpy()[:, :N], dt, bad


def run_adaptive(torch, m, t, y_host, grid, method, k, H0, tol, order):
    n, ld = y_host.shape
    N = int(np.prod(grid))
    y = torch.as_tensor(y_host, device="cuda")
    ws = torch.empty(mri.mri_adaptive_workspace_bytes(m, t, N, ld) // 8 + 1,
                     dtype=torch.float64, device="cuda")
    status = torch.zeros(ld, dtype=torch.int32, device="cuda")
    aopts = mri.adapt_opts(tol, 1e-3 * tol, 1e-3 * tol, H0, order)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = mri.mri_adaptive_run(m, t, mri.fast_opts(method=method, n_sub=k), aopts,
                              mri.ADVDIFF_RHS, mri.advdiff_params(grid, n), 0.0, T_END, N, ld, y,
                              ws, status)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return y.cpu().numpy()[:, :N], dt, mri.mri_status_count(status, N), st


def errors(y, ref, n_species):
    """(max absolute mass-fraction error, max relative temperature error, max
    relative state error with the mass-fraction floor 1e-8) over all cells."""
    ey = float(np.abs(y[:n_species] - ref[:n_species]).max())
    eT = float((np.abs(y[n_species] - ref[n_species]) / np.abs(ref[n_species])).max())
    floor = np.zeros((y.shape[0], 1))
    floor[:n_species] = 1e-8
    er = float((np.abs(y - ref) / np.maximum(np.abs(ref), floor)).max())
    return ey, eT, er


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells-per-side", type=int, default=32)
    ap.add_argument("--k", type=int, nargs="+", default=[16],
                    help="fast substeps per stage: one value, or one per method (P = 2..5)")
    ap.add_argument("--H", type=float, nargs="+", default=[1e-7, 5e-8, 2.5e-8, 1.25e-8])
    ap.add_argument("--table", choices=("kw3", "erk45a"), default="kw3",
                    help="slow table: MIS-KW3 (order 3) or MRI-GARK-ERK45a (order 4)")
    ap.add_argument("--adaptive", type=float, nargs="*", default=[],
                    help="tolerances of adaptive slow-step runs")
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the study runs on a GPU"
    torch.cuda.set_device(0)
    mech = I.make_mechanism(I.FIELD64)
    m = mri.Mech(mech)
    if len(args.k) not in (1, len(METHODS)):
        ap.error(f"--k takes 1 or {len(METHODS)} values")
    ks = args.k * len(METHODS) if len(args.k) == 1 else args.k
    tb = I.table_mis_kw3() if args.table == "kw3" else I.table_erk45a()
    t = mri.Table(tb)
    # compile every kernel ahead of the timed runs (forcing terms = table's n_gamma)
    for meth in (mri.FAST_HEUN, mri.FAST_BS3, mri.FAST_RK4, mri.FAST_CK5):
        m.specialize(128, load=True, method=meth, n_poly=tb.n_gamma)
    y0, grid = _fields(args.cells_per_side)
    H_ref = min(args.H) / 8
    k_ref = 4 * max(ks)
    ref, t_ref, bad = run(torch, m, t, y0, grid, mri.FAST_RK4, k_ref, H_ref)
    print(f"# reference: H = {H_ref:.3e}, RK4 {k_ref} substeps/stage, {t_ref:.2f} s, "
          f"flagged {bad}", flush=True)
    rows = []
    fast = (mri.FAST_HEUN, mri.FAST_BS3, mri.FAST_RK4, mri.FAST_CK5)
    for (name, P), meth, k in zip(METHODS, fast, ks):
        prev = None
        for H in args.H:
            y, dt, bad = run(torch, m, t, y0, grid, meth, k, H)
            e = errors(y, ref, mech.n_species)
            rate = None if prev is None else [float(np.log2(a / b)) for a, b in zip(prev, e)]
            prev = e
            rows.append(dict(method=name, P=P, k=k, H=H, err_Y_abs=e[0], err_T_rel=e[1],
                             err_rel=e[2], rates=rate, seconds=dt, flagged=bad))
            print(f"MRI-{P}({k}) {name:17s} H = {H:.3e}: |dY| {e[0]:.3e}  dT/T {e[1]:.3e}  "
                  f"rel {e[2]:.3e}" + (" rates " + " ".join(f"{r:.2f}" for r in rate)
                                      if rate else "") + f"  {dt * 1e3:.1f} ms  flagged {bad}",
                  flush=True)
    order = 3 if args.table == "kw3" else 4
    for (name, P), meth, k in zip(METHODS, fast, ks):
        for tol in args.adaptive:
            y, dt, bad, st = run_adaptive(torch, m, t, y0, grid, meth, k, max(args.H), tol, order)
            e = errors(y, ref, mech.n_species)
            rows.append(dict(method=name, P=P, k=k, adaptive_tol=tol, err_Y_abs=e[0],
                             err_T_rel=e[1], err_rel=e[2], seconds=dt, flagged=bad, **st))
            print(f"MRI-{P}({k}) {name:17s} adaptive tol {tol:.0e}: |dY| {e[0]:.3e}  "
                  f"dT/T {e[1]:.3e}  {st['accepted']} accepted / {st['rejected']} rejected, "
                  f"last H {st['H_last']:.2e}  {dt * 1e3:.1f} ms  flagged {bad}", flush=True)
    print(json.dumps(dict(study=f"MRI-P(k) convergence, {tb.name} slow, 21 species / 84 "
                                f"reactions, {args.cells_per_side}^3 cells, t = {T_END}",
                          rows=rows)))
    return rows


if __name__ == "__main__":
    main()
    sys.exit(0)
