"""One dispatch of each hot kernel at its benchmark size, for hardware counter
collection (run under `rocprofv3 --pmc ...`):

  1. mri_spec_main, RK4 with 50 substeps, 64^3 cells, 21 species / 84 reactions
     (the first fast stage of the 64^3 workload);
  2. mri_spec_main, RK4 with 100 substeps, 128^3 cells, 53 species / 325
     reactions (the first fast stage of the large-mechanism workload);
  3. mri_spec_main, the batched work queue over the 1000 uneven reactor sets
     (Zonneveld 4(3), with the tile and tiling variant the autotuner picks; a
     second plan takes them from the tuning cache, so that no tuning dispatches
     precede the measured one);
  4. k_infer, the fused inference over the 128^3 cells (random weights: the
     instruction stream does not depend on them);
  5. two IMEX-MRI-GARK steps (3rd-order table) of the 64^3 stiff-diffusion
     workload (its three fast stages per step and the conjugate-gradient
     kernels of the three implicit diffusion solves).

With --block B the batched plan is fixed to B threads per block instead (the
register / LDS tiling then follows the MRI_SPEC_WPE, MRI_SPEC_EXP_TABLE and
MRI_SPEC_GROUP environment knobs, which give the same code as the autotuner's
variants of those settings), so that every candidate the autotuner may pick
can be counted in a process of its own.

Each kernel is run once untimed first (run-time compilation, module load), then
once more; the second dispatch is the one to read.  Prints one JSON line with
the work of each measured dispatch (cells, substeps, attempted steps) and the
machine-code hash of each specialized kernel.

    python -m paper_2211_03293_amd.profile_kernels [--only rk4|large|batch|infer|imex]
                                                   [--block 64|128|256]
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["rk4", "large", "batch", "infer", "imex"], default=None)
    ap.add_argument("--block", type=int, choices=[64, 128, 256], default=0)
    args = ap.parse_args()
    import torch

    from . import inputs as I
    from . import mri

    torch.cuda.set_device(0)
    out = {}
    tb = I.table_mis_kw3()

    def stage(workload, key):
        cfg = I.WORKLOADS[workload]
        mech = I.make_mechanism(workload)
        m, t = mri.Mech(mech), mri.Table(tb)
        m.specialize(128, load=True)
        y = torch.as_tensor(I.initial_state(workload), device="cuda")
        n, ld = y.shape
        N = cfg.n_cells
        F = torch.empty((1, n, ld), dtype=torch.float64, device="cuda")
        rho = torch.empty((1, n, ld), dtype=torch.float64, device="cuda")
        params = mri.advdiff_params(cfg.grid, n)
        sp = torch.cuda.current_stream().cuda_stream
        rc = mri.lib.mri_advdiff_slow_rhs(0.0, y.data_ptr(), F[0].data_ptr(), N, ld,
                                          mri.C.cast(mri.C.pointer(params), mri.C.c_void_p).value,
                                          sp)
        assert rc == 0
        mri.mri_forcing_assemble(t, 1, n, ld, F, rho)
        L = float((tb.c[1] - tb.c[0]) * cfg.H)
        yo = torch.empty_like(y)
        for _ in range(2):
            mri.mri_fast_stage(m, mri.fast_opts(n_sub=cfg.n_sub), N, ld, y, yo, 1, rho, L)
        torch.cuda.synchronize()
        out[key] = dict(kernel="mri_spec_main", cells=N, n_sub=cfg.n_sub,
                        cell_substeps=N * cfg.n_sub, species=mech.n_species,
                        reactions=mech.n_reactions,
                        code_hash=m.code_hash(mri.FAST_RK4, 1, 128))

    if args.only in (None, "rk4"):
        stage(I.FIELD64, "rk4_64cube_21sp")
    if args.only in (None, "large"):
        stage(I.LARGE128, "rk4_128cube_53sp")
    if args.only in (None, "batch"):
        sizes, off, y_host, Ls = I.batch_workload()
        mech = I.make_mechanism(I.SETS1000)
        m = mri.Mech(mech)
        n, ld = y_host.shape
        y = torch.as_tensor(y_host, device="cuda")
        yo = torch.empty_like(y)
        # the choice the autotuner makes, then a plan that takes it from the
        # tuning cache (no tuning dispatches before the measured one)
        zv = dict(method=mri.FAST_ZONNEVELD43, rtol=1e-8, atol_Y=1e-8, atol_T=1e-5,
                  max_steps=2000)
        if args.block:
            plan = mri.BatchPlan(m, mri.fast_opts(block_size=args.block, **zv), off)
        else:
            tuner = mri.BatchPlan(m, mri.fast_opts(**zv), off)
            tuner.run(y, yo, ld, 0, None, Ls)
            plan = mri.BatchPlan(m, mri.fast_opts(**zv), off)
        for _ in range(2):
            plan.run(y, yo, ld, 0, None, Ls)
        torch.cuda.synchronize()
        useful, issued = plan.lane_stats()
        out["batch_1000_sets"] = dict(kernel="mri_spec_main", cells=int(off[-1]),
                                      attempted_steps=int(useful), issued_lane_steps=int(issued),
                                      tile=list(plan.tile()), code_hash=plan.code_hash(0),
                                      tuner=plan.tune_log())
    if args.only in (None, "infer"):
        cfg = I.WORKLOADS[I.FIELD128]
        y = torch.as_tensor(I.initial_state(I.FIELD128), device="cuda")
        n, ld = y.shape
        N = cfg.n_cells
        rho = torch.zeros((1, n, ld), dtype=torch.float64, device="cuda")
        rng = np.random.Generator(np.random.PCG64(1))
        widths = [89, 256, 256, 256, 22]
        params = np.concatenate([np.concatenate([
            (rng.normal(size=(widths[l + 1], widths[l])) / np.sqrt(widths[l])).ravel(),
            np.zeros(widths[l + 1])]) for l in range(4)]).astype(np.float32)
        stats = np.zeros(mri.MLP_STATS)
        stats[89:178] = 1.0
        stats[178 + 22:] = 1e-6
        sg = mri.Surrogate(widths, params, stats)
        yo = torch.empty_like(y)
        for _ in range(2):
            sg.infer(N, ld, y, yo, 1, rho, 3.3e-8)
        torch.cuda.synchronize()
        out["infer_128cube"] = dict(kernel="k_infer<false>", cells=N)
    if args.only in (None, "imex"):
        cfg = I.WORKLOADS[I.FIELD64]
        P = I.ADVDIFF_STIFF
        mech = I.make_mechanism(I.FIELD64)
        y = torch.as_tensor(I.initial_state(I.FIELD64), device="cuda")
        n, ld = y.shape
        N = cfg.n_cells
        m, t = mri.Mech(mech), mri.ImexTable(I.table_imex_mri3())
        params = mri.advdiff_params(cfg.grid, n, u=P["u"], D=P["D"], dx=P["dx"])
        cws = torch.empty(mri.diffusion_solve_workspace_bytes(params, ld), dtype=torch.uint8,
                          device="cuda")
        ctx = mri.imex_advdiff(params, cws, cg_rtol=1e-13)
        ws = torch.empty(mri.mri_imex_workspace_bytes(m, t, N, ld), dtype=torch.uint8,
                         device="cuda")
        for k in range(2):
            mri.mri_imex_slow_step(m, t, mri.fast_opts(n_sub=I.IMEX3_N_SUB), ctx, k * cfg.H,
                                   cfg.H, N, ld, y, ws)
        torch.cuda.synchronize()
        out["imex_64cube"] = dict(kernel="k_cg_*", cells=N, cg_iterations=ctx.cg_iters,
                                  fast_code_hash=m.code_hash(mri.FAST_RK4, 2, 128))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
