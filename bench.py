"""Benchmark: plain FP64 MRI fast-stage throughput on one MI355X.

Workload (one bench step = one explicit MRI-GARK slow step over the batch):
64^3 = 262,144 cells of smooth periodic synthetic fields, 21 species / 84
reversible reactions, MIS-KW3 coupling table (3 fast stages per slow step),
classic RK4 with 50 substeps per stage, H = 1e-7 s, advection-diffusion slow
RHS.  The default K = 10 steps is the workload's 10 slow steps.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: value = cell fast-stage solves per second (cell-stages/s),
plus the fast-stage kernel's roofline figures (kernel time from hipEvents around
every fast-stage launch inside the timed region) and the CPU oracle timed on a
bounded sample of the same workload.  Further legs, each in its own JSON object:
the 128^3 large mechanism (53 species / 325 reactions), the batched uneven
reactor sets (adaptive, persistent work queue) and the learned surrogate
(training on the GPU, then the gated stage against the plain FP64 stage).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-large] [--no-batch] [--no-surrogate]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell fast-stage solves/s: FP64 plain vs surrogate+fallback at 1e-4 rel err"
PEAK_FP64_TFLOPS = 78.6           # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
PEAK_BF16_TFLOPS = 2500.0         # MI355X dense BF16 MFMA
MLP_FLOPS = 2 * (89 * 256 + 256 * 256 + 256 * 256 + 256 * 22)   # one inference, 89 -> 22
# MFMA work the fused kernel executes per inference: the padded 96 -> 32 network;
# rocprofv3's SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512 per dispatch equals this times
# the cell count
MLP_FLOPS_EXECUTED = 2 * (96 * 256 + 256 * 256 + 256 * 256 + 256 * 32)
TRAIN_BATCH = 8192
F_EXP, F_LOG, F_DIV = 22, 22, 10  # flops charged per FP64 exp / log / divide


def flops_per_substep(S: int, R: int, n_poly: int = 1) -> int:
    """Algorithmic FP64 flops of one RK4 substep of one cell (FMA = 2).

    Per RHS: species S x (Z factor: fma + exp + 2 mul; den fma) = S (6 + F_exp);
    reactions R x (rate argument 2 fma + exp + 2 mul + 1 fma + 4 add) = R (12 + F_exp);
    energy S x 5 + 1; ln T, 1/T and the dT/dt divide.  Per stage and component:
    forcing (n_poly terms), accumulator fma, next-input fma; final update fma."""
    n = S + 1
    rhs = S * (6 + F_EXP) + R * (12 + F_EXP) + 5 * S + 1 + F_LOG + 2 * F_DIV + 1
    forcing = max(0, 2 * n_poly - 1)
    return 4 * rhs + 4 * n * (forcing + 4) + 2 * n


def flops_per_zv_attempt(S: int, R: int) -> int:
    """Algorithmic FP64 flops of one attempted Zonneveld 4(3) step of one cell
    (unforced): 5 RHS evaluations; per stage and component the solution, error
    and stage-5 accumulators and the next stage input (4 FMA); the WRMS error
    (scaling, weight, divide, square: 15 flops per component), the solution
    update (1 FMA per component) and the step-size factor (one pow, 44 flops)."""
    n = S + 1
    rhs = S * (6 + F_EXP) + R * (12 + F_EXP) + 5 * S + 1 + F_LOG + 2 * F_DIV + 1
    return 5 * rhs + 5 * n * 8 + 15 * n + 2 * n + 2 * F_EXP


def load_counters(workload: str, code_hash: str):
    """rocprofv3 counter figures per launch (HBM bytes, FP64 counter flops) for
    the kernel whose code object hashes to code_hash, or None when the compiled
    kernel changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "fast_stage_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_code_hash") != code_hash or d.get("workload") != workload:
        return None
    return d


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mech, y_field, rho, L_list, n_sub, n_sample=262144, n_sample_1core=8192):
    """The oracle as it stands, on n_sample cells of the same field, for the
    three fast stages of one slow step (forcing of the first stage); once with
    all the threads the job may use and once on one core (smaller sample)."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    orc = O.Oracle(mech)

    def run(n, nthreads):
        O.set_threads(nthreads)
        idx = np.linspace(0, y_field.shape[1] - 1, n).astype(np.int64)
        ys = np.ascontiguousarray(y_field[:, idx])
        rs = np.ascontiguousarray(rho[:, :, idx])
        t0 = time.perf_counter()
        for L in L_list:
            ys, _, _, _ = orc.fast_stage_soa(ys, rs, L, O.rk4_opts(n_sub))
        return time.perf_counter() - t0, O.num_threads()

    dt, used = run(n_sample, threads)
    dt1, _ = run(n_sample_1core, 1)
    cell_stages = n_sample * len(L_list)
    return dict(value=cell_stages / dt, unit="cell-stages/s", cores=used, kind="oracle",
                sample=f"{n_sample} evenly spaced cells of the 64^3 field, the 3 fast stages of "
                       f"one slow step (RK4, {n_sub} substeps/stage); {dt:.1f} s",
                one_core=dict(value=n_sample_1core * len(L_list) / dt1, unit="cell-stages/s",
                              sample=f"{n_sample_1core} cells, same stages; {dt1:.1f} s"),
                host=dict(cpu=_cpu_model(), nproc=os.cpu_count()))


def batch_leg(torch, mri, I, repeats=3):
    """Batched uneven reactor sets: 1000 sets, log-uniform sizes, adaptive
    Zonneveld 4(3) at tol 1e-8, one persistent work-queue launch per run."""
    sizes, off, y_host, Ls = I.batch_workload()
    mech = I.make_mechanism(I.SETS1000)
    m = mri.Mech(mech)
    opts = mri.fast_opts(method=mri.FAST_ZONNEVELD43, rtol=1e-8, atol_Y=1e-8, atol_T=1e-5,
                         max_steps=2000)
    plan = mri.BatchPlan(m, opts, off)
    n, ld = y_host.shape
    ntot = int(off[-1])
    y = torch.as_tensor(y_host, device="cuda")
    out = torch.empty_like(y)
    st = torch.zeros(ld, dtype=torch.int32, device="cuda")
    steps = torch.zeros(ld, dtype=torch.int32, device="cuda")
    plan.run(y, out, ld, 0, None, Ls, st, steps)          # tunes the tile, captures the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(repeats):
        plan.run(y, out, ld, 0, None, Ls, st, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / repeats
    useful, issued = plan.lane_stats()       # attempted lane-steps of the last run
    wg, nb = plan.tile()
    fpa = flops_per_zv_attempt(mech.n_species, mech.n_reactions)
    achieved = useful * fpa / (ms * 1e-3) / 1e12
    sv = steps[:ntot].cpu().numpy()
    n_bad = mri.mri_status_count(st, ntot, mri.CELL_NONFINITE | mri.CELL_MAXSTEPS | mri.CELL_TRANGE)
    return dict(workload="1000 reactor sets, sizes log-uniform in [64, 65536], 21 species / 84 "
                         "reactions, one unforced fast stage per set (L cycles through the "
                         "MIS-KW3 stage lengths, H = 1e-7 s), Zonneveld 4(3) tol 1e-8",
                cells=ntot, ms_per_run=round(ms, 3), value=round(ntot / (ms * 1e-3), 1),
                unit="cell-stages/s", accepted_steps=dict(min=int(sv.min()),
                                                          median=float(np.median(sv)),
                                                          max=int(sv.max())),
                lane_utilization=round(useful / max(issued, 1), 4), tile=dict(block=wg, blocks=nb),
                flagged_cells=n_bad, attempted_steps=int(useful),
                roofline=dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_TFLOPS,
                              unit="TFLOP/s", frac=round(achieved / PEAK_FP64_TFLOPS, 4),
                              traffic=None, kernel="mri_spec_main (batched work queue)",
                              flops_per_attempted_step=fpa))


DESCRIPTIONS = {
    "field64_s21": "plain FP64 explicit MRI-GARK (MIS-KW3) slow steps, 64^3 cells, 21 species / 84 "
       "reactions, RK4 50 substeps/stage, H = 1e-7 s, advection-diffusion slow RHS",
    "field128_s53": "plain FP64 explicit MRI-GARK (MIS-KW3) slow step, 128^3 cells, 53 species / 325 "
       "reactions, RK4 100 substeps/stage, H = 5e-8 s, advection-diffusion slow RHS",
}


def plain_leg(torch, mri, I, workload, steps, warmup, block, kernel_name):
    """K timed MRI slow steps of a field workload (W untimed before), wall time
    from events around the whole steps, fast-stage kernel time from libmri's
    per-launch events on the launch stream."""
    cfg = I.WORKLOADS[workload]
    mech = I.make_mechanism(workload)
    tb = I.table_mis_kw3()
    y_host = I.initial_state(workload)
    n, ld = y_host.shape
    N = cfg.n_cells
    kernel = dict(auto=mri.KERNEL_AUTO, specialized=mri.KERNEL_SPECIALIZED,
                  generic=mri.KERNEL_GENERIC)[kernel_name]
    m, t = mri.Mech(mech), mri.Table(tb)
    if kernel != mri.KERNEL_GENERIC:
        m.specialize(block or 128, load=True)
    opts = mri.fast_opts(n_sub=cfg.n_sub, kernel=kernel, block_size=block)
    y0 = torch.as_tensor(y_host, device="cuda")
    del y_host
    y = y0.clone()
    ws = torch.empty(mri.mri_workspace_bytes(m, t, N, ld) // 8, dtype=torch.float64,
                     device="cuda")
    status = torch.zeros(ld, dtype=torch.int32, device="cuda")
    params = mri.advdiff_params(cfg.grid, n)

    def step(k):
        mri.mri_slow_step(m, t, opts, mri.ADVDIFF_RHS, params, k * cfg.H, cfg.H, N, ld, y, ws,
                          status)

    print(f"# {workload}: warmup {warmup} steps", file=sys.stderr, flush=True)
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    y.copy_(y0)
    status.zero_()
    torch.cuda.synchronize()
    mri.timing_enable(True)
    mri.timing_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        step(k)
    e1.record()
    torch.cuda.synchronize()
    wall_ms = e0.elapsed_time(e1)
    fast_ms, n_launch = mri.timing_read(reset=True)
    mri.timing_enable(False)
    n_bad = mri.mri_status_count(status, N)
    print(f"# {workload}: timed {steps} steps: {wall_ms:.1f} ms, fast kernels "
          f"{fast_ms:.1f} ms over {n_launch} launches, flagged cells {n_bad}", file=sys.stderr,
          flush=True)
    stages_per_step = tb.s - 1
    value = N * stages_per_step * steps / (wall_ms * 1e-3)
    fps = flops_per_substep(mech.n_species, mech.n_reactions, n_poly=1)
    avg_launch_s = fast_ms * 1e-3 / max(1, n_launch)
    achieved = fps * cfg.n_sub * N / avg_launch_s / 1e12
    traffic_key = (f"mri_fast_stage rk4 {cfg.grid[0]}^3 cells S={mech.n_species} "
                   f"R={mech.n_reactions} n_sub={cfg.n_sub}")
    ctr = None
    if kernel != mri.KERNEL_GENERIC:
        ctr = load_counters(traffic_key, m.code_hash(mri.FAST_RK4, tb.n_gamma, block or 128))
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / PEAK_FP64_TFLOPS, 4),
                traffic=ctr.get("hbm_bytes_per_launch") if ctr else None,
                # the same launch time against the FP64 instructions the counters
                # saw (the algorithmic count charges 22 flops per exponential)
                frac_counters=(round(ctr["counter_fp64_flops_per_launch"] / avg_launch_s / 1e12
                                     / PEAK_FP64_TFLOPS, 4)
                               if ctr and "counter_fp64_flops_per_launch" in ctr else None),
                mcell_substep_per_s=round(N * cfg.n_sub / avg_launch_s / 1e6, 1),
                kernel="mri_spec_main (RK4, specialized)" if kernel != mri.KERNEL_GENERIC
                else "k_gen_rk4 (generic)",
                flops_per_cell_substep=fps, avg_launch_ms=round(avg_launch_s * 1e3, 4))
    return dict(value=round(value, 1), ms_per_step=round(wall_ms / steps, 3), roofline=roof,
                config=dict(workload=DESCRIPTIONS[workload], cells=N,
                            stages_per_step=stages_per_step, n_sub=cfg.n_sub,
                            flagged_cells=n_bad))


def surrogate_leg(train_steps, n_samples):
    """Learned surrogate: stage data from the 64^3 workload's plain runs, training
    with libmri's BF16 MFMA kernels, then the gated stage (tolerance 1e-4) on the
    first fast stage of the 128^3 workload against the plain FP64 stage."""
    from paper_2211_03293_amd import inputs as I
    from paper_2211_03293_amd import surrogate as S

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    data = S.generate_stage_data(n_full=n_samples, log=log)
    res = S.train(data, steps=train_steps, batch=TRAIN_BATCH, log=log,
                  log_every=max(1, train_steps // 8))
    del data
    ev = S.evaluate_stage(res["params"], res["stats"], workload=I.FIELD128, gate_tol=1e-4, log=log)
    t_inf_s = ev["infer_ms"] * 1e-3
    achieved = ev["cells"] * MLP_FLOPS / t_inf_s / 1e12
    ev.update(
        workload="128^3 cells, 21 species / 84 reactions, first MIS-KW3 fast stage "
                 "(L = H/3, H = 1e-7 s, advection-diffusion forcing); MLP 89-256-256-256-22 "
                 "BF16/FP32 trained on the 64^3 workload's stages; fallback plain RK4 "
                 "50 substeps",
        value=round(ev["cells"] / (ev["surrogate_stage_ms"] * 1e-3), 1),
        unit="cell-stages/s", plain_value=round(ev["cells"] / (ev["plain_ms"] * 1e-3), 1),
        training=dict(samples=int(3 * n_samples), steps=train_steps, batch=TRAIN_BATCH,
                      seconds=round(res["train_seconds"], 1),
                      final_val_mse=res["history"][-1][2] if res["history"] else None),
        inferences_per_s=round(ev["cells"] / t_inf_s, 1),
        roofline=dict(bound="mfma", achieved=round(achieved, 2), peak=PEAK_BF16_TFLOPS,
                      unit="TFLOP/s", frac=round(achieved / PEAK_BF16_TFLOPS, 4), traffic=None,
                      kernel="k_infer (fused 4-layer BF16 MFMA)", flops_per_inference=MLP_FLOPS,
                      frac_counters=round(ev["cells"] * MLP_FLOPS_EXECUTED / t_inf_s / 1e12
                                          / PEAK_BF16_TFLOPS, 4)),
        seconds_total=round(time.perf_counter() - t0, 1))
    return ev


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--kernel", choices=["auto", "specialized", "generic"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven-set leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 128^3 large-mechanism leg (53 species / 325 reactions)")
    ap.add_argument("--surrogate-steps", type=int, default=40000,
                    help="training steps of the surrogate leg (batch 8192)")
    ap.add_argument("--surrogate-samples", type=int, default=2_000_000,
                    help="full-stage training samples (plus twice as many half-stage ones)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 1 GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the fast stage is "
              "independent per cell, so several GPUs would each run this same kernel on their "
              "own cell slab.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_03293_amd import inputs as I
    from paper_2211_03293_amd import mri

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy kernel of known size: reads and writes 2^30 bytes per dispatch
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_per_dispatch=2 ** 30, dispatches=3)), flush=True)
        return
    plain = plain_leg(torch, mri, I, I.FIELD64, args.steps, args.warmup, args.block, args.kernel)
    out = dict(metric=METRIC, value=plain["value"], unit="cell-stages/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=plain["ms_per_step"],
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic", config=plain["config"], roofline=plain["roofline"])
    if not args.no_large:
        print("# large-mechanism leg", file=sys.stderr, flush=True)
        big = plain_leg(torch, mri, I, I.LARGE128, 1, 1, args.block, args.kernel)
        large = I.WORKLOADS[I.LARGE128]
        rhs_rate = 4 * large.n_sub * big["value"]          # 4 RHS per RK4 substep
        out["large_mechanism"] = dict(
            value=big["value"], unit="cell-stages/s", ms_per_step=big["ms_per_step"], steps=1,
            warmup=1, config=big["config"], roofline=big["roofline"],
            cell_rhs_per_s=round(rhs_rate, 1),
            paper_context=dict(
                cell_rhs_per_s=3.1e5,
                source="Table 2 (runtimes of the explicit MRI runs, Sec. 5.1), per fast "
                       "evaluation of a least-squares fit: about 0.1 s per chemistry RHS over "
                       "32^3 cells",
                hardware="one node of 2x Intel Xeon E5-2695 v4, 8 MPI ranks (Sec. 5.1)",
                mechanism="GRI-Mech 3.0, 53 species / 325 reactions (same size as this leg's "
                          "synthetic mechanism)",
                note="other hardware and another integrator; context, not the target"))
    if not args.no_batch:
        print("# batched uneven-set leg", file=sys.stderr, flush=True)
        out["batch"] = batch_leg(torch, mri, I)
    if not args.no_surrogate:
        print("# surrogate leg", file=sys.stderr, flush=True)
        out["surrogate"] = surrogate_leg(args.surrogate_steps, args.surrogate_samples)
    if not args.no_cpu_baseline:
        # forcing of the first stage of one slow step, from the oracle's own slow RHS
        from oracle import oracle as O
        cfg, tb = I.WORKLOADS[I.FIELD64], I.table_mis_kw3()
        y_host = I.initial_state(I.FIELD64)
        rho = O.advdiff(y_host, cfg.grid)[None]
        Ls = [float((tb.c[i] - tb.c[i - 1]) * cfg.H) for i in range(1, tb.s)]
        out["cpu_baseline"] = cpu_baseline(I.make_mechanism(I.FIELD64), y_host, rho, Ls, cfg.n_sub)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
