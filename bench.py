"""Benchmark: FP64 plain MRI fast stages against the learned surrogate with FP64
fallback at 1e-4 relative stage error, on one MI355X.

Headline (one bench step = one explicit MRI-GARK slow step over the batch):
128^3 = 2,097,152 cells of smooth periodic synthetic fields, 21 species / 84
reversible reactions, MIS-KW3 coupling table (3 fast stages per slow step),
H = 1e-7 s, advection-diffusion slow RHS; every fast stage taken by the gated
surrogate stage: coarse FP64 RK4 stage (4 and 2 substeps), BF16 MFMA network
correction, residual check at 1e-4, plain FP64 RK4 with 50 substeps for every
rejected cell.  The same K slow steps with the plain FP64 stage (RK4, 50
substeps) run in the same process for the comparison the metric names.  The
network is trained first (untimed) with libmri's kernels on stage data of the
64^3 workload.  Inputs are resident in HBM before the timed region.

Prints one JSON line: value = cell fast-stage solves per second (cell-stages/s)
of the surrogate + fallback path, plus its dominant kernel's roofline (the
fixed-step RK4 kernel: kernel time from libmri's HIP events on the launch
stream around every fast-stage launch inside the timed region, FP64 flops from
the algorithmic count and from rocprof counters) and the oracle timed on a
bounded sample.  Further objects: the accuracy of the surrogate on every cell
of the first slow step, the plain legs (128^3 and 64^3), the 53-species large
mechanism, the IMEX-MRI-GARK steps with stiff diffusion, the batched uneven
reactor sets.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-large] [--no-batch] [--no-plain64] [--no-imex] [--no-alt-coarse]
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
    """rocprofv3 counter figures per launch (HBM bytes, FP64 counter flops) of the
    kernel whose machine code hashes to code_hash on the named workload, or None
    when the compiled kernel changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "kernel_counters.json")
    if not os.path.exists(p):
        return None
    for d in json.load(open(p)).get("entries", []):
        if d.get("kernel_code_hash") == code_hash and d.get("workload") == workload:
            return d
    return None


def counter_flops_per_unit(code_hash: str):
    """FP64 flops per unit of work (cell-substep of a fixed-step kernel, attempted
    cell-step of the batched kernel) that the rocprof counters measured for the
    kernel with this machine code, whatever the launch size, or None."""
    p = os.path.join(ROOT, "profiles", "kernel_counters.json")
    if not os.path.exists(p):
        return None
    for d in json.load(open(p)).get("entries", []):
        if d.get("kernel_code_hash") == code_hash and d.get("counter_fp64_flops_per_unit"):
            return d["counter_fp64_flops_per_unit"]
    return None


def batch_counters_profiled_build(block: int, choice: dict):
    """Counter entry of the batched kernel taken under rocprofv3 for the same
    block size and register / LDS variant.  Under the profiler the run-time
    compilation of this kernel yields different machine code than in a plain
    run, so this entry never matches the timed kernel's hash; it is reported
    beside the algorithmic fraction, labelled with both hashes."""
    p = os.path.join(ROOT, "profiles", "kernel_counters.json")
    if not os.path.exists(p):
        return None
    if choice.get("waves_per_simd") == 1:
        name = "one wave per SIMD"
    elif choice.get("exp_table") == 0:
        name = "polynomial exponential"
    elif choice.get("sched_window") in (1, 4):
        name = "scheduling window %d" % choice["sched_window"]
    else:
        name = "built-in"
    for d in json.load(open(p)).get("entries", []):
        if (d.get("workload", "").startswith("mri_batch_run") and d.get("tile", [0])[0] == block
                and d.get("variant") == name):
            return d
    return None


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


def batch_leg(torch, mri, I, divergent, repeats=3, per_set_baseline=False):
    """Batched uneven reactor sets: 1000 sets, log-uniform sizes, adaptive
    Zonneveld 4(3) at tol 1e-8, one persistent work-queue launch per run
    (autotuned tile and register / LDS tiling, captured in a graph).  With
    per_set_baseline the same sets are also run with one fast-stage launch per
    set."""
    sizes, off, y_host, Ls = I.batch_workload(divergent=divergent)
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
    rejects = torch.zeros(ld, dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    plan.run(y, out, ld, 0, None, Ls, st, steps, rejects)   # tunes, captures the graph
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(repeats):
        plan.run(y, out, ld, 0, None, Ls, st, steps, rejects)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / repeats
    useful, issued = plan.lane_stats()       # attempted lane-steps of the last run
    trials, from_cache, choice = plan.tune_log()
    fpa = flops_per_zv_attempt(mech.n_species, mech.n_reactions)
    achieved = useful * fpa / (ms * 1e-3) / 1e12
    per_unit = counter_flops_per_unit(plan.code_hash(0))
    sv = steps[:ntot].cpu().numpy()
    rv = rejects[:ntot].cpu().numpy()
    n_bad = mri.mri_status_count(st, ntot, mri.CELL_NONFINITE | mri.CELL_TRANGE)
    n_capped = mri.mri_status_count(st, ntot, mri.CELL_MAXSTEPS)
    res = dict(workload=("1000 reactor sets, sizes log-uniform in [64, 65536], 21 species / 84 "
                         "reactions, one unforced fast stage per set, Zonneveld 4(3) tol 1e-8; "
                         + ("per-set stage lengths log-uniform in [1e-8, 1e-6] s" if divergent
                            else "L cycles through the MIS-KW3 stage lengths, H = 1e-7 s")),
               cells=ntot, ms_per_run=round(ms, 3), value=round(ntot / (ms * 1e-3), 1),
               unit="cell-stages/s",
               accepted_steps=dict(min=int(sv.min()), median=float(np.median(sv)),
                                   p99=float(np.quantile(sv, 0.99)), max=int(sv.max())),
               rejected_steps=int(rv.sum()), capped_cells=n_capped,
               exactly_once=bool(int(sv.sum()) + int(rv.sum()) == useful),
               lane_utilization=round(useful / max(issued, 1), 4),
               tile=dict(block=choice["block_size"], blocks=choice["n_blocks"],
                         waves_per_simd=choice["waves_per_simd"],
                         exp_table=choice["exp_table"], sched_window=choice["sched_window"]),
               tuner=dict(from_cache=from_cache, first_run_s=round(first_s, 2),
                          trials=[dict(t, ms=round(t["ms"], 3)) for t in trials]),
               flagged_cells=n_bad, attempted_steps=int(useful),
               roofline=dict(**fp64_roofline(achieved_alg=achieved, avg_launch_s=ms * 1e-3,
                                             counter_flops=(per_unit * useful
                                                            if per_unit else None)),
                             kernel="mri_spec_main (batched work queue)",
                             kernel_code_hash=plan.code_hash(0),
                             flops_per_attempted_step=fpa))
    if per_unit is None:
        pb = batch_counters_profiled_build(choice["block_size"], choice)
        if pb:
            ach = pb["counter_fp64_flops_per_unit"] * useful / (ms * 1e-3) / 1e12
            res["roofline"]["counters_profiled_build"] = dict(
                achieved=round(ach, 3), frac=round(ach / PEAK_FP64_TFLOPS, 4),
                counter_fp64_flops_per_attempted_step=pb["counter_fp64_flops_per_unit"],
                hbm_over_algorithmic=pb.get("hbm_over_algorithmic"),
                profiled_code_hash=pb["kernel_code_hash"], variant=pb["variant"],
                note="counters of the same block size and variant compiled under rocprofv3, "
                     "whose machine code differs from the timed kernel's")
    if per_set_baseline:
        # the same sets, one fast-stage launch per set (Zonneveld kernel,
        # specialized, default block), sets in order on one stream
        out2 = torch.empty_like(y)

        def per_set():
            for s_ in range(off.size - 1):
                a, b = int(off[s_]), int(off[s_ + 1])
                mri.mri_fast_stage(m, opts, b - a, ld, y[:, a:], out2[:, a:], 0, None,
                                   float(Ls[s_]))
        per_set()
        torch.cuda.synchronize()
        e0.record()
        per_set()
        e1.record()
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1)
        res["one_launch_per_set"] = dict(ms_per_run=round(ms1, 3),
                                         value=round(ntot / (ms1 * 1e-3), 1),
                                         speedup_of_work_queue=round(ms1 / ms, 3),
                                         max_rel_diff=float(((out2[:, :ntot] - out[:, :ntot])
                                                             .abs() / out[:, :ntot].abs()
                                                             .clamp_min(1e-12)).max().item()))
    return res


def fp64_roofline(achieved_alg, avg_launch_s, counter_flops=None, traffic=None):
    """FP64 vector roofline of a fixed-step kernel: frac from the FP64 flops the
    rocprof counters count per launch (64 x (ADD + MUL + TRANS + 2 FMA) wave
    instructions) when they were taken for this machine code, else from the
    algorithmic count; the algorithmic fraction (F_exp flops per exponential)
    is kept beside it."""
    alg = dict(achieved=round(achieved_alg, 3), frac=round(achieved_alg / PEAK_FP64_TFLOPS, 4),
               f_exp=F_EXP, f_log=F_LOG, f_div=F_DIV)
    if counter_flops:
        ach = counter_flops / avg_launch_s / 1e12
        return dict(bound="alu", achieved=round(ach, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / PEAK_FP64_TFLOPS, 4), frac_source="rocprof FP64 counters",
                    traffic=traffic, algorithmic=alg)
    return dict(bound="alu", achieved=alg["achieved"], peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                frac=alg["frac"], frac_source="algorithmic count (no counters for this code)",
                traffic=traffic, algorithmic=alg)


def counter_key(cfg, mech):
    return (f"mri_fast_stage rk4 {cfg.grid[0]}^3 cells S={mech.n_species} "
            f"R={mech.n_reactions} n_sub={cfg.n_sub}")


DESCRIPTIONS = {
    "field64_s21": "plain FP64 explicit MRI-GARK (MIS-KW3) slow steps, 64^3 cells, 21 species / 84 "
       "reactions, RK4 50 substeps/stage, H = 1e-7 s, advection-diffusion slow RHS",
    "field128_s21": "plain FP64 explicit MRI-GARK (MIS-KW3) slow steps, 128^3 cells, 21 species / "
       "84 reactions, RK4 50 substeps/stage, H = 1e-7 s, advection-diffusion slow RHS",
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
    ctr, per_unit = None, None
    if kernel != mri.KERNEL_GENERIC:
        h = m.code_hash(mri.FAST_RK4, tb.n_gamma, block or 128)
        ctr = load_counters(counter_key(cfg, mech), h)
        per_unit = counter_flops_per_unit(h)
    roof = fp64_roofline(achieved_alg=achieved, avg_launch_s=avg_launch_s,
                         counter_flops=per_unit * N * cfg.n_sub if per_unit else None,
                         traffic=ctr.get("hbm_bytes_per_launch") if ctr else None)
    roof.update(mcell_substep_per_s=round(N * cfg.n_sub / avg_launch_s / 1e6, 1),
                kernel="mri_spec_main (RK4, specialized)" if kernel != mri.KERNEL_GENERIC
                else "k_gen_rk4 (generic)",
                flops_per_cell_substep=fps, avg_launch_ms=round(avg_launch_s * 1e3, 4))
    return dict(value=round(value, 1), ms_per_step=round(wall_ms / steps, 3), roofline=roof,
                config=dict(workload=DESCRIPTIONS[workload], cells=N,
                            stages_per_step=stages_per_step, n_sub=cfg.n_sub,
                            flagged_cells=n_bad))


def imex_leg(torch, mri, I, steps=5, warmup=1, order=3):
    """IMEX-MRI-GARK steps on the 64^3 fields with the diffusion number
    H D / dx^2 = 1, where the explicit MIS-KW3 table diverges: the 3rd-order
    solve-decoupled table (three fast stages of H/3, three implicit diffusion
    stages) or the 2nd-order one (one fast stage over the step, one implicit
    stage); RK4 at the explicit workload's largest fast step H / 120.  Wall
    time per step, fast-kernel time, conjugate-gradient iterations per solve,
    and one diffusion solve timed alone for its HBM roofline (algorithmic
    traffic 11 planes per iteration: the stencil reads p and writes q, the
    update reads x, p, r, q and writes x, r, the direction update reads r, p
    and writes p).  With the 3rd-order table, the explicit table's first
    flagged step on the same state plus a 1e-6 K checkerboard is reported
    beside it."""
    cfg = I.WORKLOADS[I.FIELD64]
    P = I.ADVDIFF_STIFF
    mech = I.make_mechanism(I.FIELD64)
    N = cfg.n_cells
    y_host = I.initial_state(I.FIELD64)
    n, ld = y_host.shape
    tab = I.table_imex_mri3() if order == 3 else I.table_imex_trap2()
    n_sub = I.IMEX3_N_SUB if order == 3 else I.IMEX_N_SUB
    a_diag = float(sum(tab.gamma[k, 2, 2] / (k + 1) for k in range(tab.gamma.shape[0])))
    m, t = mri.Mech(mech), mri.ImexTable(tab)
    m.specialize(128, load=True)
    params = mri.advdiff_params(cfg.grid, n, u=P["u"], D=P["D"], dx=P["dx"])
    cws = torch.empty(mri.diffusion_solve_workspace_bytes(params, ld), dtype=torch.uint8,
                      device="cuda")
    ctx = mri.imex_advdiff(params, cws, cg_rtol=1e-13)
    ws = torch.empty(mri.mri_imex_workspace_bytes(m, t, N, ld), dtype=torch.uint8, device="cuda")
    y0 = torch.as_tensor(y_host, device="cuda")
    y = y0.clone()
    status = torch.zeros(ld, dtype=torch.int32, device="cuda")
    opts = mri.fast_opts(n_sub=n_sub)
    H = cfg.H
    for k in range(warmup):
        mri.mri_imex_slow_step(m, t, opts, ctx, k * H, H, N, ld, y, ws, status_out=status)
    torch.cuda.synchronize()
    y.copy_(y0)
    mri.timing_enable(True)
    mri.timing_read(reset=True)
    iters = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        mri.mri_imex_slow_step(m, t, opts, ctx, k * H, H, N, ld, y, ws, status_out=status)
        iters.append(ctx.cg_iters)
    e1.record()
    torch.cuda.synchronize()
    wall_ms = e0.elapsed_time(e1)
    fast_ms, n_launch = mri.timing_read(reset=True)
    mri.timing_enable(False)
    n_bad = mri.mri_status_count(status, N)
    # one diffusion solve alone, on the current state, with the first implicit
    # stage's coefficient a = gbar_33 H
    r = y.clone()
    out = torch.empty_like(r)
    mri.mri_diffusion_solve(ctx, a_diag * H, r, out, N, ld)
    torch.cuda.synchronize()
    e0.record()
    mri.mri_diffusion_solve(ctx, a_diag * H, r, out, N, ld)
    e1.record()
    torch.cuda.synchronize()
    solve_ms = e0.elapsed_time(e1)
    it = ctx.cg_iters
    bytes_alg = 11 * 8 * n * N * it
    gbs = bytes_alg / (solve_ms * 1e-3) / 1e9
    # the explicit table on the same fields with a grid-scale perturbation
    flagged_at = None
    if order == 3:
        flagged_at = explicit_flag_step(torch, mri, I, m, cfg, y0, params, N, ld, H)
    print(f"# imex (order {order}): {steps} steps {wall_ms:.1f} ms, fast kernels {fast_ms:.1f} ms, "
          f"CG iterations {iters}, solve {solve_ms:.3f} ms ({gbs:.0f} GB/s algorithmic), explicit "
          f"flagged at step {flagged_at}", file=sys.stderr, flush=True)
    return imex_result(order, n, N, steps, wall_ms, fast_ms, iters, solve_ms, gbs, it, n_bad,
                       flagged_at, n_sub)


def explicit_flag_step(torch, mri, I, m, cfg, y0, params, N, ld, H):
    """First MIS-KW3 step that flags a cell on the fields plus a 1e-6 K
    grid-scale checkerboard (None within 12 steps)."""
    te = mri.Table(I.table_mis_kw3())
    wse = torch.empty(mri.mri_workspace_bytes(m, te, N, ld) // 8, dtype=torch.float64,
                      device="cuda")
    z, yy, x = np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij")
    ye = y0.clone()
    ye[-1, :N] += torch.as_tensor(1e-6 * ((-1.0) ** (x + yy + z)).ravel(), device="cuda")
    ste = torch.zeros(ld, dtype=torch.int32, device="cuda")
    for k in range(12):
        mri.mri_slow_step(m, te, mri.fast_opts(n_sub=cfg.n_sub), mri.ADVDIFF_RHS, params, k * H, H,
                          N, ld, ye, wse, status_out=ste)
        if mri.mri_status_count(ste, N) > 0:
            return k + 1
    return None


def imex_result(order, n, N, steps, wall_ms, fast_ms, iters, solve_ms, gbs, it, n_bad, flagged_at,
                n_sub):
    table = ("3rd-order solve-decoupled table, three fast stages of H/3 with RK4 %d substeps, three "
             "implicit stages" % n_sub if order == 3 else
             "2nd-order solve-decoupled table, one fast stage over H with RK4 %d substeps, one "
             "implicit stage" % n_sub)
    out = dict(workload="IMEX-MRI-GARK steps (%s), 64^3 cells, 21 species / 84 reactions, "
                        "H = 1e-7 s, advection explicit, diffusion implicit with D = 0.1 m^2/s "
                        "(H D / dx^2 = 1)" % table,
               order=order,
               value=round(N * steps / (wall_ms * 1e-3), 1), unit="cell-steps/s",
               ms_per_step=round(wall_ms / steps, 3), fast_kernel_ms_per_step=round(
                   fast_ms / steps, 3), cg_iterations=iters, flagged_cells=n_bad,
               diffusion_solve=dict(ms=round(solve_ms, 3), iterations=it, cg_rtol=1e-13,
                                    roofline=dict(bound="hbm", achieved=round(gbs, 1),
                                                  peak=8000.0, unit="GB/s",
                                                  frac=round(gbs / 8000.0, 4),
                                                  bytes_per_iteration=11 * 8 * n * N)))
    if order == 3:
        out["explicit_mis_kw3_first_flagged_step"] = flagged_at
    return out


def train_surrogate(n_samples, train_steps, log):
    """Stage data from the 64^3 workload's plain runs and training with libmri's
    BF16 MFMA kernels (setup of the headline, not timed as a bench step)."""
    from paper_2211_03293_amd import surrogate as S
    t0 = time.perf_counter()
    data = S.generate_stage_data(n_full=n_samples, log=log)
    res = S.train(data, steps=train_steps, batch=TRAIN_BATCH, log=log,
                  log_every=max(1, train_steps // 8))
    del data
    res["setup_seconds"] = time.perf_counter() - t0
    return res


def surrogate_steps(torch, mri, I, params, stats, steps, warmup, gate_tol=1e-4, n_coarse=None,
                    check_fraction=None, stiff_limit=None):
    """K timed MRI slow steps of the 128^3 workload whose fast stages are gated
    surrogate stages (W untimed before, from the same initial state); the slow
    RHS and forcing assembly as in the plain path.  The residual check accepts
    at CHECK_FRACTION of the stage tolerance.  Nothing synchronizes inside a step: the
    fallback counts stay on the device until the timed region ends."""
    from paper_2211_03293_amd import surrogate as S
    cfg = I.WORKLOADS[I.FIELD128]
    mech = I.make_mechanism(I.FIELD128)
    tb = I.table_mis_kw3()
    y_host = I.initial_state(I.FIELD128)
    n, ld = y_host.shape
    N = cfg.n_cells
    m, t = mri.Mech(mech), mri.Table(tb)
    m.specialize(128, load=True)
    sg = mri.Surrogate(S.WIDTHS, params, stats)
    n_coarse = S.N_COARSE if n_coarse is None else n_coarse
    check_fraction = S.CHECK_FRACTION if check_fraction is None else check_fraction
    coarse = mri.fast_opts(n_sub=n_coarse, stiff_limit=S.STIFF_LIMIT if stiff_limit is None
                           else stiff_limit)
    fine = mri.fast_opts(n_sub=cfg.n_sub)
    y0 = torch.as_tensor(y_host, device="cuda")
    del y_host
    y = y0.clone()
    F = torch.empty((tb.s - 1, n, ld), dtype=torch.float64, device="cuda")
    rho = torch.empty((1, n, ld), dtype=torch.float64, device="cuda")
    ws = torch.empty(mri.Surrogate.workspace_bytes(N, ld, 1) // 8 + 1, dtype=torch.float64,
                     device="cuda")
    status = torch.zeros(ld, dtype=torch.int32, device="cuda")
    n_fb = torch.zeros(max(steps, warmup) * (tb.s - 1), dtype=torch.int32, device="cuda")
    params_ad = mri.advdiff_params(cfg.grid, n)
    uptr = mri.C.cast(mri.C.pointer(params_ad), mri.C.c_void_p).value

    def step(k):
        sp = torch.cuda.current_stream().cuda_stream
        for i in range(1, tb.s):
            rc = mri.lib.mri_advdiff_slow_rhs(k * cfg.H + tb.c[i - 1] * cfg.H, y.data_ptr(),
                                              F[i - 1].data_ptr(), N, ld, uptr, sp)
            assert rc == 0
            mri.mri_forcing_assemble(t, i, n, ld, F, rho)
            L = float((tb.c[i] - tb.c[i - 1]) * cfg.H)
            j = k * (tb.s - 1) + i - 1
            sg.stage(m, coarse, fine, check_fraction * gate_tol, N, ld, y, y, 1, rho, L, ws,
                     None, None,
                     status, n_fb[j:j + 1])

    print(f"# surrogate steps: warmup {warmup}", file=sys.stderr, flush=True)
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    y.copy_(y0)
    n_fb.zero_()
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
    fb = n_fb[:steps * (tb.s - 1)].cpu().numpy()
    n_bad = mri.mri_status_count(status, N)
    print(f"# surrogate steps: timed {steps} steps: {wall_ms:.1f} ms, RK4 kernels {fast_ms:.1f} ms "
          f"over {n_launch} launches, fallback cells per stage {fb.tolist()}", file=sys.stderr,
          flush=True)
    stages = steps * (tb.s - 1)
    value = N * stages / (wall_ms * 1e-3)
    # the dominant kernel: the fixed-step RK4 kernel of the coarse stages (n and
    # n/2 substeps over every cell) and of the fallback (n_sub over the rejected
    # cells); algorithmic flops per cell-substep as for the plain path
    fps = flops_per_substep(mech.n_species, mech.n_reactions, n_poly=1)
    cell_substeps = stages * N * (n_coarse + n_coarse // 2) + int(fb.sum()) * cfg.n_sub
    fast_s = fast_ms * 1e-3
    per_unit = counter_flops_per_unit(m.code_hash(mri.FAST_RK4, tb.n_gamma, 128))
    roof = fp64_roofline(achieved_alg=fps * cell_substeps / fast_s / 1e12,
                         avg_launch_s=fast_s / max(1, n_launch),
                         counter_flops=(per_unit * cell_substeps / max(1, n_launch)
                                        if per_unit else None))
    roof.update(kernel="mri_spec_main (RK4, specialized): coarse, half and fallback stages",
                launches=n_launch, kernel_ms=round(fast_ms, 3),
                share_of_step_time=round(fast_ms / wall_ms, 3), flops_per_cell_substep=fps,
                cell_substeps=cell_substeps)
    return dict(value=round(value, 1), ms_per_step=round(wall_ms / steps, 3), roofline=roof,
                fallback_cells=int(fb.sum()), fallback_frac=float(fb.sum()) / (N * stages),
                flagged_cells=n_bad, cells=N, stages_per_step=tb.s - 1)


def alt_coarse_leg(n_samples, train_steps, log, steps=10, warmup=2):
    """The same pipeline with the other coarse setting (N_COARSE_ALT substeps,
    check at CHECK_FRACTION_ALT of the tolerance): a network trained on that
    coarse stage against the zero correction on every cell of the first slow
    step of the 128^3 workload, and the headline's slow steps."""
    from paper_2211_03293_amd import inputs as I
    from paper_2211_03293_amd import surrogate as S
    nc, frac = S.N_COARSE_ALT, S.CHECK_FRACTION_ALT
    data = S.generate_stage_data(n_full=n_samples, n_coarse=nc, log=log)
    res = S.train(data, steps=train_steps, batch=TRAIN_BATCH, log=log,
                  log_every=max(1, train_steps // 2))
    del data
    ev = S.evaluate(res["params"], res["stats"], workload=I.FIELD128, gate_tol=1e-4,
                    check_tol=frac * 1e-4, n_coarse=nc, repeats=1, log=log)
    keys = ("ms", "fallback_frac", "false_accepts", "max_err", "speedup_vs_plain")
    import torch
    from paper_2211_03293_amd import mri
    log(f"# the {nc}-substep configuration over the headline's slow steps")
    run = surrogate_steps(torch, mri, I, res["params"], res["stats"], steps, warmup, n_coarse=nc,
                          check_fraction=frac)
    return dict(n_coarse=nc, check_tol=frac * 1e-4,
                slow_steps=dict(steps=steps, ms_per_step=run["ms_per_step"], value=run["value"],
                                fallback_frac=run["fallback_frac"]),
                learned={k: ev["learned"][k] for k in keys},
                no_network={k: ev["no_network"][k] for k in keys},
                fallback_reduction=round(1.0 - ev["learned"]["fallback_frac"]
                                         / max(ev["no_network"]["fallback_frac"], 1e-30), 3),
                errors=ev["errors"])


def surrogate_eval(params, stats, log, gate_tol=1e-4):
    """Accuracy on every cell of the three fast stages of the first slow step
    against the plain FP64 stage, the no-network comparison, the cheapest plain
    substep count within the tolerance, and the fused inference's roofline."""
    from paper_2211_03293_amd import inputs as I
    from paper_2211_03293_amd import surrogate as S
    ev = S.evaluate(params, stats, workload=I.FIELD128, gate_tol=gate_tol, log=log)
    t_inf_s = ev["infer_ms"] * 1e-3 / ev["stages"]
    n = ev["cells"] // ev["stages"]
    achieved = n * MLP_FLOPS / t_inf_s / 1e12
    ev.update(
        workload="every cell of the three MIS-KW3 fast stages of the 128^3 workload's first "
                 "slow step, against the plain FP64 RK4 stage (50 substeps)",
        inferences_per_s=round(n / t_inf_s, 1),
        roofline=dict(bound="mfma", achieved=round(achieved, 2), peak=PEAK_BF16_TFLOPS,
                      unit="TFLOP/s", frac=round(achieved / PEAK_BF16_TFLOPS, 4), traffic=None,
                      kernel="k_infer (fused 4-layer BF16 MFMA)", flops_per_inference=MLP_FLOPS,
                      frac_executed_mfma=round(n * MLP_FLOPS_EXECUTED / t_inf_s / 1e12
                                               / PEAK_BF16_TFLOPS, 4)))
    return ev


def cpu_baseline_surrogate(params, stats, n_sample=262144):
    """The oracle's gated surrogate stage (RK4 at N_COARSE and N_COARSE / 2
    substeps, the network in its bfloat16-emulating mode, the residual check,
    plain RK4 with 50 substeps for rejected cells) on evenly spaced cells of the
    first fast stage of the 128^3 workload, with all the threads the job may
    use."""
    from oracle import oracle as O
    from paper_2211_03293_amd import inputs as I
    from paper_2211_03293_amd import surrogate as S
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    O.set_threads(threads)
    cfg, tb = I.WORKLOADS[I.FIELD128], I.table_mis_kw3()
    y_host = I.initial_state(I.FIELD128)
    idx = np.linspace(0, cfg.n_cells - 1, n_sample).astype(np.int64)
    rho = O.advdiff(y_host, cfg.grid)[None][:, :, idx] * (tb.gamma[0][1][0] / tb.c[1])
    ys = np.ascontiguousarray(y_host[:, idx])
    del y_host
    orc = O.Oracle(I.make_mechanism(I.FIELD128))
    L = float(tb.c[1] * cfg.H)
    t0 = time.perf_counter()
    _, acc, _, _ = O.sur_stage(orc, S.WIDTHS, np.asarray(params, np.float64), stats, ys,
                               np.ascontiguousarray(rho), L, S.N_COARSE, cfg.n_sub,
                               S.CHECK_FRACTION * 1e-4, stiff_limit=S.STIFF_LIMIT)
    dt = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="cell-stages/s", cores=O.num_threads(), kind="oracle",
                sample=f"{n_sample} evenly spaced cells of the 128^3 field, first MIS-KW3 fast "
                       f"stage, the oracle's gated surrogate stage ({int((~acc).sum())} plain "
                       f"fallbacks); {dt:.1f} s",
                host=dict(cpu=_cpu_model(), nproc=os.cpu_count()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--kernel", choices=["auto", "specialized", "generic"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven-set leg")
    ap.add_argument("--no-plain64", action="store_true", help="skip the 64^3 plain leg")
    ap.add_argument("--no-imex", action="store_true", help="skip the IMEX (stiff diffusion) leg")
    ap.add_argument("--no-alt-coarse", action="store_true",
                    help="skip the surrogate leg with the other coarse-stage setting")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 128^3 large-mechanism leg (53 species / 325 reactions)")
    ap.add_argument("--surrogate-steps", type=int, default=40000,
                    help="training steps of the surrogate (batch 8192)")
    ap.add_argument("--surrogate-samples", type=int, default=2_000_000,
                    help="stage samples (start state, forcing, coarse and plain stage results)")
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
    from paper_2211_03293_amd import surrogate as S

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

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    log("# surrogate training (setup)")
    res = train_surrogate(args.surrogate_samples, args.surrogate_steps, log)
    sur = surrogate_steps(torch, mri, I, res["params"], res["stats"], args.steps, args.warmup)
    log("# plain steps on the same workload")
    plain = plain_leg(torch, mri, I, I.FIELD128, args.steps, args.warmup, args.block,
                      args.kernel)
    out = dict(metric=METRIC, value=sur["value"], unit="cell-stages/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=sur["ms_per_step"],
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64+bf16",
               data="synthetic",
               config=dict(workload="surrogate + FP64 fallback at 1e-4: explicit MRI-GARK "
                                    "(MIS-KW3) slow steps, 128^3 cells, 21 species / 84 reactions, "
                                    "H = 1e-7 s, advection-diffusion slow RHS; each fast stage: "
                                    f"coarse FP64 RK4 ({S.N_COARSE} and {S.N_COARSE // 2} "
                                    "substeps), BF16 MLP correction 89-256-256-256-22, residual "
                                    f"check {1e-4 * S.CHECK_FRACTION:g} for a 1e-4 stage error, "
                                    "FP64 RK4 50 substeps for rejected cells",
                           cells=sur["cells"], stages_per_step=sur["stages_per_step"],
                           stage_tol=1e-4, check_tol=1e-4 * S.CHECK_FRACTION),
               plain_value=plain["value"], plain_ms_per_step=plain["ms_per_step"],
               speedup_vs_plain=round(sur["value"] / plain["value"], 3),
               fallback_frac=sur["fallback_frac"], flagged_cells=sur["flagged_cells"],
               roofline=sur["roofline"])
    log("# surrogate accuracy (every cell of the first slow step)")
    ev = surrogate_eval(res["params"], res["stats"], log)
    ev["training"] = dict(samples=int(args.surrogate_samples), steps=args.surrogate_steps,
                          batch=TRAIN_BATCH, seconds=round(res["train_seconds"], 1),
                          setup_seconds=round(res["setup_seconds"], 1),
                          final_val_mse=res["history"][-1][2] if res["history"] else None)
    out["surrogate"] = ev
    log(f"# accuracy on every cell of the last timed slow step (step {args.steps})")
    late = S.evaluate(res["params"], res["stats"], workload=I.FIELD128, gate_tol=1e-4,
                      repeats=1, log=log, step=args.steps - 1)
    keys = ("fallback_frac", "false_accepts", "max_err", "speedup_vs_plain")
    ev["last_step"] = dict(step=args.steps, learned={k: late["learned"][k] for k in keys},
                           no_network={k: late["no_network"][k] for k in keys},
                           errors=late["errors"])
    if not args.no_alt_coarse:
        log(f"# the other coarse setting: {S.N_COARSE_ALT} substeps")
        out[f"surrogate_coarse{S.N_COARSE_ALT}"] = alt_coarse_leg(
            args.surrogate_samples, args.surrogate_steps, log, args.steps, args.warmup)
    out["plain_128cube"] = dict(value=plain["value"], ms_per_step=plain["ms_per_step"],
                                roofline=plain["roofline"], config=plain["config"])
    if not args.no_plain64:
        log("# 64^3 plain leg")
        p64 = plain_leg(torch, mri, I, I.FIELD64, args.steps, args.warmup, args.block,
                        args.kernel)
        out["plain_64cube"] = dict(value=p64["value"], ms_per_step=p64["ms_per_step"],
                                   roofline=p64["roofline"], config=p64["config"])
    if not args.no_large:
        log("# large-mechanism leg")
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
    if not args.no_imex:
        log("# IMEX legs (stiff diffusion)")
        out["imex"] = imex_leg(torch, mri, I, order=3)
        out["imex_order2"] = imex_leg(torch, mri, I, order=2)
    if not args.no_batch:
        log("# batched uneven-set legs (the standard one tunes; the divergent one takes its "
            "choice from the tuning cache)")
        out["batch"] = batch_leg(torch, mri, I, divergent=False)
        out["batch_divergent"] = batch_leg(torch, mri, I, divergent=True, per_set_baseline=True)
    if not args.no_cpu_baseline:
        log("# CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline_surrogate(res["params"], res["stats"])
        from oracle import oracle as O
        cfg, tb = I.WORKLOADS[I.FIELD64], I.table_mis_kw3()
        y_host = I.initial_state(I.FIELD64)
        rho = O.advdiff(y_host, cfg.grid)[None]
        Ls = [float((tb.c[i] - tb.c[i - 1]) * cfg.H) for i in range(1, tb.s)]
        out["cpu_baseline_plain"] = cpu_baseline(I.make_mechanism(I.FIELD64), y_host, rho, Ls,
                                                 cfg.n_sub, n_sample=65536, n_sample_1core=4096)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
