"""Learned fast-stage surrogate: stage data from the plain FP64 method, training
with libmri's own BF16 MFMA forward / backward / Adam kernels, and evaluation
of the gated surrogate stage against the plain FP64 stage.

Every arithmetic step runs in libmri kernels; this module only orders the
calls, draws random sample indices and moves tensors.

Stage data (the 64^3 workload, 21 species / 84 reactions): the workload's MRI
slow steps are replayed stage by stage (slow RHS, forcing assembly, plain RK4
fast stage).  In every fast stage a random subset of cells is recorded as a
full-stage sample (Y0, rho, L -> Y1) and, for the step-doubling gate, as two
half-stage samples (Y0, rho, L/2 -> Yh) and (Yh, rho, L/2 -> Yhh) integrated by
the same plain method with half the substeps.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs as I
from . import mri

# the training network reads the padded feature rows written by mri_mlp_featurize
# (96 columns, the last 7 always zero)
WIDTHS = [mri.MLP_KPAD, 256, 256, 256, mri.MLP_OUTPUTS]


def _torch():
    import torch
    return torch


class StageData:
    """Stage samples on the device, SoA with leading dimension n (= count)."""

    def __init__(self, Y0, RHO, L, Y1):
        self.Y0, self.RHO, self.L, self.Y1 = Y0, RHO, L, Y1
        self.n = L.numel()


def generate_stage_data(n_full=1_000_000, workload=I.FIELD64, seed=None, log=print):
    """Full- and half-stage samples from the workload's MRI run (n_full full-stage
    samples spread evenly over all fast stages, plus 2 n_full half-stage ones)."""
    torch = _torch()
    cfg = I.WORKLOADS[workload]
    mech = I.make_mechanism(workload)
    tb = I.table_mis_kw3()
    m, t = mri.Mech(mech), mri.Table(tb)
    m.specialize(128, load=True)
    y_host = I.initial_state(workload)
    n, ld = y_host.shape
    N = cfg.n_cells
    y = torch.as_tensor(y_host, device="cuda")
    F = torch.empty((tb.s - 1, n, ld), dtype=torch.float64, device="cuda")
    rho = torch.empty((1, n, ld), dtype=torch.float64, device="cuda")
    params = mri.advdiff_params(cfg.grid, n)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(1000 * I.WORKLOADS[workload].seed_base + 5 if seed is None else seed)
    n_stages = cfg.n_slow_steps * (tb.s - 1)
    per = int(math.ceil(n_full / n_stages))
    buf = {k: [] for k in ("Y0", "RHO", "L", "Y1")}
    opts_full = mri.fast_opts(n_sub=cfg.n_sub)
    opts_half = mri.fast_opts(n_sub=max(1, cfg.n_sub // 2))
    sp = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    for step in range(cfg.n_slow_steps):
        tn = step * cfg.H
        for i in range(1, tb.s):
            # slow evaluation of the current stage value (F_(i-1))
            rc = mri.lib.mri_advdiff_slow_rhs(tn + tb.c[i - 1] * cfg.H, y.data_ptr(),
                                              F[i - 1].data_ptr(), N, ld,
                                              mri.C.cast(mri.C.pointer(params),
                                                         mri.C.c_void_p).value, sp)
            assert rc == 0
            mri.mri_forcing_assemble(t, i, n, ld, F, rho)
            L = float((tb.c[i] - tb.c[i - 1]) * cfg.H)
            idx = torch.randperm(N, generator=gen)[:per].to("cuda")
            k = idx.numel()
            y0s = y[:, idx].contiguous()
            rs = rho[:, :, idx].contiguous()
            y_next = torch.empty_like(y)
            mri.mri_fast_stage(m, opts_full, N, ld, y, y_next, 1, rho, L)
            y1s = y_next[:, idx].contiguous()
            yh = torch.empty_like(y0s)
            mri.mri_fast_stage(m, opts_half, k, k, y0s, yh, 1, rs, 0.5 * L)
            yhh = torch.empty_like(y0s)
            mri.mri_fast_stage(m, opts_half, k, k, yh, yhh, 1, rs, 0.5 * L)
            buf["Y0"] += [y0s, y0s, yh]
            buf["RHO"] += [rs, rs, rs]
            buf["L"] += [torch.full((k,), L, dtype=torch.float64, device="cuda"),
                         torch.full((k,), 0.5 * L, dtype=torch.float64, device="cuda"),
                         torch.full((k,), 0.5 * L, dtype=torch.float64, device="cuda")]
            buf["Y1"] += [y1s, yh, yhh]
            y = y_next
    torch.cuda.synchronize()
    data = StageData(torch.cat(buf["Y0"], 1).contiguous(), torch.cat(buf["RHO"], 2).contiguous(),
                     torch.cat(buf["L"]).contiguous(), torch.cat(buf["Y1"], 1).contiguous())
    log(f"# stage data: {data.n} samples ({n_stages} stages x {per} cells x 3) in "
        f"{time.time() - t0:.1f} s")
    return data


def init_params(seed=4004):
    """He-style initial weights (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for l in range(len(WIDTHS) - 1):
        ni, no = WIDTHS[l], WIDTHS[l + 1]
        fan_in = mri.MLP_FEATURES if l == 0 else ni
        std = math.sqrt(2.0 / fan_in) if l < len(WIDTHS) - 2 else math.sqrt(1.0 / fan_in)
        W = rng.normal(0.0, std, size=(no, ni)).astype(np.float32)
        if l == 0:
            W[:, mri.MLP_FEATURES:] = 0.0
        out.append(W.ravel())
        out.append(np.zeros(no, dtype=np.float32))
    return np.concatenate(out)


def train(data: StageData, steps=20000, batch=4096, lr=2e-3, lr_min=2e-5, seed=5005,
          val_frac=0.05, log=print, log_every=2000):
    """Adam with cosine learning-rate decay on the standardized MSE."""
    torch = _torch()
    stats = torch.empty(mri.MLP_STATS, dtype=torch.float64, device="cuda")
    mri.mri_mlp_feature_stats(data.n, data.n, data.Y0, 1, data.RHO, data.L, data.Y1, stats)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    perm = torch.randperm(data.n, generator=gen)
    n_val = int(data.n * val_frac)
    val_idx = perm[:n_val].to(torch.int32).to("cuda")
    tr_idx = perm[n_val:].to(torch.int32).to("cuda")
    net = mri.MLP(WIDTHS, init_params(), max_batch=batch)
    X = torch.empty((batch, mri.MLP_KPAD), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((batch, mri.MLP_OUTPUTS), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    t0 = time.time()
    n_tr = tr_idx.numel()
    order = torch.randperm(n_tr, generator=gen).to("cuda")
    pos = 0
    for it in range(steps):
        if pos + batch > n_tr:
            order = torch.randperm(n_tr, generator=gen).to("cuda")
            pos = 0
        bidx = tr_idx[order[pos:pos + batch]].contiguous()
        pos += batch
        mri.mri_mlp_featurize(batch, bidx, data.n, data.Y0, 1, data.RHO, data.L, data.Y1, stats,
                              X, T)
        net.forward(X)
        net.backward(T, loss)
        cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / steps))
        net.adam_step(cur)
        if (it + 1) % log_every == 0 or it == steps - 1:
            torch.cuda.synchronize()
            tl = loss.item() / log_every
            loss.zero_()
            vl = evaluate_loss(net, data, val_idx, stats, batch)
            hist.append((it + 1, tl, vl))
            log(f"# step {it + 1}: train mse {tl:.3e}  val mse {vl:.3e}  ({time.time() - t0:.1f} s)")
    params = net.params()
    return dict(params=params, stats=stats.cpu().numpy(), history=hist, net=net,
                train_seconds=time.time() - t0)


def evaluate_loss(net, data, idx, stats, batch):
    torch = _torch()
    X = torch.empty((batch, mri.MLP_KPAD), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((batch, mri.MLP_OUTPUTS), dtype=torch.float32, device="cuda")
    Y = torch.empty((batch, mri.MLP_OUTPUTS), dtype=torch.float32, device="cuda")
    tot, cnt = 0.0, 0
    for a in range(0, idx.numel() - batch + 1, batch):
        b = idx[a:a + batch].contiguous()
        mri.mri_mlp_featurize(batch, b, data.n, data.Y0, 1, data.RHO, data.L, data.Y1, stats, X, T)
        net.forward(X, Y)
        tot += float(((Y - T) ** 2).mean().item()) * batch
        cnt += batch
    return tot / max(cnt, 1)


def stage_error(y_pred, y_ref, n_species, floor=1e-8):
    """Per-cell stage error: max over components of |pred - ref| / max(|ref|, floor)
    (floor for mass fractions; temperature relative)."""
    torch = _torch()
    fl = torch.zeros((y_ref.shape[0], 1), dtype=y_ref.dtype, device=y_ref.device)
    fl[:n_species] = floor
    return ((y_pred - y_ref).abs() / torch.maximum(y_ref.abs(), fl)).amax(0)


def stage_inputs(workload=I.FIELD128, stage=1):
    """State, forcing and stage length of one fast stage of the workload's first
    slow step (slow RHS by the advection-diffusion kernel, forcing assembly by
    libmri), as device tensors."""
    torch = _torch()
    cfg = I.WORKLOADS[workload]
    tb = I.table_mis_kw3()
    t = mri.Table(tb)
    y_host = I.initial_state(workload)
    n, ld = y_host.shape
    N = cfg.n_cells
    y = torch.as_tensor(y_host, device="cuda")
    F = torch.empty((tb.s - 1, n, ld), dtype=torch.float64, device="cuda")
    rho = torch.empty((1, n, ld), dtype=torch.float64, device="cuda")
    params = mri.advdiff_params(cfg.grid, n)
    sp = torch.cuda.current_stream().cuda_stream
    rc = mri.lib.mri_advdiff_slow_rhs(0.0, y.data_ptr(), F[0].data_ptr(), N, ld,
                                      mri.C.cast(mri.C.pointer(params), mri.C.c_void_p).value, sp)
    assert rc == 0
    mri.mri_forcing_assemble(t, stage, n, ld, F, rho)
    L = float((tb.c[stage] - tb.c[stage - 1]) * cfg.H)
    return y, rho, L, N, ld


def evaluate_stage(params, stats, workload=I.FIELD128, gate_tol=1e-4, repeats=3, log=print):
    """Gated surrogate stage against the plain FP64 stage on every cell of the
    workload's first fast stage: fallback fraction, false accepts, error of the
    accepted cells, wall times and the fused inference kernel time."""
    torch = _torch()
    cfg = I.WORKLOADS[workload]
    mech = I.make_mechanism(workload)
    m = mri.Mech(mech)
    m.specialize(128, load=True)
    y, rho, L, N, ld = stage_inputs(workload)
    opts = mri.fast_opts(n_sub=cfg.n_sub)
    ref = torch.empty_like(y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mri.mri_fast_stage(m, opts, N, ld, y, ref, 1, rho, L)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(repeats):
        mri.mri_fast_stage(m, opts, N, ld, y, ref, 1, rho, L)
    e1.record()
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / repeats
    sg = mri.Surrogate([mri.MLP_KPAD, 256, 256, 256, mri.MLP_OUTPUTS], params, stats)
    raw = torch.empty_like(y)
    sg.infer(N, ld, y, raw, 1, rho, L)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(repeats):
        sg.infer(N, ld, y, raw, 1, rho, L)
    e1.record()
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / repeats
    ws = torch.empty(mri.Surrogate.workspace_bytes(N, ld, 1) // 8 + 1, dtype=torch.float64,
                     device="cuda")
    used = torch.zeros(ld, dtype=torch.int32, device="cuda")
    gv = torch.zeros(ld, dtype=torch.float32, device="cuda")
    out = torch.empty_like(y)
    nf = sg.stage(m, opts, gate_tol, N, ld, y, out, 1, rho, L, ws, used, gv)
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        t1 = time.perf_counter()
        nf = sg.stage(m, opts, gate_tol, N, ld, y, out, 1, rho, L, ws, used, gv)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t1) * 1e3)
    t_sur = float(np.median(times))
    err = stage_error(out[:, :N], ref[:, :N], mech.n_species)
    err6 = stage_error(out[:, :N], ref[:, :N], mech.n_species, floor=1e-6)
    acc = used[:N] == 0
    n_acc = int(acc.sum().item())
    err_raw = stage_error(raw[:, :N], ref[:, :N], mech.n_species)

    def q(x, p):
        return float(torch.quantile(x.float()[:1 << 24], p).item()) if x.numel() else None

    # fair comparison: the cheapest plain substep count whose stage result is
    # within gate_tol of the workload's own (n_sub) result on every cell
    cheapest = None
    alt = torch.empty_like(y)
    for n_sub in sorted(c for c in (5, 8, 10, 13, 16, 20, 25, 32, 40) if c < cfg.n_sub):
        o2 = mri.fast_opts(n_sub=n_sub)
        mri.mri_fast_stage(m, o2, N, ld, y, alt, 1, rho, L)
        torch.cuda.synchronize()
        e = float(torch.nan_to_num(stage_error(alt[:, :N], ref[:, :N], mech.n_species),
                                   nan=float("inf")).max().item())
        if e <= gate_tol:
            e0.record()
            mri.mri_fast_stage(m, o2, N, ld, y, alt, 1, rho, L)
            e1.record()
            torch.cuda.synchronize()
            cheapest = dict(n_sub=n_sub, max_err=e, ms=round(e0.elapsed_time(e1), 3))
            break
    res = dict(cells=N, gate_tol=gate_tol, fallback_cells=int(nf), fallback_frac=nf / N,
               accepted_cells=n_acc,
               false_accepts=int(((err > gate_tol) & acc).sum().item()),
               max_err_accepted=float(err[acc].max().item()) if n_acc else None,
               p999_err_accepted=q(err[acc], 0.999) if n_acc else None,
               max_err_accepted_floor_1e6=float(err6[acc].max().item()) if n_acc else None,
               max_err_all=float(err.max().item()),
               raw_err_median=q(err_raw, 0.5), raw_err_p90=q(err_raw, 0.9),
               raw_frac_within_tol=float((err_raw <= gate_tol).float().mean().item()),
               plain_ms=round(t_plain, 3), surrogate_stage_ms=round(t_sur, 3),
               infer_ms=round(t_inf, 4), speedup=round(t_plain / t_sur, 3),
               plain_cheapest_within_tol=cheapest)
    log(f"# surrogate stage on {N} cells at gate {gate_tol:g}: fallback {nf / N:.3f}, "
        f"false accepts {res['false_accepts']}, plain {t_plain:.2f} ms, gated {t_sur:.2f} ms, "
        f"one inference {t_inf:.3f} ms")
    return res
