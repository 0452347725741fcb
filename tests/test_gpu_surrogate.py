"""GPU checks of the surrogate: MFMA GEMM layout, forward and gradients against
the oracle MLP (bfloat16-emulating mode), the fused inference kernel against
the training forward, Adam, the gate's limiting cases and a short training run."""
import math

import numpy as np
import pytest

from paper_2211_03293_amd import inputs as I

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


def _rand_net(widths, seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [(rng.normal(size=(widths[l + 1], widths[l])) * scale / math.sqrt(widths[l])).astype(np.float32)
          for l in range(len(widths) - 1)]
    bs = [(rng.normal(size=widths[l + 1]) * 0.1).astype(np.float32) for l in range(len(widths) - 1)]
    return Ws, bs, rng


def _pack(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(Ws, bs)]).astype(np.float32)


def _relnorm(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_single_layer_gemm_is_exact_in_bf16_inputs(torch, mri, oracle_mod):
    """Y = X W^T + b with bf16 X and W: FP32 accumulation of exact bf16 products."""
    widths = [77, 45]
    Ws, bs, rng = _rand_net(widths, 1)
    X = rng.normal(size=(133, 77)).astype(np.float32)
    Xq = oracle_mod.bf16_round(X)
    Wq = oracle_mod.bf16_round(Ws[0])
    net = mri.MLP(widths, _pack(Ws, bs), max_batch=133)
    Xd = torch.as_tensor(Xq, device="cuda").to(torch.bfloat16)
    Y = torch.empty((133, 45), dtype=torch.float32, device="cuda")
    net.forward(Xd, Y)
    torch.cuda.synchronize()
    ref = Xq.astype(np.float64) @ Wq.astype(np.float64).T + bs[0]
    np.testing.assert_allclose(Y.cpu().numpy(), ref, rtol=2e-5, atol=2e-5)


def test_mlp_forward_and_gradients_match_oracle(torch, mri, oracle_mod):
    O = oracle_mod
    widths = [89, 256, 256, 256, 22]
    Ws, bs, rng = _rand_net(widths, 2)
    p = _pack(Ws, bs)
    B = 192
    X = O.bf16_round(rng.normal(size=(B, 89)).astype(np.float32))
    T = rng.normal(size=(B, 22)).astype(np.float32)
    net = mri.MLP(widths, p, max_batch=B)
    Xd = torch.as_tensor(X, device="cuda").to(torch.bfloat16)
    Y = torch.empty((B, 22), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.forward(Xd, Y)
    net.backward(torch.as_tensor(T, device="cuda"), loss)
    torch.cuda.synchronize()
    y_o = O.mlp_forward(widths, p.astype(np.float64), X.astype(np.float64), bf16=True)
    l_o, g_o = O.mlp_loss_grad(widths, p.astype(np.float64), X.astype(np.float64),
                               T.astype(np.float64), bf16=True)
    e_fwd = _relnorm(Y.cpu().numpy(), y_o)
    assert e_fwd < 5e-3, e_fwd
    assert loss.item() == pytest.approx(l_o, rel=1e-2)
    g = net.grads()
    off = 0
    worst = 0.0
    for l in range(4):
        ni, no = widths[l], widths[l + 1]
        for sz in (no * ni, no):
            e = _relnorm(g[off:off + sz], g_o[off:off + sz])
            worst = max(worst, e)
            off += sz
    print(f"forward rel err {e_fwd:.2e}, worst gradient tensor rel err {worst:.2e}")
    assert worst < 2e-2, worst


def test_adam_step(torch, mri):
    widths = [8, 4]
    Ws, bs, rng = _rand_net(widths, 3)
    p0 = _pack(Ws, bs)
    net = mri.MLP(widths, p0, max_batch=16)
    X = torch.as_tensor(rng.normal(size=(16, 8)), dtype=torch.bfloat16, device="cuda")
    T = torch.as_tensor(rng.normal(size=(16, 4)), dtype=torch.float32, device="cuda")
    net.forward(X)
    net.backward(T)
    torch.cuda.synchronize()
    g = net.grads().astype(np.float64)
    net.adam_step(1e-2, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    m = 0.1 * g
    v = 0.001 * g * g
    ref = p0 - 1e-2 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    np.testing.assert_allclose(net.params(), ref, rtol=1e-5, atol=1e-6)


def _cells(torch, mri, n_cells, seed):
    mech = I.make_mechanism(I.FIELD64)
    rng = np.random.Generator(np.random.PCG64(seed))
    y = I.independent_cells(n_cells, mech.n_species, rng)
    rho = (rng.normal(size=(1, *y.shape)) * 1e3)
    rho[:, :mech.n_species] -= rho[:, :mech.n_species].mean(axis=1, keepdims=True)
    return mech, y, rho


@pytest.mark.parametrize("n_poly", [1, 2])
def test_fused_inference_matches_training_forward(torch, mri, n_poly):
    """The fused kernel (activations in registers, permuted inputs) reproduces the
    training-path forward on the same features, for the full and both half
    stages; with two forcing terms the half stages see the forcing polynomial
    re-expanded on each half (first half: r0 + r1 tau/2; second half:
    r0 + r1/2 + r1 tau/2), which the training path is given explicitly."""
    widths = [89, 256, 256, 256, 22]
    Ws, bs, rng = _rand_net(widths, 5)
    p = _pack(Ws, bs)
    mech, y, rho1 = _cells(torch, mri, 1000, 6)
    rho = np.concatenate([rho1, 0.5 * rho1[::-1, ::-1]]) if n_poly == 2 else rho1
    n, ld = y.shape
    yd = torch.as_tensor(y, device="cuda")
    rd = torch.as_tensor(rho, device="cuda")
    L = 3e-8
    stats = torch.empty(mri.MLP_STATS, dtype=torch.float64, device="cuda")
    Lv = torch.full((ld,), L, dtype=torch.float64, device="cuda")
    mri.mri_mlp_feature_stats(1000, ld, yd, n_poly, rd, Lv, yd, stats)
    st = stats.cpu().numpy()
    st[2 * 89 + 2 * 22:] = rng.uniform(0.5, 2.0, 22) * 1e-3      # y_std
    st[2 * 89:2 * 89 + 22] = rng.normal(size=22) * 1e-4         # y_mean
    stats = torch.as_tensor(st, device="cuda")
    sg = mri.Surrogate(widths, p, st)
    # the training path reads 96 padded feature columns
    W1p = np.zeros((256, 96), np.float32)
    W1p[:, :89] = Ws[0]
    net = mri.MLP([96] + widths[1:], _pack([W1p] + Ws[1:], bs), max_batch=ld)
    X = torch.empty((ld, 96), dtype=torch.bfloat16, device="cuda")
    Y = torch.empty((ld, 22), dtype=torch.float32, device="cuda")
    for half, Lh in ((0, L), (1, 0.5 * L), (2, 0.5 * L)):
        out = torch.empty_like(yd)
        sg.infer(1000, ld, yd, out, n_poly, rd, L, half=half)
        Lv.fill_(Lh)
        rh = rho.copy()
        if n_poly == 2 and half == 1:
            rh[1] = 0.5 * rho[1]
        elif n_poly == 2 and half == 2:
            rh[0] = rho[0] + 0.5 * rho[1]
            rh[1] = 0.5 * rho[1]
        mri.mri_mlp_featurize(ld, None, ld, yd, n_poly, torch.as_tensor(rh, device="cuda"), Lv,
                              None, stats, X)
        net.forward(X, Y)
        torch.cuda.synchronize()
        d = st[2 * 89:2 * 89 + 22][:, None] + st[2 * 89 + 44:][:, None] * Y.cpu().numpy().T.astype(np.float64)
        # species: log-increment of Y + 1e-8; T: plain increment
        d_out = np.log(np.maximum(out.cpu().numpy()[:22] + 1e-8, 1e-300)) - np.log(np.maximum(y[:22], 0) + 1e-8)
        d_out[21] = out.cpu().numpy()[21] - y[21]
        e = _relnorm(d_out[:, :1000], d[:, :1000])
        print(f"half={half}: fused vs training forward rel err {e:.2e}")
        assert e < 2e-2


def test_gate_limits(torch, mri):
    """gate_tol = 0 sends every cell to the FP64 fallback (bitwise the plain
    stage); gate_tol = inf accepts every cell (the doubled prediction)."""
    widths = [89, 256, 256, 256, 22]
    Ws, bs, rng = _rand_net(widths, 7, scale=0.5)
    p = _pack(Ws, bs)
    mech, y, rho = _cells(torch, mri, 700, 8)
    n, ld = y.shape
    st = np.zeros(mri.MLP_STATS)
    st[89:2 * 89] = 1.0
    st[2 * 89 + 22:2 * 89 + 44] = 1.0
    st[2 * 89 + 44:] = 1e-6
    sg = mri.Surrogate(widths, p, st)
    m = mri.Mech(mech)
    yd = torch.as_tensor(y, device="cuda")
    rd = torch.as_tensor(rho, device="cuda")
    L = 2e-8
    opts = mri.fast_opts(n_sub=10)
    plain = torch.empty_like(yd)
    mri.mri_fast_stage(m, opts, 700, ld, yd, plain, 1, rd, L)
    ws = torch.empty(mri.Surrogate.workspace_bytes(700, ld, 1) // 8 + 1, dtype=torch.float64,
                     device="cuda")
    used = torch.zeros(ld, dtype=torch.int32, device="cuda")
    out = torch.zeros_like(yd)
    nf = sg.stage(m, opts, 0.0, 700, ld, yd, out, 1, rd, L, ws, used)
    torch.cuda.synchronize()
    assert nf == 700 and int(used[:700].sum().item()) == 700
    assert torch.equal(out[:, :700], plain[:, :700])
    out2 = torch.zeros_like(yd)
    nf = sg.stage(m, opts, float("inf"), 700, ld, yd, out2, 1, rd, L, ws, used)
    mid = torch.empty_like(yd)
    dbl = torch.empty_like(yd)
    sg.infer(700, ld, yd, mid, 1, rd, L, half=1)
    sg.infer(700, ld, mid, dbl, 1, rd, L, half=2)
    torch.cuda.synchronize()
    assert nf == 0 and int(used[:700].sum().item()) == 0
    assert torch.equal(out2[:, :700], dbl[:, :700])
    # in place (y_out aliases y_in) gives the same result
    yy = yd.clone()
    sg.stage(m, opts, 0.0, 700, ld, yy, yy, 1, rd, L, ws)
    torch.cuda.synchronize()
    assert torch.equal(yy[:, :700], plain[:, :700])


def test_trained_network_gain(torch, mri):
    """What training buys, on every cell of the first fast stage of the 128^3
    workload (errors judged against the plain FP64 stage): the trained network's
    median stage error is far below the untrained one's; the gated stage at
    1e-4 returns the plain FP64 result bitwise on every rejected cell and never
    accepts a cell the gate should not (mass-sum residual and step doubling both
    within the tolerance); with the gate open it is several times faster than
    the plain stage at a median error of a few per mille."""
    from paper_2211_03293_amd import surrogate as S
    import time
    data = S.generate_stage_data(n_full=200_000, log=print)
    res = S.train(data, steps=4000, batch=4096, log=print, log_every=2000)
    del data
    cfg = I.WORKLOADS[I.FIELD128]
    mech = I.make_mechanism(I.FIELD128)
    m = mri.Mech(mech)
    m.specialize(128, load=True)
    y, rho, L, N, ld = S.stage_inputs(I.FIELD128)
    opts = mri.fast_opts(n_sub=cfg.n_sub)
    ref = torch.empty_like(y)
    mri.mri_fast_stage(m, opts, N, ld, y, ref, 1, rho, L)
    widths = [mri.MLP_KPAD, 256, 256, 256, mri.MLP_OUTPUTS]
    med = {}
    for name, params in (("untrained", S.init_params()), ("trained", res["params"])):
        sg = mri.Surrogate(widths, params, res["stats"])
        out = torch.empty_like(y)
        sg.infer(N, ld, y, out, 1, rho, L)
        torch.cuda.synchronize()
        err = S.stage_error(out[:, :N], ref[:, :N], mech.n_species)
        med[name] = float(torch.median(err).item())
    print(f"median stage error: untrained {med['untrained']:.3e}, trained {med['trained']:.3e}")
    assert med["trained"] < 0.1 * med["untrained"]
    assert med["trained"] < 2e-2
    sg = mri.Surrogate(widths, res["params"], res["stats"])
    ws = torch.empty(mri.Surrogate.workspace_bytes(N, ld, 1) // 8 + 1, dtype=torch.float64,
                     device="cuda")
    used = torch.zeros(ld, dtype=torch.int32, device="cuda")
    gv = torch.zeros(ld, dtype=torch.float32, device="cuda")
    out = torch.empty_like(y)
    nf = sg.stage(m, opts, 1e-4, N, ld, y, out, 1, rho, L, ws, used, gv)
    torch.cuda.synchronize()
    rej = used[:N] == 1
    assert int(rej.sum().item()) == nf
    assert torch.equal(out[:, :N][:, rej], ref[:, :N][:, rej])
    acc = ~rej
    assert bool((gv[:N][acc] <= 1e-4).all().item())
    print(f"gate 1e-4: {nf} of {N} cells fall back to the plain FP64 stage")
    # gate open: every cell takes the doubled prediction
    times = {}
    for name, fn in (("plain", lambda: mri.mri_fast_stage(m, opts, N, ld, y, ref, 1, rho, L)),
                     ("open gate", lambda: sg.stage(m, opts, float("inf"), N, ld, y, out, 1, rho,
                                                    L, ws, used, gv))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) * 1e3
    err = S.stage_error(out[:, :N], ref[:, :N], mech.n_species)
    med_open = float(torch.median(err).item())
    print(f"plain {times['plain']:.2f} ms, open gate {times['open gate']:.2f} ms, "
          f"median error {med_open:.3e}")
    assert times["open gate"] * 2.0 < times["plain"]
    assert med_open < 2e-2
