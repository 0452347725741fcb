"""Pins for the oracle's surrogate MLP: the backward pass against central finite
differences of the forward loss (FP64), bfloat16 rounding against torch's
conversion, SiLU and its derivative against closed forms, and the BF16 mode
against the FP64 mode within bfloat16 precision."""
import math

import numpy as np
import pytest


def _net(widths, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [rng.normal(size=(widths[l + 1], widths[l])) / math.sqrt(widths[l])
          for l in range(len(widths) - 1)]
    bs = [rng.normal(size=widths[l + 1]) * 0.1 for l in range(len(widths) - 1)]
    return Ws, bs, rng


def test_backward_matches_finite_differences(oracle_mod):
    O = oracle_mod
    widths = [7, 9, 8, 5]
    Ws, bs, rng = _net(widths, 1)
    p = O.mlp_pack(Ws, bs)
    X = rng.normal(size=(6, widths[0]))
    T = rng.normal(size=(6, widths[-1]))
    loss, g = O.mlp_loss_grad(widths, p, X, T)
    idx = rng.choice(p.size, size=60, replace=False)
    for i in idx:
        e = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += e
        pm[i] -= e
        lp, _ = O.mlp_loss_grad(widths, pp, X, T)
        lm, _ = O.mlp_loss_grad(widths, pm, X, T)
        fd = (lp - lm) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])
    # the loss itself is the mean squared error of the forward output
    Y = O.mlp_forward(widths, p, X)
    assert loss == pytest.approx(np.mean((Y - T) ** 2), rel=1e-13)


def test_forward_single_layer_is_affine(oracle_mod):
    O = oracle_mod
    rng = np.random.Generator(np.random.PCG64(2))
    W, b = rng.normal(size=(3, 4)), rng.normal(size=3)
    X = rng.normal(size=(5, 4))
    Y = O.mlp_forward([4, 3], O.mlp_pack([W], [b]), X)
    np.testing.assert_allclose(Y, X @ W.T + b, rtol=1e-14)


def test_bf16_rounding_matches_torch(oracle_mod):
    import torch
    rng = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([rng.normal(size=20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.3895314e38, np.inf,
                                  -np.inf], np.float32)]).astype(np.float32)
    # exact ties: bf16 value +- half an ulp
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ours = oracle_mod.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_silu_and_derivative(oracle_mod):
    for z in (-30.0, -2.5, -1e-3, 0.0, 0.7, 4.0, 25.0):
        assert oracle_mod.silu(z) == pytest.approx(z / (1 + math.exp(-z)), rel=1e-15, abs=1e-300)
        e = 1e-6
        fd = (oracle_mod.silu(z + e) - oracle_mod.silu(z - e)) / (2 * e)
        assert oracle_mod.silu_grad(z) == pytest.approx(fd, rel=1e-7, abs=1e-12)


def test_bf16_mode_tracks_fp64_mode(oracle_mod):
    O = oracle_mod
    widths = [89, 256, 256, 256, 22]
    Ws, bs, rng = _net(widths, 4)
    p = O.mlp_pack(Ws, bs)
    X = rng.normal(size=(16, widths[0]))
    T = rng.normal(size=(16, widths[-1]))
    y64 = O.mlp_forward(widths, p, X)
    y16 = O.mlp_forward(widths, p, X, bf16=True)
    rel = np.linalg.norm(y16 - y64) / np.linalg.norm(y64)
    assert 1e-4 < rel < 3e-2          # bfloat16 carries ~3 significant digits
    _, g64 = O.mlp_loss_grad(widths, p, X, T)
    _, g16 = O.mlp_loss_grad(widths, p, X, T, bf16=True)
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) < 5e-2


def test_bf16_mode_rounding_points_hand_computed(oracle_mod):
    """A 2-2-1 network whose output, worked out by hand, moves when any single
    rounding point of the bfloat16 mode is switched off.

    Hidden pre-activations are near 64, where SiLU(z) = z / (1 + e^-z) equals z
    in double precision (e^-64 < 2^-53), so every step is exact dyadic
    arithmetic.  bfloat16 spacing in [64, 128) is 1/2, FP32 spacing 2^-17.
      x = (1 + 2^-8 + 2^-10, 1) -> bf16 (1 + 2^-7, 1)
      W1 = [[64.375, 0], [0, 64]] -> bf16 [[64.5, 0], [0, 64]],  b1 = (1/4, 0)
      z1 = 64.5 (1 + 2^-7) + 1/4 = 65.25390625 -> bf16 65.5 (above the midpoint
           65.25 between 65 and 65.5);  z2 = 64 -> 64
      W2 = [[1, 2^-30]], b2 = 2^-18 + 2^-44 (the 2^-44 is below FP32
      resolution at 2^-18 but above FP64 resolution at 65.5)
      acc = 65.5 + 2^-24 -> FP32 65.5;  b2 -> FP32 2^-18;
      65.5 + 2^-18 is half an FP32 ulp above 65.5: ties to even -> y = 65.5.
    With one rounding point off:
      input   z1 = 64.5 (1 + 2^-8 + 2^-10) + 1/4 = 65.0649... -> 65   -> y = 65
      weight  z1 = 64.375 (1 + 2^-7) + 1/4 = 65.1279...      -> 65   -> y = 65
      act     h1 = 65.25390625 (no bf16), tie again rounds to even -> y = 65.25390625
      acc     65.5 + 2^-24 + 2^-18 above the tie            -> y = 65.5 + 2^-17
      bias    65.5 + 2^-18 + 2^-44 above the tie            -> y = 65.5 + 2^-17
      sum     65.5 + 2^-18 kept in FP64                     -> y = 65.5 + 2^-18
    """
    O = oracle_mod
    widths = [2, 2, 1]
    W1 = np.array([[64.375, 0.0], [0.0, 64.0]])
    b1 = np.array([0.25, 0.0])
    W2 = np.array([[1.0, 2.0 ** -30]])
    b2 = np.array([2.0 ** -18 + 2.0 ** -44])
    p = O.mlp_pack([W1, W2], [b1, b2])
    X = np.array([[1.0 + 2.0 ** -8 + 2.0 ** -10, 1.0]])
    expect = {
        O.R_ALL: 65.5,
        O.R_ALL & ~O.R_INPUT: 65.0,
        O.R_ALL & ~O.R_WEIGHT: 65.0,
        O.R_ALL & ~O.R_ACT: 65.25390625,
        O.R_ALL & ~O.R_ACC: 65.5 + 2.0 ** -17,
        O.R_ALL & ~O.R_BIAS: 65.5 + 2.0 ** -17,
        O.R_ALL & ~O.R_SUM: 65.5 + 2.0 ** -18,
    }
    for mode, want in expect.items():
        got = O.mlp_forward(widths, p, X, bf16=mode)[0, 0]
        assert got == want, (mode, got, want)
    # True selects every rounding point
    assert O.mlp_forward(widths, p, X, bf16=True)[0, 0] == 65.5
