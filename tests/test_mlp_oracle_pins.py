"""Pins of the warm-start network oracle (oracle/mlp_oracle.py) against
things other than itself: torch's bfloat16 cast (round to nearest even),
float64 central finite differences of the loss, torch.optim.Adam, and a
hand-computed masked-MSE case."""
import numpy as np
import pytest
import torch

import workload as W
from oracle import mlp_oracle as M


def test_bf16_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-38).astype(np.float32),      # subnormal range
        np.array([1 + 2**-8, 1 + 3 * 2**-8, -(1 + 2**-8), 2**-126 * (1 + 2**-8), 3.0, 0.0, -0.0,
                  1 - 2**-9, 65504.0, 1e-40], dtype=np.float32),   # exact ties and edges
    ])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = M.bf16(x.astype(np.float64))
    assert np.array_equal(got, ref)
    # the two ties round to even: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    assert M.bf16(np.array([1 + 2**-8]))[0] == 1.0
    assert M.bf16(np.array([1 + 3 * 2**-8]))[0] == 1 + 2**-6


def test_dsilu_finite_difference():
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.abs(fd - M.dsilu(z)).max() < 1e-8


def _data(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, size=(B, 4))
    T = rng.normal(0, 0.3, size=(B, 64))
    n = rng.integers(1, 65, size=B)
    return X, T, n


def test_backward_matches_finite_differences_unrounded():
    """With the bfloat16 rounding switched off the loss is smooth; the backward
    pass must equal central differences in every parameter block."""
    p = W.mlp_init(3).astype(np.float64) * 2.0
    X, T, n = _data(6, 1)
    L, g = M.loss_and_grad(p, X, T, n, rounding=False)
    assert abs(L - M.loss(p, X, T, n, rounding=False)) < 1e-14
    rng = np.random.default_rng(2)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    idx = np.concatenate([rng.integers(offs[k], offs[k + 1], 40) for k in range(len(M.SHAPES))])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss(p + e, X, T, n, rounding=False) - M.loss(p - e, X, T, n, rounding=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_rounded_gradient_close_to_unrounded():
    """bfloat16 rounding perturbs the gradient only at the 1e-2 relative level."""
    p = W.mlp_init(4).astype(np.float64)
    X, T, n = _data(64, 5)
    _, g0 = M.loss_and_grad(p, X, T, n, rounding=False)
    _, g1 = M.loss_and_grad(p, X, T, n, rounding=True)
    assert np.linalg.norm(g1 - g0) <= 3e-2 * np.linalg.norm(g0)


def test_masked_mse_closed_form():
    """W3 = 0: Y = b3 for every sample, so the loss is the masked mean of
    (b3[k] - T[b,k])^2 over the first n_b entries."""
    p = M.unpack(W.mlp_init(0).astype(np.float64))
    p["W3"][:] = 0.0
    p["b3"][:] = np.linspace(-1, 1, 64)
    flat = M.pack(p)
    T = np.zeros((2, 64))
    T[0, :3] = [0.5, 0.0, 1.0]
    n = np.array([3, 1])
    b = np.linspace(-1, 1, 64)
    want = ((b[0] - 0.5) ** 2 + b[1] ** 2 + (b[2] - 1.0) ** 2 + b[0] ** 2) / 4.0
    assert abs(M.loss(flat, np.zeros((2, 4)), T, n) - want) < 1e-15
    # its gradient with respect to b3: 2 sum_b M (b3 - T) / N (bfloat16-rounded G3)
    _, g = M.loss_and_grad(flat, np.zeros((2, 4)), T, n)
    gb3 = g[-64:]
    ref = np.zeros(64)
    ref[:3] += M.bf16(2 * (b[:3] - T[0, :3]) / 4)
    ref[0] += M.bf16(2 * b[0] / 4)
    assert np.allclose(gb3, ref, atol=0, rtol=0)


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(4)]
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads):
        opt.zero_grad()
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = M.adam_step(p, g, m, v, k + 1, 3e-3)
    assert np.abs(p - t.detach().numpy()).max() < 1e-14


def test_param_count():
    assert M.N_PARAMS == 25408 == len(W.mlp_init(0))
