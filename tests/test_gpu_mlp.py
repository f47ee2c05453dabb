"""Warm-start network on the GPU (fock_mlp_*, bf16 MFMA kernels) against the
FP64 oracle of the same precision contract, and the warm start's effect on
held-out ADAPT runs.

Tolerances: both sides round the same quantities to bf16, but the device
rounds FP32 values accumulated in another order than the oracle's FP64
values, so a value lying within ~1e-7 relative of a bf16 rounding boundary can
round the other way (one bf16 ulp = 2^-8 relative).  Such flips are rare and
each moves one hidden activation by one ulp, so
  * forward: |Y - Y_oracle| <= 5e-3 max|Y| elementwise, and the median
    difference <= 1e-5 max|Y| (FP32 accumulation);
  * loss: relative 1e-5; gradients: ||g - g_oracle|| <= 1e-2 ||g_oracle||
    for every parameter block (error signals are bf16 too);
  * Adam: the FP32 update equals the FP64 one to 1e-6 relative.
"""
import sys

import numpy as np
import pytest
import torch

import workload as W
from oracle import mlp_oracle as M
from paper_2606_05297_amd import lib

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def batch(B, seed):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0.5, 1.5, B), rng.uniform(0, 1, B), rng.uniform(0, 0.5, B),
                  rng.integers(1, 65, B) / 64.0], axis=1).astype(np.float32)
    T = rng.normal(0, 0.4, size=(B, 64)).astype(np.float32)
    n = rng.integers(1, 65, size=B).astype(np.int32)
    return X, T, n


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


BLOCKS = [(name, int(np.prod(s))) for name, s in M.SHAPES]


@pytest.mark.parametrize("B", [1, 63, 64, 200, 1000])
def test_forward_parity(B):
    say("mlp forward", B)
    p = W.mlp_init(11) * 1.5
    X, _, _ = batch(B, B)
    net = lib.Mlp(1024, p)
    Y = net.forward(cuda(X)).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(p.astype(np.float64), X.astype(np.float64))
    scale = np.abs(ref).max()
    d = np.abs(Y - ref)
    assert d.max() <= 5e-3 * scale, d.max() / scale
    assert np.median(d) <= 1e-5 * scale
    net.close()


@pytest.mark.parametrize("B", [37, 512, 4096])
def test_loss_and_gradient_parity(B):
    say("mlp gradient", B)
    p = W.mlp_init(5) * 1.5
    X, T, n = batch(B, 100 + B)
    net = lib.Mlp(4096, p)
    L, g = net.loss_grad(cuda(X), cuda(T), cuda(n))
    Lr, gr = M.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n)
    assert abs(L - Lr) <= 1e-5 * Lr
    o = 0
    for name, sz in BLOCKS:
        a, b = g[o:o + sz].astype(np.float64), gr[o:o + sz]
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), (name, np.linalg.norm(a - b) / np.linalg.norm(b))
        o += sz
    net.close()


def test_adam_step_parity_and_param_roundtrip():
    say("mlp adam")
    p = W.mlp_init(2)
    X, T, n = batch(300, 9)
    net = lib.Mlp(512, p)
    assert np.array_equal(net.params(), p)
    _, g = net.loss_grad(cuda(X), cuda(T), cuda(n))
    net.adam_step(cuda(X), cuda(T), cuda(n), 1e-3)
    got = net.params().astype(np.float64)
    want, _, _ = M.adam_step(p.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, 1e-3)
    assert np.abs(got - want).max() <= 1e-6 * max(1.0, np.abs(want).max())
    # a second step uses the carried moments (t = 2)
    _, g2 = net.loss_grad(cuda(X), cuda(T), cuda(n))
    m = 0.1 * g.astype(np.float64)
    v = 0.001 * g.astype(np.float64) ** 2
    net.adam_step(cuda(X), cuda(T), cuda(n), 1e-3)
    want2, _, _ = M.adam_step(got, g2.astype(np.float64), m, v, 2, 1e-3)
    assert np.abs(net.params() - want2).max() <= 1e-6 * max(1.0, np.abs(want2).max())
    net.close()


def test_training_reduces_loss_and_rejects_bad_batches():
    say("mlp training")
    rng = np.random.default_rng(4)
    B = 2048
    X = np.stack([np.ones(B), rng.uniform(0, 1, B), rng.uniform(0, 0.5, B), rng.integers(1, 65, B) / 64],
                 axis=1).astype(np.float32)
    k = np.arange(64)[None, :]
    T = (0.5 * np.sin(3 * X[:, 1:2] + 0.1 * k) * X[:, 2:3] + 0.2 * X[:, 3:4]).astype(np.float32)
    n = (X[:, 3] * 64).round().astype(np.int32)
    net = lib.Mlp(B, W.mlp_init(0))
    Xd, Td, nd = cuda(X), cuda(T), cuda(n)
    L0, _ = net.loss_grad(Xd, Td, nd, grad=False)
    for _ in range(300):
        net.adam_step(Xd, Td, nd, 3e-3)
    L1, _ = net.loss_grad(Xd, Td, nd, grad=False)
    say("loss", L0, "->", L1)
    assert L1 < 0.05 * L0
    with pytest.raises(lib.FockError):
        net.forward(cuda(np.zeros((B + 1, 4), np.float32)))
    with pytest.raises(lib.FockError):
        net.adam_step(Xd, Td[:, :32].contiguous(), nd, 1e-3)
    net.close()


def test_warm_start_gain_on_held_out_points():
    """Reduced warm-start study: the network trained on the converged angles
    of 48 training points proposes the starting angles of 8 held-out points
    ("delta" proposals: own angles plus the predicted re-optimisation shift,
    network angle for the new slot).  Asserted: training fits, the library's
    fallback rule holds for every accepted proposal (start energy not above
    the plain start), the network is accepted on most of the first four steps
    (where the held-out points share their operator sequence with the
    training points), and accepted starts are strictly lower on average.
    BFGS iterations with and without the network are printed (not asserted:
    a start that is lower in energy but not converged in the old angles does
    not shorten BFGS)."""
    from paper_2606_05297_amd import warmstart as WS
    steps = 8
    tr = W.warmstart_points("train")[:48]
    he = W.warmstart_points("held")[:8]
    say("warm start: data")
    _, ang = WS.run_sweep(tr, steps)
    X, T, n = WS.dataset(tr, ang)
    say("warm start: train", len(X))
    net, hist = WS.train(X, T, n, epochs=800, batch=256, lr=2e-3)
    say("loss", hist[0], hist[-1])
    assert hist[-1][1] < 0.5 * hist[0][1]
    say("warm start: plain vs proposals")
    plain, _ = WS.run_sweep(he, steps)
    warm, _ = WS.run_sweep(he, steps, net=net, mode="delta")
    sp, sw = WS.summarise(plain), WS.summarise(warm)
    say("plain", {k: v for k, v in sp.items() if k != "final_E"})
    say("warm", {k: v for k, v in sw.items() if k != "final_E"})
    nacc = 0
    for r in warm:
        for x in r:
            if x.get("accepted"):
                nacc += 1
                assert x["E_prop"] <= x["E_plain"]
    assert nacc > 0
    assert sw["acceptance_steps_1_4"] >= 0.5
    assert sw["mean_start_energy_gain_accepted"] > 0.0
    net.close()


def test_warm_start_after_selection_on_nearby_points_l6():
    """The benchmark's warm-start procedure at L=6, d=8 (262,144 amplitudes):
    plain ADAPT on 8 points around (Delta, K) = (0.5, 0.2) by the batched
    sweep, training on the steps that follow the majority operator sequence,
    then 12 steps of the centre point with proposals after selection, against
    the same 12 steps without the network (both with Hessian recycling).
    Asserted: training fits; every kept proposal starts no higher than the
    plain start; the network's run selects the same operators and ends at the
    same energy (1e-5 relative); BFGS evaluations with and without the network
    are printed with the proposal counts."""
    from paper_2606_05297_amd import warmstart as WS
    steps = 12
    cfg = dict(W.config("kk_l8_d8"), L=6, pool=W.pool(6, "nn", False, W.KITAEV_TYPES))
    h = lib.ham_from(cfg)
    psi0 = torch.zeros(8**6, dtype=torch.complex64, device="cuda")
    psi0[0] = 1.0
    rng = np.random.default_rng(5)
    pts = [dict(cfg, Delta=cfg["Delta"] * f1, K=cfg["K"] * f2) for f1, f2 in rng.uniform(0.9, 1.1, (8, 2))]
    say("warm start after selection: data")
    recs, ang = WS.run_sweep(pts, steps)
    seq, agree = WS.consensus(recs)
    X, T, nv = WS.dataset_agreeing(pts, ang, agree)
    say("samples", len(X), "sequence", seq, "agree", agree)
    net, hist = WS.train(X, T, nv, epochs=300, batch=256)
    assert hist[-1][1] < 0.5 * hist[0][1]
    plain, _, _, _ = WS.adapt_with_network(cfg, h, psi0, steps, net, [], recycle_hessian=True)
    warm, made, kept, _ = WS.adapt_with_network(cfg, h, psi0, steps, net, seq, recycle_hessian=True)
    net.close()
    for r in warm:
        if r.get("accepted"):
            assert r["E_prop"] <= r["E_plain"]
    assert made > 0 and kept > 0
    ep = sum(r["bfgs_evals"] for r in plain)
    ew = sum(r["bfgs_evals"] for r in warm)
    same = [r["k_sel"] for r in warm] == [r["k_sel"] for r in plain]
    say(f"BFGS evaluations over {steps} steps: plain {ep}, with network {ew}; proposals {made}, kept {kept}; "
        f"same operators: {same}; final E plain {plain[-1]['E']:.8f}, with network {warm[-1]['E']:.8f}")
