"""Learned warm start for ADAPT on the Kitaev-Kerr chain (L=6, d=8, open).

    python -m paper_2606_05297_amd.warmstart [--train 256] [--held 64] [--steps 64]
           [--epochs 400] [--out report.json]

1. Data: the batched sweep runs plain ADAPT (initial angles {theta_prev, 0})
   on the training points; after every step n the converged angles theta^(n)
   become one sample: features (J, Delta, K, n / 64) -> target theta^(n)
   padded to 64, with the first n entries valid.
2. Training: the network 4 -> 128 -> 128 -> 64 (libfock fock_mlp_*: bf16
   MFMA forward and backward kernels, Adam on FP32 master weights) on the GPU,
   mini-batches from a seeded permutation.
3. Evaluation on held-out points: the plain sweep and a sweep that, before
   every step n + 1, proposes the network's first n + 1 angles for
   (J, Delta, K, (n + 1) / 64); the library keeps a proposal only if its
   energy is not above the plain start, so the method never gets worse at the
   start of a step.  Reported: proposal acceptance rate, BFGS iterations and
   evaluations per step, ADAPT iterations to the gradient threshold (or the
   cap), final energies, and |E - E_ED| where exact energies are supplied.

Every GPU computation runs in libfock; this module only moves arrays.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NOUT = 64


def _entries(points, lib, torch):
    out = []
    for p in points:
        n = p["d"] ** p["L"]
        psi0 = torch.zeros(n, dtype=torch.complex64, device="cuda")
        psi0[0] = 1.0  # vacuum
        out.append(dict(ham=lib.ham_from(p), pool=p["pool"], psi0=psi0, warm_ops=[], warm_theta0=np.zeros(0)))
    return out


def run_sweep(points, steps, net=None, grid=None, log=None, mode="delta"):
    """ADAPT on every point for up to `steps` iterations (batched sweep);
    with `net`, proposals from the network before every step.  Returns per
    point the list of step records and the angles after every step.

    Proposal for step n + 1 of a point with current angles theta (n of them)
    and network outputs y(m) = net(J, Delta, K, m / 64):
      mode "full":  y(n + 1)[: n + 1];
      mode "delta": theta + y(n + 1)[: n] - y(n)[: n] for the existing angles
                    (the network's predicted re-optimisation shift) and
                    y(n + 1)[n] for the new one."""
    import torch

    from paper_2606_05297_amd import lib
    import workload as W

    sw = lib.Sweep(_entries(points, lib, torch), max_iters=steps)
    if grid:
        sw.set_grid(grid)
    npts = len(points)
    recs = [[] for _ in range(npts)]
    angles = [[] for _ in range(npts)]
    done = [False] * npts
    nparams = [0] * npts
    Xp = torch.zeros((npts, 4), dtype=torch.float32, device="cuda")
    for it in range(steps + 1):
        if all(done):
            break
        if net is not None:
            feats = np.stack([W.mlp_features(p["J"], p["Delta"], p["K"], nparams[k] + 1) for k, p in enumerate(points)])
            Xp.copy_(torch.from_numpy(feats))
            Y = net.forward(Xp).cpu().numpy().astype(np.float64)
            if mode == "delta":
                feats0 = np.stack([W.mlp_features(p["J"], p["Delta"], p["K"], nparams[k]) for k, p in enumerate(points)])
                Xp.copy_(torch.from_numpy(feats0))
                Y0 = net.forward(Xp).cpu().numpy().astype(np.float64)
            for k in range(npts):
                m = nparams[k]
                if done[k] or m + 1 > NOUT:
                    continue
                if mode == "delta" and m > 0:
                    th = np.append(angles[k][-1] + Y[k, :m] - Y0[k, :m], Y[k, m])
                else:
                    th = Y[k, :m + 1]
                sw.propose(k, th)
        reps, na = sw.step()
        for k in range(npts):
            if done[k]:
                continue
            r = dict(reps[k])
            if net is not None and r["k_sel"] >= 0:
                r.update(sw.last_proposal(k))
            recs[k].append(r)
            if r["converged"] or r["capped"]:
                done[k] = True
                continue
            _, th = sw.ansatz(k)
            nparams[k] = len(th)
            angles[k].append(th.copy())
        if log:
            log(f"step {it + 1}: active {na}")
    sw.close()
    return recs, angles


def dataset(points, angles):
    """Samples (features, padded target, number of valid targets) from the
    converged angles of every step."""
    import workload as W

    X, T, n = [], [], []
    for p, ang in zip(points, angles):
        for th in ang:
            m = len(th)
            if m > NOUT:
                continue
            X.append(W.mlp_features(p["J"], p["Delta"], p["K"], m))
            t = np.zeros(NOUT, dtype=np.float32)
            t[:m] = th
            T.append(t)
            n.append(m)
    return np.array(X, dtype=np.float32), np.array(T, dtype=np.float32), np.array(n, dtype=np.int32)


def consensus(recs):
    """Majority operator sequence of the training trajectories and, per point,
    how many of its first steps follow it.  A slot-wise angle regression only
    means something while the circuits agree, so training keeps those steps."""
    seq, agree = [], [0] * len(recs)
    alive = list(range(len(recs)))
    step = 0
    while alive:
        ks = [recs[k][step]["k_sel"] for k in alive if step < len(recs[k]) and recs[k][step]["k_sel"] >= 0]
        if not ks:
            break
        vals, cnt = np.unique(ks, return_counts=True)
        best = int(vals[np.argmax(cnt)])
        seq.append(best)
        nxt = []
        for k in alive:
            if step < len(recs[k]) and recs[k][step]["k_sel"] == best:
                agree[k] = step + 1
                nxt.append(k)
        alive = nxt
        step += 1
    return seq, agree


def dataset_agreeing(points, angles, agree):
    """dataset() restricted to each point's first agree[k] steps."""
    return dataset(points, [ang[:a] for ang, a in zip(angles, agree)])


def adapt_with_network(cfg, h, psi0, steps, net, seq, **adapt_kw):
    """Steps 1..steps of one ADAPT run (lib.Adapt on ham h from device psi0)
    where every step selects first and, while the chosen circuit follows the
    operator sequence seq the network was trained on, proposes previous
    angles + the network's predicted shift and its predicted new angle
    ("delta"), kept by the library only if not above the plain start.
    Returns (step reports, proposals made, proposals kept, seconds)."""
    import torch

    from paper_2606_05297_amd import lib
    import workload as W

    Xd = torch.zeros((2, 4), dtype=torch.float32, device="cuda")
    ad = lib.Adapt(h, cfg["pool"], psi0, max_iters=cfg["max_iters"], **adapt_kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps, made, kept, on_seq = [], 0, 0, True
    for step in range(steps):
        sel = ad.select()
        if sel["converged"] or sel["capped"]:
            reps.append(sel)
            break
        n = sel["n_params"] - 1
        on_seq = on_seq and step < len(seq) and sel["k_sel"] == seq[step]
        use = on_seq and n + 1 <= NOUT
        if use:
            Xd.copy_(torch.from_numpy(np.stack([W.mlp_features(cfg["J"], cfg["Delta"], cfg["K"], n + 1),
                                                W.mlp_features(cfg["J"], cfg["Delta"], cfg["K"], max(n, 1))])))
            Y = net.forward(Xd).cpu().numpy().astype(np.float64)
            _, th = ad.ansatz()
            ad.propose(np.append(th[:n] + Y[0, :n] - Y[1, :n], Y[0, n]) if n > 0 else Y[0, :1])
            made += 1
        r = ad.finish()
        if use:
            r.update(ad.last_proposal())
            kept += int(r["accepted"])
        reps.append(r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ad.close()
    return reps, made, kept, dt


def train(X, T, n, epochs=400, batch=1024, lr=2e-3, seed=0, log=None):
    """Adam on the GPU; returns (network, loss history per epoch)."""
    import torch

    from paper_2606_05297_amd import lib
    import workload as W

    B = len(X)
    net = lib.Mlp(max(batch, B), W.mlp_init(seed))
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    nd = torch.from_numpy(n).cuda()
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(B)).cuda()
        for b0 in range(0, B, batch):
            idx = perm[b0:b0 + batch]
            net.adam_step(Xd[idx].contiguous(), Td[idx].contiguous(), nd[idx].contiguous(), lr)
        if ep % 50 == 0 or ep == epochs - 1:
            loss, _ = net.loss_grad(Xd, Td, nd, grad=False)
            hist.append((ep, loss))
            if log:
                log(f"epoch {ep}: loss {loss:.3e}")
    return net, hist


def summarise(recs):
    it = [len(r) for r in recs]
    steps = [x for r in recs for x in r if x["k_sel"] >= 0]
    out = {
        "adapt_steps_total": len(steps),
        "bfgs_iters_per_step": float(np.mean([x["bfgs_iters"] for x in steps])) if steps else 0.0,
        "bfgs_evals_per_step": float(np.mean([x["bfgs_evals"] for x in steps])) if steps else 0.0,
        "converged_points": int(sum(1 for r in recs if r and r[-1]["converged"])),
        "iterations_per_point": float(np.mean(it)),
        "final_E": [r[-1]["E"] if r else None for r in recs],
    }
    acc = [x["accepted"] for x in steps if "accepted" in x]
    if acc:
        out["proposal_acceptance"] = float(np.mean(acc))
        for lo, hi in ((1, 4), (5, 16), (17, 64)):
            a = [x["accepted"] for x in steps if "accepted" in x and lo <= x["iter"] <= hi]
            if a:
                out[f"acceptance_steps_{lo}_{hi}"] = float(np.mean(a))
        gain = [x["E_plain"] - x["E_prop"] for x in steps if x.get("accepted")]
        out["mean_start_energy_gain_accepted"] = float(np.mean(gain)) if gain else 0.0
    for lo, hi in ((1, 4), (5, 16), (17, 64)):
        it = [x["bfgs_iters"] for x in steps if lo <= x["iter"] <= hi]
        if it:
            out[f"bfgs_iters_steps_{lo}_{hi}"] = float(np.mean(it))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--held", type=int, default=64)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--mode", choices=["full", "delta"], default="delta")
    ap.add_argument("--ed", default=None, help="JSON with exact energies of the held-out points (list 'E0')")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch

    import workload as W

    torch.cuda.set_device(0)

    def log(m):
        print(f"[warmstart] {m}", file=sys.stderr, flush=True)

    tr = W.warmstart_points("train")[: args.train]
    he = W.warmstart_points("held")[: args.held]
    t0 = time.perf_counter()
    _, ang = run_sweep(tr, args.steps, log=log)
    t_data = time.perf_counter() - t0
    X, T, n = dataset(tr, ang)
    log(f"{len(X)} samples from {len(tr)} points in {t_data:.1f} s")
    t0 = time.perf_counter()
    net, hist = train(X, T, n, args.epochs, args.batch, args.lr, log=log)
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    plain, _ = run_sweep(he, args.steps, log=log)
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    warm, _ = run_sweep(he, args.steps, net=net, mode=args.mode, log=log)
    t_warm = time.perf_counter() - t0
    rep = {"mode": args.mode, "train_points": len(tr), "held_points": len(he), "max_steps": args.steps, "samples": int(len(X)),
           "loss_history": hist, "t_data_s": t_data, "t_train_s": t_train, "t_plain_s": t_plain, "t_warm_s": t_warm,
           "plain": summarise(plain), "warm": summarise(warm)}
    if args.ed:
        E0 = np.array(json.load(open(args.ed))["E0"])[: len(he)]
        for key in ("plain", "warm"):
            fe = np.array(rep[key]["final_E"], dtype=np.float64)
            rep[key]["mean_abs_dE_vs_ed"] = float(np.mean(np.abs(fe - E0)))
    net.close()
    line = json.dumps(rep)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
