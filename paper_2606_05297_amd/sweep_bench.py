"""Sweep benchmark: the 96-point parameter sweep (Bose-Hubbard L in {4,6,8},
d in {4,6}, U/J log-spaced over [0.5, 20], ring, warm-up layer; Kitaev-Kerr
L in {4,6}, d = 8, seeded (Delta, K), open) run for K ADAPT iterations
(a) point by point with adapt_step and (b) batched with fock_sweep_step
(persistent batched launches, graph-replayed BFGS rounds, autotuned grid).
Creation (incl. the warm-up optimisation) is outside the timed regions.
Prints one JSON line: point-steps per second of both, the speed-up, and
whether every point's energies agree bit for bit.

    python -m paper_2606_05297_amd.sweep_bench [--steps K] [--points N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--points", type=int, default=96)
    ap.add_argument("--cache", default=None, help="autotune cache file (JSON lines)")
    args = ap.parse_args()
    import numpy as np
    import torch

    import workload as W
    from paper_2606_05297_amd import lib

    torch.cuda.set_device(0)
    pts = W.sweep_points()[: args.points]
    entries = []
    for p in pts:
        n = p["d"] ** p["L"]
        psi0 = torch.zeros(n, dtype=torch.complex64, device="cuda")
        psi0[W.fock_index(p["L"], p["d"], p["occ"])] = 1.0
        wops = W.warmup_ops(p["L"], p["periodic"]) if p["warm"] else []
        wth = W.warmup_theta0(len(wops), p["warm_seed"]) if p["warm"] else np.zeros(0)
        entries.append(dict(ham=lib.ham_from(p), pool=p["pool"], psi0=psi0, warm_ops=wops, warm_theta0=wth))
    K = args.steps
    amps = sum(p["d"] ** p["L"] for p in pts)
    print(f"[sweep_bench] {len(pts)} points, {amps} amplitudes, {K} steps", file=sys.stderr, flush=True)

    # (a) point by point, gates one per pass on complex64 states like the batched
    # kernels (bitwise comparable: fusion and real-state evaluations off)
    fused = lib.get_gate_fusion()
    lib.set_gate_fusion(lib.FUSE_OFF)
    lib.set_real_states(lib.REAL_OFF)
    singles = [lib.Adapt(e["ham"], e["pool"], e["psi0"], max_iters=40, warm_ops=e["warm_ops"],
                         warm_theta0=e["warm_theta0"]) for e in entries]
    torch.cuda.synchronize()
    E_seq = np.zeros((len(pts), K))
    steps_seq = 0
    t0 = time.perf_counter()
    for k, a in enumerate(singles):
        for s in range(K):
            r = a.step()
            E_seq[k, s] = r["E"]
            steps_seq += 1
            if r["converged"] or r["capped"]:  # finished: its energy stays
                E_seq[k, s + 1:] = r["E"]
                break
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for a in singles:
        a.close()
    lib.set_gate_fusion(fused)
    lib.set_real_states(lib.REAL_AUTO)
    print(f"[sweep_bench] sequential {t_seq:.2f} s", file=sys.stderr, flush=True)

    # (b) batched
    sw = lib.Sweep(entries, max_iters=40)
    grid = sw.autotune(args.cache)
    torch.cuda.synchronize()
    E_bat = np.zeros((len(pts), K))
    steps_bat = 0
    t0 = time.perf_counter()
    done = np.zeros(len(pts), dtype=bool)
    for s in range(K):
        if done.all():
            break
        reps, na = sw.step()
        steps_bat += na
        for k in range(len(pts)):
            if done[k]:
                continue
            E_bat[k, s:] = reps[k]["E"]
            done[k] = bool(reps[k]["converged"] or reps[k]["capped"])
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    sw.close()
    print(f"[sweep_bench] batched {t_bat:.2f} s (grid {grid})", file=sys.stderr, flush=True)
    out = {"points": len(pts), "amplitudes": amps, "steps": K, "sequential_point_steps_per_s": steps_seq / t_seq,
           "batched_point_steps_per_s": steps_bat / t_bat, "speedup": (steps_bat / t_bat) / (steps_seq / t_seq),
           "bitwise_equal": bool(np.array_equal(E_seq, E_bat)), "autotuned_grid": grid,
           "max_abs_dE": float(np.abs(E_seq - E_bat).max()), "points_finished_early": int(done.sum())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
