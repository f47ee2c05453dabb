"""Kernel micro-benchmark of libfock on one GPU (used for rocprofv3 runs).

    python -m paper_2606_05297_amd.kbench [--workload kk_l8_d8|bh_l8_d6] [--iters N] [--kernels ...]

Runs each kernel family on seeded synthetic states of the workload's size,
rotating three state buffers (working set larger than the 256 MiB Infinity
Cache at L=8, d=8), and prints per-kernel launches, average duration (HIP
events on the launch stream) and algorithmic GB/s.  A plain device copy of
one state is timed alongside as the bandwidth reference.
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

NAMES = {0: "apply_h", 1: "pool_grads", 2: "gate2", 3: "gate2_adjoint", 4: "diag_gate", 6: "mlp_forward",
         7: "mlp_train_step", 8: "gate2_dense_mfma", 9: "score"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="kk_l8_d8")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--kernels", default="copy,apply_h,pool,score,gate,adjoint,m4,dense,mlp")
    ap.add_argument("--mlp-batch", type=int, default=16384)
    ap.add_argument("--lib", default=None, help="path of an alternative libfock.so build")
    ap.add_argument("--schedule", type=int, default=None, help="stencil tile schedule (fock_set_stencil_schedule)")
    ap.add_argument("--stencil", type=int, default=None, help="H psi work split (fock_set_stencil_variant)")
    ap.add_argument("--store-L", type=int, default=None,
                    help="adapt_store leg: chain length of the Kitaev-Kerr run (default: the workload's L)")
    ap.add_argument("--store-steps", type=int, default=4, help="adapt_store leg: ADAPT steps per run")
    ap.add_argument("--hot", action="store_true",
                    help="apply H psi to one state and one output buffer every time (input stays cache-resident, "
                         "as inside an ADAPT step) instead of rotating over three")
    args = ap.parse_args()
    import numpy as np
    import torch

    import workload as W
    from paper_2606_05297_amd import lib

    torch.cuda.set_device(0)
    if args.lib:
        lib.load(args.lib)
    if args.schedule is not None:
        lib.set_stencil_schedule(args.schedule)
    if args.stencil is not None:
        lib.set_stencil_variant(args.stencil)
    cfg = W.config(args.workload)
    h = lib.ham_from(cfg)
    L, d = cfg["L"], cfg["d"]
    n = d**L
    sector = cfg["sector"]
    states = [torch.from_numpy(W.random_state(L, d, seed=s, sector=sector)).to("cuda") for s in range(3)]
    outs = [torch.empty_like(states[0]) for _ in range(3)]
    ws = lib.workspace(h, len(cfg["pool"]), 64)
    want = set(args.kernels.split(","))
    res = {}
    lib.prof_reset()
    lib.prof_enable(True)
    if "copy" in want:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        outs[0].copy_(states[0])
        torch.cuda.synchronize()
        ev0.record()
        for k in range(args.iters):
            outs[k % 3].copy_(states[k % 3])
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.iters
        res["copy"] = {"avg_us": ms * 1e3, "GBs": 16.0 * n / (ms * 1e-3) / 1e9}
        print(f"[kbench] copy done", file=sys.stderr, flush=True)
    if "stream" in want:
        # streaming ceiling: 1 GiB buffers (4x the 256 MiB Infinity Cache) and, for
        # contrast, 128 MiB buffers that stay cache-resident between launches
        res["stream"] = {}
        for mib in (1024, 128):
            a = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
            b = torch.empty_like(a).fill_(2.0)
            for grid in (1024, 4096, 16384):
                for kind, name, mult in ((0, "copy", 2), (1, "read", 1), (2, "update", 2)):
                    ms = lib.stream_probe(kind, a, b, grid=grid, iters=max(5, args.iters // 2))
                    res["stream"][f"{name}_{mib}MiB_g{grid}"] = {
                        "avg_us": ms * 1e3, "GBs": mult * (mib << 20) / (ms * 1e-3) / 1e9}
            del a, b
        torch.cuda.synchronize()
        print(f"[kbench] stream done", file=sys.stderr, flush=True)
    if "apply_h" in want:
        for k in range(args.iters):
            j = 0 if args.hot else k % 3
            lib.apply_H(h, states[j], outs[j], ws, energy=(k == args.iters - 1))
        print(f"[kbench] apply_h done", file=sys.stderr, flush=True)
    if "pool" in want:
        for k in range(3):
            lib.apply_H(h, states[k], outs[k], ws, energy=False)
        for k in range(args.iters):
            lib.pool_grads(h, cfg["pool"], states[k % 3], outs[k % 3], ws)
        print(f"[kbench] pool done", file=sys.stderr, flush=True)
    if "score" in want:
        for k in range(args.iters):
            lib.score(h, cfg["pool"], states[k % 3], outs[k % 3], ws)
        print(f"[kbench] score done", file=sys.stderr, flush=True)
    if "gate" in want:
        pairs = [(0, 1), (3, 4), (L - 2, L - 1), (1, 2)]
        types = ["HR", "PR"] if cfg["Delta"] != 0 else ["HR", "DH"]
        for k in range(args.iters):
            for (i, j) in pairs:
                for t in types:
                    lib.apply_gate2(L, d, (t, i, j), 0.37, states[k % 3], ws)
        torch.cuda.synchronize()
        print(f"[kbench] gate done", file=sys.stderr, flush=True)
    if "dense" in want:
        lib.set_gate_variant(lib.GATE_DENSE_MFMA)
        pairs = [(0, 1), (3, 4), (L - 2, L - 1), (1, 2)]
        types = ["HR", "PR"] if cfg["Delta"] != 0 else ["HR", "DH"]
        for k in range(max(1, args.iters // 2)):
            for (i, j) in pairs:
                for t in types:
                    lib.apply_gate2(L, d, (t, i, j), 0.37, states[k % 3], ws)
        torch.cuda.synchronize()
        lib.set_gate_variant(lib.GATE_BLOCK)
        print(f"[kbench] dense done", file=sys.stderr, flush=True)
    if "adjoint" in want:
        ops, th = W.random_circuit(cfg["pool"], 8, seed=3)
        for k in range(max(1, args.iters // 4)):
            lib.energy_grad_adjoint(h, ops, th, states[k % 3], outs[(k + 1) % 3], outs[(k + 2) % 3], ws)
        print(f"[kbench] adjoint done", file=sys.stderr, flush=True)
    if "m4" in want:
        # one energy + adjoint-gradient evaluation of a 30-gate circuit (gates drawn
        # from the pool with default_rng(3), angles U[-0.5, 0.5]) on the complex64
        # tensor, against the plain method's central-difference gradient (2n energy
        # evaluations); then a 30-gate HR / PR circuit on real parity-halved states,
        # gate by gate and with fused runs.  Wall time per call (results on the host).
        nm4, reps = 30, max(3, args.iters // 4)
        rng = np.random.default_rng(3)
        pool = cfg["pool"]
        ops = [pool[k] for k in rng.integers(0, len(pool), nm4)]
        th = rng.uniform(-0.5, 0.5, nm4)
        ws30 = lib.workspace(h, 0, nm4)

        def per_call(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        t_adj = per_call(lambda: lib.energy_grad_adjoint(h, ops, th, states[0], outs[1], outs[2], ws30))
        t_en = per_call(lambda: lib.energy_grad_adjoint(h, ops, th, states[0], outs[1], outs[2], ws30, grad=False))
        m4 = {"n": nm4, "complex_full": {
            "adjoint_ms": 1e3 * t_adj, "algorithmic_GB": (48 * nm4 + 16) * n / 1e9,
            "GBs": (48 * nm4 + 16) * n / t_adj / 1e9, "energy_ms": 1e3 * t_en,
            "fd_gradient_ms": 1e3 * 2 * nm4 * t_en, "adjoint_speedup_vs_fd": 2 * nm4 * t_en / t_adj}}
        if L == 8 and d == 8 and not cfg["periodic"]:
            rp = [o for o in pool if o[0] in ("HR", "PR")]
            ops_r = [rp[k] for k in rng.integers(0, len(rp), nm4)]
            half = torch.empty(n // 2, dtype=torch.complex64, device="cuda")
            sr = states[0].real.to(torch.complex64)
            sr /= torch.linalg.vector_norm(sr)
            lib.sector_pack(L, d, lib.LAYOUT_EVEN, sr, half)
            x0 = half.real.contiguous()
            a, b = torch.empty_like(x0), torch.empty_like(x0)
            hr = lib.ham_from(cfg, layout=lib.LAYOUT_EVEN | lib.LAYOUT_REAL)
            wsr = lib.workspace(hr, 0, nm4)
            for mode, name in ((lib.RFUSE_OFF, "real_halved_gate_by_gate"), (lib.RFUSE_ON, "real_halved_fused")):
                lib.set_real_fusion(mode)
                t = per_call(lambda: lib.energy_grad_adjoint(hr, ops_r, th, x0, a, b, wsr))
                m4[name] = {"adjoint_ms": 1e3 * t, "runs": len(lib.real_fusion_plan(hr, ops_r)),
                            "algorithmic_GB": (24 * nm4 + 8) * (n // 2) / 1e9}
            lib.set_real_fusion(lib.RFUSE_ON)
        res["m4"] = m4
        print(f"[kbench] m4 done", file=sys.stderr, flush=True)
    if "mlp" in want:
        B = args.mlp_batch
        rng = np.random.default_rng(0)
        X = torch.from_numpy(rng.uniform(0, 1, (B, 4)).astype(np.float32)).cuda()
        T = torch.from_numpy(rng.normal(0, 0.3, (B, 64)).astype(np.float32)).cuda()
        nv = torch.from_numpy(rng.integers(1, 65, B).astype(np.int32)).cuda()
        net = lib.Mlp(B, W.mlp_init(0))
        Y = torch.empty((B, 64), dtype=torch.float32, device="cuda")
        for k in range(args.iters):
            net.forward(X, Y)
            net.adam_step(X, T, nv, 1e-3)
        torch.cuda.synchronize()
        net.close()
        print(f"[kbench] mlp done", file=sys.stderr, flush=True)
    if "adapt_store" in want:
        # ADAPT steps with the forward-state store off and on, alternating twice
        # (Kitaev-Kerr chain of the workload's parameters, nearest-neighbour pool)
        Ls = args.store_L or L
        cs = dict(cfg, L=Ls, pool=W.pool(Ls, "nn", False, W.KITAEV_TYPES))
        hs = lib.ham_from(cs)
        p0 = torch.zeros(d**Ls, dtype=torch.complex64, device="cuda")
        p0[0] = 1.0
        res["adapt_store"] = []
        lib.prof_enable(False)
        for mode in (lib.STORE_OFF, lib.STORE_ON, lib.STORE_OFF, lib.STORE_ON):
            lib.set_state_store(mode)
            ad = lib.Adapt(hs, cs["pool"], p0, max_iters=60, recycle_hessian=True)
            lib.prof_reset()
            lib.prof_enable(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = [ad.step() for _ in range(args.store_steps)]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lib.prof_enable(False)
            us = {}
            for nm, kid in (("gate2", 2), ("gate2_adjoint", 3), ("apply_h", 0)):
                q = lib.prof_query(kid)
                us[nm] = 1e3 * q["ms"] / q["launches"] if q["launches"] else None
            res["adapt_store"].append({"L": Ls, "store": mode, "states_kept": ad.state_store(),
                                       "steps_per_s": args.store_steps / dt, "E": rs[-1]["E"],
                                       "bfgs_evals": int(sum(r["bfgs_evals"] for r in rs)), "avg_us": us})
            ad.close()
        lib.set_state_store(lib.STORE_AUTO)
        lib.prof_reset()
        print(f"[kbench] adapt_store done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    lib.prof_enable(False)
    for kid, name in NAMES.items():
        p = lib.prof_query(kid)
        if p["launches"]:
            avg = p["ms"] / p["launches"]
            res[name] = {"launches": p["launches"], "avg_us": avg * 1e3,
                         "GBs": (p["bytes"] / p["launches"]) / (avg * 1e-3) / 1e9}
            if kid in (6, 7):  # recorded "bytes" are the kernels' algorithmic FLOPs
                res[name] = {"launches": p["launches"], "avg_us": avg * 1e3, "batch": args.mlp_batch,
                             "TFLOPs": (p["bytes"] / p["launches"]) / (avg * 1e-3) / 1e12}
                res[name]["mfma_frac_bf16"] = res[name]["TFLOPs"] / 2500.0
            if kid == 8:  # dense GEMM: (2 d^2)^2 x 2 flop per fibre, d^(L-2) fibres
                fl = (2 * d * d) ** 2 * 2 * d ** (L - 2)
                res[name]["TFLOPs"] = fl / (avg * 1e-3) / 1e12
                res[name]["mfma_frac_fp32"] = res[name]["TFLOPs"] / 157.3
    print(json.dumps({"workload": args.workload, "iters": args.iters, "schedule": lib.get_stencil_schedule(),
                      "stencil": lib.get_stencil_variant(), "kernels": res}), flush=True)


if __name__ == "__main__":
    main()
