"""CV-ADAPT-VQE at the paper's own parameters (Sec. V): energy error against
exact diagonalisation as a function of the number of ADAPT gates.

    python -m paper_2606_05297_amd.paper_runs [--gates 160] [--cases name,...] [--out file]

Cases: workload.paper_cases() (Kitaev chain N_S = 3..5 at mu = -3.1 and -2.7,
Kitaev chain with Kerr term, Bose-Hubbard N_S = 4 with 12 bosons at
Lambda = +-4).  Each run appends operators until `gates` have been added or
the energy error drops below 1e-10 (the paper's stopping rule; the gradient
threshold is disabled), with the inverse Hessian recycled across steps.
Exact ground energies: tests/golden/paper_cases_ed.json (written from the FP64
oracle by tests/golden/make_ed_reference.py --paper-cases).  States are
complex64, so the energy error levels off near 1e-6 |E0| instead of the
paper's 1e-10.  Prints one JSON line per case.
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


def fock_vector(L, d, occ):
    import torch

    import workload as W

    x = torch.zeros(d**L, dtype=torch.complex64)
    x[W.fock_index(L, d, occ)] = 1.0
    return x.to("cuda")


def run_case(p, E0, gates, log):
    import workload as W
    from paper_2606_05297_amd import lib

    h = lib.ham(p["L"], p["d"], p["periodic"], p["J"], p["U"], p["mu"], p["Delta"], p["K"])
    wops = W.warmup_ops(p["L"], p["periodic"]) if p["warm"] else []
    wth = W.warmup_theta0(len(wops), p["warm_seed"]) if p["warm"] else np.zeros(0)
    ad = lib.Adapt(h, p["pool"], fock_vector(p["L"], p["d"], p["occ"]), max_iters=gates, grad_tol=1e-14,
                   warm_ops=wops, warm_theta0=wth, recycle_hessian=True)
    dE, iters, sel = [], [], []
    t0 = time.perf_counter()
    for k in range(gates):
        r = ad.step()
        dE.append(abs(r["E"] - E0))
        iters.append(int(r["bfgs_iters"]))
        if r["k_sel"] >= 0:
            sel.append(p["pool"][r["k_sel"]][0])
        if log and (k + 1) % 20 == 0:
            log(f"{p['name']}: {k + 1} gates, dE = {dE[-1]:.3e}")
        if r["converged"] or r["capped"] or dE[-1] < 1e-10:
            break
    dt = time.perf_counter() - t0
    ad.close()
    dE = np.array(dE)

    def first_below(t):
        k = np.nonzero(dE < t * abs(E0))[0]
        return int(k[0]) + 1 if k.size else None

    return {"case": p["name"], "L": p["L"], "d": p["d"], "E0": E0, "warmup_gates": len(wops),
            "pool_size": len(p["pool"]), "gates": int(dE.size), "dE": [float(x) for x in dE],
            "dE_min": float(dE.min()), "gates_to_rel_1e-3": first_below(1e-3), "gates_to_rel_1e-5": first_below(1e-5),
            "bfgs_iters": iters, "selected_types": {t: sel.count(t) for t in sorted(set(sel))}, "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gates", type=int, default=160)
    ap.add_argument("--cases", default=None, help="comma-separated case names (default: all)")
    ap.add_argument("--ed", default=os.path.join(ROOT, "tests", "golden", "paper_cases_ed.json"))
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch

    import workload as W

    torch.cuda.set_device(0)
    ed = json.load(open(args.ed))
    want = set(args.cases.split(",")) if args.cases else None

    def log(m):
        print(f"[paper_runs] {m}", file=sys.stderr, flush=True)

    lines = []
    for p in W.paper_cases():
        if want and p["name"] not in want:
            continue
        res = run_case(p, ed[p["name"]]["E0"], args.gates, log)
        line = json.dumps(res)
        print(line, flush=True)
        lines.append(line)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
