"""CV-ADAPT-VQE at the paper's own parameters (Sec. V): energy error against
exact diagonalisation as a function of the number of ADAPT gates.

    python -m paper_2606_05297_amd.paper_runs [--gates 160] [--cases name,...] [--fp64 [--two-param]]
        [--warm-seeds 0,1,...] [--warm-fixed] [--no-hessian-recycling] [--out file]

Cases: workload.paper_cases() (Kitaev chain N_S = 3..5 at mu = -3.1 and -2.7,
Kitaev chain with Kerr term, Bose-Hubbard N_S = 4 with 12 bosons at
Lambda = +-4).  Each run appends operators until `gates` have been added or
the energy error drops below 1e-10 (the paper's stopping rule; the gradient
threshold is disabled), with the inverse Hessian recycled across steps
(--no-hessian-recycling: every BFGS starts from the identity).
Exact ground energies: tests/golden/paper_cases_ed.json (written from the FP64
oracle by tests/golden/make_ed_reference.py --paper-cases).  complex64 states
(default) stop resolving the per-iteration BFGS gains near 1e-7 |E|; --fp64
runs the complex128 driver (adapt64_*), which follows the paper's convergence.
--two-param (with --fp64) takes the paper's two-parameter pool (beam splitter
and two-mode squeezer on every pair, single-mode squeezer and rotation on
every site, plus the Kerr-type terms where the Hamiltonian has them).
--warm-seeds 0,1,... runs each case with a warm-up layer once per seed of its
initial warm-up angles (the paper keeps the best seed per configuration,
Appendix C); --warm-fixed (with --fp64) keeps those angles fixed instead of
optimising them (Appendix D compares both).  Prints one JSON line per run.
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


def fock_vector(L, d, occ, dtype="complex64"):
    import torch

    import workload as W

    x = torch.zeros(d**L, dtype=getattr(torch, dtype))
    x[W.fock_index(L, d, occ)] = 1.0
    return x.to("cuda")


def run_case(p, E0, gates, log, fp64=False, two_param=False, warm_fixed=False, recycle=True):
    import workload as W
    from paper_2606_05297_amd import lib

    h = lib.ham(p["L"], p["d"], p["periodic"], p["J"], p["U"], p["mu"], p["Delta"], p["K"])
    wops = W.warmup_ops(p["L"], p["periodic"]) if p["warm"] else []
    wth = W.warmup_theta0(len(wops), p["warm_seed"]) if p["warm"] else np.zeros(0)
    pool = p["pool2"] if two_param else p["pool"]
    if fp64:
        ad = lib.Adapt64(h, pool, fock_vector(p["L"], p["d"], p["occ"], dtype="complex128"), max_iters=gates,
                         grad_tol=1e-14, recycle_hessian=recycle, warm_ops=wops, warm_theta0=wth,
                         warm_fixed=warm_fixed and bool(wops))
    else:
        ad = lib.Adapt(h, p["pool"], fock_vector(p["L"], p["d"], p["occ"]), max_iters=gates, grad_tol=1e-14,
                       warm_ops=wops, warm_theta0=wth, recycle_hessian=recycle)
    ad_warm = ad.warm_report()
    dE, iters, sel, npar = [], [], [], 0
    t0 = time.perf_counter()
    for k in range(gates):
        r = ad.step()
        dE.append(abs(r["E"] - E0))
        iters.append(int(r["bfgs_iters"]))
        npar = int(r["n_params"])
        if r["k_sel"] >= 0:
            sel.append(pool[r["k_sel"]][0])
        if log and (k + 1) % 5 == 0:
            log(f"{p['name']} (warm-up seed {p['warm_seed']}): {k + 1} gates, dE = {dE[-1]:.3e}")
        if r["converged"] or r["capped"] or dE[-1] < 1e-10:
            break
    dt = time.perf_counter() - t0
    ad.close()
    dE = np.array(dE)

    def first_below(t):
        k = np.nonzero(dE < t * abs(E0))[0]
        return int(k[0]) + 1 if k.size else None

    return {"case": p["name"], "state": "complex128" if fp64 else "complex64", "L": p["L"], "d": p["d"], "E0": E0,
            "warmup_gates": len(wops), "warm_seed": p["warm_seed"] if p["warm"] else None,
            "warmup": ("fixed" if warm_fixed else "optimised") if wops else None, "hessian_recycling": recycle,
            "E_after_warmup": float(ad_warm["E"]),
            "pool": "two-parameter" if two_param else "one-parameter", "pool_size": len(pool), "gates": int(dE.size),
            "params": npar, "dE": [float(x) for x in dE],
            "dE_min": float(dE.min()), "gates_to_rel_1e-3": first_below(1e-3), "gates_to_rel_1e-5": first_below(1e-5),
            "bfgs_iters": iters, "selected_types": {t: sel.count(t) for t in sorted(set(sel))}, "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gates", type=int, default=160)
    ap.add_argument("--cases", default=None, help="comma-separated case names (default: all)")
    ap.add_argument("--ed", default=os.path.join(ROOT, "tests", "golden", "paper_cases_ed.json"))
    ap.add_argument("--out", default=None)
    ap.add_argument("--fp64", action="store_true",
                    help="complex128 states (adapt64_*)")
    ap.add_argument("--two-param", action="store_true", help="the two-parameter pool (needs --fp64)")
    ap.add_argument("--warm-fixed", action="store_true",
                    help="keep the warm-up angles at their seeded initial values (needs --fp64)")
    ap.add_argument("--no-hessian-recycling", action="store_true",
                    help="start every BFGS from the identity instead of the previous inverse Hessian")
    ap.add_argument("--warm-seeds", default=None,
                    help="comma-separated seeds of the warm-up angles, one run each (cases with a warm-up layer; "
                         "default: the case's own seed)")
    args = ap.parse_args()
    if (args.two_param or args.warm_fixed) and not args.fp64:
        ap.error("--two-param and --warm-fixed need --fp64")
    import torch

    import workload as W

    torch.cuda.set_device(0)
    ed = json.load(open(args.ed))
    want = set(args.cases.split(",")) if args.cases else None

    def log(m):
        print(f"[paper_runs] {m}", file=sys.stderr, flush=True)

    if args.out:
        open(args.out, "w").close()
    for p in W.paper_cases():
        if want and p["name"] not in want:
            continue
        if args.two_param and "pool2" not in p:
            log(f"{p['name']}: skipped (no two-parameter pool)")
            continue
        seeds = [p["warm_seed"]]
        if p["warm"] and args.warm_seeds:
            seeds = [int(x) for x in args.warm_seeds.split(",")]
        for seed in seeds:
            q = dict(p, warm_seed=seed)
            res = run_case(q, ed[p["name"]]["E0"], args.gates, log, fp64=args.fp64, two_param=args.two_param,
                           warm_fixed=args.warm_fixed, recycle=not args.no_hessian_recycling)
            line = json.dumps(res)
            print(line, flush=True)
            if args.out:  # one line per finished run, so a cut-off call keeps what it finished
                with open(args.out, "a") as fh:
                    fh.write(line + "\n")


if __name__ == "__main__":
    main()
