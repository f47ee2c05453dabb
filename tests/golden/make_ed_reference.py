"""Write tests/golden/ed_reference.json: exact-diagonalisation ground energies
of the benchmark workloads in their symmetry sectors, computed by the FP64
oracle only (dense eigh for small sectors, Lanczos otherwise).

    python tests/golden/make_ed_reference.py [names...]
    python tests/golden/make_ed_reference.py --warmstart-held [--jobs N]
    python tests/golden/make_ed_reference.py --paper-cases

The second form writes tests/golden/warmstart_held_ed.json: the even-parity
ground energies of the 64 held-out Kitaev-Kerr L=6 d=8 warm-start points (in
the order of workload.warmstart_points("held")).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workload as W  # noqa: E402

OUT = os.path.join(HERE, "ed_reference.json")
OUT_HELD = os.path.join(HERE, "warmstart_held_ed.json")
OUT_PAPER = os.path.join(HERE, "paper_cases_ed.json")


def paper_cases():
    """Ground energies of workload.paper_cases() in their sectors (dense eigh)."""
    res = {}
    for p in W.paper_cases():
        h = O.Ham(p["L"], p["d"], p["periodic"], p["J"], p["U"], p["mu"], p["Delta"], p["K"])
        t = time.time()
        gs = O.ground_state(h, p["sector"], want_vector=False, tol=1e-12)
        res[p["name"]] = dict(E0=gs["E0"], sector=list(p["sector"]), dim=int(gs["dim"]),
                              method="eigh" if gs["dim"] <= 20000 else "eigsh", seconds=round(time.time() - t, 1))
        print(p["name"], res[p["name"]], flush=True)
    with open(OUT_PAPER, "w") as f:
        json.dump(res, f, indent=1)


def held_one(k):
    p = W.warmstart_points("held")[k]
    h = O.Ham(p["L"], p["d"], p["periodic"], p["J"], p["U"], p["mu"], p["Delta"], p["K"])
    t = time.time()
    gs = O.ground_state(h, p["sector"], want_vector=False, tol=1e-10)
    print(f"held {k}: Delta={p['Delta']:.4f} K={p['K']:.4f} E0={gs['E0']:.10f} ({time.time() - t:.0f} s)", flush=True)
    return gs["E0"]


def held(jobs):
    from concurrent.futures import ProcessPoolExecutor
    pts = W.warmstart_points("held")
    with ProcessPoolExecutor(jobs) as ex:
        E0 = list(ex.map(held_one, range(len(pts))))
    with open(OUT_HELD, "w") as f:
        json.dump({"E0": E0, "Delta": [p["Delta"] for p in pts], "K": [p["K"] for p in pts],
                   "sector": list(pts[0]["sector"]), "L": pts[0]["L"], "d": pts[0]["d"],
                   "method": "eigsh (tol 1e-10) on the even-parity sector"}, f, indent=1)


def entries():
    c = W.config("bh_l3_d4")
    yield "bh_l3_d4", c, {}
    c = W.config("bh_l8_d6")
    for U in c["U_values"]:
        yield f"bh_l8_d6_U{U:g}", c, {"U": U}
    yield "warm_l6_d8", W.config("warm_l6_d8"), {}
    yield "kk_l8_d8", W.config("kk_l8_d8"), {}


def main(names):
    res = {}
    if os.path.exists(OUT):
        res = json.load(open(OUT))
    for name, c, over in entries():
        if names and name not in names:
            continue
        p = dict(c)
        p.update(over)
        h = O.Ham(p["L"], p["d"], p["periodic"], p["J"], p["U"], p["mu"], p["Delta"], p["K"])
        t = time.time()
        gs = O.ground_state(h, p["sector"], want_vector=False, tol=1e-10)
        res[name] = dict(E0=gs["E0"], sector=list(p["sector"]), dim=int(gs["dim"]),
                         ham=dict(L=h.L, d=h.d, periodic=h.periodic, J=h.J, U=h.U, mu=h.mu, Delta=h.Delta, K=h.K),
                         method="eigh" if gs["dim"] <= 20000 else "eigsh", seconds=round(time.time() - t, 1))
        print(name, res[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    if "--paper-cases" in sys.argv:
        paper_cases()
    elif "--warmstart-held" in sys.argv:
        j = sys.argv.index("--jobs") if "--jobs" in sys.argv else -1
        held(int(sys.argv[j + 1]) if j >= 0 else 4)
    else:
        main(sys.argv[1:])
