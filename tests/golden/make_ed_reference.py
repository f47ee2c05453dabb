"""Write tests/golden/ed_reference.json: exact-diagonalisation ground energies
of the benchmark workloads in their symmetry sectors, computed by the FP64
oracle only (dense eigh for small sectors, Lanczos otherwise).

    python tests/golden/make_ed_reference.py [names...]
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
    main(sys.argv[1:])
