"""Operator tiling (Appendix B): learn which pool operators matter on a small
lattice with CV-ADAPT-VQE, then tile them over a larger lattice.

An operator's *shape* is its generator type and its relative geometry: the
mode distance j - i of a two-mode operator (on a ring of L sites the ring
distance min(j - i, L - (j - i)), so that translated copies share a shape),
or nothing for a single-mode one.
Tiling a set of shapes over a lattice takes every operator of that lattice's
full pool whose shape is in the set, in the full pool's order (so the tie
break of the selection rule, lowest pool index, acts as on the full pool).

    learn_shapes(...)   steps 1-3: ADAPT on the small lattice; after every
                        step, every operator whose gradient is within the
                        selection tie band of the largest is collected (the
                        operators the selection could equally have chosen)
    tile_pool(...)      step 4
    learn_shapes64(...) steps 1-3 on complex128 states (the shapes of the
                        operators ADAPT selects; on a ring, translated copies
                        share a shape, so the selection covers them)

Every gradient, energy and BFGS evaluation runs on the GPU through the C ABI.

    python -m paper_2606_05297_amd.tiling --small bkc_N4_mu-3.1 --large bkc_N5_mu-3.1 [--gates 160]

learns shapes on the small paper case (complex128), tiles the large case's pool
and runs complex128 ADAPT with the tiled pool; prints one JSON line (shapes,
pool sizes, energy errors against tests/golden/paper_cases_ed.json).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from . import lib


def shape_of(op, ring_L: int | None = None) -> tuple:
    """(type, distance); ring_L: the number of sites of a periodic lattice."""
    t, i, j = op
    if j < 0:
        return (t, None)
    dist = j - i
    return (t, min(dist, ring_L - dist) if ring_L else dist)


def ring_of(h) -> int | None:
    """Number of sites if the Hamiltonian's chain is a ring (periodic, L >= 3)."""
    return h.L if h.periodic and h.L >= 3 else None


def learn_shapes(h, pool, psi0, steps: int, tie: float = 1e-4, max_iters: int = 60, warm_ops=(),
                 warm_theta0=(), grad_tol: float = 1e-3) -> tuple[set, list]:
    """Runs up to `steps` ADAPT iterations of the small-lattice problem and
    returns (shapes, selected), `selected` being the operators ADAPT chose.

    Before each step the pool gradients are evaluated on the current ansatz
    state; every operator with |g_k| >= (1 - tie) max |g| contributes its shape
    (this covers operators related by a lattice symmetry, whose gradients are
    degenerate with the selected one)."""
    import torch

    L, d = h.L, h.d
    ring = ring_of(h)
    ad = lib.Adapt(h, pool, psi0, max_iters=max_iters, warm_ops=warm_ops, warm_theta0=warm_theta0,
                   grad_tol=grad_tol)
    n_amp = d**L
    a = torch.empty(n_amp, dtype=torch.complex64, device=psi0.device)
    b = torch.empty_like(a)
    ws = lib.workspace(h, len(pool), max_iters + len(warm_ops) + 1)
    shapes, selected = set(), []
    try:
        for _ in range(steps):
            ops, th = ad.ansatz()
            lib.energy_grad_adjoint(h, ops, th, psi0, a, b, ws, grad=False)  # a = psi, b = H psi
            g = np.abs(lib.pool_grads(h, pool, a, b, ws))
            if g.max() > 0:
                for k in np.nonzero(g >= (1.0 - tie) * g.max())[0]:
                    shapes.add(shape_of(pool[int(k)], ring))
            rep = ad.step()
            if rep["k_sel"] >= 0:
                selected.append(pool[rep["k_sel"]])
                shapes.add(shape_of(pool[rep["k_sel"]], ring))
            if rep["converged"] or rep["capped"]:
                break
    finally:
        ad.close()
    return shapes, selected


def tile_pool(full_pool, shapes, ring_L: int | None = None) -> list:
    """The operators of `full_pool` whose shape was learned, in pool order
    (ring_L: the large lattice's size if it is a ring)."""
    return [op for op in full_pool if shape_of(op, ring_L) in shapes]


def learn_shapes64(h, pool, psi0, max_iters: int, E0: float | None = None, stop_dE: float = 1e-10,
                   **adapt_kw) -> tuple[set, list]:
    """ADAPT on complex128 states (lib.Adapt64) for up to `max_iters` steps, or
    until E - E0 < stop_dE when E0 is given; returns (shapes of the selected
    operators, the selected operators)."""
    ring = ring_of(h)
    ad = lib.Adapt64(h, pool, psi0, max_iters=max_iters, **adapt_kw)
    shapes, selected = set(), []
    try:
        for _ in range(max_iters):
            r = ad.step()
            if r["k_sel"] >= 0:
                selected.append(pool[r["k_sel"]])
                shapes.add(shape_of(pool[r["k_sel"]], ring))
            if r["converged"] or r["capped"] or (E0 is not None and r["E"] - E0 < stop_dE):
                break
    finally:
        ad.close()
    return shapes, selected


def main():
    import argparse

    import torch

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workload as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--small", required=True, help="paper case to learn on (workload.paper_cases name)")
    ap.add_argument("--large", required=True, help="paper case to tile to")
    ap.add_argument("--gates", type=int, default=160)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    ed = json.load(open(os.path.join(root, "tests", "golden", "paper_cases_ed.json")))
    cases = {c["name"]: c for c in W.paper_cases()}
    small, large = cases[args.small], cases[args.large]

    def setup(p):
        h = lib.ham(p["L"], p["d"], p["periodic"], p["J"], p["U"], p["mu"], p["Delta"], p["K"])
        psi0 = torch.zeros(p["d"] ** p["L"], dtype=torch.complex128)
        psi0[W.fock_index(p["L"], p["d"], p["occ"])] = 1.0
        return h, psi0.to("cuda")

    kw = dict(grad_tol=1e-14, recycle_hessian=True)
    hs, ps = setup(small)
    shapes, _ = learn_shapes64(hs, small["pool"], ps, args.gates, E0=ed[small["name"]]["E0"], **kw)
    tiled = tile_pool(large["pool"], shapes, ring_of(lib.ham(large["L"], large["d"], large["periodic"])))
    hl, pl = setup(large)
    E0 = ed[large["name"]]["E0"]
    ad = lib.Adapt64(hl, tiled, pl, max_iters=args.gates, **kw)
    dE = []
    try:
        for _ in range(args.gates):
            r = ad.step()
            dE.append(r["E"] - E0)
            if r["converged"] or r["capped"] or dE[-1] < 1e-10:
                break
    finally:
        ad.close()
    print(json.dumps({"small": args.small, "large": args.large, "shapes": sorted(map(list, shapes), key=str),
                      "pool_full": len(large["pool"]), "pool_tiled": len(tiled), "dE": dE}), flush=True)


if __name__ == "__main__":
    main()
