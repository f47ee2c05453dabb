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

Every gradient, energy and BFGS evaluation runs on the GPU through the C ABI.
"""
from __future__ import annotations

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
