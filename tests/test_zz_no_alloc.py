"""The allocation-free H psi entry point (fock_apply_H_noalloc) against
fock_apply_H: two calls in a row, the second on a smaller lattice (the shared
scratch array keeps the first call's partials), both through the C ABI; the
outputs must agree bit for bit, and the device's free memory must not change
across the allocation-free calls."""
import sys

import numpy as np
import pytest
import torch

import workload as W
from paper_2606_05297_amd import lib

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


CASES = [
    # the slab path (L=8, d=8 ring with every term), then a smaller open chain (row kernel)
    dict(L=8, d=8, periodic=True, J=0.8, U=1.1, mu=0.3, Delta=0.45, K=0.15, sector=None, seed=3),
    dict(L=6, d=8, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.5, K=0.2, sector=("parity", 0), seed=4),
]


def test_apply_H_noalloc_matches_apply_H_two_calls():
    lib.load()
    refs = []
    for c in CASES:  # reference results first (fock_apply_H may allocate its staging on first use)
        h = lib.ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"])
        x = torch.from_numpy(W.random_state(c["L"], c["d"], seed=c["seed"], sector=c["sector"])).cuda()
        y = torch.empty_like(x)
        ws = lib.workspace(h, 0, 0)
        E, n2 = lib.apply_H(h, x, y, ws)
        refs.append((h, x, y.clone(), E, n2))
    outs = [(torch.empty_like(x), torch.full((2,), float("nan"), dtype=torch.float64, device="cuda"))
            for (_, x, _, _, _) in refs]
    torch.cuda.synchronize()
    lib.apply_H_noalloc(refs[1][0], refs[1][1], outs[1][0], outs[1][1])  # first use on this device
    torch.cuda.synchronize()
    for yo, res in outs:
        yo.fill_(float("nan"))
        res.fill_(float("nan"))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k in (0, 1):  # large, then smaller: nothing is allocated between the two free-memory reads
        h, x, _, _, _ = refs[k]
        say("noalloc call", k, "L", h.L, "d", h.d)
        lib.apply_H_noalloc(h, x, outs[k][0], outs[k][1])
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for k in (0, 1):
        _, _, y, E, n2 = refs[k]
        yo, res = outs[k]
        assert torch.equal(yo, y), k
        r = res.cpu().numpy()
        assert r[0] == E and r[1] == n2, (k, r, E, n2)
    # without the result buffer only H psi is written
    h, x, y, _, _ = refs[1]
    yo = torch.empty_like(x)
    lib.apply_H_noalloc(h, x, yo)
    torch.cuda.synchronize()
    assert torch.equal(yo, y)
