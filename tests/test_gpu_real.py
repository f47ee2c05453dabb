"""GPU parity of real-state evaluations (adapt_real): ADAPT runs whose
evaluations run their HR / PR gates and reverse steps on float32 amplitudes,
against the same runs in complex64 (FOCK_REAL_OFF) and against the FP64 oracle
replaying the GPU's own ansatz.

H has real matrix elements and HR, PR are real antisymmetric, so the states
of such runs are real; the two paths differ only by FP32 rounding (and by the
gate tables' imaginary rounding noise, which the real path drops).  Bars: same
selections, energies within 1e-6 relative of the complex run, pool-gradient
norms within 1e-4, and the oracle replay at 1e-5 |E|."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workload as W
from paper_2606_05297_amd import lib

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).to("cuda")


def oham(c):
    return O.Ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"])


def pair_runs(hl, pool, psi0, steps, sector=lib.SECTOR_AUTO, **kw):
    """The same run with real states allowed and switched off."""
    prev = lib.get_sector_layout()
    lib.set_sector_layout(sector)
    try:
        a = lib.Adapt(hl, pool, dev(psi0), **kw)
        lib.set_real_states(lib.REAL_OFF)
        try:
            b = lib.Adapt(hl, pool, dev(psi0), **kw)
        finally:
            lib.set_real_states(lib.REAL_AUTO)
    finally:
        lib.set_sector_layout(prev)
    assert b.real() is False
    ra = rb = None
    for _ in range(steps):
        ra, rb = a.step(), b.step()
        assert ra["k_sel"] == rb["k_sel"]
        assert abs(ra["E"] - rb["E"]) <= 1e-6 * max(1.0, abs(rb["E"]))
        assert abs(ra["g_norm2"] - rb["g_norm2"]) <= 1e-4 * max(1.0, rb["g_norm2"])
        if ra["converged"]:
            break
    return a, b, ra


@pytest.mark.parametrize("sector", [lib.SECTOR_AUTO, lib.SECTOR_OFF], ids=["halved", "full"])
def test_real_states_match_complex_kitaev_l8_d8(sector):
    """The benchmark's run (Kitaev-Kerr L=8 d=8 from the vacuum, Hessian
    recycling) on real states, parity-halved (the default) and full: every gate
    of its ansatz is HR or PR, so every evaluation runs on float32 states."""
    c = W.config("kk_l8_d8")
    ho, hl = oham(c), lib.ham_from(c)
    psi0 = O.fock_state(8, 8, c["occ"])
    say("real vs complex, kk_l8_d8, sector mode", sector)
    a, b, ra = pair_runs(hl, c["pool"], psi0, 6, sector=sector, max_iters=c["max_iters"], recycle_hessian=True)
    assert a.real() is True
    assert a.layout() == (lib.LAYOUT_EVEN if sector == lib.SECTOR_AUTO else lib.LAYOUT_FULL)
    ops, th = a.ansatz()
    assert {o[0] for o in ops} <= {"HR", "PR"}
    psi = O.ansatz_state(psi0, ops, th, 8, 8)
    E = np.vdot(psi, O.apply_H_slices(ho, psi)).real / np.vdot(psi, psi).real
    assert abs(ra["E"] - E) <= 1e-5 * abs(E)
    a.close()
    b.close()


def test_real_states_odd_start_fd_and_small_chains():
    """An odd-parity real start (parity-halved, odd sector) with central-
    difference gradients; an L=6 chain (full layout, pipelined mode-0 real
    kernels); an L=4 chain, whose (0,1) pair has too few fibers for the real
    mode-0 kernel, so evaluations containing it run in complex64."""
    c = W.config("kk_l8_d8")
    odd = O.fock_state(8, 8, [0, 0, 0, 0, 0, 0, 0, 1])
    say("real vs complex: odd start, FD gradients")
    a, b, ra = pair_runs(lib.ham_from(c), c["pool"], odd, 3, max_iters=3, grad_mode=1)
    assert a.real() is True and a.layout() == lib.LAYOUT_ODD
    ops, th = a.ansatz()
    Eo = O.energy_of(oham(c), odd, ops, th)
    assert abs(ra["E"] - Eo) <= 1e-5 * max(1.0, abs(Eo))
    a.close()
    b.close()
    for L in (6, 4):
        cc = dict(L=L, d=8, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.5, K=0.2)
        pool = W.pool(L, "nn", False, W.KITAEV_TYPES)
        psi0 = O.fock_state(L, 8, [0] * L)
        say("real vs complex, L", L)
        a, b, ra = pair_runs(lib.ham_from(cc), pool, psi0, 5, max_iters=8)
        assert a.real() is True and a.layout() == lib.LAYOUT_FULL
        ops, th = a.ansatz()
        Eo = O.energy_of(oham(cc), psi0, ops, th)
        assert abs(ra["E"] - Eo) <= 1e-5 * max(1.0, abs(Eo))
        a.close()
        b.close()


def test_real_states_fallbacks():
    """A complex psi0 keeps no real states; a warm-up layer with HI gates keeps
    them but runs every evaluation in complex64 (its gates are not real), with
    the same results as the run without real states."""
    c = W.config("kk_l8_d8")
    L = 6
    cc = dict(L=L, d=8, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.5, K=0.2)
    hl = lib.ham_from(cc)
    pool = W.pool(L, "nn", False, W.KITAEV_TYPES)
    psi_c = W.random_state(L, 8, seed=3, sector=("parity", 0))
    say("real-state fallbacks")
    a = lib.Adapt(hl, pool, dev(psi_c), max_iters=2)
    assert a.real() is False
    a.close()
    warm = [("HI", 0, 1), ("HI", 2, 3)]
    psi0 = O.fock_state(L, 8, [0] * L)
    a, b, ra = pair_runs(hl, pool, psi0, 3, max_iters=3, warm_ops=warm, warm_theta0=np.array([0.02, -0.03]))
    assert a.real() is True
    ops, th = a.ansatz()
    assert ops[:2] == warm
    Eo = O.energy_of(oham(cc), psi0, ops, th)
    assert abs(ra["E"] - Eo) <= 1e-5 * max(1.0, abs(Eo))
    a.close()
    b.close()
    del c
