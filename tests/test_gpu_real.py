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


def stored_index(L, d, sigma):
    """Full flat index of every stored amplitude of the parity-halved layout
    (from its definition, as in test_gpu_sector.py)."""
    nlow = d ** (L - 1)
    c = np.arange(d**L // 2, dtype=np.int64)
    low, m = c % nlow, c // nlow
    s, x = np.zeros_like(low), low.copy()
    for _ in range(L - 1):
        s += x % d
        x //= d
    return low + (2 * m + (s + sigma) % 2) * nlow


def real_state(seed, sigma=0):
    """A real, normalised state of L=8, d=8 and parity sigma (the real part of
    a seeded sector state)."""
    psi = W.random_state(8, 8, seed=seed, sector=("parity", sigma)).real.astype(np.float64)
    return psi / np.linalg.norm(psi)


HAM = dict(L=8, d=8, periodic=False, J=0.8, U=1.1, mu=0.3, Delta=0.45, K=0.15)
REAL_LAYOUTS = [lib.LAYOUT_FULL | lib.LAYOUT_REAL, lib.LAYOUT_EVEN | lib.LAYOUT_REAL]


def ham_real(layout):
    c = HAM
    return (O.Ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"]),
            lib.ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"], layout=layout))


@pytest.mark.parametrize("layout", REAL_LAYOUTS, ids=["full", "halved"])
def test_real_apply_H_l8_d8(layout):
    """H psi on float32 states (FOCK_LAYOUT_REAL) on every stored amplitude,
    with the energy and norm, against the oracle on the full tensor (open
    chain with hopping, pairing, U, K and mu)."""
    ho, hl = ham_real(layout)
    say("real H psi, layout", layout)
    psi = real_state(81)
    idx = stored_index(8, 8, 0) if layout & 3 else np.arange(8**8)
    x = torch.from_numpy(psi[idx].astype(np.float32)).to("cuda")
    y = torch.full_like(x, float("nan"))
    ws = lib.workspace(hl, 0, 0)
    E, n2 = lib.apply_H(hl, x, y, ws)
    p128 = psi.astype(np.float32).astype(np.complex128)
    href = O.apply_H_slices(ho, p128)
    assert np.abs(href.imag).max() == 0.0
    got = y.cpu().numpy().astype(np.float64)
    hs = href.real[idx]
    assert np.isfinite(got).all()
    assert np.abs(got - hs).max() <= 2e-5 * np.abs(hs).max()
    Eref = np.vdot(p128, href).real
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - np.vdot(p128, p128).real) <= 1e-6


@pytest.mark.parametrize("layout", REAL_LAYOUTS + [lib.LAYOUT_ODD | lib.LAYOUT_REAL], ids=["full", "halved", "odd"])
def test_real_energy_and_adjoint_l8_d8(layout):
    """Energy, final state and every dE/dtheta of an HR / PR circuit on float32
    states (20 gates over all seven bonds, the mode-0 pair and the top pair
    included) against the oracle's FP64 reverse sweep on the full tensor; the
    parity-halved layout in both sectors."""
    ho, hl = ham_real(layout)
    pool = W.pool(8, "nn", False, ("HR", "PR"))
    ops, th = W.random_circuit(pool, 16, seed=91)
    ops = ops + [("HR", 0, 1), ("PR", 0, 1), ("HR", 6, 7), ("PR", 6, 7)]
    th = np.concatenate([th, [0.21, -0.17, 0.33, -0.29]])
    say("real adjoint, layout", layout, len(ops))
    sigma = 1 if (layout & 3) == lib.LAYOUT_ODD else 0
    psi0 = real_state(93, sigma)
    idx = stored_index(8, 8, sigma) if layout & 3 else np.arange(8**8)
    x0 = torch.from_numpy(psi0[idx].astype(np.float32)).to("cuda")
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, 0, len(ops))
    p0 = psi0.astype(np.float32).astype(np.complex128)
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws, grad=False)
    psi_n = O.ansatz_state(p0, ops, th, 8, 8)
    assert np.abs(psi_n.imag).max() < 1e-12
    assert np.abs(a.cpu().numpy() - psi_n.real[idx]).max() <= 1e-5 * np.abs(psi_n).max() * len(ops) ** 0.5
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    Eref, gref, n2ref = O.energy_and_grad_adjoint(ho, p0, ops, th, apply_h=O.apply_H_slices)
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - n2ref) <= 1e-6 * len(ops)
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max()), np.abs(g - gref).max()
    with pytest.raises(lib.FockError) as e:  # a complex gate on real states
        lib.energy_grad_adjoint(hl, [("HI", 0, 1)], np.array([0.1]), x0, a, b, ws)
    assert e.value.code == -3


# Runs chosen to cover every fused tile kind (a = 0, 1, >= 2), gates on both
# tile pairs, a run from psi0 and one at the end, a run split at 8 gates, the
# window below the top pair (a = 4) and, in the full layout only, the top
# window (a = 5); the top pair of the halved layout stays a single gate.
FUSE_OPS = ([("PR", 0, 1), ("HR", 1, 2), ("HR", 0, 1), ("PR", 6, 7),
             ("HR", 3, 4), ("PR", 3, 4), ("HR", 2, 3),
             ("HR", 1, 2), ("PR", 1, 2), ("PR", 2, 3),
             ("PR", 5, 6), ("HR", 4, 5), ("PR", 5, 6), ("HR", 6, 7)]
            + [("HR", 3, 4)] * 9
            + [("PR", 5, 6), ("PR", 6, 7), ("HR", 5, 6), ("PR", 5, 6), ("HR", 0, 1), ("PR", 0, 1)])


def fused_pair(hl, ops, th, x0, grad):
    """The same evaluation with fused runs of real gates and gate by gate."""
    outs = []
    ws = lib.workspace(hl, 0, len(ops))
    for mode in (lib.RFUSE_ON, lib.RFUSE_OFF):
        lib.set_real_fusion(mode)
        try:
            a, b = torch.full_like(x0, float("nan")), torch.full_like(x0, float("nan"))
            E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws, grad=grad)
            torch.cuda.synchronize()
            outs.append((E, n2, g, a, b))
        finally:
            lib.set_real_fusion(lib.RFUSE_ON)
    return outs


_FUSED_ORACLE = {}


def fused_oracle(ho, psi0, th):
    """The oracle's energy, gradients, norm and final state of FUSE_OPS (the
    same for both layouts: computed once)."""
    if not _FUSED_ORACLE:
        p0 = psi0.astype(np.float32).astype(np.complex128)
        Eref, gref, n2ref = O.energy_and_grad_adjoint(ho, p0, FUSE_OPS, th, apply_h=O.apply_H_slices)
        _FUSED_ORACLE["r"] = (Eref, gref, n2ref, O.ansatz_state(p0, FUSE_OPS, th, 8, 8))
    return _FUSED_ORACLE["r"]


@pytest.mark.parametrize("layout", REAL_LAYOUTS, ids=["full", "halved"])
def test_real_fused_runs_match_gate_by_gate_l8_d8(layout):
    """Fused runs against the per-gate kernels on the same evaluation: the final
    state bit for bit (same block arithmetic in LDS), the energy and norm, phi
    and lambda after the reverse sweep bit for bit, gradients to FP32 rounding
    of the per-tile partial sums; then the fused evaluation against the
    oracle's FP64 reverse sweep."""
    assert lib.get_real_fusion() == lib.RFUSE_ON
    ho, hl = ham_real(layout)
    rng = np.random.default_rng(95)
    th = rng.uniform(-0.4, 0.4, len(FUSE_OPS))
    psi0 = real_state(97)
    idx = stored_index(8, 8, 0) if layout & 3 else np.arange(8**8)
    x0 = torch.from_numpy(psi0[idx].astype(np.float32)).to("cuda")
    say("fused vs gate by gate, layout", layout, len(FUSE_OPS))
    (Ef, nf, _, af, _), (Eu, nu, _, au, _) = fused_pair(hl, FUSE_OPS, th, x0, grad=False)
    assert torch.equal(af, au)
    assert Ef == Eu and nf == nu
    (Ef, nf, gf, pf, lf), (Eu, nu, gu, pu, lu) = fused_pair(hl, FUSE_OPS, th, x0, grad=True)
    assert Ef == Eu and nf == nu
    assert torch.equal(pf, pu) and torch.equal(lf, lu)
    assert np.abs(gf - gu).max() <= 2e-5 * max(1.0, np.abs(gu).max()), np.abs(gf - gu).max()
    Eref, gref, n2ref, psi_n = fused_oracle(ho, psi0, th)
    assert np.abs(af.cpu().numpy() - psi_n.real[idx]).max() <= 1e-5 * np.abs(psi_n).max() * len(FUSE_OPS) ** 0.5
    assert abs(Ef - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(nf - n2ref) <= 1e-6 * len(FUSE_OPS)
    assert np.abs(gf - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max()), np.abs(gf - gref).max()


def test_real_fused_adapt_l7_d8():
    """ADAPT on an L=7 chain (2^21 amplitudes, full layout: the smallest state
    the fused runs take) with fused runs and gate by gate: the same selections,
    energies to FP32 rounding, and the oracle replay of the final ansatz."""
    L = 7
    cc = dict(L=L, d=8, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.5, K=0.2)
    hl = lib.ham_from(cc)
    pool = W.pool(L, "nn", False, W.KITAEV_TYPES)
    psi0 = O.fock_state(L, 8, [0] * L)
    assert len(lib.real_fusion_plan(hl, [("PR", 0, 1), ("PR", 1, 2)])) == 1
    say("fused vs gate by gate ADAPT, L", L)
    a = lib.Adapt(hl, pool, dev(psi0), max_iters=30, recycle_hessian=True)
    b = lib.Adapt(hl, pool, dev(psi0), max_iters=30, recycle_hessian=True)
    assert a.real() and b.real()
    ra = None
    try:
        for _ in range(9):
            ra = a.step()
            lib.set_real_fusion(lib.RFUSE_OFF)
            try:
                rb = b.step()
            finally:
                lib.set_real_fusion(lib.RFUSE_ON)
            assert ra["k_sel"] == rb["k_sel"]
            assert abs(ra["E"] - rb["E"]) <= 1e-6 * max(1.0, abs(rb["E"]))
        ops, th = a.ansatz()
        runs = lib.real_fusion_plan(hl, ops)
        assert any(r[1] >= 0 for r in runs) and len(runs) < len(ops)
        Eo = O.energy_of(oham(cc), psi0, ops, th)
        assert abs(ra["E"] - Eo) <= 1e-5 * max(1.0, abs(Eo))
    finally:
        a.close()
        b.close()
