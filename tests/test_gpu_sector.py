"""GPU parity of the parity-halved layout (FOCK_LAYOUT_EVEN / _ODD) against the
FP64 oracle, through the C ABI.

A state of total parity sigma keeps, of the top mode, only m = 0..3 with
n_7 = 2 m + ((n_0 + .. + n_6 + sigma) mod 2).  The index map used here is
computed in NumPy from that definition (digit sums of the flat index), apart
from both the oracle and the kernels; the oracle works on the full d^L tensor
and its results are read at the stored indices.

Tolerances as the full-layout tests: H psi elementwise 2e-5 max|H psi|,
energies 1e-5 max(1, |E|), norms 1e-6, gradients 1e-4 max(1, |g|_inf); the
conversions are exact (bitwise)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workload as W
from paper_2606_05297_amd import lib

pytestmark = pytest.mark.gpu

LAYOUT = {0: lib.LAYOUT_EVEN, 1: lib.LAYOUT_ODD}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def stored_index(L, d, sigma):
    """Full flat index of every stored amplitude c = low + m d^(L-1)."""
    nlow = d ** (L - 1)
    c = np.arange(d**L // 2, dtype=np.int64)
    low, m = c % nlow, c // nlow
    s, x = np.zeros_like(low), low.copy()
    for _ in range(L - 1):
        s += x % d
        x //= d
    return low + (2 * m + (s + sigma) % 2) * nlow


def total_parity(L, d):
    idx = np.arange(d**L, dtype=np.int64)
    s = np.zeros_like(idx)
    for _ in range(L):
        s += idx % d
        idx //= d
    return s % 2


def test_stored_index_is_the_parity_sector():
    """The NumPy index map lists each amplitude of the sector exactly once."""
    for L in (3, 8):
        par = total_parity(L, 8)
        for sigma in (0, 1):
            idx = stored_index(L, 8, sigma)
            assert len(np.unique(idx)) == len(idx) == 8**L // 2
            assert np.all(par[idx] == sigma)


@pytest.mark.parametrize("L", [4, 8])
@pytest.mark.parametrize("sigma", [0, 1])
def test_sector_pack_unpack_bitwise(L, sigma):
    say("sector pack/unpack", L, sigma)
    psi = W.random_state(L, 8, seed=40 + L + sigma, sector=("parity", sigma))
    full = dev(psi)
    half = torch.full((8**L // 2,), float("nan"), dtype=torch.complex64, device="cuda")
    lib.sector_pack(L, 8, LAYOUT[sigma], full, half)
    got = half.cpu().numpy()
    assert np.array_equal(got, psi[stored_index(L, 8, sigma)])
    back = torch.full_like(full, float("nan"))
    lib.sector_unpack(L, 8, LAYOUT[sigma], half, back)
    assert np.array_equal(back.cpu().numpy(), psi)


# open chain with every term: hopping, pairing, U, K and mu (on-site terms of
# the top mode depend on its reconstructed level)
HAM = dict(L=8, d=8, periodic=False, J=0.8, U=1.1, mu=0.3, Delta=0.45, K=0.15)
POOL_ALL = W.pool(8, "nn", False, ("HR", "HI", "DH", "PR", "PI"))


def hams(sigma):
    c = HAM
    ho = O.Ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"])
    hl = lib.ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"], layout=LAYOUT[sigma])
    return ho, hl


@pytest.mark.parametrize("sigma", [0, 1])
def test_sector_apply_H_and_score_l8_d8(sigma):
    """H psi on the 8,388,608 stored amplitudes, energy, norm and all 35 pool
    gradients (HR, HI, DH, PR, PI on the seven bonds), from fock_score (fused)
    and from fock_apply_H + fock_pool_grads, against the oracle on the full
    tensor."""
    ho, hl = hams(sigma)
    say("sector H psi / score", sigma)
    psi = W.random_state(8, 8, seed=50 + sigma, sector=("parity", sigma))
    idx = stored_index(8, 8, sigma)
    x = dev(psi[idx])
    y = torch.full((8**8 // 2,), float("nan"), dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(POOL_ALL), 0)
    g, E, n2 = lib.score(hl, POOL_ALL, x, y, ws)
    p128 = psi.astype(np.complex128)
    href = O.apply_H_slices(ho, p128)
    assert np.count_nonzero(href[total_parity(8, 8) != sigma]) == 0
    got = host(y)
    hs = href[idx]
    assert np.isfinite(got).all()
    assert np.abs(got - hs).max() <= 2e-5 * np.abs(hs).max()
    Eref = np.vdot(p128, href).real
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - np.vdot(p128, p128).real) <= 1e-6
    gref = np.array([2 * np.vdot(href, O.apply_generator(op, p128, 8, 8)).real for op in POOL_ALL])
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max()), np.abs(g - gref).max()
    y2 = torch.full_like(y, float("nan"))
    E2, n22 = lib.apply_H(hl, x, y2, ws)
    assert np.abs(host(y2) - hs).max() <= 2e-5 * np.abs(hs).max()
    assert abs(E2 - Eref) <= 1e-5 * max(1.0, abs(Eref))
    g2 = lib.pool_grads(hl, POOL_ALL, x, y2, ws)
    assert np.abs(g2 - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max())


@pytest.mark.parametrize("sigma,ngates", [(0, 24), (1, 10)])
def test_sector_energy_and_adjoint_l8_d8(sigma, ngates):
    """Energy and every dE/dtheta of a circuit drawn from the 35-entry pool
    (every type on every bond, the top pair (6,7) included) in the
    parity-halved layout, against the oracle's FP64 reverse sweep on the full
    tensor; the final state (psi_work) at the stored indices against the
    oracle's circuit state."""
    ho, hl = hams(sigma)
    ops, th = W.random_circuit(POOL_ALL, ngates, seed=60 + sigma)
    ops = ops + [("HR", 6, 7), ("PI", 6, 7), ("DH", 6, 7), ("PR", 6, 7), ("HI", 6, 7)]
    th = np.concatenate([th, [0.31, -0.27, 0.19, 0.23, -0.35]])
    say("sector adjoint", sigma, len(ops))
    psi0 = W.random_state(8, 8, seed=70 + sigma, sector=("parity", sigma))
    idx = stored_index(8, 8, sigma)
    x0 = dev(psi0[idx])
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, 0, len(ops))
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws, grad=False)
    p0 = psi0.astype(np.complex128)
    psi_n = O.ansatz_state(p0, ops, th, 8, 8)
    assert np.abs(host(a) - psi_n[idx]).max() <= 1e-5 * np.abs(psi_n).max() * len(ops) ** 0.5
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    Eref, gref, n2ref = O.energy_and_grad_adjoint(ho, p0, ops, th, apply_h=O.apply_H_slices)
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - n2ref) <= 1e-6 * len(ops)
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max()), np.abs(g - gref).max()


def test_sector_layout_rejections():
    """Calls and ops the parity-halved layout does not take fail with
    FOCK_ERR_UNSUPPORTED before any launch on the state."""
    ho, hl = hams(0)
    x = torch.zeros(8**8 // 2, dtype=torch.complex64, device="cuda")
    x[0] = 1.0
    a, b = torch.empty_like(x), torch.empty_like(x)
    ws = lib.workspace(hl, 4, 4)
    for op in [("KERR", 3, -1), ("CK", 1, 2), ("HR", 5, 7), ("SR", 2, -1)]:
        with pytest.raises(lib.FockError) as e:
            lib.energy_grad_adjoint(hl, [op], np.array([0.1]), x, a, b, ws)
        assert e.value.code == -3
    with pytest.raises(lib.FockError) as e:
        lib.score(hl, [("HR", 0, 2)], x, a, ws)
    assert e.value.code == -3
    with pytest.raises(lib.FockError) as e:
        lib.score(hl, [("KERR", 0, -1)], x, a, ws)
    assert e.value.code == -3


def oham(c):
    return O.Ham(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"])


def test_adapt_sector_layout_matches_full_layout():
    """The benchmark's ADAPT run (Kitaev-Kerr L=8 d=8 from the vacuum) with the
    parity-halved layout (chosen by default) and with the full layout
    (SECTOR_OFF): same selections, energies within 1e-6 relative, and the
    halved run's energy after step 6 replays on the oracle."""
    c = W.config("kk_l8_d8")
    ho, hl = oham(c), lib.ham_from(c)
    psi0 = O.fock_state(8, 8, c["occ"])
    say("adapt kk_l8_d8 halved vs full")
    assert lib.get_sector_layout() == lib.SECTOR_AUTO
    a = lib.Adapt(hl, c["pool"], dev(psi0), max_iters=c["max_iters"], recycle_hessian=True)
    try:
        lib.set_sector_layout(lib.SECTOR_OFF)
        b = lib.Adapt(hl, c["pool"], dev(psi0), max_iters=c["max_iters"], recycle_hessian=True)
    finally:
        lib.set_sector_layout(lib.SECTOR_AUTO)
    assert a.layout() == lib.LAYOUT_EVEN and b.layout() == lib.LAYOUT_FULL
    for _ in range(6):
        ra, rb = a.step(), b.step()
        assert ra["k_sel"] == rb["k_sel"]
        assert abs(ra["E"] - rb["E"]) <= 1e-6 * abs(rb["E"])
        assert abs(ra["g_norm2"] - rb["g_norm2"]) <= 1e-4 * max(1.0, rb["g_norm2"])
    ops, th = a.ansatz()
    psi = O.ansatz_state(psi0, ops, th, 8, 8)
    E = np.vdot(psi, O.apply_H_slices(ho, psi)).real / np.vdot(psi, psi).real
    assert abs(ra["E"] - E) <= 1e-5 * abs(E)
    a.close()
    b.close()


def test_adapt_sector_layout_odd_start_and_fallbacks():
    """An odd-parity start gives LAYOUT_ODD; a start with both parities, or a
    pool entry the layout does not take, keeps the full layout.  With the
    forward states kept (STORE_ON, read-only reverse step on the top pair) the
    odd run selects and converges like the in-place sweep."""
    c = W.config("kk_l8_d8")
    hl = lib.ham_from(c)
    odd = O.fock_state(8, 8, [0, 0, 0, 0, 0, 0, 0, 1])
    mixed = (O.fock_state(8, 8, [0] * 8) + O.fock_state(8, 8, [0, 0, 0, 0, 0, 0, 0, 1])) / np.sqrt(2)
    say("adapt layouts: odd start, mixed start, Kerr pool entry")
    try:
        lib.set_state_store(lib.STORE_ON)
        a = lib.Adapt(hl, c["pool"], dev(odd), max_iters=4)
    finally:
        lib.set_state_store(lib.STORE_AUTO)
    b = lib.Adapt(hl, c["pool"], dev(odd), max_iters=4)
    m = lib.Adapt(hl, c["pool"], dev(mixed), max_iters=1)
    k = lib.Adapt(hl, c["pool"] + [("KERR", 3, -1)], dev(odd), max_iters=1)
    assert a.layout() == lib.LAYOUT_ODD and b.layout() == lib.LAYOUT_ODD and a.state_store() > 0
    assert m.layout() == lib.LAYOUT_FULL and k.layout() == lib.LAYOUT_FULL
    for _ in range(3):
        ra, rb = a.step(), b.step()
        assert ra["k_sel"] == rb["k_sel"]
        assert abs(ra["E"] - rb["E"]) <= 1e-6 * max(1.0, abs(rb["E"]))
    ho = oham(c)
    ops, th = a.ansatz()
    Eo = O.energy_of(ho, odd, ops, th)
    assert abs(ra["E"] - Eo) <= 1e-5 * max(1.0, abs(Eo))
    for x in (a, b, m, k):
        x.close()

