"""GPU parity of the HIP kernels (through the C ABI) against the FP64 oracle.

Tolerances (FP32 state arithmetic with FP64 reductions):
  * H psi elementwise: |d| <= 2e-5 * max|H psi|  (about 30 FP32 terms per amplitude);
  * energies: |dE| <= 1e-5 * max(1, |E|)  (the required energy tolerance);
  * norms: |d| <= 1e-6;
  * pool and adjoint gradients: |dg| <= 1e-4 * max(1, max|g|)  (required gradient tolerance);
  * gates elementwise: |d| <= 1e-5 * max|psi|; leakage out of a conserved
    sector must be exactly zero (bit-exact, integer-like structure).
"""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def ham_pair(L, d, per, J=1.0, U=0.0, mu=0.0, Delta=0.0, K=0.0):
    return O.Ham(L, d, per, J, U, mu, Delta, K), lib.ham(L, d, per, J, U, mu, Delta, K)


SMALL = [
    # (L, d, periodic, J, U, mu, Delta, K)
    (1, 5, False, 1.0, 1.3, 0.2, 0.0, 0.0),
    (2, 4, True, 1.0, 2.0, 0.0, 0.0, 0.0),
    (2, 3, False, 0.7, 0.0, 0.1, 0.6, 0.3),
    (3, 4, False, 1.0, 2.0, 0.0, 0.0, 0.0),
    (3, 3, True, 1.0, 0.5, 0.3, 0.4, 0.1),
    (4, 5, False, 1.0, 0.0, 0.0, 0.5, 0.2),
    (5, 4, True, 0.9, 1.7, 0.4, 0.3, 0.1),
    (4, 7, True, 1.0, 0.0, -0.2, 0.5, 0.2),
    (3, 16, False, 1.0, 0.0, 0.0, 0.5, 0.2),
    (6, 6, True, 1.0, 4.0, 0.0, 0.0, 0.0),
    (6, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2),
    (7, 5, False, 1.0, 0.0, 0.3, 0.45, 0.15),
]


@pytest.fixture
def schedule(request):
    prev = lib.get_stencil_schedule()
    lib.set_stencil_schedule(request.param)
    yield request.param
    lib.set_stencil_schedule(prev)


SMALL_2P = SMALL + [(7, 5, True, 1.0, 0.0, 0.3, 0.45, 0.15), (8, 4, True, 1.0, 1.5, 0.0, 0.0, 0.0),
                    (6, 6, False, 1.0, 0.0, 0.0, 0.5, 0.2)]


@pytest.mark.parametrize("schedule", [0, 4], indirect=True, ids=["1pass", "2pass"])
@pytest.mark.parametrize("case", SMALL_2P, ids=lambda c: f"L{c[0]}d{c[1]}{'p' if c[2] else 'o'}")
def test_apply_H_parity(case, schedule):
    L, d, per, J, U, mu, Dl, K = case
    say("apply_H", case, "schedule", schedule)
    ho, hl = ham_pair(L, d, per, J, U, mu, Dl, K)
    psi = W.random_state(L, d, seed=L * 100 + d)
    ref = O.apply_H(ho, psi.astype(np.complex128))
    x, y = dev(psi), torch.empty(d**L, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl)
    E, n2 = lib.apply_H(hl, x, y, ws)
    got = host(y)
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()
    Eref = np.vdot(psi.astype(np.complex128), ref).real
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - 1.0) <= 1e-6
    # determinism: bit-identical on a second call
    E2, n22 = lib.apply_H(hl, x, y, ws)
    assert E2 == E and n22 == n2


@pytest.fixture
def stencil(request):
    prev = lib.get_stencil_variant()
    lib.set_stencil_variant(request.param)
    yield request.param
    lib.set_stencil_variant(prev)


LANE_CASES = [
    # (L, d, periodic, J, U, mu, Delta, K): d = 8 open chains, the lane split's domain
    (4, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2),    # a single tile, no bond leaves it
    (5, 8, False, 1.0, 0.0, 0.3, 0.45, 0.15),  # only the bond (3,4) leaves the tile
    (6, 8, False, 0.8, 1.2, 0.2, 0.0, 0.0),    # Bose-Hubbard, open, Delta = 0
    (7, 8, False, -0.6, 0.4, -0.3, 0.7, 0.25),
]


@pytest.mark.parametrize("case", LANE_CASES, ids=lambda c: f"L{c[0]}d{c[1]}o")
def test_apply_H_lane_split_parity(case):
    """Four-lanes-per-row H psi against the oracle; against the row split to
    FP32 rounding; deterministic; a ring chain (outside its domain) runs the
    row split and matches it bit for bit."""
    L, d, per, J, U, mu, Dl, K = case
    say("apply_H lanes", case)
    ho, hl = ham_pair(L, d, per, J, U, mu, Dl, K)
    psi = W.random_state(L, d, seed=L * 100 + d + 7)
    ref = O.apply_H(ho, psi.astype(np.complex128))
    x = dev(psi)
    ys = {}
    prev = lib.get_stencil_variant()
    try:
        for v in (lib.STENCIL_ROWS, lib.STENCIL_LANES):
            lib.set_stencil_variant(v)
            y = torch.empty(d**L, dtype=torch.complex64, device="cuda")
            ws = lib.workspace(hl)
            E, n2 = lib.apply_H(hl, x, y, ws)
            ys[v] = (host(y), E, n2)
            E2, n22 = lib.apply_H(hl, x, y, ws)
            assert E2 == E and n22 == n2
        got, E, n2 = ys[lib.STENCIL_LANES]
        assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()
        Eref = np.vdot(psi.astype(np.complex128), ref).real
        assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
        assert abs(n2 - 1.0) <= 1e-6
        rows = ys[lib.STENCIL_ROWS][0]
        assert np.abs(got - rows).max() <= 4e-6 * np.abs(ref).max()
        # a ring of the same size is outside the lane split: the row kernel runs
        ho_r, hl_r = ham_pair(L, d, True, J, U, mu, Dl, K)
        out = []
        for v in (lib.STENCIL_ROWS, lib.STENCIL_LANES):
            lib.set_stencil_variant(v)
            y = torch.empty(d**L, dtype=torch.complex64, device="cuda")
            lib.apply_H(hl_r, x, y, lib.workspace(hl_r))
            out.append(host(y))
        assert np.array_equal(out[0], out[1])
    finally:
        lib.set_stencil_variant(prev)


SQ_CASES = [
    # (L, d, J, U, mu, Delta, K): open chains, squeezers on every site
    (5, 6, 1.0, 0.0, 0.1, 0.5, 0.2),
    (4, 8, 0.8, 0.5, 0.0, 0.4, 0.1),
    (5, 7, 1.0, 0.0, 0.0, 0.5, 0.25),   # ragged: 2401 fibres per mode
]


@pytest.mark.parametrize("case", SQ_CASES, ids=lambda c: f"L{c[0]}d{c[1]}")
def test_squeezer_energy_adjoint_and_pool_parity(case):
    """Circuits and pools with the single-mode squeezers SR, SI (with the
    Kitaev generators, CK and K): energy, adjoint gradient and pool gradients
    against the oracle; a chunk of squeezer entries alone is scored too."""
    L, d, J, U, mu, Dl, K = case
    say("squeezers", case)
    ho, hl = ham_pair(L, d, False, J, U, mu, Dl, K)
    pool = W.pool(L, "nn", False, W.KITAEV_TYPES + ("CK",)) + W.site_ops(L, ("SR", "SI", "KERR"))
    ops, th = W.random_circuit(pool, 12, seed=L * 7 + d)
    ops = ops[:10] + [("SR", 0, -1), ("SI", L - 1, -1)]
    th = np.concatenate([th[:10], [0.31, -0.27]])
    psi0 = W.random_state(L, d, seed=3, sector=("parity", 0))
    x0 = dev(psi0)
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, len(pool), len(ops))
    E, _, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    Eo, go, _ = O.energy_and_grad_adjoint(ho, psi0.astype(np.complex128), ops, th)
    assert abs(E - Eo) <= 1e-5 * max(1.0, abs(Eo))
    assert np.abs(g - go).max() <= 1e-4 * max(1.0, np.abs(go).max())
    psi = W.random_state(L, d, seed=9)
    x, y = dev(psi), torch.empty(d**L, dtype=torch.complex64, device="cuda")
    lib.apply_H(hl, x, y, ws)
    gp = lib.pool_grads(hl, pool, x, y, ws)
    ref = O.pool_gradients(ho, psi.astype(np.complex128), pool)
    assert np.abs(gp - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    only = W.site_ops(L, ("SI", "SR"))
    gs = lib.pool_grads(hl, only, x, y, ws)
    refs = O.pool_gradients(ho, psi.astype(np.complex128), only)
    assert np.abs(gs - refs).max() <= 1e-4 * max(1.0, np.abs(refs).max())


POOL_CASES = [
    (3, 4, False, 1.0, 2.0, 0.0, 0.0, 0.0, "all", ("HR", "HI", "DH", "PR", "PI")),
    (4, 5, True, 1.0, 0.7, 0.2, 0.5, 0.2, "nn+nnn", ("HR", "HI", "DH", "PR", "PI")),
    (5, 4, False, 1.0, 0.0, 0.0, 0.5, 0.2, "all", W.KITAEV_TYPES),
    (4, 7, True, 1.0, 3.0, 0.0, 0.0, 0.0, "nn+nnn", W.BH_TYPES + ("CK",)),
    (6, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2, "nn", W.KITAEV_TYPES + ("CK",)),
    (2, 6, False, 1.0, 1.0, 0.3, 0.3, 0.1, "all", ("HR", "HI", "DH", "PR", "PI")),
]


@pytest.mark.parametrize("case", POOL_CASES, ids=lambda c: f"L{c[0]}d{c[1]}{c[8]}")
def test_pool_grads_parity(case):
    L, d, per, J, U, mu, Dl, K, kind, types = case
    say("pool_grads", case[:9])
    ho, hl = ham_pair(L, d, per, J, U, mu, Dl, K)
    pool = W.pool(L, kind, per, types) + [("KERR", r, -1) for r in range(L)] + [("ROT", 0, -1), ("ROT", L - 1, -1)]
    psi = W.random_state(L, d, seed=7 + L + d)
    x, y = dev(psi), torch.empty(d**L, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(pool))
    lib.apply_H(hl, x, y, ws)
    g = lib.pool_grads(hl, pool, x, y, ws)
    ref = O.pool_gradients(ho, psi.astype(np.complex128), pool)
    assert np.abs(g - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    g2 = lib.pool_grads(hl, pool, x, y, ws)
    assert np.array_equal(g, g2)


def test_pool_grads_large_pool_chunks():
    """More than 256 entries and duplicates force several launches."""
    L, d = 5, 3
    ho, hl = ham_pair(L, d, True, 1.0, 0.5, 0.1, 0.4, 0.1)
    base = W.pool(L, "all", True, ("HR", "HI", "DH", "PR", "PI", "CK"))
    pool = base * 5 + [("KERR", 1, -1), ("CK", 0, 4)]
    say("pool_grads chunks", len(pool))
    psi = W.random_state(L, d, seed=3)
    x, y = dev(psi), torch.empty(d**L, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(pool))
    lib.apply_H(hl, x, y, ws)
    g = lib.pool_grads(hl, pool, x, y, ws)
    ref = O.pool_gradients(ho, psi.astype(np.complex128), pool)
    assert np.abs(g - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


GATE_OPS = [("HR", 0, 1), ("HI", 1, 3), ("DH", 0, 2), ("DH", 2, 3), ("PR", 0, 3), ("PI", 1, 2), ("KERR", 0, -1),
            ("KERR", 2, -1), ("ROT", 3, -1), ("ROT", 0, -1), ("CK", 0, 2), ("CK", 1, 3), ("SR", 0, -1), ("SI", 2, -1),
            ("SR", 3, -1)]


@pytest.mark.parametrize("d", [2, 3, 5, 8, 12, 16])
@pytest.mark.parametrize("opx", GATE_OPS, ids=lambda o: f"{o[0]}{o[1]}{o[2]}")
def test_gate_parity_and_leakage(opx, d):
    L = 4
    say("gate", opx, d)
    psi = W.random_state(L, d, seed=11 + d)
    ws = lib.workspace(lib.ham(L, d), 0, 1)
    for adj in (False, True):
        x = dev(psi)
        lib.apply_gate2(L, d, opx, 0.37, x, ws, adjoint=adj)
        got = host(x)
        ref = O.apply_gate(opx, 0.37, psi.astype(np.complex128), L, d, adjoint=adj)
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(psi).max()
    # exact zero leakage from a conserved sector
    sector = ("parity", 0) if opx[0] in ("PR", "PI", "SR", "SI") else ("N", 3)
    ps = W.random_state(L, d, seed=5, sector=sector)
    x = dev(ps)
    lib.apply_gate2(L, d, opx, 0.9, x, ws)
    out = host(x)
    outside = np.ones(d**L, dtype=bool)
    outside[O.sector_indices(L, d, sector)] = False
    assert np.count_nonzero(out[outside]) == 0
    assert abs(np.vdot(out, out).real - np.vdot(ps, ps).real) < 2e-6


def test_gate_then_adjoint_is_identity_ragged():
    L, d = 5, 7  # 16807 amplitudes: fibers do not fill whole workgroups
    psi = W.random_state(L, d, seed=2)
    x = dev(psi)
    ws = lib.workspace(lib.ham(L, d), 0, 1)
    for o in [("HR", 1, 4), ("PR", 0, 4), ("DH", 3, 4), ("KERR", 4, -1), ("CK", 0, 3), ("SR", 2, -1), ("SI", 0, -1)]:
        say("gate roundtrip", o)
        lib.apply_gate2(L, d, o, 1.1, x, ws)
        lib.apply_gate2(L, d, o, 1.1, x, ws, adjoint=True)
    assert np.abs(host(x) - psi).max() < 2e-6


ADJ_CASES = [
    (3, 4, False, 1.0, 2.0, 0.0, 0.0, 0.0, W.BH_TYPES, ("N", 3), 8),
    (4, 5, False, 1.0, 0.0, 0.0, 0.5, 0.2, W.KITAEV_TYPES, ("parity", 0), 12),
    (5, 4, True, 1.0, 1.2, 0.1, 0.3, 0.1, ("HR", "HI", "DH", "PR", "PI"), None, 10),
    (5, 5, True, 1.0, 2.0, 0.0, 0.0, 0.0, W.BH_TYPES + ("CK",), ("N", 5), 10),
    (6, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2, W.KITAEV_TYPES, ("parity", 0), 6),
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=lambda c: f"L{c[0]}d{c[1]}n{c[10]}")
def test_energy_and_adjoint_parity(case):
    L, d, per, J, U, mu, Dl, K, types, sector, n = case
    say("adjoint", case[:8], n)
    ho, hl = ham_pair(L, d, per, J, U, mu, Dl, K)
    pool = W.pool(L, "nn", per, types) + [("KERR", 0, -1), ("ROT", L - 1, -1)]
    ops, th = W.random_circuit(pool, n, seed=L + d)
    psi0 = W.random_state(L, d, seed=9, sector=sector)
    x0 = dev(psi0)
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, 0, n)
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    Eref, gref, n2ref = O.energy_and_grad_adjoint(ho, psi0.astype(np.complex128), ops, th)
    assert abs(E - Eref / n2ref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - n2ref) <= 2e-6
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max())
    # forward-only call leaves psi and H psi in the work buffers
    E2, _, _ = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws, grad=False)
    assert E2 == E
    psi_n = O.ansatz_state(psi0.astype(np.complex128), ops, th, L, d)
    assert np.abs(host(a) - psi_n).max() <= 1e-5
    assert np.array_equal(host(x0), psi0.astype(np.complex128))  # psi0 untouched
    # repeated call: bit-identical
    E3, _, g3 = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    assert E3 == E and np.array_equal(g3, g)


DIAG_RUN_CASES = [(3, 5, False, 12), (4, 4, True, 12), (5, 3, False, 12), (4, 3, False, 40)]


@pytest.mark.parametrize("case", DIAG_RUN_CASES, ids=lambda c: f"L{c[0]}d{c[1]}n{c[3]}")
def test_phase_gate_runs_energy_and_adjoint(case):
    """Runs of consecutive single-mode phase gates (Kerr and rotation on mode 0
    and on higher modes) go through one diagonal pass forward and one in the
    reverse sweep; ragged row counts (d^(L-1) not a multiple of the workgroup)
    and a 40-gate run (split at 32 gates).  Energy, every gradient and the final
    state against the oracle, which applies the gates one by one."""
    L, d, per, n = case
    ho, hl = ham_pair(L, d, per, 1.0, 0.7, 0.2, 0.3, 0.1)
    rng = np.random.default_rng(L * 10 + d)
    if n == 12:
        ops = [("HR", 0, 1), ("KERR", 0, -1), ("ROT", 2, -1), ("KERR", 1, -1), ("ROT", 0, -1),
               ("KERR", L - 1, -1), ("HI", 1, 2), ("ROT", 1, -1), ("KERR", 2, -1), ("PR", 0, L - 1),
               ("ROT", 0, -1), ("ROT", 0, -1)]
    else:
        ops = [("HR", 0, 1)] + [(("KERR", "ROT")[int(rng.integers(2))], int(rng.integers(L)), -1)
                                for _ in range(n - 2)] + [("PI", 1, 2)]
    th = rng.uniform(-0.6, 0.6, len(ops))
    say("phase-gate runs", case)
    psi0 = W.random_state(L, d, seed=4, sector=None)
    x0 = dev(psi0)
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, 0, len(ops))
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    Eref, gref, n2ref = O.energy_and_grad_adjoint(ho, psi0.astype(np.complex128), ops, th)
    assert abs(E - Eref / n2ref) <= 1e-5 * max(1.0, abs(Eref))
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max()), np.abs(g - gref).max()
    lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws, grad=False)
    psi_n = O.ansatz_state(psi0.astype(np.complex128), ops, th, L, d)
    assert np.abs(host(a) - psi_n).max() <= 1e-5


def test_adjoint_matches_gpu_finite_differences():
    """dE/dtheta from the reverse sweep vs central differences (h = 1e-4 in the
    angle, required step) of the GPU energy, Kitaev-Kerr chain."""
    L, d = 5, 8
    _, hl = ham_pair(L, d, False, 1.0, 0.0, 0.0, 0.5, 0.2)
    ops, th = W.random_circuit(W.pool(L, "nn", False, W.KITAEV_TYPES), 8, seed=1)
    x0 = dev(W.random_state(L, d, seed=4, sector=("parity", 0)))
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, 0, len(ops))
    E, _, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    say("adjoint vs gpu fd")
    h = 1e-3  # FP32 energies: 1e-4 steps leave ~1e-3 noise; 1e-3 keeps truncation ~1e-6
    for k in range(len(ops)):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        ep = lib.energy_grad_adjoint(hl, ops, tp, x0, a, b, ws, grad=False)[0]
        em = lib.energy_grad_adjoint(hl, ops, tm, x0, a, b, ws, grad=False)[0]
        assert abs((ep - em) / (2 * h) - g[k]) <= 2e-3 * max(1.0, abs(E))


# ---------------------------------------------------------------- full workload sizes

@pytest.fixture(scope="module")
def kk_full():
    c = W.config("kk_l8_d8")
    ho, hl = ham_pair(c["L"], c["d"], c["periodic"], c["J"], c["U"], c["mu"], c["Delta"], c["K"])
    psi = W.random_state(8, 8, seed=0, sector=("parity", 0))
    return c, ho, hl, psi


SLAB_CASES = [
    # (periodic, J, U, mu, Delta, K, state sector): the benchmark's chain, and a ring with every term on
    (False, 1.0, 0.0, 0.0, 0.5, 0.2, ("parity", 0)),
    (True, 0.8, 1.1, 0.3, 0.45, 0.15, None),
]


@pytest.mark.parametrize("case", SLAB_CASES, ids=["kk_open", "ring_all_terms"])
def test_slab_stencil_full_vector_l8_d8(case):
    """The two-pass slab H psi (default at L=8, d=8) against the oracle on all
    16,777,216 amplitudes: open Kitaev-Kerr chain on an even-parity state, and
    a ring with hopping, pairing, on-site U, K and mu on a state with every
    amplitude non-zero (all boundary digits n_r = 0, 7 exercised).  Also the
    energy, the norm, and agreement with the one-pass row kernel."""
    per, J, U, mu, Dl, K, sector = case
    ho, hl = ham_pair(8, 8, per, J, U, mu, Dl, K)
    say("slab full vector", case)
    assert lib.get_stencil_variant() == lib.STENCIL_SLAB
    psi = W.random_state(8, 8, seed=7, sector=sector)
    x, y = dev(psi), torch.empty(8**8, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, 0, 0)
    y.fill_(float("nan"))  # every output amplitude must be written
    E, n2 = lib.apply_H(hl, x, y, ws)
    got = host(y)
    p128 = psi.astype(np.complex128)
    ref = O.apply_H_slices(ho, p128)
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()
    Eref = np.vdot(p128, ref).real
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref))
    assert abs(n2 - np.vdot(p128, p128).real) <= 1e-6
    if sector is not None:  # H keeps the parity sector: odd amplitudes exactly zero
        odd = O.sector_indices(8, 8, ("parity", 1))
        assert np.count_nonzero(got[odd]) == 0
    lib.set_stencil_variant(lib.STENCIL_ROWS)
    try:
        y2 = torch.empty_like(y)
        E2, _ = lib.apply_H(hl, x, y2, ws)
    finally:
        lib.set_stencil_variant(lib.STENCIL_SLAB)
    assert np.abs(host(y2) - got).max() <= 2e-5 * np.abs(ref).max()
    assert abs(E2 - E) <= 1e-5 * max(1.0, abs(E))


def test_slab_pool_ring_all_types_l8_d8():
    """Slab pool scoring (default at L=8, d=8) on a ring with hopping, pairing,
    U, K and mu: every two-mode generator type (HR, HI, DH, PR, PI) on all
    eight nearest-neighbour pairs including the ring pair (0, 7), plus Kerr,
    rotation and cross-Kerr entries on several modes, on a state with every
    amplitude non-zero; against the oracle's 2 Re <H psi|A_k psi> (FP64) and
    against the one-pass pool kernel."""
    per, J, U, mu, Dl, K = True, 0.8, 1.1, 0.3, 0.45, 0.15
    ho, hl = ham_pair(8, 8, per, J, U, mu, Dl, K)
    pool = W.pool(8, "nn", True, ("HR", "HI", "DH", "PR", "PI"))
    pool += [("KERR", 0, -1), ("ROT", 3, -1), ("KERR", 7, -1), ("CK", 0, 7), ("CK", 2, 5), ("ROT", 5, -1),
             ("KERR", 3, -1), ("CK", 3, 6), ("CK", 1, 3), ("ROT", 4, -1), ("CK", 3, 4)]
    assert ("HR", 0, 7) in pool
    say("slab pool ring, all types")
    psi = W.random_state(8, 8, seed=11, sector=None)
    x, y = dev(psi), torch.empty(8**8, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(pool), 0)
    lib.apply_H(hl, x, y, ws)
    g = lib.pool_grads(hl, pool, x, y, ws)
    p128 = psi.astype(np.complex128)
    ref = O.pool_gradients(ho, p128, pool, apply_h=O.apply_H_slices)
    assert np.abs(g - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max()), np.abs(g - ref).max()
    lib.set_stencil_variant(lib.STENCIL_ROWS)
    try:
        y2 = torch.empty_like(y)
        lib.apply_H(hl, x, y2, ws)
        g2 = lib.pool_grads(hl, pool, x, y2, ws)
    finally:
        lib.set_stencil_variant(lib.STENCIL_SLAB)
    assert np.abs(g2 - g).max() <= 1e-4 * max(1.0, np.abs(ref).max())


SCORE_CASES = [
    # the benchmark's chain and pool; a ring with every two-mode type and diagonal entries
    (False, 1.0, 0.0, 0.0, 0.5, 0.2, ("parity", 0), "kk"),
    (True, 0.8, 1.1, 0.3, 0.45, 0.15, None, "all"),
]


@pytest.mark.parametrize("case", SCORE_CASES, ids=["kk_open_pool28", "ring_all_types"])
def test_fused_scoring_l8_d8(case):
    """fock_score (fused H psi + pool scoring at L=8, d=8) against the oracle
    (H psi on every amplitude, energy, norm, every pool gradient) and against
    fock_apply_H followed by fock_pool_grads."""
    per, J, U, mu, Dl, K, sector, kind = case
    ho, hl = ham_pair(8, 8, per, J, U, mu, Dl, K)
    if kind == "kk":
        pool = W.config("kk_l8_d8")["pool"]
    else:
        pool = W.pool(8, "nn", True, ("HR", "HI", "DH", "PR", "PI"))
        pool += [("KERR", 0, -1), ("ROT", 3, -1), ("CK", 0, 7), ("CK", 2, 5), ("KERR", 3, -1), ("CK", 3, 6),
                 ("CK", 1, 3), ("KERR", 4, -1)]
    say("fused scoring", kind)
    psi = W.random_state(8, 8, seed=21, sector=sector)
    x = dev(psi)
    y = torch.full((8**8,), float("nan"), dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(pool), 0)
    g, E, n2 = lib.score(hl, pool, x, y, ws)
    p128 = psi.astype(np.complex128)
    href = O.apply_H_slices(ho, p128)
    got = host(y)
    assert np.abs(got - href).max() <= 2e-5 * np.abs(href).max()
    Eref = np.vdot(p128, href).real
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref)) and abs(n2 - np.vdot(p128, p128).real) <= 1e-6
    gref = np.array([2 * np.vdot(href, O.apply_generator(op, p128, 8, 8)).real for op in pool])
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max()), np.abs(g - gref).max()
    y2 = torch.empty_like(y)
    E2, _ = lib.apply_H(hl, x, y2, ws)
    g2 = lib.pool_grads(hl, pool, x, y2, ws)
    assert np.abs(g2 - g).max() <= 1e-4 * max(1.0, np.abs(gref).max())
    assert abs(E2 - E) <= 1e-5 * max(1.0, abs(E))


@pytest.mark.parametrize("stencil", [0, 1, 2], indirect=True, ids=["rows", "lanes", "slab"])
def test_full_kitaev_l8_d8_apply_H_sampled_and_energy(kk_full, stencil):
    c, ho, hl, psi = kk_full
    say("full kk apply_H, stencil", stencil)
    x, y = dev(psi), torch.empty(8**8, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(c["pool"]), 64)
    E, n2 = lib.apply_H(hl, x, y, ws)
    got = host(y)
    p128 = psi.astype(np.complex128)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.integers(0, 8**8, 1500), [0, 1, 7, 8, 8**7, 8**8 - 1, 8**8 - 8, 8**7 - 1]])
    ref = np.array([O.apply_H_at(ho, p128, int(k)) for k in idx])
    assert np.abs(got[idx] - ref).max() <= 2e-5 * max(np.abs(ref).max(), 1e-30)
    full = O.apply_H_slices(ho, p128)
    Eref = np.vdot(p128, full).real
    assert abs(E - Eref) <= 1e-5 * abs(Eref)
    # parity leakage of H psi is exactly zero
    odd = O.sector_indices(8, 8, ("parity", 1))
    assert np.count_nonzero(got[odd]) == 0


def test_full_kitaev_l8_d8_pool_grads(kk_full):
    c, ho, hl, psi = kk_full
    say("full kk pool")
    x, y = dev(psi), torch.empty(8**8, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(c["pool"]), 64)
    lib.apply_H(hl, x, y, ws)
    g = lib.pool_grads(hl, c["pool"], x, y, ws)
    p128 = psi.astype(np.complex128)
    h128 = O.apply_H_slices(ho, p128)
    assert len(c["pool"]) == 28
    ref = np.array([2 * np.vdot(h128, O.apply_generator(op, p128, 8, 8)).real for op in c["pool"]])
    assert np.abs(g - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


def test_full_kitaev_l8_d8_adjoint(kk_full):
    """Adjoint gradients at the benchmark's size and depth: a 24-gate circuit
    drawn from the 28-entry pool (every generator type, all seven bonds) on
    L=8 d=8; energy to 1e-5 |E| and every dE/dtheta_k to 1e-4 max(1, |g|_inf)
    against the oracle's FP64 reverse sweep."""
    c, ho, hl, psi = kk_full
    say("full kk adjoint, 24 gates")
    ops, th = W.random_circuit(c["pool"], 24, seed=3)
    assert {o[0] for o in ops} == {"HR", "HI", "PI", "PR"}
    psi0 = W.random_state(8, 8, seed=0, sector=("parity", 0))
    x0 = dev(psi0)
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, len(c["pool"]), 64)
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    Eref, gref, n2ref = O.energy_and_grad_adjoint(ho, psi0.astype(np.complex128), ops, th, apply_h=O.apply_H_slices)
    assert abs(E - Eref) <= 1e-5 * abs(Eref)
    assert np.abs(g - gref).max() <= 1e-4 * max(1.0, np.abs(gref).max())


def test_full_kitaev_l8_d8_adjoint_vs_fp64_finite_differences(kk_full):
    """The GPU adjoint gradient of a 3-gate circuit at L=8 d=8 against FP64
    central differences of the oracle's energy with the step 1e-4 of the
    Kitaev-Kerr workload (no FP32 noise in the difference quotient)."""
    c, ho, hl, psi = kk_full
    ops, th = W.random_circuit(c["pool"], 3, seed=5)
    psi0 = W.random_state(8, 8, seed=2, sector=("parity", 0))
    x0 = dev(psi0)
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, len(c["pool"]), 64)
    E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
    p0 = psi0.astype(np.complex128)

    def e64(t):
        s = O.ansatz_state(p0, ops, t, 8, 8)
        return np.vdot(s, O.apply_H_slices(ho, s)).real / np.vdot(s, s).real

    h = 1e-4
    for k in range(len(ops)):
        say("fp64 fd parameter", k)
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (e64(tp) - e64(tm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-4 * max(1.0, abs(fd)), (k, fd, g[k])


def test_full_bose_hubbard_l8_d6_sampled():
    c = W.config("bh_l8_d6")
    ho, hl = ham_pair(8, 6, True, 1.0, 4.0, 0.0, 0.0, 0.0)
    say("full bh apply_H + pool")
    psi = W.random_state(8, 6, seed=1, sector=("N", 8))
    x, y = dev(psi), torch.empty(6**8, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(c["pool"]), 64)
    E, n2 = lib.apply_H(hl, x, y, ws)
    got = host(y)
    p128 = psi.astype(np.complex128)
    full = O.apply_H(ho, p128)
    assert np.abs(got - full).max() <= 2e-5 * np.abs(full).max()
    assert abs(E - np.vdot(p128, full).real) <= 1e-5 * max(1.0, abs(np.vdot(p128, full).real))
    g = lib.pool_grads(hl, c["pool"], x, y, ws)
    ref = O.pool_gradients(ho, p128, c["pool"])
    assert np.abs(g - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    outside = np.ones(6**8, dtype=bool)
    outside[O.sector_indices(8, 6, ("N", 8))] = False
    assert np.count_nonzero(got[outside]) == 0


def test_stencil_schedules_bitwise_equal_and_autotune(kk_full, tmp_path):
    """H psi, E, norm and pool gradients are bit-identical under every tile
    schedule (partials are indexed by tile, not by workgroup); the autotuner
    returns a valid scheme and its cache is hit on the second call."""
    c, ho, hl, psi = kk_full
    say("schedules kk L8 d8")
    x, y = dev(psi), torch.empty(8**8, dtype=torch.complex64, device="cuda")
    ws = lib.workspace(hl, len(c["pool"]), 64)
    prev = lib.get_stencil_schedule()
    try:
        base = None
        for s in range(4):  # schemes 0-3 only reorder tiles
            lib.set_stencil_schedule(s)
            E, n2 = lib.apply_H(hl, x, y, ws)
            g = lib.pool_grads(hl, c["pool"], x, y, ws)
            cur = (E, n2, host(y), g)
            if base is None:
                base = cur
            else:
                assert cur[0] == base[0] and cur[1] == base[1], s
                assert np.array_equal(cur[2], base[2]), s
                assert np.array_equal(cur[3], base[3]), s
        # two passes: same values to FP32 rounding, the exact ones at sampled rows
        lib.set_stencil_schedule(4)
        E4, n24 = lib.apply_H(hl, x, y, ws)
        got = host(y)
        assert abs(E4 - base[0]) <= 1e-5 * abs(base[0]) and abs(n24 - base[1]) <= 1e-6
        p128 = psi.astype(np.complex128)
        rng = np.random.default_rng(7)
        idx = np.concatenate([rng.integers(0, 8**8, 1000), [0, 8**8 - 1, 8**7, 8**7 - 1]])
        ref = np.array([O.apply_H_at(ho, p128, int(k)) for k in idx])
        assert np.abs(got[idx] - ref).max() <= 2e-5 * np.abs(ref).max()
        assert np.abs(got - base[2]).max() <= 2e-5 * np.abs(base[2]).max()
        cache = str(tmp_path / "stencil.jsonl")
        best = lib.autotune_stencil(hl, x, y, ws, cache)
        say("autotuned schedule", best)
        assert 0 <= best < 5 and lib.get_stencil_schedule() == best
        lib.set_stencil_schedule(0)
        assert lib.autotune_stencil(hl, x, y, ws, cache) == best
    finally:
        lib.set_stencil_schedule(prev)


FUSE_CASES = [
    # (L, d, periodic, J, U, mu, Delta, K, ops as (type, i, j))
    (5, 4, True, 1.0, 0.7, 0.1, 0.4, 0.2,
     [("HR", 0, 1), ("PR", 1, 2), ("HI", 2, 3), ("KERR", 2, -1), ("DH", 0, 1), ("PI", 3, 4), ("ROT", 0, -1),
      ("HR", 0, 4), ("CK", 1, 2), ("SR", 1, -1), ("PR", 3, 4), ("CK", 0, 1), ("HR", 0, 1), ("SI", 0, -1)]),
    (6, 6, True, 1.0, 4.0, 0.0, 0.0, 0.0,
     [("HR", 0, 1), ("HR", 1, 2), ("HR", 2, 3), ("HR", 3, 4), ("HR", 4, 5), ("HR", 0, 5), ("KERR", 5, -1),
      ("ROT", 5, -1), ("DH", 4, 5), ("HI", 1, 2), ("HR", 0, 1)]),
    (6, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2,
     [("PR", 0, 1), ("PR", 1, 2), ("PR", 2, 3), ("PR", 3, 4), ("PR", 4, 5), ("HR", 0, 1), ("PR", 1, 2),
      ("PR", 0, 1), ("PI", 2, 3), ("HI", 2, 3)]),
]


@pytest.mark.parametrize("case", FUSE_CASES, ids=lambda c: f"L{c[0]}d{c[1]}")
def test_gate_fusion_matches_unfused_and_oracle(case):
    """Fused gate groups (one pass per run of gates sharing a tile) give the
    per-gate kernels' energy and gradients to rounding, and the oracle's to
    the stated tolerances."""
    L, d, per, J, U, mu, Dl, K, ops = case
    say("fusion", L, d, len(ops))
    ho, hl = ham_pair(L, d, per, J, U, mu, Dl, K)
    rng = np.random.default_rng(L * 10 + d)
    th = rng.uniform(-0.6, 0.6, len(ops))
    psi0 = W.random_state(L, d, seed=11, sector=("parity", 0) if Dl != 0 else ("N", L))
    x0 = dev(psi0)
    a, b = torch.empty_like(x0), torch.empty_like(x0)
    ws = lib.workspace(hl, 0, len(ops))
    prev = lib.get_gate_fusion()
    res = {}
    try:
        for mode in (lib.FUSE_ALL, lib.FUSE_FORWARD, lib.FUSE_OFF):
            lib.set_gate_fusion(mode)
            E, n2, g = lib.energy_grad_adjoint(hl, ops, th, x0, a, b, ws)
            res[mode] = (E, g, host(a))
    finally:
        lib.set_gate_fusion(prev)
    Er, gr, _ = O.energy_and_grad_adjoint(ho, psi0.astype(np.complex128), ops, th)
    Eu, gu, _ = res[lib.FUSE_OFF]
    for mode in (lib.FUSE_ALL, lib.FUSE_FORWARD):
        Ef, gf, phif = res[mode]
        assert abs(Ef - Eu) <= 1e-6 * max(1.0, abs(Eu)), mode
        assert np.abs(gf - gu).max() <= 1e-5 * max(1.0, np.abs(gu).max()), mode
        assert abs(Ef - Er) <= 1e-5 * max(1.0, abs(Er)), mode
        assert np.abs(gf - gr).max() <= 1e-4 * max(1.0, np.abs(gr).max()), mode
        # after the reverse sweep phi is back at psi0 (U^+ ... U^+ U ... U = 1)
        assert np.abs(phif - psi0).max() <= 1e-5, mode


@pytest.mark.parametrize("d", [4, 6, 8])
def test_dense_mfma_gate_variant(d):
    """The dense matrix-core gate gives the block kernel's and the oracle's
    result (forward and adjoint), on a ragged tile count and on mode 0."""
    L = 5 if d == 8 else 6
    say("dense gate", L, d)
    psi = W.random_state(L, d, seed=d)
    p128 = psi.astype(np.complex128)
    ws = lib.workspace(lib.ham(L, d), 0, 1)
    prev = lib.get_gate_variant()
    try:
        for o in [("HR", 0, 1), ("PR", 1, 3), ("DH", L - 2, L - 1), ("PI", 0, L - 1), ("HI", 2, 3), ("CK", 0, 2)]:
            for adj in (False, True):
                th = 0.41 if not adj else -0.23
                out = {}
                for v in (lib.GATE_BLOCK, lib.GATE_DENSE_MFMA):
                    lib.set_gate_variant(v)
                    x = dev(psi)
                    lib.apply_gate2(L, d, o, th, x, ws, adjoint=adj)
                    out[v] = host(x)
                ref = O.apply_gate(o, th, p128, L, d, adjoint=adj)
                assert np.abs(out[lib.GATE_DENSE_MFMA] - ref).max() <= 1e-5 * np.abs(ref).max(), (o, adj)
                assert np.abs(out[lib.GATE_DENSE_MFMA] - out[lib.GATE_BLOCK]).max() <= 2e-6 * np.abs(ref).max()
    finally:
        lib.set_gate_variant(prev)


def test_maximum_size_product_state_apply_H_gate_energy():
    """Largest state the library accepts with L <= 24, d <= 16: d^L = 7^11 =
    1,977,326,743 amplitudes (2^31 limit; 15.8 GB per state), Kitaev-Kerr with mu,
    ring.  The input is a product state built on the device from seeded factors;
    the oracle gives exact (H psi) and gate outputs at sampled indices, including
    both ends of the index range, and the exact energy."""
    L, d = 11, 7
    ho, hl = ham_pair(L, d, True, 1.0, 0.0, 0.2, 0.45, 0.15)
    fac = W.product_factors(L, d, seed=17)
    say("max size", L, d, d**L)
    t = torch.from_numpy(fac[-1]).cuda()
    for f in reversed(fac[:-1]):
        t = (t[:, None] * torch.from_numpy(f).cuda()[None, :]).reshape(-1)
    n = d**L
    assert t.numel() == n
    y = torch.empty_like(t)
    ws = lib.workspace(hl, 0, 1)
    E, n2 = lib.apply_H(hl, t, y, ws)
    Eref = O.product_energy(ho, fac)
    assert abs(E - Eref) <= 1e-5 * max(1.0, abs(Eref)), (E, Eref)
    assert abs(n2 - 1.0) <= 1e-4
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.integers(0, n, 300), [0, 1, d - 1, n - 1, n - d, n // 2]]).astype(np.int64)
    got = y[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = np.array([O.product_H_at(ho, fac, int(k)) for k in idx])
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()
    del y
    for o in [("PR", 0, 1), ("HR", L - 2, L - 1), ("DH", 3, 7)]:
        x = t.clone()
        lib.apply_gate2(L, d, o, 0.3, x, ws)
        got = x[torch.from_numpy(idx).cuda()].cpu().numpy()
        ref = np.array([O.product_gate_at(o, 0.3, fac, L, d, int(k)) for k in idx])
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max(), o
        del x


def test_event_timing_samples_one_launch_in_k():
    """Event timing with a sampling interval k times launches 0, k, 2k, ... of
    each kernel family: 8 gate launches give 2 timed ones at k = 4 and 8 at
    k = 1, each with a positive duration; nothing is timed while disabled."""
    L, d = 6, 4
    x = dev(W.random_state(L, d, seed=3))
    ws = lib.workspace(lib.ham(L, d), 0, 1)
    say("event sampling")
    try:
        for k, want in ((4, 2), (1, 8)):
            lib.prof_set_sample(k)
            lib.prof_reset()
            lib.prof_enable(True)
            for _ in range(8):
                lib.apply_gate2(L, d, ("HR", 2, 3), 0.3, x, ws)
            torch.cuda.synchronize()
            lib.prof_enable(False)
            p = lib.prof_query(2)  # FOCK_K_GATE
            assert p["launches"] == want and p["ms"] > 0.0, (k, p)
        lib.prof_reset()
        lib.apply_gate2(L, d, ("HR", 2, 3), 0.3, x, ws)
        torch.cuda.synchronize()
        assert lib.prof_query(2)["launches"] == 0
    finally:
        lib.prof_enable(False)
        lib.prof_set_sample(1)


def test_prepare_then_calls_allocate_no_device_memory():
    """After fock_prepare(L, d) the gate, H psi (every tile schedule) and
    adjoint calls on (L, d) change the device's free memory by nothing (the
    library's kernels are loaded by an earlier call on another cutoff)."""
    L, d = 5, 7
    h0 = lib.ham(3, 4)
    x0 = torch.zeros(64, dtype=torch.complex64, device="cuda")
    x0[0] = 1.0
    lib.apply_H(h0, x0, torch.empty_like(x0), lib.workspace(h0))
    hl = lib.ham(L, d, False, 1.0, 0.5, 0.1, 0.3, 0.2)
    psi = dev(W.random_state(L, d, seed=5))
    y, a, b = torch.empty_like(psi), torch.empty_like(psi), torch.empty_like(psi)
    ws = lib.workspace(hl, 0, 4)
    ops = [("HR", 0, 1), ("PI", 2, 3), ("KERR", 4, -1), ("SR", 1, -1)]
    th = np.array([0.1, -0.2, 0.3, 0.05])
    lib.prepare(L, d)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    prev = lib.get_stencil_schedule()
    try:
        for sc in (0, 1, 2, 3, 4):
            lib.set_stencil_schedule(sc)
            lib.apply_H(hl, psi, y, ws)
    finally:
        lib.set_stencil_schedule(prev)
    lib.apply_gate2(L, d, ("HR", 1, 3), 0.2, psi, ws)
    lib.energy_grad_adjoint(hl, ops, th, psi, a, b, ws)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
