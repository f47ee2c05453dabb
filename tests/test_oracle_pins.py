"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: hand-derived
matrix elements, closed forms (free bosons, Bogoliubov-de Gennes, two-mode
squeezed vacuum, binomial beam-splitter output), symmetry invariants,
independent constructions (Kronecker-built matrices vs tensor stencils) and
finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_c(n, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(n) + 1j * r.standard_normal(n)


# ---------------------------------------------------------------- ladder ops (Sec. II.A)

@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_ladder_action(d):
    a = O.ladder(d)
    for m in range(d):
        e = np.zeros(d)
        e[m] = 1.0
        v = a @ e
        want = np.zeros(d)
        if m > 0:
            want[m - 1] = math.sqrt(m)
        assert np.array_equal(v, want)
        w = a.T @ e
        want = np.zeros(d)
        if m < d - 1:  # truncation: a^+ |d-1> = 0
            want[m + 1] = math.sqrt(m + 1)
        assert np.allclose(w, want, atol=0, rtol=1e-15)
    assert np.allclose(a.T @ a, np.diag(np.arange(d)))
    comm = a @ a.T - a.T @ a
    assert np.allclose(comm, np.diag([1.0] * (d - 1) + [-(d - 1.0)]))


# ---------------------------------------------------------------- Hamiltonian constructions

CASES = [(1, 5, False), (2, 4, False), (2, 3, True), (3, 4, False), (3, 3, True), (4, 3, True), (3, 5, True)]


@pytest.mark.parametrize("L,d,per", CASES)
def test_three_constructions_of_H_agree(L, d, per):
    h = O.Ham(L, d, per, J=0.8, U=0.7, mu=0.3, Delta=0.45, K=0.2)
    H = O.ham_matrix(h, sparse=False)
    assert np.abs(H - H.T).max() == 0.0
    x = rand_c(d**L, L * 10 + d)
    y = H @ x
    assert np.allclose(O.apply_H(h, x), y, atol=1e-12)
    assert np.allclose(O.apply_H_slices(h, x), y, atol=1e-12)


def test_bose_hubbard_two_sites_by_hand():
    """L=2, d=3, N=2 sector {|2,0>, |1,1>, |0,2>}: on-site U/2 n(n-1) gives U on the doubly
    occupied states, hopping <1,1|a_0^+ a_1|0,2> = sqrt(2). Eigenvalues: U (antisymmetric
    combination) and (U +- sqrt(U^2 + 16 J^2)) / 2."""
    J, U = 1.3, 2.1
    h = O.Ham(2, 3, False, J=J, U=U)
    gs = O.ground_state(h, ("N", 2))
    want = sorted([U, (U + math.sqrt(U * U + 16 * J * J)) / 2, (U - math.sqrt(U * U + 16 * J * J)) / 2])
    idx = O.sector_indices(2, 3, ("N", 2))
    Hs = O.ham_matrix(h, sparse=False)[np.ix_(idx, idx)]
    assert np.allclose(np.linalg.eigvalsh(Hs), want, atol=1e-13)
    assert abs(gs["E0"] - want[0]) < 1e-13


def test_symmetries():
    """[H, N_tot] = 0 for Bose-Hubbard (Sec. III.A); [H, P] = 0 for the Kitaev chain (Sec. III.B)."""
    L, d = 3, 4
    occ = O.occupations(L, d).sum(axis=1)
    Ntot = np.diag(occ.astype(float))
    P = np.diag((-1.0) ** occ)
    hb = O.ham_matrix(O.Ham(L, d, True, J=1.0, U=3.0, mu=0.4), sparse=False)
    hk = O.ham_matrix(O.Ham(L, d, False, J=1.0, Delta=0.6, K=0.3, mu=0.2), sparse=False)
    assert np.abs(hb @ Ntot - Ntot @ hb).max() < 1e-13
    assert np.abs(hk @ P - P @ hk).max() < 1e-13
    assert np.abs(hk @ Ntot - Ntot @ hk).max() > 0.1  # pairing breaks U(1)


def test_zero_hopping_is_diagonal_closed_form():
    L, d = 3, 4
    h = O.Ham(L, d, True, J=0.0, U=1.7, mu=0.6, K=0.25)
    H = O.ham_matrix(h, sparse=False)
    occ = O.occupations(L, d)
    want = ((1.7 / 2 + 0.25) * occ * (occ - 1) - 0.6 * occ).sum(axis=1)
    assert np.allclose(H, np.diag(want), atol=1e-14)
    # N = L ground state of the repulsive chain at J = 0 is |1..1> with E0 = 0
    gs = O.ground_state(O.Ham(L, d, True, J=0.0, U=2.0), ("N", L))
    assert abs(gs["E0"]) < 1e-14
    assert abs(abs(gs["vec"][W.fock_index(L, d, [1] * L)]) - 1) < 1e-12


@pytest.mark.parametrize("per", [True, False])
def test_free_bosons(per):
    """U = 0: one-boson energies are the tight-binding band, for any cutoff d >= 2;
    N bosons condense into the lowest orbital when d >= N + 1."""
    L = 5
    for d in (2, 4):
        h = O.Ham(L, d, per, J=1.0)
        idx = O.sector_indices(L, d, ("N", 1))
        Hs = O.ham_matrix(h, sparse=False)[np.ix_(idx, idx)]
        assert np.allclose(np.linalg.eigvalsh(Hs), O.free_boson_single_particle(L, 1.0, per), atol=1e-12)
    N = 3
    h = O.Ham(4, N + 1, per, J=1.0)
    gs = O.ground_state(h, ("N", N))
    assert abs(gs["E0"] - N * O.free_boson_single_particle(4, 1.0, per)[0]) < 1e-11


def test_bdg_closed_forms_agree():
    """Ring dispersion (Appendix A) and the dynamical-matrix route give the same E0."""
    for L in (3, 4, 6):
        a = O.bdg_ground_energy_periodic(L, 1.0, -3.1, 0.5)
        b = O.bdg_ground_energy(L, 1.0, -3.1, 0.5, periodic=True)
        assert abs(a - b) < 1e-12
    with pytest.raises(ValueError):
        O.bdg_ground_energy_periodic(4, 1.0, 0.0, 0.5)  # mu = 0 violates mu < -2(J + Delta)


@pytest.mark.parametrize("per", [True, False])
def test_truncated_kitaev_approaches_bdg(per):
    """The truncated Kitaev chain (even sector) converges to the untruncated Bogoliubov
    ground energy as the cutoff grows, monotonically from above (variational)."""
    L = 3
    exact = O.bdg_ground_energy(L, 1.0, -3.1, 0.5, periodic=per)
    errs = []
    for d in (6, 8, 10, 14):
        h = O.Ham(L, d, per, J=1.0, mu=-3.1, Delta=0.5)
        errs.append(O.ground_state(h, ("parity", 0))["E0"] - exact)
    assert errs[0] > errs[1] > errs[2] > errs[3] > -1e-10
    assert errs[3] < 1e-5


def test_eigh_and_lanczos_agree():
    h = O.Ham(4, 5, False, J=1.0, Delta=0.5, K=0.2)
    a = O.ground_state(h, ("parity", 0))
    b = O.ground_state(h, ("parity", 0), dense_max=10)
    c = O.ground_state(h, ("parity", 0), matrix_free=True)
    assert abs(a["E0"] - b["E0"]) < 1e-10 and abs(a["E0"] - c["E0"]) < 1e-10
    assert abs(abs(np.dot(a["vec"], c["vec"])) - 1) < 1e-8


# ---------------------------------------------------------------- gates (Sec. II.B, Sec. IV.B)

@pytest.mark.parametrize("g", O.GEN_TYPES)
def test_generators_antihermitian_and_gates_unitary(g):
    d = 4
    A = O.generator_local(g, d)
    assert np.abs(A + A.conj().T).max() < 1e-14
    U = O.gate_local(g, d, 0.37)
    assert np.abs(U.conj().T @ U - np.eye(U.shape[0])).max() < 1e-13
    assert np.abs(O.gate_local(g, d, 0.22) @ O.gate_local(g, d, 0.15) - U).max() < 1e-13
    h = 1e-5
    dU = (O.gate_local(g, d, h) - O.gate_local(g, d, -h)) / (2 * h)
    assert np.abs(dU - A).max() < 1e-10 * np.abs(A).max() ** 3  # central-difference error h^2 |A|^3 / 6


def test_generator_matrix_elements_by_hand():
    """Spot matrix elements from the ladder action, local index n_i*d + n_j."""
    d = 4
    li = lambda ni, nj: ni * d + nj  # noqa: E731
    HR = O.generator_local("HR", d)
    assert HR[li(2, 1), li(1, 2)] == pytest.approx(math.sqrt(2) * math.sqrt(2))   # a_i^+ a_j
    assert HR[li(0, 3), li(1, 2)] == pytest.approx(-math.sqrt(1) * math.sqrt(3))  # -a_j^+ a_i
    DH = O.generator_local("DH", d)
    # N_i a_i^+ a_j |1,2> = 2 * sqrt(2) sqrt(2) |2,1>
    assert DH[li(2, 1), li(1, 2)] == pytest.approx(1j * 2 * 2)
    # a_j^+ a_i N_i |1,2> = 1 * sqrt(1) * sqrt(3) |0,3>
    assert DH[li(0, 3), li(1, 2)] == pytest.approx(1j * math.sqrt(3))
    PR = O.generator_local("PR", d)
    assert PR[li(0, 1), li(1, 2)] == pytest.approx(math.sqrt(2))           # a_i a_j
    assert PR[li(2, 3), li(1, 2)] == pytest.approx(-math.sqrt(2) * math.sqrt(3))  # -a_i^+ a_j^+
    assert PR[li(3, 3), li(2, 3)] == 0.0   # truncation kills a^+ |3>


def test_cross_kerr_closed_forms():
    """CK = i N_i N_j: diagonal with entries i n_i n_j (local index n_i d + n_j);
    exp(theta CK) multiplies each amplitude by exp(i theta n_i n_j), checked on a
    random three-mode state with the digits read off the flat index."""
    d = 4
    CK = O.generator_local("CK", d)
    assert CK[2 * d + 3, 2 * d + 3] == pytest.approx(6j)
    assert np.count_nonzero(CK - np.diag(np.diag(CK))) == 0
    L, th = 3, 0.61
    psi = rand_c(d**L, 11)
    for (i, j) in [(0, 1), (0, 2), (1, 2)]:
        out = O.apply_gate(("CK", i, j), th, psi, L, d)
        want = psi.copy()
        for k in range(d**L):
            n = [(k // d**r) % d for r in range(L)]
            want[k] *= np.exp(1j * th * n[i] * n[j])
        assert np.abs(out - want).max() < 1e-13


@pytest.mark.parametrize("g,phase", [("SR", 1.0), ("SI", 1j)])
def test_single_mode_squeezed_vacuum(g, phase):
    """exp(theta A)|0> with A = (e^{-i phi} a^2 - e^{i phi} a^+2)/2 is the squeezed
    vacuum sum_n (-e^{i phi} tanh theta)^n sqrt((2n)!)/(2^n n!) / sqrt(cosh theta) |2n>
    as d grows; SR has phi = 0, SI phi = -pi/2 (so -e^{i phi} = i)."""
    L, d, th = 1, 48, 0.3
    psi = O.apply_gate((g, 0, -1), th, O.fock_state(L, d, [0]), L, d)
    want = np.zeros(d, dtype=complex)
    for n in range(d // 2):
        want[2 * n] = ((-1.0 if g == "SR" else phase) * math.tanh(th)) ** n * \
            math.sqrt(math.factorial(2 * n)) / (2**n * math.factorial(n)) / math.sqrt(math.cosh(th))
    assert np.abs(psi - want).max() < 1e-10


def test_beam_splitter_binomial_closed_form():
    """exp(theta HR)|n, 0> = sum_k sqrt(C(n,k)) cos^(n-k) (-sin)^k |n-k, k> (exact for n <= d-1)."""
    L, d, th = 2, 6, 0.41
    for n in range(d):
        psi = O.apply_gate(("HR", 0, 1), th, O.fock_state(L, d, [n, 0]), L, d)
        want = np.zeros(d * d, dtype=complex)
        for k in range(n + 1):
            want[W.fock_index(L, d, [n - k, k])] = math.sqrt(math.comb(n, k)) * math.cos(th) ** (n - k) * (-math.sin(th)) ** k
        assert np.abs(psi - want).max() < 1e-13


def test_two_mode_squeezed_vacuum():
    """exp(r (a_i a_j - a_i^+ a_j^+))|0,0> -> sum_n (-tanh r)^n / cosh r |n,n> as d grows."""
    L, d, r = 2, 24, 0.3
    psi = O.apply_gate(("PR", 0, 1), r, O.fock_state(L, d, [0, 0]), L, d)
    want = np.zeros(d * d, dtype=complex)
    for n in range(d):
        want[W.fock_index(L, d, [n, n])] = (-math.tanh(r)) ** n / math.cosh(r)
    assert np.abs(psi - want).max() < 1e-10


@pytest.mark.parametrize("g,sector", [("HR", ("N", 3)), ("HI", ("N", 3)), ("DH", ("N", 3)),
                                      ("PR", ("parity", 0)), ("PI", ("parity", 0)),
                                      ("KERR", ("N", 3)), ("ROT", ("parity", 1)),
                                      ("CK", ("N", 3)), ("CK", ("parity", 1)),
                                      ("SR", ("parity", 0)), ("SI", ("parity", 1))])
def test_gates_preserve_sector(g, sector):
    L, d = 3, 4
    psi = W.random_state(L, d, 7, sector=sector, dtype=np.complex128)
    op = (g, 0, 2) if g not in O.SINGLE_MODE else (g, 1, -1)
    out = O.apply_gate(op, 0.83, psi, L, d)
    assert O.leakage(out, L, d, sector) == 0.0
    assert abs(np.vdot(out, out).real - 1.0) < 1e-13


# ---------------------------------------------------------------- pool gradients (Eq. grad)

def test_pool_gradient_fock_state_closed_form():
    """Fock product state, hopping rotation on a bond:
    g = -2J [(n_i+1) n_j [n_i<d-1] - n_i (n_j+1) [n_j<d-1]]; zero on non-bonds;
    HI and DH vanish (purely imaginary generators on a real state with real H)."""
    L, d, J = 4, 4, 0.9
    h = O.Ham(L, d, False, J=J, U=1.1)
    occ = [3, 0, 2, 1]
    psi = O.fock_state(L, d, occ)
    pool = W.pool(L, "all", False, W.BH_TYPES + ("CK",))
    g = O.pool_gradients(h, psi, pool)
    for k, (t, i, j) in enumerate(pool):
        if t == "HR" and j == i + 1:
            ni, nj = occ[i], occ[j]
            want = -2 * J * ((ni + 1) * nj * (ni < d - 1) - ni * (nj + 1) * (nj < d - 1))
        else:
            want = 0.0
        assert abs(g[k] - want) < 1e-12, (t, i, j)


def test_pool_gradient_kitaev_vacuum():
    """Vacuum: only the two-mode squeezer PR on bonds has a gradient, -2 Delta."""
    L, d, Dl = 4, 4, 0.35
    h = O.Ham(L, d, False, J=1.0, Delta=Dl, K=0.2)
    pool = W.pool(L, "all", False, W.KITAEV_TYPES) + W.site_ops(L, ("SR", "SI", "KERR"))
    g = O.pool_gradients(h, O.fock_state(L, d, [0] * L), pool)
    for k, (t, i, j) in enumerate(pool):
        want = -2 * Dl if (t == "PR" and j == i + 1) else 0.0
        assert abs(g[k] - want) < 1e-13


def test_pool_gradient_equals_commutator_and_fd():
    L, d = 3, 3
    h = O.Ham(L, d, True, J=1.0, U=0.8, Delta=0.4, K=0.1, mu=0.2)
    psi = rand_c(d**L, 3)
    psi /= np.linalg.norm(psi)
    pool = W.pool(L, "all", True, ("HR", "HI", "DH", "PR", "PI", "CK")) + [("KERR", 1, -1), ("ROT", 2, -1),
                                                                          ("SR", 0, -1), ("SI", 2, -1)]
    g = O.pool_gradients(h, psi, pool)
    assert np.allclose(g, O.commutator_gradients(h, psi, pool), atol=1e-12)
    for k, op in enumerate(pool):
        e = lambda t: O.energy(h, O.apply_gate(op, t, psi, L, d))[0]  # noqa: E731
        fd = (e(1e-5) - e(-1e-5)) / 2e-5
        assert abs(fd - g[k]) < 1e-7


def test_real_state_imaginary_generators_vanish():
    L, d = 3, 4
    h = O.Ham(L, d, False, J=1.0, U=0.5, Delta=0.3)
    psi = np.random.default_rng(1).standard_normal(d**L).astype(complex)
    pool = W.pool(L, "all", False, ("HR", "HI", "DH", "PR", "PI"))
    g = O.pool_gradients(h, psi, pool)
    for k, (t, _, _) in enumerate(pool):
        if t in ("HI", "DH", "PI"):
            assert abs(g[k]) < 1e-12


# ---------------------------------------------------------------- adjoint

def test_adjoint_matches_finite_differences():
    L, d = 3, 4
    h = O.Ham(L, d, False, J=1.0, Delta=0.5, K=0.2)
    pool = W.pool(L, "nn", False, W.KITAEV_TYPES) + [("KERR", 0, -1), ("ROT", 2, -1), ("DH", 0, 2), ("CK", 0, 2),
                                                     ("CK", 1, 2), ("SR", 1, -1), ("SI", 0, -1)]
    ops, th = W.random_circuit(pool, 9, 4)
    psi0 = O.fock_state(L, d, [0] * L)
    E, g, n2 = O.energy_and_grad_adjoint(h, psi0, ops, th)
    fd = O.fd_gradient(h, psi0, ops, th, h=1e-4)
    assert abs(n2 - 1) < 1e-13
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(g).max())
    assert abs(E - O.energy_of(h, psi0, ops, th)) < 1e-13
    # the sliced H psi gives the same sweep (open and ring lattices)
    E2, g2, _ = O.energy_and_grad_adjoint(h, psi0, ops, th, apply_h=O.apply_H_slices)
    assert abs(E2 - E) < 1e-12 and np.abs(g2 - g).max() < 1e-12
    hr = O.Ham(4, 3, True, J=1.0, U=0.7, mu=0.2, Delta=0.3, K=0.1)
    opr, thr = W.random_circuit(W.pool(4, "nn", True, W.KITAEV_TYPES), 6, 8)
    p0 = W.random_state(4, 3, seed=1, sector=("parity", 0)).astype(complex)
    Ea, ga, _ = O.energy_and_grad_adjoint(hr, p0, opr, thr)
    Eb, gb, _ = O.energy_and_grad_adjoint(hr, p0, opr, thr, apply_h=O.apply_H_slices)
    assert abs(Ea - Eb) < 1e-12 and np.abs(ga - gb).max() < 1e-12
    pr = W.pool(4, "nn", True, W.KITAEV_TYPES)
    psr = O.ansatz_state(p0, opr, thr, 4, 3)
    assert np.abs(O.pool_gradients(hr, psr, pr) - O.pool_gradients(hr, psr, pr, apply_h=O.apply_H_slices)).max() < 1e-12


# ---------------------------------------------------------------- ADAPT

def test_bfgs_single_gate_closed_form():
    """H = -J(a_0^+ a_1 + h.c.), psi0 = |1,0>: E(theta) = J sin(2 theta), minimum -J."""
    h = O.Ham(2, 2, False, J=1.0)
    x, E, _, _ = O.bfgs(h, O.fock_state(2, 2, [1, 0]), [("HR", 0, 1)], [0.1], gtol=1e-10)
    assert abs(E + 1.0) < 1e-12 and abs(x[0] + math.pi / 4) < 1e-6


def test_adapt_kitaev_small_is_variational_and_monotone():
    L, d = 3, 4
    h = O.Ham(L, d, False, J=1.0, Delta=0.5, K=0.2)
    E0 = O.ground_state(h, ("parity", 0))["E0"]
    pool = W.pool(L, "nn", False, W.KITAEV_TYPES)
    recs = O.adapt(h, O.fock_state(L, d, [0] * L), pool, max_iters=12)
    Es = [r["E"] for r in recs]
    assert all(b <= a + 1e-10 for a, b in zip(Es, Es[1:]))
    assert min(Es) >= E0 - 1e-9
    assert recs[0]["k"] == pool.index(("PR", 0, 1))  # -2 Delta ties on both bonds: lowest index


def test_select_tie_band():
    assert O.select_operator(np.array([0.5, -1.0, 1.0 - 5e-5, 0.2])) == 1
    assert O.select_operator(np.array([0.99, -1.0])) == 1
    assert O.select_operator(np.array([-1.0 + 1e-5, 1.0])) == 0


def test_golden_fixtures():
    """Hand-derived fixtures stored with their derivation and citation."""
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        cases = json.load(f)
    for c in cases:
        h = O.Ham(**c["ham"])
        if c["kind"] == "sector_spectrum":
            idx = O.sector_indices(h.L, h.d, tuple(c["sector"]))
            Hs = O.ham_matrix(h, sparse=False)[np.ix_(idx, idx)]
            assert np.allclose(np.linalg.eigvalsh(Hs), c["eigenvalues"], atol=1e-12), c["name"]
        elif c["kind"] == "pool_gradient":
            psi = O.fock_state(h.L, h.d, c["occ"])
            g = O.pool_gradients(h, psi, [tuple(o) for o in c["pool"]])
            assert np.allclose(g, c["g"], atol=1e-12), c["name"]


def test_product_state_oracle_functions():
    """The product-state shortcuts equal the general oracle on the explicit
    vector: (H psi) at every index, the energy, and gates at every index."""
    import workload as W
    for (L, d, per, U, mu, Dl, K) in [(4, 3, True, 1.2, 0.3, 0.4, 0.1), (3, 5, False, 0.0, 0.0, 0.5, 0.2)]:
        h = O.Ham(L, d, per, 1.0, U, mu, Dl, K)
        fac = W.product_factors(L, d, seed=L + d)
        psi = W.product_state(fac, dtype=np.complex128)
        Hpsi = O.apply_H(h, psi)
        for k in range(d**L):
            assert abs(O.product_H_at(h, fac, k) - Hpsi[k]) < 1e-12
        E = np.vdot(psi, Hpsi).real / np.vdot(psi, psi).real
        assert abs(O.product_energy(h, fac) - E) < 1e-12
        for op in [("PR", 0, 1), ("DH", 1, L - 1), ("KERR", 1, -1)]:
            out = O.apply_gate(op, 0.37, psi, L, d)
            for k in range(d**L):
                assert abs(O.product_gate_at(op, 0.37, fac, L, d, k) - out[k]) < 1e-12


@pytest.mark.parametrize("t", ["BS", "TMS", "SQ"])
def test_two_parameter_gates_are_rotation_conjugated_fixed_phase_gates(t):
    """The paper's two-parameter gates (Sec. II.B), built directly as
    exp(theta A(phi)), equal the phi = 0 gate conjugated by phase rotations
    R(a) = exp(i a N): BS(theta, phi) = R_2(phi) exp(-theta HR) R_2(-phi),
    S2(theta, phi) = R_2(-phi) exp(theta PR) R_2(phi) and
    S(theta, phi) = R(phi/2) exp(theta SR) R(-phi/2), on the truncated space,
    for several angles (a wrong sign of phi, a missing factor 1/2 or a
    transposed mode order fails)."""
    import scipy.linalg

    d = 5
    a = O.ladder(d)
    ad = a.T
    I = np.eye(d)
    rng = np.random.default_rng(7)
    for _ in range(4):
        th, ph = rng.uniform(-1.5, 1.5, 2)
        if t == "BS":
            A = np.exp(1j * ph) * np.kron(a, ad) - np.exp(-1j * ph) * np.kron(ad, a)
            R = lambda x: np.kron(I, O.gate_local("ROT", d, x))  # noqa: E731  (rotation of mode 2)
            M = R(ph) @ O.gate_local("HR", d, -th) @ R(-ph)
        elif t == "TMS":
            A = np.exp(1j * ph) * np.kron(a, a) - np.exp(-1j * ph) * np.kron(ad, ad)
            R = lambda x: np.kron(I, O.gate_local("ROT", d, x))  # noqa: E731
            M = R(-ph) @ O.gate_local("PR", d, th) @ R(ph)
        else:
            A = 0.5 * (np.exp(-1j * ph) * a @ a - np.exp(1j * ph) * ad @ ad)
            M = O.gate_local("ROT", d, ph / 2) @ O.gate_local("SR", d, th) @ O.gate_local("ROT", d, -ph / 2)
        U = scipy.linalg.expm(th * A)
        assert np.abs(U - M).max() < 1e-12


# ---------------------------------------------------------------- HVA-CV-VQE baseline

def test_hva_single_boson_two_sites_reaches_hopping_ground_state():
    """One HVA layer (Sec. IV.A) on two sites holding one boson: HI(0,1), Kerr
    and rotation phases give cos t e^{ia}|1,0> + i sin t e^{ib}|0,1>, whose
    energy 2J cos t sin t sin(b - a) has the closed-form minimum -J (t = pi/4,
    b - a = -pi/2), the exact ground energy."""
    h = O.Ham(2, 3, False, J=1.0)
    layer = W.hva_layer(2, False, "bh")
    assert layer == [("HI", 0, 1), ("KERR", 0, -1), ("KERR", 1, -1), ("ROT", 0, -1), ("ROT", 1, -1)]
    recs = O.hva(h, O.fock_state(2, 3, [1, 0]), layer, W.hva_inits(len(layer), 1, seed=0), gtol=1e-10)
    assert abs(recs[0]["E"] - (-1.0)) < 1e-9


def test_hva_pairing_two_modes_reaches_bogoliubov_energy():
    """Two modes with pairing only (J = 0, mu < 0): H = eps (n_0 + n_1) +
    Delta (a_0 a_1 + h.c.) with eps = -mu has the Bogoliubov ground energy
    sqrt(eps^2 - Delta^2) - eps (a two-mode squeezed vacuum); one Kitaev HVA
    layer (PI, HI, rotations) from the vacuum reaches it at d = 16, where the
    truncation is negligible."""
    eps, dl = 2.0, 0.5
    h = O.Ham(2, 16, False, J=0.0, mu=-eps, Delta=dl)
    layer = W.hva_layer(2, False, "bkc")
    assert layer == [("PI", 0, 1), ("HI", 0, 1), ("ROT", 0, -1), ("ROT", 1, -1)]
    recs = O.hva(h, O.fock_state(2, 16, [0, 0]), layer, W.hva_inits(len(layer), 1, seed=3), gtol=1e-10)
    assert abs(recs[0]["E"] - (np.sqrt(eps**2 - dl**2) - eps)) < 1e-9


def test_hva_zero_start_is_stationary_and_layers_repeat():
    """All-zero angles leave a Fock start unchanged (every gradient vanishes
    there: the HVA generators are off-diagonal or diagonal phases), so BFGS stops
    at once with the start's diagonal energy; each layer repeats the same gates."""
    h = O.Ham(3, 4, True, J=1.0, U=2.0)
    layer = W.hva_layer(3, True, "bh")
    assert len(layer) == 9
    recs = O.hva(h, O.fock_state(3, 4, [2, 1, 0]), layer, [np.zeros(9), np.zeros(9)], gtol=1e-10)
    assert abs(recs[-1]["E"] - (2.0 / 2 * 2 * 1)) < 1e-12  # (U/2) n(n-1) at n = 2
    assert recs[-1]["ops"] == layer + layer and np.all(recs[-1]["theta"] == 0.0)
    assert W.hva_layer(4, True, "bkck") == ([("PI", i, j) for i, j in [(0, 1), (1, 2), (2, 3), (0, 3)]] +
                                            [("HI", i, j) for i, j in [(0, 1), (1, 2), (2, 3), (0, 3)]] +
                                            [("KERR", r, -1) for r in range(4)] + [("ROT", r, -1) for r in range(4)])
