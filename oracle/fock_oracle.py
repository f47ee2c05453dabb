"""FP64 CPU oracle for the truncated-Fock statevector path of CV-ADAPT-VQE.

TEST INFRASTRUCTURE ONLY. This module is imported by the test suite, by the
smoke check and by the CPU-baseline leg of the benchmark.  The product path
(the HIP library and its Python binding) never imports, links or calls it, and
it shares no code, tables or constants with that path.

Everything here is plain NumPy/SciPy in complex128/float64, written to be read
against the paper:

* Fock space, truncated ladder operators: Sec. II.A (ladder action on |n>,
  truncation to D levels).
* Bose-Hubbard and bosonic Kitaev(+Kerr) Hamiltonians: Sec. III, Eqs.
  (BoseHubbard), (BosonicKitaevChain), (BosonicKitaevChain_Kerr), with the sign
  conventions of the build's configurations (+U/2 n(n-1), +Delta(aa+h.c.),
  +K n(n-1)); the pairing sign is a gauge choice a_r -> i a_r and leaves the
  spectrum unchanged.
* Gates O = exp(theta A): Sec. II.B and Sec. IV.B (single-parameter gate form);
  the truncated generator is exponentiated exactly (no renormalisation).
* Pool gradient g = <psi|[H, A]|psi> = 2 Re <H psi | A psi>: Sec. IV.B, Eq. (grad).
* ADAPT loop (select largest |g|, append, re-optimise all parameters with
  BFGS, L-infinity gradient tolerance min(1e-6, 1e-5 |g_sel|), at most 1000
  iterations): Sec. IV.B and Sec. V.A.
* Exact diagonalisation in a fixed boson-number or parity sector: Sec. III.A
  (N_tot conservation), Sec. III.B (global parity).
* Bogoliubov-de Gennes ground energy of the quadratic chain: Appendix A.

Index convention: a basis state |n_0, ..., n_{L-1}> sits at flat index
sum_r n_r d^r (mode 0 has stride 1).  Two-mode local matrices on the ordered
pair (i, j) use the local index n_i * d + n_j (i.e. numpy.kron(X_i, Y_j)).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Iterable, Sequence

import numpy as np
import scipy.linalg
import scipy.optimize
import scipy.sparse
import scipy.sparse.linalg

# --------------------------------------------------------------------------
# Model description
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class Ham:
    """Lattice Hamiltonian parameters.

    H = sum_bonds [ -J (a_i^+ a_j + a_j^+ a_i) + Delta (a_i a_j + a_i^+ a_j^+) ]
        + sum_r [ (U/2 + K) N_r (N_r - 1) - mu N_r ]
    Bose-Hubbard: Delta = K = 0.  Kitaev + Kerr: U = 0.
    """

    L: int
    d: int
    periodic: bool = False
    J: float = 1.0
    U: float = 0.0
    mu: float = 0.0
    Delta: float = 0.0
    K: float = 0.0


GEN_TYPES = ("HR", "HI", "DH", "PR", "PI", "KERR", "ROT", "CK", "SR", "SI")
SINGLE_MODE = ("KERR", "ROT", "SR", "SI")


def bonds(L: int, periodic: bool) -> list[tuple[int, int]]:
    """Nearest-neighbour bonds of the chain; the periodic wrap bond joins modes
    L-1 and 0 and is added once, only for L >= 3 (for L = 2 it would repeat
    the bond (0, 1))."""
    out = [(r, r + 1) for r in range(L - 1)]
    if periodic and L >= 3:
        out.append((0, L - 1))
    return out


# --------------------------------------------------------------------------
# Single-mode operators (Sec. II.A)
# --------------------------------------------------------------------------


def ladder(d: int) -> np.ndarray:
    """Truncated annihilation operator: a|m> = sqrt(m)|m-1> for m = 1..d-1."""
    a = np.zeros((d, d))
    for m in range(1, d):
        a[m - 1, m] = np.sqrt(m)
    return a


def number(d: int) -> np.ndarray:
    return np.diag(np.arange(d, dtype=float))


def onsite(ham: Ham) -> np.ndarray:
    """Diagonal single-site term (U/2 + K) N (N - 1) - mu N."""
    n = np.arange(ham.d, dtype=float)
    return np.diag((ham.U / 2.0 + ham.K) * n * (n - 1.0) - ham.mu * n)


# --------------------------------------------------------------------------
# Full-space operators by Kronecker products (small lattices only)
# --------------------------------------------------------------------------


def embed(ops: dict, L: int, d: int, sparse: bool = True):
    """Kronecker embedding of single-mode matrices {mode: matrix}; mode L-1 is the
    leftmost factor so that mode 0 is the fastest-varying index."""
    eye = np.eye(d)
    mats = [ops.get(r, eye) for r in range(L - 1, -1, -1)]
    if sparse:
        out = scipy.sparse.csr_matrix(mats[0])
        for m in mats[1:]:
            out = scipy.sparse.kron(out, scipy.sparse.csr_matrix(m), format="csr")
        return out
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def ham_matrix(ham: Ham, sparse: bool = True):
    """H assembled term by term from Kronecker products of the truncated ladder
    operators (construction independent of the stencil forms below)."""
    L, d = ham.L, ham.d
    a = ladder(d)
    ad = a.T
    H = embed({}, L, d, sparse) * 0.0
    for (i, j) in bonds(L, ham.periodic):
        if ham.J != 0.0:
            H = H - ham.J * (embed({i: ad, j: a}, L, d, sparse) + embed({i: a, j: ad}, L, d, sparse))
        if ham.Delta != 0.0:
            H = H + ham.Delta * (embed({i: a, j: a}, L, d, sparse) + embed({i: ad, j: ad}, L, d, sparse))
    os_ = onsite(ham)
    for r in range(L):
        H = H + embed({r: os_}, L, d, sparse)
    return H


# --------------------------------------------------------------------------
# Matrix-free application on the d^L tensor
# --------------------------------------------------------------------------


def _axis(L: int, r: int) -> int:
    # C-order reshape of the flat vector puts mode L-1 first.
    return L - 1 - r


def apply_1(mat: np.ndarray, r: int, psi: np.ndarray, L: int, d: int) -> np.ndarray:
    """Apply a d x d matrix to mode r."""
    T = psi.reshape((d,) * L)
    ax = _axis(L, r)
    out = np.tensordot(mat, T, axes=([1], [ax]))
    return np.moveaxis(out, 0, ax).reshape(-1)


def apply_2(mat: np.ndarray, i: int, j: int, psi: np.ndarray, L: int, d: int) -> np.ndarray:
    """Apply a d^2 x d^2 matrix (local index n_i*d + n_j) to the ordered mode pair (i, j)."""
    T = psi.reshape((d,) * L)
    M = mat.reshape(d, d, d, d)
    ai, aj = _axis(L, i), _axis(L, j)
    out = np.tensordot(M, T, axes=([2, 3], [ai, aj]))
    return np.moveaxis(out, [0, 1], [ai, aj]).reshape(-1)


def apply_H(ham: Ham, psi: np.ndarray) -> np.ndarray:
    """H psi term by term, each term a product of single-mode ladder matrices
    applied along tensor axes."""
    L, d = ham.L, ham.d
    a = ladder(d)
    ad = a.T
    psi = np.asarray(psi)
    out = np.zeros(psi.shape, dtype=np.result_type(psi.dtype, float))
    for (i, j) in bonds(L, ham.periodic):
        if ham.J != 0.0:
            out -= ham.J * apply_1(ad, i, apply_1(a, j, psi, L, d), L, d)
            out -= ham.J * apply_1(a, i, apply_1(ad, j, psi, L, d), L, d)
        if ham.Delta != 0.0:
            out += ham.Delta * apply_1(a, i, apply_1(a, j, psi, L, d), L, d)
            out += ham.Delta * apply_1(ad, i, apply_1(ad, j, psi, L, d), L, d)
    os_ = onsite(ham)
    for r in range(L):
        out += apply_1(os_, r, psi, L, d)
    return out


def apply_H_slices(ham: Ham, psi: np.ndarray) -> np.ndarray:
    """H psi by shifted tensor slices (faster form used for large-sector
    Lanczos).  Each term adds coef(n) * psi[n + shift] for the neighbour it
    connects, the coefficient being the product of the two ladder factors."""
    L, d = ham.L, ham.d
    T = np.asarray(psi).reshape((d,) * L)
    out = np.zeros_like(T, dtype=np.result_type(T.dtype, float))
    sq = np.sqrt(np.arange(d + 1, dtype=float))

    def view(arr, sel):
        return arr[tuple(sel)]

    def bshape(ax, vec):
        shp = [1] * L
        shp[ax] = vec.shape[0]
        return vec.reshape(shp)

    for (i, j) in bonds(L, ham.periodic):
        ai, aj = _axis(L, i), _axis(L, j)
        # Each entry: (shift in n_i, shift in n_j, coefficient) for out[n] += c psi[n + shift].
        terms = []
        if ham.J != 0.0:
            terms.append((-1, +1, -ham.J))  # a_i^+ a_j : out[n] <- psi[n - e_i + e_j] sqrt(n_i) sqrt(n_j+1)
            terms.append((+1, -1, -ham.J))  # a_j^+ a_i
        if ham.Delta != 0.0:
            terms.append((+1, +1, ham.Delta))  # a_i a_j : out[n] <- psi[n + e_i + e_j] sqrt(n_i+1) sqrt(n_j+1)
            terms.append((-1, -1, ham.Delta))  # a_i^+ a_j^+
        for (di, dj, c) in terms:
            o_sel = [slice(None)] * L
            p_sel = [slice(None)] * L
            ci = _coef_range(di, d, sq)
            cj = _coef_range(dj, d, sq)
            o_sel[ai], p_sel[ai] = ci[0], ci[1]
            o_sel[aj], p_sel[aj] = cj[0], cj[1]
            coef = c * bshape(ai, ci[2]) * bshape(aj, cj[2])
            view(out, o_sel)[...] += coef * view(T, p_sel)
    n = np.arange(d, dtype=float)
    diag1 = (ham.U / 2.0 + ham.K) * n * (n - 1.0) - ham.mu * n
    for r in range(L):
        out += bshape(_axis(L, r), diag1) * T
    return out.reshape(-1)


def _coef_range(shift: int, d: int, sq: np.ndarray):
    """Output slice, input slice and ladder factor along one axis for a term that
    reads psi at n + shift.  shift = -1 is a creation (factor sqrt(n)), shift = +1
    an annihilation (factor sqrt(n + 1))."""
    if shift == -1:  # out index n in 1..d-1 reads n-1; a^+ factor sqrt(n)
        return slice(1, d), slice(0, d - 1), sq[1:d]
    # out index n in 0..d-2 reads n+1; a factor sqrt(n+1)
    return slice(0, d - 1), slice(1, d), sq[1:d]


# --------------------------------------------------------------------------
# Generators and gates (Sec. II.B, Sec. IV.B)
# --------------------------------------------------------------------------


def generator_local(gtype: str, d: int) -> np.ndarray:
    """Anti-Hermitian generator A as a local matrix.

    Two-mode (ordered pair (i, j), local index n_i*d + n_j):
      HR = a_i^+ a_j - a_j^+ a_i          (beam splitter, phi = pi)
      HI = i (a_i^+ a_j + a_j^+ a_i)      (beam splitter, phi = pi/2)
      DH = i (N_i a_i^+ a_j + a_j^+ a_i N_i)   (density-assisted hop)
      PR = a_i a_j - a_i^+ a_j^+          (two-mode squeezer, phi = 0)
      PI = i (a_i a_j + a_i^+ a_j^+)      (two-mode squeezer, phi = pi/2)
      CK = i N_i N_j                      (cross-Kerr, Sec. II.B)
    Single-mode: KERR = i N^2, ROT = i N, and the squeezer's generator
    (theta/2)(e^{-i phi} a^2 - e^{i phi} a^+2) / theta at two phases:
      SR = (a^2 - a^+2) / 2               (phi = 0)
      SI = i (a^2 + a^+2) / 2             (phi = -pi/2)
    """
    a = ladder(d)
    ad = a.T
    N = number(d)
    if gtype == "HR":
        return np.kron(ad, a) - np.kron(a, ad)
    if gtype == "HI":
        return 1j * (np.kron(ad, a) + np.kron(a, ad))
    if gtype == "DH":
        return 1j * (np.kron(N @ ad, a) + np.kron(a @ N, ad))
    if gtype == "PR":
        return np.kron(a, a) - np.kron(ad, ad)
    if gtype == "PI":
        return 1j * (np.kron(a, a) + np.kron(ad, ad))
    if gtype == "CK":
        return 1j * np.kron(N, N)
    if gtype == "SR":
        return 0.5 * (a @ a - ad @ ad)
    if gtype == "SI":
        return 0.5j * (a @ a + ad @ ad)
    if gtype == "KERR":
        return 1j * (N @ N)
    if gtype == "ROT":
        return 1j * N
    raise ValueError(gtype)


def apply_local(mat: np.ndarray, op, psi: np.ndarray, L: int, d: int) -> np.ndarray:
    gtype, i, j = op
    if gtype in SINGLE_MODE:
        return apply_1(mat, i, psi, L, d)
    return apply_2(mat, i, j, psi, L, d)


def apply_generator(op, psi: np.ndarray, L: int, d: int) -> np.ndarray:
    return apply_local(generator_local(op[0], d), op, psi, L, d)


def gate_local(gtype: str, d: int, theta: float) -> np.ndarray:
    """O(theta) = exp(theta A) of the truncated generator (exactly unitary)."""
    return scipy.linalg.expm(theta * generator_local(gtype, d))


def apply_gate(op, theta: float, psi: np.ndarray, L: int, d: int, adjoint: bool = False) -> np.ndarray:
    t = -theta if adjoint else theta  # O(theta)^+ = exp(-theta A) for anti-Hermitian A
    return apply_local(gate_local(op[0], d, t), op, psi, L, d)


def ansatz_state(psi0: np.ndarray, ops: Sequence, thetas: Sequence[float], L: int, d: int) -> np.ndarray:
    """psi = O_n(theta_n) ... O_1(theta_1) psi0; the newest gate acts last (Sec. IV.B)."""
    psi = np.asarray(psi0, dtype=complex)
    for op, th in zip(ops, thetas):
        psi = apply_gate(op, th, psi, L, d)
    return psi


# --------------------------------------------------------------------------
# Energy, pool gradients, parameter gradients
# --------------------------------------------------------------------------


def energy(ham: Ham, psi: np.ndarray) -> tuple[float, float]:
    """(<psi|H|psi>, <psi|psi>)."""
    h = apply_H(ham, psi)
    return float(np.vdot(psi, h).real), float(np.vdot(psi, psi).real)


def pool_gradients(ham: Ham, psi: np.ndarray, pool: Sequence, apply_h=None) -> np.ndarray:
    """g_k = <psi|[H, A_k]|psi> = 2 Re <H psi|A_k psi> for anti-Hermitian A_k (Eq. grad).
    apply_h: as in energy_and_grad_adjoint (apply_H by default)."""
    L, d = ham.L, ham.d
    h = (apply_h or apply_H)(ham, psi)
    return np.array([2.0 * np.vdot(h, apply_generator(op, psi, L, d)).real for op in pool])


def commutator_gradients(ham: Ham, psi: np.ndarray, pool: Sequence) -> np.ndarray:
    """Same quantity evaluated literally as <psi|(H A - A H)|psi> on the dense
    matrices (small lattices; an independent check of the 2 Re form)."""
    L, d = ham.L, ham.d
    H = ham_matrix(ham, sparse=False)
    out = []
    for op in pool:
        A = np.zeros((d**L, d**L), dtype=complex)
        for c in range(d**L):
            e = np.zeros(d**L, dtype=complex)
            e[c] = 1.0
            A[:, c] = apply_generator(op, e, L, d)
        C = H @ A - A @ H
        out.append(np.vdot(psi, C @ psi).real)
    return np.array(out)


def energy_and_grad_adjoint(ham: Ham, psi0: np.ndarray, ops: Sequence, thetas: Sequence[float], apply_h=None):
    """E(theta) = <psi|H|psi> and dE/dtheta_k = 2 Re <lambda_k|A_k phi_k> by one
    reverse sweep, with phi_k = O_k ... O_1 psi0 and
    lambda_k = O_{k+1}^+ ... O_n^+ H psi_n (uses dO_k/dtheta_k = A_k O_k).
    apply_h: which of the oracle's H psi constructions to use (apply_H by
    default; apply_H_slices is the same operator, several times faster on
    large lattices, and pinned against apply_H and the dense matrix)."""
    L, d = ham.L, ham.d
    phi = ansatz_state(psi0, ops, thetas, L, d)
    lam = (apply_h or apply_H)(ham, phi)
    E = float(np.vdot(phi, lam).real)
    n2 = float(np.vdot(phi, phi).real)
    g = np.zeros(len(ops))
    for k in range(len(ops) - 1, -1, -1):
        g[k] = 2.0 * np.vdot(lam, apply_generator(ops[k], phi, L, d)).real
        phi = apply_gate(ops[k], thetas[k], phi, L, d, adjoint=True)
        lam = apply_gate(ops[k], thetas[k], lam, L, d, adjoint=True)
    return E, g, n2


def energy_of(ham: Ham, psi0, ops, thetas) -> float:
    psi = ansatz_state(psi0, ops, thetas, ham.L, ham.d)
    return energy(ham, psi)[0]


def fd_gradient(ham: Ham, psi0, ops, thetas, h: float = 1e-4) -> np.ndarray:
    """Central finite differences of E(theta)."""
    th = np.array(thetas, dtype=float)
    g = np.zeros(len(th))
    for k in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        g[k] = (energy_of(ham, psi0, ops, tp) - energy_of(ham, psi0, ops, tm)) / (2.0 * h)
    return g


# --------------------------------------------------------------------------
# States and sectors
# --------------------------------------------------------------------------


def fock_state(L: int, d: int, occ: Sequence[int]) -> np.ndarray:
    psi = np.zeros(d**L, dtype=complex)
    psi[sum(int(n) * d**r for r, n in enumerate(occ))] = 1.0
    return psi


def occupations(L: int, d: int) -> np.ndarray:
    """occ[idx, r] = n_r of flat index idx."""
    idx = np.arange(d**L)
    return np.stack([(idx // d**r) % d for r in range(L)], axis=1)


def sector_indices(L: int, d: int, sector) -> np.ndarray:
    """sector = ("N", k): total boson number k; ("parity", p): total number mod 2 == p."""
    tot = occupations(L, d).sum(axis=1)
    kind, val = sector
    if kind == "N":
        return np.nonzero(tot == val)[0]
    if kind == "parity":
        return np.nonzero(tot % 2 == val)[0]
    raise ValueError(kind)


def leakage(psi: np.ndarray, L: int, d: int, sector) -> float:
    """Total probability outside the sector."""
    mask = np.ones(d**L, dtype=bool)
    mask[sector_indices(L, d, sector)] = False
    return float(np.sum(np.abs(psi[mask]) ** 2))


# --------------------------------------------------------------------------
# Exact diagonalisation in a symmetry sector
# --------------------------------------------------------------------------


def ground_state(ham: Ham, sector, dense_max: int = 20000, tol: float = 1e-12, seed: int = 0,
                 want_vector: bool = True, matrix_free: bool | None = None):
    """Lowest eigenpair of H restricted to a sector (ED ground truth).

    Dense eigh for sector dimension <= dense_max, else Lanczos (eigsh, 'SA').
    Returns dict(E0, E1 (dense only), vec (full-space, normalised), dim).
    """
    L, d = ham.L, ham.d
    idx = sector_indices(L, d, sector)
    dim = idx.size
    if matrix_free is None:
        matrix_free = d**L > 3_000_000
    if not matrix_free:
        H = ham_matrix(ham, sparse=True)
        Hs = H[idx][:, idx]
        if dim <= dense_max:
            w, v = np.linalg.eigh(Hs.toarray())
            vec = np.zeros(d**L)
            vec[idx] = v[:, 0]
            return dict(E0=float(w[0]), E1=float(w[1]) if dim > 1 else None, vec=vec, dim=dim)
        op = Hs
    else:
        full = d**L

        def mv(x):
            y = np.zeros(full)
            y[idx] = np.asarray(x).reshape(-1)
            return apply_H_slices(ham, y)[idx]

        op = scipy.sparse.linalg.LinearOperator((dim, dim), matvec=mv, dtype=float)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(dim)
    w, v = scipy.sparse.linalg.eigsh(op, k=1, which="SA", tol=tol, v0=v0)
    vec = np.zeros(d**L) if want_vector else None
    if want_vector:
        vec[idx] = v[:, 0]
    return dict(E0=float(w[0]), E1=None, vec=vec, dim=dim)


# --------------------------------------------------------------------------
# Closed forms used as pins
# --------------------------------------------------------------------------


def bdg_ground_energy_periodic(L: int, J: float, mu: float, Delta: float) -> float:
    """Untruncated ground energy of the quadratic chain on a ring (Appendix A):
    E0 = 1/2 sum_k (E(k) - xi_k), E(k) = sqrt(xi_k^2 - Delta_k^2),
    xi_k = -2J cos k - mu, Delta_k = 2 Delta cos k, k = 2 pi m / L."""
    k = 2.0 * np.pi * np.arange(L) / L
    xi = -2.0 * J * np.cos(k) - mu
    dk = 2.0 * Delta * np.cos(k)
    if np.any(xi <= np.abs(dk)):
        raise ValueError("unstable chain: xi_k <= |Delta_k|")
    return float(0.5 * np.sum(np.sqrt(xi**2 - dk**2) - xi))


def bdg_ground_energy(L: int, J: float, mu: float, Delta: float, periodic: bool) -> float:
    """Untruncated ground energy of H = sum A_ij a_i^+ a_j + 1/2 sum B_ij (a_i a_j + h.c.)
    from the positive eigenvalues w of the dynamical matrix [[A, B], [-B, -A]]:
    E0 = (sum w - tr A) / 2 (textbook Bogoliubov result for real symmetric A, B)."""
    A = -mu * np.eye(L)
    B = np.zeros((L, L))
    for (i, j) in bonds(L, periodic):
        A[i, j] += -J
        A[j, i] += -J
        B[i, j] += Delta
        B[j, i] += Delta
    Dm = np.block([[A, B], [-B, -A]])
    w = np.linalg.eigvals(Dm)
    if np.max(np.abs(w.imag)) > 1e-9:
        raise ValueError("unstable chain: complex normal-mode frequencies")
    w = np.sort(w.real)
    pos = w[L:]
    if pos.min() <= 0:
        raise ValueError("unstable chain")
    return float(0.5 * (pos.sum() - np.trace(A)))


def free_boson_single_particle(L: int, J: float, periodic: bool) -> np.ndarray:
    """One-boson energies of the hopping chain: -2J cos(2 pi k / L) (ring),
    -2J cos(pi k / (L + 1)), k = 1..L (open)."""
    if periodic:
        return np.sort(-2.0 * J * np.cos(2.0 * np.pi * np.arange(L) / L))
    return np.sort(-2.0 * J * np.cos(np.pi * np.arange(1, L + 1) / (L + 1)))


# --------------------------------------------------------------------------
# ADAPT loop (Sec. IV.B; BFGS settings of Sec. V.A)
# --------------------------------------------------------------------------


def select_operator(g: np.ndarray, tau: float = 1e-4) -> int:
    """Largest |g_k|; among entries within the relative band (1 - tau) max|g| the
    lowest pool index is taken (deterministic resolution of symmetry ties)."""
    a = np.abs(g)
    m = a.max()
    return int(np.nonzero(a >= (1.0 - tau) * m)[0][0])


def bfgs(ham: Ham, psi0, ops, theta0, gtol: float, maxiter: int = 1000):
    """SciPy BFGS on E(theta) with the adjoint gradient; L-infinity stopping rule."""
    cnt = {"n": 0}

    def f(th):
        cnt["n"] += 1
        E, g, _ = energy_and_grad_adjoint(ham, psi0, ops, th)
        return E, g

    res = scipy.optimize.minimize(f, np.array(theta0, dtype=float), jac=True, method="BFGS",
                                  options={"gtol": gtol, "norm": np.inf, "maxiter": maxiter})
    return res.x, float(res.fun), int(res.nit), cnt["n"]


def adapt(ham: Ham, psi0, pool, max_iters: int, grad_tol: float = 1e-3, warm_ops=(), warm_theta0=(),
          tau: float = 1e-4, warm_gtol: float = 1e-9, callback=None):
    """CV-ADAPT-VQE from psi0.

    Optional warm-up layer (Sec. IV.B, Appendix C): its parameters are first
    optimised alone, then re-optimised with every later BFGS.
    Returns a list of per-iteration records.
    """
    ops = list(warm_ops)
    theta = np.array(warm_theta0, dtype=float)
    records = []
    if len(ops):
        theta, E, nit, nev = bfgs(ham, psi0, ops, theta, gtol=warm_gtol)
        records.append(dict(iter=0, warm=True, E=E, bfgs_iters=nit, bfgs_evals=nev, theta=theta.copy()))
    for it in range(1, max_iters + 2):
        psi = ansatz_state(psi0, ops, theta, ham.L, ham.d)
        g = pool_gradients(ham, psi, pool)
        gnorm = float(np.linalg.norm(g))
        if gnorm < grad_tol or it > max_iters:
            records.append(dict(iter=it, converged=gnorm < grad_tol, g=g, gnorm=gnorm,
                                E=energy(ham, psi)[0], theta=theta.copy(), ops=list(ops)))
            break
        k = select_operator(g, tau)
        gsel = abs(g[k])
        ops.append(pool[k])
        theta = np.append(theta, 0.0)
        gtol = min(1e-6, 1e-5 * gsel)
        theta, E, nit, nev = bfgs(ham, psi0, ops, theta, gtol=gtol)
        rec = dict(iter=it, k=k, g_sel=gsel, gnorm=gnorm, g=g, E=E, bfgs_iters=nit, bfgs_evals=nev,
                   theta=theta.copy(), ops=list(ops))
        records.append(rec)
        if callback:
            callback(rec)
    return records


def hva(ham: Ham, psi0, layer_ops, layer_inits, gtol: float = 1e-9, maxiter: int = 1000):
    """HVA-CV-VQE (Sec. IV.A, Eq. (HVA_ansatz)): psi = prod_l prod_k exp(theta_lk A_k) psi0
    with the same layer of generators A_k (the Hamiltonian's own terms) repeated.
    Grown one layer at a time (Sec. V.A): layer l enters with the angles
    layer_inits[l-1], the earlier layers start from their previous optimum, and
    BFGS (L-infinity tolerance gtol, at most maxiter iterations) re-optimises all
    angles.  Returns one record per layer."""
    ops, theta, out = [], np.zeros(0), []
    for l, init in enumerate(layer_inits):
        ops = ops + list(layer_ops)
        theta = np.concatenate([theta, np.asarray(init, dtype=float)])
        theta, E, nit, nev = bfgs(ham, psi0, ops, theta, gtol=gtol, maxiter=maxiter)
        out.append(dict(layers=l + 1, E=E, theta=theta.copy(), ops=list(ops), bfgs_iters=nit, bfgs_evals=nev))
    return out


# --------------------------------------------------------------------------
# Single matrix rows (sampled checks on states too large for the full oracle)
# --------------------------------------------------------------------------


def ham_column(ham: Ham, occ: Sequence[int]) -> dict:
    """H |occ> as {flat index: coefficient}, term by term from the ladder
    matrices acting on the occupied levels.  H is real symmetric, so this is
    also row `occ` of H: (H psi)[occ] = sum_k coef_k psi[k]."""
    L, d = ham.L, ham.d
    a = ladder(d)
    ad = a.T
    out: dict = {}

    def add(new_occ, c):
        if c == 0.0:
            return
        idx = sum(int(n) * d**r for r, n in enumerate(new_occ))
        out[idx] = out.get(idx, 0.0) + c

    occ = list(occ)
    for (i, j) in bonds(L, ham.periodic):
        for (mi, mj, c) in ((ad, a, -ham.J), (a, ad, -ham.J), (a, a, ham.Delta), (ad, ad, ham.Delta)):
            if c == 0.0:
                continue
            # single-mode matrices map |n> to column n: entries mi[:, n_i]
            for ni2 in range(d):
                vi = mi[ni2, occ[i]]
                if vi == 0.0:
                    continue
                for nj2 in range(d):
                    vj = mj[nj2, occ[j]]
                    if vj == 0.0:
                        continue
                    new = list(occ)
                    new[i], new[j] = ni2, nj2
                    add(new, c * vi * vj)
    dg = onsite(ham)
    add(occ, float(sum(dg[n, n] for n in occ)))
    return out


# --------------------------------------------------------------------------
# Product states psi[n] = prod_r f_r[n_r]: exact values at chosen indices without
# forming the d^L vector (used at the largest sizes the library accepts).

def _product_amp(factors, occ) -> complex:
    v = 1.0 + 0.0j
    for f, n in zip(factors, occ):
        v *= complex(f[n])
    return v


def product_H_at(ham: Ham, factors, flat_index: int) -> complex:
    """(H psi)[flat_index] for the product state of `factors` (one length-d
    vector per mode): the row of H from ham_column, contracted with the
    product amplitudes."""
    L, d = ham.L, ham.d
    occ = [(flat_index // d**r) % d for r in range(L)]
    tot = 0.0 + 0.0j
    for k, c in ham_column(ham, occ).items():
        tot += c * _product_amp(factors, [(k // d**r) % d for r in range(L)])
    return complex(tot)


def product_energy(ham: Ham, factors) -> float:
    """<psi|H|psi> / <psi|psi> of a product state from single-mode expectation
    values: every bond term is a product of two one-mode expectations times
    the norms of the other modes (Sec. III Hamiltonians)."""
    L, d = ham.L, ham.d
    f = [np.asarray(x, dtype=np.complex128) for x in factors]
    a = ladder(d)
    ad = a.T
    nrm = [np.vdot(x, x).real for x in f]
    ex = lambda x, M: np.vdot(x, M @ x)
    N = number(d)
    onsite_m = (0.5 * ham.U + ham.K) * (N @ N - N) - ham.mu * N
    E = 0.0 + 0.0j
    for (i, j) in bonds(L, ham.periodic):
        rest = np.prod([nrm[r] for r in range(L) if r not in (i, j)])
        for (mi, mj, c) in ((ad, a, -ham.J), (a, ad, -ham.J), (a, a, ham.Delta), (ad, ad, ham.Delta)):
            E += c * ex(f[i], mi) * ex(f[j], mj) * rest
    for r in range(L):
        E += ex(f[r], onsite_m) * np.prod([nrm[s] for s in range(L) if s != r])
    return float(E.real / np.prod(nrm))


def product_gate_at(op, theta: float, factors, L: int, d: int, flat_index: int) -> complex:
    """(O(theta) psi)[flat_index] for a product state: the gate's local matrix
    (exp of the truncated generator) applied to the factors of its modes."""
    gtype, i, j = op
    occ = [(flat_index // d**r) % d for r in range(L)]
    rest = _product_amp([f for r, f in enumerate(factors) if r not in (i, j)],
                        [n for r, n in enumerate(occ) if r not in (i, j)])
    G = gate_local(gtype, d, theta)
    if j is None or j < 0:
        v = G[occ[i], :] @ np.asarray(factors[i], dtype=np.complex128)
    else:
        loc = np.kron(np.asarray(factors[i], dtype=np.complex128), np.asarray(factors[j], dtype=np.complex128))
        v = G[occ[i] * d + occ[j], :] @ loc
    return complex(rest * v)


def apply_H_at(ham: Ham, psi: np.ndarray, flat_index: int) -> complex:
    """(H psi)[flat_index] from one row of H."""
    L, d = ham.L, ham.d
    occ = [(flat_index // d**r) % d for r in range(L)]
    return complex(sum(c * psi[k] for k, c in ham_column(ham, occ).items()))
