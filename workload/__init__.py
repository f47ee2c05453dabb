"""Seeded synthetic inputs and run configurations.

This module only produces inputs: seeded random states, seeded initial angles,
operator-pool enumerations and the parameter sets of the benchmark workloads.
It holds none of the method's arithmetic and is shared by the tests, the
benchmark and the smoke check, which hand the same inputs to the HIP path and
to the oracle.
"""
from __future__ import annotations

import numpy as np

# Generator type codes (same order on every side of the boundary).
HR, HI, DH, PR, PI, KERR, ROT, CK, SR, SI, BS, TMS, SQ = range(13)
TYPE_NAMES = ("HR", "HI", "DH", "PR", "PI", "KERR", "ROT", "CK", "SR", "SI", "BS", "TMS", "SQ")


def pairs(L: int, kind: str, periodic: bool) -> list[tuple[int, int]]:
    """Mode pairs (i < j) in lexicographic order.

    kind: "all" (every i < j), "nn" (nearest neighbours, ring wrap added for a
    periodic chain with L >= 3), "nn+nnn" (nearest and next-nearest)."""
    out = set()
    if kind == "all":
        out = {(i, j) for i in range(L) for j in range(i + 1, L)}
    else:
        dists = [1] if kind == "nn" else [1, 2]
        for dist in dists:
            for r in range(L):
                s = r + dist
                if s < L:
                    out.add((r, s))
                elif periodic and L >= 3 and (dist < L):
                    a, b = sorted((r, s % L))
                    if a != b:
                        out.add((a, b))
    return sorted(out)


def pool(L: int, kind: str, periodic: bool, types) -> list[tuple[str, int, int]]:
    """Pool = pairs (lexicographic) x generator types (in the listed order)."""
    return [(t, i, j) for (i, j) in pairs(L, kind, periodic) for t in types]


BH_TYPES = ("HR", "HI", "DH")


def site_ops(L: int, types) -> list[tuple[str, int, int]]:
    """Single-mode pool entries (j = -1): every site x types, sites in order."""
    return [(t, r, -1) for r in range(L) for t in types]
KITAEV_TYPES = ("HR", "HI", "PI", "PR")


def warmup_ops(L: int, periodic: bool) -> list[tuple[str, int, int]]:
    """One Hamiltonian-variational layer for the Bose-Hubbard chain, built from
    exp(-i theta H_k) of the Hamiltonian's own terms (Sec. IV.A): the hopping
    term's generator i(a_i^+ a_j + h.c.) (HI) on every bond, then a Kerr phase
    and a rotation on every site (the on-site interaction and number terms)."""
    bl = [(r, r + 1) for r in range(L - 1)]
    if periodic and L >= 3:
        bl.append((0, L - 1))
    ops = [("HI", i, j) for (i, j) in bl]
    ops += [("KERR", r, -1) for r in range(L)]
    ops += [("ROT", r, -1) for r in range(L)]
    return ops


def hva_layer(L: int, periodic: bool, model: str) -> list[tuple[str, int, int]]:
    """One layer of the Hamiltonian variational ansatz (Sec. IV.A, Table I and
    the HVA circuit figure): exp(-i theta H_k) for each of the Hamiltonian's
    terms, one angle per gate, in the figure's order.  The hopping term gives the
    generator i(a_i^+ a_j + h.c.) (HI), the pairing term i(a_i a_j + h.c.) (PI),
    the on-site terms Kerr (i N^2) and rotation (i N) phases.
      "bh":  HI on every bond, KERR and ROT on every site        (3 N_S gates)
      "bkc": PI on every bond, HI on every bond, ROT on every site (3 N_S gates)
      "bkck": as "bkc" with KERR on every site before the rotations (4 N_S gates)
    Bonds in order (r, r+1), then the ring bond (0, L-1) when periodic."""
    bl = [(r, r + 1) for r in range(L - 1)]
    if periodic and L >= 3:
        bl.append((0, L - 1))
    sites = range(L)
    if model == "bh":
        return [("HI", i, j) for (i, j) in bl] + [("KERR", r, -1) for r in sites] + [("ROT", r, -1) for r in sites]
    if model in ("bkc", "bkck"):
        ops = [("PI", i, j) for (i, j) in bl] + [("HI", i, j) for (i, j) in bl]
        if model == "bkck":
            ops += [("KERR", r, -1) for r in sites]
        return ops + [("ROT", r, -1) for r in sites]
    raise ValueError(model)


def hva_inits(n_layer: int, layers: int, seed: int) -> list[np.ndarray]:
    """Initial angles of each new HVA layer, uniform in [-0.05, 0.05] (Sec. V.A)."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(-0.05, 0.05, size=n_layer) for _ in range(layers)]


def warmup_theta0(n: int, seed: int) -> np.ndarray:
    """Initial warm-up angles uniform in [-0.05, 0.05]."""
    return np.random.default_rng(seed).uniform(-0.05, 0.05, size=n)


def random_state(L: int, d: int, seed: int, sector=None, dtype=np.complex64) -> np.ndarray:
    """i.i.d. complex normal amplitudes, optionally zeroed outside a sector
    (("N", k) or ("parity", p)), normalised in float64, then cast to dtype."""
    rng = np.random.default_rng(seed)
    n = d**L
    psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    if sector is not None:
        idx = np.arange(n)
        tot = np.zeros(n, dtype=np.int64)
        for _ in range(L):
            tot += idx % d
            idx //= d
        kind, val = sector
        keep = (tot == val) if kind == "N" else (tot % 2 == val)
        psi[~keep] = 0.0
    psi /= np.sqrt(np.vdot(psi, psi).real)
    return psi.astype(dtype)


def random_angles(n: int, seed: int, lo: float = -0.5, hi: float = 0.5) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def random_circuit(pool_ops, n: int, seed: int):
    rng = np.random.default_rng(seed)
    sel = rng.integers(0, len(pool_ops), size=n)
    th = rng.uniform(-0.5, 0.5, size=n)
    return [pool_ops[k] for k in sel], th


def fock_index(L: int, d: int, occ) -> int:
    return int(sum(int(n) * d**r for r, n in enumerate(occ)))


# --------------------------------------------------------------------------
# Workloads (sizes, parameters, pools, caps, seeds)
# --------------------------------------------------------------------------

def config(name: str) -> dict:
    """Parameter sets of the five workloads.

    bh_l3_d4     Bose-Hubbard open chain L=3, d=4, J=1, U=2, |1,1,1>, all-pairs pool.
    bh_l8_d6     Bose-Hubbard ring L=8, d=6, N=8, U in {1,4,16}, nn+nnn pool.
    kk_l8_d8     Kitaev-Kerr open chain L=8, d=8, J=1, Delta=0.5, K=0.2, vacuum, nn pool.
    sweep96      96 mixed points (see sweep_points()).
    warm_l6_d8   Kitaev-Kerr open chain L=6, d=8 for the learned warm start.
    """
    if name == "bh_l3_d4":
        return dict(L=3, d=4, periodic=False, J=1.0, U=2.0, mu=0.0, Delta=0.0, K=0.0,
                    occ=[1, 1, 1], sector=("N", 3), pool=pool(3, "all", False, BH_TYPES),
                    max_iters=30, warm=True, warm_seed=0)
    if name == "bh_l8_d6":
        return dict(L=8, d=6, periodic=True, J=1.0, U=4.0, mu=0.0, Delta=0.0, K=0.0,
                    occ=[1] * 8, sector=("N", 8), pool=pool(8, "nn+nnn", True, BH_TYPES),
                    max_iters=60, warm=True, warm_seed=1, U_values=(1.0, 4.0, 16.0))
    if name == "kk_l8_d8":
        return dict(L=8, d=8, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.5, K=0.2,
                    occ=[0] * 8, sector=("parity", 0), pool=pool(8, "nn", False, KITAEV_TYPES),
                    max_iters=60, warm=False, warm_seed=2)
    if name == "warm_l6_d8":
        return dict(L=6, d=8, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.5, K=0.2,
                    occ=[0] * 6, sector=("parity", 0), pool=pool(6, "nn", False, KITAEV_TYPES),
                    max_iters=64, warm=False, warm_seed=3)
    raise KeyError(name)


def sweep_points(seed: int = 20260605) -> list[dict]:
    """96 points: 48 Bose-Hubbard (L in {4,6,8} x d in {4,6} x 8 values of U/J
    log-spaced over [0.5, 20], ring, N = L from |1..1>, nn+nnn pool, warm-up
    layer) and 48 Kitaev-Kerr (L in {4,6}, d = 8, open, 24 seeded draws of
    (Delta, K) uniform in [0,1] x [0,0.5] per L, vacuum start, nn pool)."""
    pts = []
    us = np.geomspace(0.5, 20.0, 8)
    for L in (4, 6, 8):
        for d in (4, 6):
            for U in us:
                pts.append(dict(model="bh", L=L, d=d, periodic=True, J=1.0, U=float(U), mu=0.0,
                                Delta=0.0, K=0.0, occ=[1] * L, sector=("N", L),
                                pool=pool(L, "nn+nnn", True, BH_TYPES), warm=True, max_iters=40))
    rng = np.random.default_rng(seed)
    for L in (4, 6):
        draws = rng.uniform([0.0, 0.0], [1.0, 0.5], size=(24, 2))
        for (Dl, K) in draws:
            pts.append(dict(model="kk", L=L, d=8, periodic=False, J=1.0, U=0.0, mu=0.0,
                            Delta=float(Dl), K=float(K), occ=[0] * L, sector=("parity", 0),
                            pool=pool(L, "nn", False, KITAEV_TYPES), warm=False, max_iters=40))
    for k, p in enumerate(pts):
        p["warm_seed"] = 1000 + k
    return pts


def warmstart_points(split: str) -> list[dict]:
    """Kitaev-Kerr L=6, d=8 points for the learned warm start: 256 training
    points (seed 1) and 64 held-out points (seed 2), (Delta, K) uniform in
    [0,1] x [0,0.5]."""
    n, seed = (256, 1) if split == "train" else (64, 2)
    rng = np.random.default_rng(seed)
    draws = rng.uniform([0.0, 0.0], [1.0, 0.5], size=(n, 2))
    base = config("warm_l6_d8")
    out = []
    for (Dl, K) in draws:
        p = dict(base)
        p["Delta"], p["K"] = float(Dl), float(K)
        out.append(p)
    return out


def paper_cases() -> list[dict]:
    """The paper's own ADAPT runs (Sec. V), in this library's sign conventions.

    Kitaev chain (BKC): periodic, d = 6, J = 1, Delta = 0.5, mu in {-3.1, -2.7},
    N_S in {3, 4, 5}, vacuum; pool: beam splitters and two-mode squeezers on all
    pairs, single-mode squeezers and rotations on every site.
    BKC + Kerr: the paper's -(U/2) N(N-1) with U = -1 is K = 0.5 here; mu = -2.7,
    N_S in {3, 4, 5}; the pool adds cross-Kerr on all pairs and Kerr on every site.
    Bose-Hubbard: periodic, N_S = 4, 12 bosons, d = 13, Lambda = N U / J = +-4
    in the paper's sign, i.e. U = -Lambda / 12 here; |3,3,3,3> for Lambda < 0
    and |6,0,6,0> for Lambda > 0; nearest-neighbour beam splitters and cross-Kerr,
    Kerr and rotations on every site, after the warm-up layer."""
    out = []
    gauss = ("HR", "HI", "PR", "PI")
    for mu in (-3.1, -2.7):
        for L in (3, 4, 5):
            out.append(dict(name=f"bkc_N{L}_mu{mu:g}", model="kk", L=L, d=6, periodic=True, J=1.0, U=0.0, mu=mu,
                            Delta=0.5, K=0.0, occ=[0] * L, sector=("parity", 0), warm=False, warm_seed=0,
                            pool=pool(L, "all", True, gauss) + site_ops(L, ("SR", "SI", "ROT"))))
    for L in (3, 4, 5):
        out.append(dict(name=f"bkck_N{L}_mu-2.7", model="kk", L=L, d=6, periodic=True, J=1.0, U=0.0, mu=-2.7,
                        Delta=0.5, K=0.5, occ=[0] * L, sector=("parity", 0), warm=False, warm_seed=0,
                        pool=pool(L, "all", True, gauss + ("CK",)) + site_ops(L, ("SR", "SI", "ROT", "KERR"))))
    # the same Kitaev pools with the paper's two-parameter gates (one BS, TMS, SQ entry per pair or site)
    for p in out:
        tp = ("BS", "TMS") + (("CK",) if p["K"] else ())
        sp = ("SQ", "ROT") + (("KERR",) if p["K"] else ())
        p["pool2"] = pool(p["L"], "all", True, tp) + site_ops(p["L"], sp)
    for lam in (4.0, -4.0):
        occ = [3, 3, 3, 3] if lam < 0 else [6, 0, 6, 0]
        out.append(dict(name=f"bh_N4_lam{lam:+g}", model="bh", L=4, d=13, periodic=True, J=1.0, U=-lam / 12.0,
                        mu=0.0, Delta=0.0, K=0.0, occ=occ, sector=("N", 12), warm=True, warm_seed=7,
                        pool=pool(4, "nn", True, ("HR", "HI", "CK")) + site_ops(4, ("KERR", "ROT")),
                        # the paper's number-conserving pool with its two-parameter beam splitter
                        pool2=pool(4, "nn", True, ("BS", "CK")) + site_ops(4, ("KERR", "ROT"))))
    return out


# ---------------------------------------------------------------- warm-start network inputs

MLP_SHAPES = [((128, 4), 4), ((128,), 4), ((128, 128), 128), ((128,), 128), ((64, 128), 128), ((64,), 128)]


def mlp_init(seed: int = 0) -> np.ndarray:
    """Seeded float32 initial parameters of the 4 -> 128 -> 128 -> 64 network,
    uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)] (W1, b1, W2, b2, W3, b3, W
    stored [out x in] row-major)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp, fan_in in MLP_SHAPES:
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, size=shp).astype(np.float32).ravel())
    return np.concatenate(parts)


def mlp_features(J: float, Delta: float, K: float, step: int) -> np.ndarray:
    """Network input of an ADAPT point at step n: (J, Delta, K, n / 64)."""
    return np.array([J, Delta, K, step / 64.0], dtype=np.float32)


def product_factors(L: int, d: int, seed: int = 0) -> list:
    """Seeded single-mode factors f_r (complex64, length d, unit norm) of the
    product state psi[n] = prod_r f_r[n_r] used at the largest sizes."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(L):
        v = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        v /= np.linalg.norm(v)
        out.append(v.astype(np.complex64))
    return out


def product_state(factors, dtype=np.complex64) -> np.ndarray:
    """The full product vector (index sum_r n_r d^r, mode 0 fastest)."""
    psi = np.asarray(factors[-1], dtype=np.complex128)
    for f in reversed(factors[:-1]):
        psi = np.kron(psi, np.asarray(f, dtype=np.complex128))
    return psi.astype(dtype)
