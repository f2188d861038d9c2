"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only draws random numbers and arranges them into integral arrays
and test vectors. It holds none of the sigma-build or Davidson arithmetic, so
both sides of every parity test can take their inputs from here without
sharing any of the method's code.

Conventions (the readings used throughout this repository):
  * one-electron integrals h[p, q] are Hermitian (real symmetric for real
    problems);
  * two-electron integrals use the chemists' (Mulliken) order,
    g[p, q, r, s] = (pq|rs), with H = sum h_pq a+_p a_q
    + 1/2 sum (pq|rs) a+_p a+_r a_s a_q;
  * the second argument of every normal draw is a standard deviation.

Draw order (identical for every caller):
  1. diagonal of h: uniform(-2, 0, M), sorted ascending;
  2. off-diagonal of h in upper-triangle row-major order (p < q): one normal
     draw of length M(M-1)/2 for real problems; for complex problems a draw
     for the real parts followed by one for the imaginary parts, each with
     standard deviation 0.1/sqrt(2);
  3. two-electron factor: real problems draw F ~ N(0, 0.05) of shape
     (R, M(M+1)/2) over packed pairs pq = p(p+1)/2 + q (p >= q); complex
     problems draw A = N(0, s) + 1j N(0, s) of shape (R, M, M) (real part
     first) and take the Hermitian part L = (A + A^H)/2.  In both cases
     (pq|rs) = sum_P L[P, p, q] L[P, r, s].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Integrals", "SpaceSpec", "real_integrals", "complex_integrals",
    "kramers_integrals", "test_vector", "CONFIGS", "TSPACES", "config",
    "serving_requests",
]


@dataclass
class Integrals:
    """One- and two-electron integrals of a synthetic Hamiltonian.

    h: (M, M) Hermitian; g: (M, M, M, M) with g[p,q,r,s] = (pq|rs).
    spin_free: when True, h and g are over M spatial orbitals and the
    determinant space is built over 2M spin-orbitals (alpha block first).
    """
    h: np.ndarray
    g: np.ndarray
    spin_free: bool = False
    e_core: float = 0.0

    @property
    def n_orb(self) -> int:
        return int(self.h.shape[0])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.h) or np.iscomplexobj(self.g)


@dataclass
class SpaceSpec:
    """A determinant space: contiguous subspaces of sizes `sub`, N electrons,
    inclusive per-subspace occupation windows [lo_k, hi_k]."""
    n_elec: int
    sub: list
    lo: list = field(default_factory=list)
    hi: list = field(default_factory=list)

    def __post_init__(self):
        if not self.lo:
            self.lo = [0] * len(self.sub)
        if not self.hi:
            self.hi = list(self.sub)

    @property
    def n_spin_orb(self) -> int:
        return int(sum(self.sub))

    def categories(self):
        """Occupation tuples of the space, in lexicographic order."""
        out = []

        def rec(k, acc, left):
            if k == len(self.sub):
                if left == 0:
                    out.append(tuple(acc))
                return
            for n in range(max(self.lo[k], 0), min(self.hi[k], self.sub[k], left) + 1):
                rec(k + 1, acc + [n], left - n)
        rec(0, [], self.n_elec)
        return out

    def n_dets(self) -> int:
        return sum(math.prod(math.comb(m, n) for m, n in zip(self.sub, c))
                   for c in self.categories())


def _diag_and_offdiag(rng, M, complex_):
    d = rng.uniform(-2.0, 0.0, M)
    d.sort()
    n = M * (M - 1) // 2
    iu = np.triu_indices(M, k=1)
    if complex_:
        re = rng.normal(0.0, 0.1 / math.sqrt(2.0), n)
        im = rng.normal(0.0, 0.1 / math.sqrt(2.0), n)
        h = np.zeros((M, M), dtype=np.complex128)
        h[iu] = re + 1j * im
        h = h + h.conj().T
        h[np.diag_indices(M)] = d
    else:
        off = rng.normal(0.0, 0.1, n)
        h = np.zeros((M, M))
        h[iu] = off
        h = h + h.T
        h[np.diag_indices(M)] = d
    return h


def real_integrals(M: int, seed: int, rank: int = 16, sigma_f: float = 0.05) -> Integrals:
    """Real symmetric h and 8-fold symmetric (pq|rs) = sum_P L_pq L_rs."""
    rng = np.random.default_rng(seed)
    h = _diag_and_offdiag(rng, M, False)
    npair = M * (M + 1) // 2
    F = rng.normal(0.0, sigma_f, (rank, npair))
    L = np.zeros((rank, M, M))
    for p in range(M):
        for q in range(p + 1):
            L[:, p, q] = F[:, p * (p + 1) // 2 + q]
            L[:, q, p] = F[:, p * (p + 1) // 2 + q]
    g = np.einsum("Ppq,Prs->pqrs", L, L)
    return Integrals(h=h, g=np.ascontiguousarray(g))


def complex_integrals(M: int, seed: int, rank: int = 16, sigma_f: float = 0.05) -> Integrals:
    """Hermitian complex h and (pq|rs) = sum_P L^P_pq L^P_rs with L^P Hermitian,
    so (pq|rs) = (qp|sr)^* and (pq|rs) = (rs|pq)."""
    rng = np.random.default_rng(seed)
    h = _diag_and_offdiag(rng, M, True)
    A = rng.normal(0.0, sigma_f, (rank, M, M)) + 1j * rng.normal(0.0, sigma_f, (rank, M, M))
    L = 0.5 * (A + A.conj().transpose(0, 2, 1))
    g = np.einsum("Ppq,Prs->pqrs", L, L)
    return Integrals(h=h, g=np.ascontiguousarray(g))


def kramers_integrals(n_pairs: int, seed: int, rank: int = 16, sigma_f: float = 0.05) -> Integrals:
    """Time-reversal-symmetric spinor integrals over 2*n_pairs spinors.

    Spinor order: the n unbarred spinors first, then their n Kramers
    partners.  h = [[A, B], [-B*, A*]] with A Hermitian and B antisymmetric;
    the two-electron part is a real rank-`rank` spatial factor expanded over
    the pairs, (p_s q_s | r_t s_t) = (pq|rs) for both spinor blocks s, t.
    """
    n = n_pairs
    rng = np.random.default_rng(seed)
    A = _diag_and_offdiag(rng, n, True)
    X = rng.normal(0.0, 0.05, (n, n)) + 1j * rng.normal(0.0, 0.05, (n, n))
    B = 0.5 * (X - X.T)
    h = np.block([[A, B], [-B.conj(), A.conj()]])
    npair = n * (n + 1) // 2
    F = rng.normal(0.0, sigma_f, (rank, npair))
    L = np.zeros((rank, n, n))
    for p in range(n):
        for q in range(p + 1):
            L[:, p, q] = F[:, p * (p + 1) // 2 + q]
            L[:, q, p] = F[:, p * (p + 1) // 2 + q]
    gs = np.einsum("Ppq,Prs->pqrs", L, L)
    M = 2 * n
    g = np.zeros((M, M, M, M), dtype=np.complex128)
    for s in range(2):
        for t in range(2):
            g[s * n:(s + 1) * n, s * n:(s + 1) * n, t * n:(t + 1) * n, t * n:(t + 1) * n] = gs
    return Integrals(h=h.astype(np.complex128), g=g)


def test_vector(n_dets: int, seed: int, complex_: bool = True) -> np.ndarray:
    """Normalised N(0,1) vector in canonical determinant order (ascending
    occupation bitstring), drawn from default_rng(seed + 100)."""
    rng = np.random.default_rng(seed + 100)
    if complex_:
        c = rng.normal(size=n_dets) + 1j * rng.normal(size=n_dets)
    else:
        c = rng.normal(size=n_dets)
    return c / np.linalg.norm(c)


# ---------------------------------------------------------------------------
# Workload configurations.  Sizes follow the problem statement of each
# workload; "3p" is the 40-spinor three-subspace space with N = 11 (the
# literal N = 14 reading holds 1.93e10 determinants, more than one vector of
# complex FP64 fits in one GPU's memory).
# ---------------------------------------------------------------------------
CONFIGS = {
    # spin-free real FCI: 8 spatial orbitals, 4 alpha + 4 beta
    "c1": dict(kind="real_sf", M=8, seed=1001, space=SpaceSpec(8, [8, 8], [4, 4], [4, 4]), roots=1),
    # complex spinor FCI: 24 spinors, 8 electrons
    "c2": dict(kind="complex", M=24, seed=2002, rank=32, sigma_f=0.03,
               space=SpaceSpec(8, [24]), roots=2),
    # three-subspace categorical space, 40 spinors, 11 electrons
    "c3p": dict(kind="complex", M=40, seed=3003, rank=16, sigma_f=0.05,
                space=SpaceSpec(11, [12, 16, 12], [2, 4, 2], [6, 10, 6]), roots=1),
    # literal reading: same partition with 14 electrons
    "c3lit": dict(kind="complex", M=40, seed=3003, rank=16, sigma_f=0.05,
                  space=SpaceSpec(14, [12, 16, 12], [2, 4, 2], [6, 10, 6]), roots=1),
}

# Tiny spaces used for exhaustive checks.
TSPACES = {
    "T2": dict(kind="complex", M=8, seed=12, space=SpaceSpec(3, [8])),
    "T3": dict(kind="complex", M=10, seed=13, space=SpaceSpec(4, [4, 6], [1, 1], [3, 3])),
    "T4": dict(kind="complex", M=12, seed=14, space=SpaceSpec(5, [4, 4, 4], [1, 1, 1], [2, 3, 2])),
    "T8": dict(kind="complex", M=12, seed=18, space=SpaceSpec(4, [4, 4, 4])),
    "T8fci": dict(kind="complex", M=12, seed=18, space=SpaceSpec(4, [12])),
}


def config(name: str) -> tuple:
    """(Integrals, SpaceSpec, n_roots) for a named workload."""
    cfg = CONFIGS.get(name) or TSPACES[name]
    kind = cfg["kind"]
    if kind == "real_sf":
        ints = real_integrals(cfg["M"], cfg["seed"])
        ints.spin_free = True
    elif kind == "complex":
        ints = complex_integrals(cfg["M"], cfg["seed"], cfg.get("rank", 16), cfg.get("sigma_f", 0.05))
    else:
        raise ValueError(kind)
    return ints, cfg["space"], cfg.get("roots", 1)


def serving_requests(n: int, seed: int = 5000, min_dets: int = 10_000, max_dets: int = 100_000_000,
                     M_range=(16, 32), N_range=(6, 12), sub_range=(1, 3), root_range=(1, 4)):
    """Request descriptors for the continuous-batching workload.

    Request j draws from default_rng(seed + 1 + j): M ~ U{M_range}, number of
    subspaces ~ U{sub_range} with a near-equal contiguous split, N ~ U{N_range},
    roots ~ U{root_range}; for more than one subspace, window k is
    round(N m_k / M) -/+ w with w ~ U{1..3}, clipped to [0, m_k].  A draw whose
    determinant count falls outside [min_dets, max_dets] (or is empty) is
    redrawn from the same generator.  Integrals: complex, rank 16, s = 0.05,
    seeded with the request seed.
    """
    out = []
    for j in range(n):
        rseed = seed + 1 + j
        rng = np.random.default_rng(rseed)
        while True:
            M = int(rng.integers(M_range[0], M_range[1] + 1))
            K = int(rng.integers(sub_range[0], sub_range[1] + 1))
            N = int(rng.integers(N_range[0], N_range[1] + 1))
            k = int(rng.integers(root_range[0], root_range[1] + 1))
            base, rem = divmod(M, K)
            sub = [base + (1 if i < rem else 0) for i in range(K)]
            if K == 1:
                lo, hi = [0], [M]
            else:
                w = int(rng.integers(1, 4))
                lo, hi = [], []
                for m in sub:
                    c = int(round(N * m / M))
                    lo.append(max(0, c - w))
                    hi.append(min(m, c + w))
            sp = SpaceSpec(N, sub, lo, hi)
            nd = sp.n_dets() if sp.categories() else 0
            if min_dets <= nd <= max_dets and N <= M:
                break
        out.append(dict(seed=rseed, M=M, space=sp, roots=k, n_dets=nd))
    return out
