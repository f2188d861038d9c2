"""Second-quantised Hamiltonian by literal operator application (oracle only).

This is the definition of H used to pin the Slater-Condon code:
  H = e_core + sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q.
Basis states are occupation integers b (bit p set <=> orbital p occupied) and
  a_p |b>  = (-1)^{#occupied below p} |b - e_p>   (0 if p empty)
  a+_p |b> = (-1)^{#occupied below p} |b + e_p>   (0 if p occupied),
the Jordan-Wigner convention matching |b> = a+_{i1}...a+_{iN}|0>, i1<...<iN.
Every term of the sum is applied to every basis state of the N-electron
sector, so the cost is C(M,N) * M^4; only for M <= 10.
"""
from __future__ import annotations

import itertools

import numpy as np


def apply_annihilate(b: int, p: int):
    if not (b >> p) & 1:
        return None
    sign = -1 if bin(b & ((1 << p) - 1)).count("1") % 2 else 1
    return b ^ (1 << p), sign


def apply_create(b: int, p: int):
    if (b >> p) & 1:
        return None
    sign = -1 if bin(b & ((1 << p) - 1)).count("1") % 2 else 1
    return b | (1 << p), sign


def apply_string(b: int, ops):
    """Apply a product of operators, rightmost first.  ops: list of ('c'|'a', p)
    written left to right as in the operator product."""
    sign = 1
    for kind, p in reversed(ops):
        r = apply_create(b, p) if kind == "c" else apply_annihilate(b, p)
        if r is None:
            return None
        b, s = r
        sign *= s
    return b, sign


def operator_matrix(M: int, ops):
    """Dense 2^M x 2^M matrix of an operator product (for the CAR check)."""
    dim = 1 << M
    A = np.zeros((dim, dim))
    for b in range(dim):
        r = apply_string(b, ops)
        if r is not None:
            A[r[0], b] += r[1]
    return A


def sector_hamiltonian(h, g, n_elec: int, e_core: float = 0.0):
    """H on the full N-electron sector; returns (sorted states, dense H)."""
    M = h.shape[0]
    states = sorted(sum(1 << i for i in occ) for occ in itertools.combinations(range(M), n_elec))
    index = {b: i for i, b in enumerate(states)}
    n = len(states)
    H = np.zeros((n, n), dtype=np.complex128)
    for j, b in enumerate(states):
        H[j, j] += e_core
        for p in range(M):
            for q in range(M):
                if h[p, q] == 0:
                    continue
                r = apply_string(b, [("c", p), ("a", q)])
                if r is not None:
                    H[index[r[0]], j] += h[p, q] * r[1]
        for p in range(M):
            for q in range(M):
                for rr in range(M):
                    for s in range(M):
                        v = g[p, q, rr, s]
                        if v == 0:
                            continue
                        r = apply_string(b, [("c", p), ("c", rr), ("a", s), ("a", q)])
                        if r is not None:
                            H[index[r[0]], j] += 0.5 * v * r[1]
    return np.array(states, dtype=np.uint64), H


def project(states, H, dets):
    """Rows/columns of H (over `states`) belonging to the determinant list."""
    pos = {int(b): i for i, b in enumerate(states)}
    idx = np.array([pos[int(b)] for b in dets], dtype=np.int64)
    return H[np.ix_(idx, idx)]
