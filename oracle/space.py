"""Explicit enumeration of a determinant space (oracle; test infrastructure only).

A determinant is the occupation bitstring b of N electrons over M spin-orbitals
(bit p set <=> orbital p occupied), standing for a+_{i1}...a+_{iN}|0> with
ascending indices.  The orbitals are split into contiguous subspaces; the
space keeps every determinant whose electron count in subspace k lies in the
inclusive window [lo_k, hi_k] (the distributed-active-space partition of the
Results section and Fig. 2A).  Determinants are returned sorted ascending,
which is the oracle's own order and the canonical order of the seeded test
vectors.
"""
from __future__ import annotations

import itertools

import numpy as np


def masks(sub):
    out, off = [], 0
    for m in sub:
        out.append(((1 << m) - 1) << off)
        off += m
    return out


def enumerate_dets(n_elec: int, sub, lo=None, hi=None) -> np.ndarray:
    """All N-subsets of range(M) whose per-subspace popcounts lie in the
    windows, as sorted uint64 bitstrings."""
    M = int(sum(sub))
    lo = list(lo) if lo is not None else [0] * len(sub)
    hi = list(hi) if hi is not None else list(sub)
    mk = masks(sub)
    out = []
    for occ in itertools.combinations(range(M), n_elec):
        b = 0
        for i in occ:
            b |= 1 << i
        ok = True
        for k, m in enumerate(mk):
            c = bin(b & m).count("1")
            if c < lo[k] or c > hi[k]:
                ok = False
                break
        if ok:
            out.append(b)
    arr = np.array(sorted(out), dtype=np.uint64)
    return arr


def occupations(b: int, M: int):
    return [i for i in range(M) if (int(b) >> i) & 1]
