"""The documented CI-vector layout, written out independently of the library.

Categories in lexicographic order of (n_1..n_K); inside a category, row-major
over the local string ranks with subspace 1 slowest; the local rank of a
string is its position among the masks of equal popcount sorted ascending.
Used by the tests to move seeded vectors between the oracle's order
(ascending bitstring) and the library's layout.
"""
import itertools
import math

import numpy as np


def categories(n_elec, sub, lo, hi):
    out = []
    for t in itertools.product(*[range(max(l, 0), min(h, m) + 1) for m, l, h in zip(sub, lo, hi)]):
        if sum(t) == n_elec:
            out.append(t)
    return sorted(out)


def local_masks(m, n):
    return sorted(sum(1 << i for i in c) for c in itertools.combinations(range(m), n))


def layout_dets(n_elec, sub, lo=None, hi=None):
    lo = list(lo) if lo is not None else [0] * len(sub)
    hi = list(hi) if hi is not None else list(sub)
    offs = np.cumsum([0] + list(sub))[:-1]
    out = []
    for t in categories(n_elec, sub, lo, hi):
        lists = [local_masks(m, n) for m, n in zip(sub, t)]
        for combo in itertools.product(*lists):
            b = 0
            for k, mk in enumerate(combo):
                b |= int(mk) << int(offs[k])
            out.append(b)
    return np.array(out, dtype=np.uint64)


class Perm:
    """Maps vectors between oracle order (sorted dets) and library layout."""

    def __init__(self, sorted_dets, lib_dets):
        self.idx = np.searchsorted(sorted_dets, lib_dets)
        assert np.all(sorted_dets[self.idx] == lib_dets)

    def to_lib(self, x_oracle):
        return x_oracle[self.idx]

    def to_oracle(self, x_lib):
        out = np.empty_like(x_lib)
        out[self.idx] = x_lib
        return out


def local_rank(mask):
    """Position of `mask` among the masks of equal popcount sorted ascending:
    the number of smaller masks with as many bits, counted by choosing, for
    each set bit i (at bit position b), the masks that agree above b and have
    0 at b: C(b, i + 1) of them."""
    r, i = 0, 0
    b = 0
    while mask:
        if mask & 1:
            r += math.comb(b, i + 1)
            i += 1
        mask >>= 1
        b += 1
    return r


def address(bits, n_elec, sub, lo=None, hi=None):
    """Vector address of determinant `bits` under the documented layout, or -1."""
    lo = list(lo) if lo is not None else [0] * len(sub)
    hi = list(hi) if hi is not None else list(sub)
    bits = int(bits)
    loc, occ, off = [], [], 0
    for m in sub:
        s = (bits >> off) & ((1 << m) - 1)
        loc.append(s)
        occ.append(bin(s).count("1"))
        off += m
    cats = categories(n_elec, sub, lo, hi)
    t = tuple(occ)
    if t not in cats:
        return -1
    base = 0
    for c in cats:
        if c == t:
            break
        base += math.prod(math.comb(m, n) for m, n in zip(sub, c))
    a, stride = 0, 1
    for k in reversed(range(len(sub))):
        a += local_rank(loc[k]) * stride
        stride *= math.comb(sub[k], t[k])
    return base + a


def _rank_table(m):
    """local_rank of every m-bit mask (the same sum of binomials as
    local_rank, evaluated for all masks at once)."""
    masks = np.arange(1 << m, dtype=np.int64)
    rank = np.zeros(1 << m, dtype=np.int64)
    seen = np.zeros(1 << m, dtype=np.int64)   # set bits below the current position
    for b in range(m):
        bit = (masks >> b) & 1
        comb = np.array([math.comb(b, i + 1) for i in range(m + 1)], dtype=np.int64)
        rank += bit * comb[seen]
        seen += bit
    return rank


def address_array(bits, n_elec, sub, lo=None, hi=None):
    """address() for an array of determinants at once (NumPy); -1 outside
    the space."""
    lo = list(lo) if lo is not None else [0] * len(sub)
    hi = list(hi) if hi is not None else list(sub)
    bits = np.asarray(bits, dtype=np.uint64)
    cats = categories(n_elec, sub, lo, hi)
    base, b = {}, 0
    for c in cats:
        base[c] = b
        b += math.prod(math.comb(m, n) for m, n in zip(sub, c))
    locs, occs, off = [], [], 0
    for m in sub:
        s = ((bits >> np.uint64(off)) & np.uint64((1 << m) - 1)).astype(np.int64)
        locs.append(s)
        occs.append(np.array([bin(int(x)).count("1") for x in range(1 << m)], dtype=np.int64)[s])
        off += m
    out = np.full(len(bits), -1, dtype=np.int64)
    if len(bits) == 0:
        return out
    occ = np.stack(occs, axis=1)
    tables = {m: _rank_table(m) for m in set(sub)}
    # group the determinants by occupation tuple (one pass per tuple present)
    uniq, inv = np.unique(occ, axis=0, return_inverse=True)
    inv = np.asarray(inv).reshape(-1)
    order = np.argsort(inv, kind="stable")
    bounds = np.searchsorted(inv[order], np.arange(len(uniq) + 1))
    for u in range(len(uniq)):
        c = tuple(int(x) for x in uniq[u])
        if c not in base:
            continue
        sel = order[bounds[u]:bounds[u + 1]]
        a = np.zeros(len(sel), dtype=np.int64)
        stride = 1
        for k in reversed(range(len(sub))):
            a += tables[sub[k]][locs[k][sel]] * stride
            stride *= math.comb(sub[k], c[k])
        out[sel] = base[c] + a
    return out
