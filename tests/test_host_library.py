"""Host-side checks of libstpci (no GPU): exported symbols, space and table
logic, work counts, layout, validation, and the host eigensolver."""
import glob
import math
import os
import re

import numpy as np
import pytest

import paper_2505_20375_amd as stpci
import synth
from oracle import space as ospace
from tests import layout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(hdr).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(stpci_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert "stpci_sigma" in names and "stpci_davidson" in names
    for n in sorted(names):
        assert hasattr(stpci._lib, n), n


def host_ctx(n_elec, sub, lo=None, hi=None):
    c = stpci.Context(device=-1)
    c.set_space(n_elec, sub, lo, hi)
    return c


@pytest.mark.parametrize("name", ["c1", "c2", "c3p", "c3lit"])
def test_space_sizes(name):
    sp = synth.CONFIGS[name]["space"]
    c = host_ctx(sp.n_elec, sp.sub, sp.lo, sp.hi)
    info = c.space_info()
    assert info.n_dets == sp.n_dets()
    assert info.n_cat == len(sp.categories())
    if name == "c3p":
        assert info.n_dets == 1365867360 and info.n_cat == 10
        assert info.w_sigma_macs == pytest.approx(3.80e11 + 1.144e14, rel=2e-3)
    if name == "c2":
        assert info.nnz_h == pytest.approx(2.566e9, rel=1e-3)


@pytest.mark.parametrize("n,sub,lo,hi", [
    (3, [8], None, None),
    (4, [4, 6], [1, 1], [3, 3]),
    (5, [4, 4, 4], [1, 1, 1], [2, 3, 2]),
    (4, [4, 4, 4], None, None),
    (8, [8, 8], [4, 4], [4, 4]),
])
def test_layout_and_address_to_det(n, sub, lo, hi):
    c = host_ctx(n, sub, lo, hi)
    ref = layout.layout_dets(n, sub, lo, hi)
    info = c.space_info()
    assert info.n_dets == len(ref)
    got = np.array([c.address_to_det(i) for i in range(len(ref))], dtype=np.uint64)
    assert np.array_equal(got, ref)
    # same determinant set as the oracle's enumeration
    assert np.array_equal(np.sort(got), ospace.enumerate_dets(n, sub, lo, hi))
    cats = layout.categories(n, sub, lo or [0] * len(sub), hi or list(sub))
    off = 0
    for i, t in enumerate(cats):
        occ, o, nd = c.category(i)
        assert occ == t and o == off
        assert nd == math.prod(math.comb(m, k) for m, k in zip(sub, t))
        off += nd


def brute_counts(n, sub, lo, hi):
    """W1, W2 and structural nnz(H) by explicit enumeration of bitstrings."""
    M = sum(sub)
    lo = lo or [0] * len(sub)
    hi = hi or list(sub)
    dets = ospace.enumerate_dets(n, sub, lo, hi)
    inset = set(int(b) for b in dets)
    allN = ospace.enumerate_dets(n, [M])
    W1 = W2 = 0
    for J in allN:
        J = int(J)
        deg = 0
        for y in range(M):
            if not (J >> y) & 1:
                continue
            for x in range(M):
                if x != y and (J >> x) & 1:
                    continue
                K = (J & ~(1 << y)) | (1 << x)
                if K in inset:
                    deg += 1
        W2 += deg * deg
        if J in inset:
            W1 += deg
    nnz = 0
    for L in dets:
        for K in dets:
            if bin(int(L) ^ int(K)).count("1") <= 4:
                nnz += 1
    return W1, W2, nnz


@pytest.mark.parametrize("n,sub,lo,hi", [
    (3, [7], None, None),
    (4, [4, 6], [1, 1], [3, 3]),
    (4, [3, 3, 3], [1, 0, 1], [2, 2, 2]),
])
def test_work_counts_match_brute_force(n, sub, lo, hi):
    c = host_ctx(n, sub, lo, hi)
    info = c.space_info()
    W1, W2, nnz = brute_counts(n, sub, lo, hi)
    assert info.w_sigma_macs == W1 + W2
    assert info.nnz_h == nnz


def test_invalid_inputs_are_rejected():
    c = stpci.Context(device=-1)
    with pytest.raises(stpci.StpciError) as e:
        c.set_space(9, [4, 4], [0, 0], [4, 4])  # 9 electrons cannot fit
    assert e.value.status in (stpci.EINVAL,)
    with pytest.raises(stpci.StpciError):
        c.set_space(4, [4, 4], [3, 3], [4, 4])  # windows exclude every pattern
    ints = synth.complex_integrals(4, 1)
    bad = ints.h.copy()
    bad[0, 1] += 0.1
    with pytest.raises(stpci.StpciError) as e:
        c.set_integrals(bad, ints.g)
    assert e.value.status == stpci.EINVAL
    g2 = ints.g.copy()
    g2[0, 1, 2, 3] += 0.01
    with pytest.raises(stpci.StpciError):
        c.set_integrals(ints.h, g2)
    c.set_integrals(ints.h, ints.g)
    with pytest.raises(stpci.StpciError) as e:
        c.sigma(0, 0)
    # device calls on a host-only context report a state error, not a crash
    assert e.value.status in (stpci.EINVAL, stpci.ESTATE)


def test_report_and_precision_arguments_are_checked():
    """Argument checks of the reporting calls and of the precision codes
    (host-only context: nothing touches a device)."""
    import ctypes
    c = stpci.Context(device=-1)
    n = ctypes.c_int()
    assert stpci._lib.stpci_dav_sigma_count(c._h, 3, ctypes.byref(n)) == stpci.EINVAL
    assert stpci._lib.stpci_dav_sigma_count(c._h, -1, ctypes.byref(n)) == stpci.EINVAL
    assert stpci._lib.stpci_dav_sigma_count(None, 0, ctypes.byref(n)) == stpci.EINVAL
    for p in (stpci.FP64, stpci.FP32, stpci.BF16):
        assert stpci._lib.stpci_dav_sigma_count(c._h, p, ctypes.byref(n)) == stpci.OK
        assert n.value == 0
    buf = (ctypes.c_double * 4)()
    assert stpci._lib.stpci_dav_history_dc(c._h, -1, buf) == stpci.EINVAL
    assert stpci._lib.stpci_dav_history_dc(c._h, 4, None) == stpci.EINVAL
    assert stpci._lib.stpci_dav_history_dc(c._h, 4, buf) == stpci.OK
    c.set_space(2, [4])
    assert c.history() == 0
    # an unknown precision code is rejected before any device work
    with pytest.raises(stpci.StpciError):
        c.sigma(0, 0, precision=7)


def test_host_eigensolver_matches_lapack():
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 17, 40):
        Z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        A = Z + Z.conj().T
        w, V = stpci.heev(A)
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-11 * max(1, np.abs(A).max()))
        assert np.allclose(A @ V, V * w, atol=1e-10 * max(1, np.abs(A).max()))
        assert np.allclose(V.conj().T @ V, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("name,cap", [("T2", 1 << 40), ("T3", 1 << 40), ("T4", 1 << 40), ("T8", 1 << 40),
                                      ("c1", 1 << 40), ("c2", 5000), ("c3p", 300)])
def test_kernel_move_arithmetic_on_host(name, cap):
    """The move enumeration, signs and target addresses that the sigma kernels
    compute (same code, compiled for the host) agree with the global
    fermion-sign rule and stay inside the space."""
    sp = (synth.CONFIGS.get(name) or synth.TSPACES[name])["space"]
    c = host_ctx(sp.n_elec, sp.sub, sp.lo, sp.hi)
    n, bad = c.test_moves(cap)
    assert n > 0 and bad == 0


@pytest.mark.parametrize("name,cap", [("T2", 1 << 40), ("T3", 1 << 40), ("T4", 1 << 40), ("T8", 1 << 40),
                                      ("c1", 1 << 40), ("c2", 3000), ("c3p", 200)])
def test_pair_kernel_arithmetic_on_host(name, cap):
    """The pair-slot enumeration, signs and target addresses of the pair
    kernel (same code, compiled for the host) agree with the global fermion
    sign of a+_p a+_r on the occupation bits and stay inside the space."""
    sp = (synth.CONFIGS.get(name) or synth.TSPACES[name])["space"]
    c = host_ctx(sp.n_elec, sp.sub, sp.lo, sp.hi)
    n, bad = c.test_pairs(cap)
    assert n > 0 and bad == 0


@pytest.mark.parametrize("name,cap", [("T3", 1 << 40), ("T4", 1 << 40), ("T8", 1 << 40), ("c1", 1 << 40),
                                      ("c2_12_12", 40), ("c2_8_8_8", 40), ("c3p", 3)])
def test_spectator_batched_arithmetic_on_host(name, cap):
    """The padded pair lists, member tables, entry signs and target addresses
    of the spectator-batched kernel (same code, compiled for the host): an
    entry vanishes exactly when its pair meets an orbital occupied in the
    member, otherwise it holds K' + {p, r} with the global fermion sign of
    a+_p a+_r; each member meets every pair that leads into the space once;
    the item streams cover every column chunk once."""
    if name.startswith("c2_"):
        sub = [int(x) for x in name[3:].split("_")]
        c = host_ctx(8, sub, None, None)
    else:
        sp = (synth.CONFIGS.get(name) or synth.TSPACES[name])["space"]
        c = host_ctx(sp.n_elec, sp.sub, sp.lo, sp.hi)
    n, bad = c.test_sb(cap)
    assert n > 0 and bad == 0


def test_spectator_batched_kernel_refuses_one_subspace():
    c = host_ctx(5, [12], None, None)
    with pytest.raises(Exception):
        c.test_sb()


@pytest.mark.parametrize("n,sub,lo,hi,ok", [
    (3, [3], None, None, True), (3, [8], None, None, True), (4, [12], None, None, True),
    (8, [24], None, None, True), (10, [16], None, None, True), (7, [8], None, None, True),
    (2, [8], None, None, False), (5, [4, 4, 4], [1, 1, 1], [2, 3, 2], False), (4, [6, 6], None, None, False),
])
def test_pair_groups_on_host(n, sub, lo, hi, ok):
    """Items of the grouped pair kernel: every (N-2)-electron intermediate in
    exactly one item, each member the item's core plus one electron; spaces of
    several subspaces or fewer than three electrons are refused."""
    c = host_ctx(n, sub, lo, hi)
    if not ok:
        with pytest.raises(Exception):
            c.test_pair_groups()
        return
    items, bad, unit = c.test_pair_groups()
    assert items > 0 and bad == 0 and unit in (4, 8)


def brute_pair_counts(n, sub, lo, hi):
    """sum over (N-2)-electron bit strings K' of deg(K')^2, deg = pairs p < r
    empty in K' with K' + {p, r} in the space."""
    M = sum(sub)
    inset = set(int(b) for b in ospace.enumerate_dets(n, sub, lo, hi))
    W = 0
    nk = 0
    maxd = 0
    for K in ospace.enumerate_dets(n - 2, [M]):
        K = int(K)
        d = sum(1 for r in range(M) for p in range(r)
                if not (K >> p) & 1 and not (K >> r) & 1 and (K | 1 << p | 1 << r) in inset)
        if d:
            W += d * d
            nk += 1
            maxd = max(maxd, d)
    return W, nk, maxd


@pytest.mark.parametrize("n,sub,lo,hi", [
    (3, [7], None, None),
    (4, [4, 6], [1, 1], [3, 3]),
    (5, [3, 3, 3], [1, 0, 1], [2, 2, 2]),
    (2, [3, 4], [0, 1], [1, 2]),
])
def test_pair_counts_match_brute_force(n, sub, lo, hi):
    c = host_ctx(n, sub, lo, hi)
    W, nk, maxd = brute_pair_counts(n, sub, lo, hi)
    w, npi, md = c.pair_counts()
    assert (w, npi, md) == (W, nk, maxd)


@pytest.mark.parametrize("n,sub,lo,hi", [
    (5, [4, 4, 4], [1, 1, 1], [2, 3, 2]),
    (4, [4, 6], [1, 1], [3, 3]),
    (3, [9], None, None),
])
def test_layout_address_formula(n, sub, lo, hi):
    """The closed-form address of the test layout module agrees with its
    explicit enumeration (and therefore with the library, test above)."""
    ref = layout.layout_dets(n, sub, lo, hi)
    for a, b in enumerate(ref):
        assert layout.address(int(b), n, sub, lo, hi) == a


def test_exponential_search_equals_lower_bound():
    """The exponential search of Alg. sigmaBuild (as the compressed sigma
    build runs it) returns the lower bound of x in a[i:], i.e.
    numpy.searchsorted(a[i:], x, 'left') + i, on random sorted arrays with
    repeated values, from random start positions, for values below, inside
    and above the range, and for empty ranges."""
    import paper_2505_20375_amd as stpci
    rng = np.random.default_rng(41)
    checked = 0
    for n in (0, 1, 2, 3, 7, 64, 1000, 4097):
        a = np.sort(rng.integers(0, max(2 * n, 4), n).astype(np.uint32))
        for _ in range(200 if n else 3):
            i = int(rng.integers(0, n + 1))
            x = int(rng.integers(0, max(2 * n, 4) + 3))
            ref = i + int(np.searchsorted(a[i:], np.uint32(x), side="left"))
            assert stpci.test_exp_search(a, i, x) == ref, (n, i, x)
            checked += 1
        if n:
            assert stpci.test_exp_search(a, 0, int(a[-1]) + 1) == n
            assert stpci.test_exp_search(a, 0, 0) == 0
            assert stpci.test_exp_search(a, n, 0) == n
    assert stpci.test_exp_search(np.zeros(4, np.uint32), 5, 0) == -1
    assert checked > 1000


def test_sigma_kernel_names():
    """The selectable sigma kernels; the removed one-move forms and unknown
    names are refused with STPCI_EINVAL."""
    import paper_2505_20375_amd as stpci
    c = stpci.Context(device=-1)
    for name in ("auto", "pair", "pair_atomic", "pair_mf64", "pair_valu", "pair_grp", "pair_sb", "tile", "rowtile"):
        c.set_sigma_kernel(name)
    for name in ("wave", "simple", "bogus", ""):
        with pytest.raises(stpci.StpciError):
            c.set_sigma_kernel(name)
    del c


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: a request for several exits with status 2
    and says why, before touching a device."""
    import subprocess
    import sys
    from pathlib import Path
    root = Path(__file__).resolve().parents[1]
    p = subprocess.run([sys.executable, str(root / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=root)
    assert p.returncode == 2
    assert "exactly one GPU" in p.stderr and p.stdout == ""
