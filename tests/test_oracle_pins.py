"""Pins of the CPU oracle against things other than itself.

Each check is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign or index, a transposed operand) fails at least one:
  * the fermion operators satisfy the canonical anticommutation relations;
  * the Slater-Condon matrix equals the literal second-quantised H on tiny
    spaces (windows included), element by element;
  * special cases with closed forms: one electron, g = 0, N = M;
  * invariants: Hermiticity, orbital-rotation invariance of the FCI spectrum,
    spin-ladder structure of a spin-free problem, Kramers degeneracy;
  * the oracle sigma equals the dense product, the oracle Davidson equals
    LAPACK eigh;
  * the gap-theorem bound reproduces the paper's worked example.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import bounds, csc, davidson, dense, fock, space, spinfree

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_ints(M, seed, complex_=True):
    return (synth.complex_integrals(M, seed, rank=6, sigma_f=0.2) if complex_
            else synth.real_integrals(M, seed, rank=6, sigma_f=0.2))


def test_car_relations():
    M = 4
    a = [fock.operator_matrix(M, [("a", p)]) for p in range(M)]
    ad = [fock.operator_matrix(M, [("c", p)]) for p in range(M)]
    eye = np.eye(1 << M)
    for p in range(M):
        assert np.allclose(ad[p], a[p].T)
        for q in range(M):
            assert np.allclose(a[p] @ ad[q] + ad[q] @ a[p], eye * (p == q))
            assert np.allclose(a[p] @ a[q] + a[q] @ a[p], 0)


@pytest.mark.parametrize("M,N,sub,lo,hi,cplx", [
    (6, 3, [6], None, None, True),
    (7, 3, [3, 4], [1, 1], [2, 2], True),
    (8, 4, [2, 3, 3], [0, 1, 1], [2, 2, 3], True),
    (6, 2, [6], None, None, False),
    (8, 3, [4, 4], [1, 0], [3, 2], False),
])
def test_slater_condon_equals_second_quantisation(M, N, sub, lo, hi, cplx):
    ints = rand_ints(M, 17 + M + N, cplx)
    states, Hf = fock.sector_hamiltonian(ints.h, ints.g, N, e_core=0.3)
    dets = space.enumerate_dets(N, sub, lo, hi)
    Hsc = dense.hamiltonian(dets, ints.h, ints.g, e_core=0.3)
    Href = fock.project(states, Hf, dets)
    assert np.max(np.abs(Hsc - Href)) < 1e-13
    assert np.max(np.abs(Hsc - Hsc.conj().T)) < 1e-13


def test_sigma_equals_dense_product():
    ints = rand_ints(9, 5)
    dets = space.enumerate_dets(4, [4, 5], [1, 1], [3, 3])
    H = dense.hamiltonian(dets, ints.h, ints.g)
    c = synth.test_vector(len(dets), 9)
    s = csc.sigma(dets, ints.h, ints.g, c)
    assert np.linalg.norm(s - H @ c) <= 1e-13 * np.linalg.norm(H @ c)
    rows = np.array([0, 3, len(dets) - 1])
    assert np.allclose(csc.sigma_rows(dets, ints.h, ints.g, c, rows), s[rows], atol=1e-14)
    assert np.allclose(csc.diag(dets, ints.h, ints.g), np.diag(H).real, atol=1e-14)


def test_one_electron_is_h():
    ints = rand_ints(7, 3)
    dets = space.enumerate_dets(1, [7])
    H = dense.hamiltonian(dets, ints.h, ints.g, e_core=-1.5)
    # dets sorted ascending: |1<<0>, |1<<1>, ... so H = h + e_core exactly
    assert np.max(np.abs(H - (ints.h + (-1.5) * np.eye(7)))) < 1e-15


def test_zero_two_electron_spectrum():
    ints = rand_ints(7, 4)
    g0 = np.zeros_like(ints.g)
    dets = space.enumerate_dets(3, [7])
    w = np.linalg.eigvalsh(dense.hamiltonian(dets, ints.h, g0))
    e = np.linalg.eigvalsh(ints.h)
    ref = sorted(sum(e[list(c)]) for c in __import__("itertools").combinations(range(7), 3))
    assert np.allclose(w, ref, atol=1e-12)


def test_full_occupation_closed_form():
    ints = rand_ints(5, 8)
    dets = space.enumerate_dets(5, [5])
    H = dense.hamiltonian(dets, ints.h, ints.g)
    h, g = ints.h, ints.g
    e = np.trace(h) + 0.5 * sum(g[i, i, j, j] - g[i, j, j, i] for i in range(5) for j in range(5) if i != j)
    assert H.shape == (1, 1) and abs(H[0, 0] - e) < 1e-13


def rotate(h, g, U):
    h2 = U.conj().T @ h @ U
    g2 = np.einsum("ap,bq,cr,ds,abcd->pqrs", U.conj(), U, U.conj(), U, g, optimize=True)
    return h2, g2


def test_rotation_invariance():
    ints = rand_ints(8, 21)
    rng = np.random.default_rng(3)
    Z = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
    U, _ = np.linalg.qr(Z)
    h2, g2 = rotate(ints.h, ints.g, U)
    dets = space.enumerate_dets(3, [8])
    w1 = np.linalg.eigvalsh(dense.hamiltonian(dets, ints.h, ints.g))
    w2 = np.linalg.eigvalsh(dense.hamiltonian(dets, h2, g2))
    assert np.allclose(w1, w2, atol=1e-11)
    # a transposed two-electron index changes the spectrum (the check bites)
    w3 = np.linalg.eigvalsh(dense.hamiltonian(dets, h2, g2.transpose(0, 1, 3, 2)))
    assert np.max(np.abs(w3 - w1)) > 1e-4


def test_block_rotation_invariance_das():
    """A windowed space is invariant under unitaries that act inside each subspace."""
    ints = rand_ints(8, 22)
    rng = np.random.default_rng(4)
    U = np.zeros((8, 8), dtype=complex)
    for a, b in [(0, 3), (3, 8)]:
        Z = rng.normal(size=(b - a, b - a)) + 1j * rng.normal(size=(b - a, b - a))
        U[a:b, a:b] = np.linalg.qr(Z)[0]
    h2, g2 = rotate(ints.h, ints.g, U)
    dets = space.enumerate_dets(4, [3, 5], [1, 1], [2, 3])
    w1 = np.linalg.eigvalsh(dense.hamiltonian(dets, ints.h, ints.g))
    w2 = np.linalg.eigvalsh(dense.hamiltonian(dets, h2, g2))
    assert np.allclose(w1, w2, atol=1e-11)


def test_spin_ladder_spin_free():
    """Spin-free H: every M_s = 1 eigenvalue reappears in the M_s = 0 sector."""
    ints = synth.real_integrals(4, 31, rank=6, sigma_f=0.2)
    hs, gs = spinfree.expand(ints.h, ints.g)
    d0 = space.enumerate_dets(4, [4, 4], [2, 2], [2, 2])
    d1 = space.enumerate_dets(4, [4, 4], [3, 1], [3, 1])
    w0 = np.linalg.eigvalsh(dense.hamiltonian(d0, hs, gs, real=True))
    w1 = np.linalg.eigvalsh(dense.hamiltonian(d1, hs, gs, real=True))
    for e in w1:
        assert np.min(np.abs(w0 - e)) < 1e-10
    # and the ground state is a singlet (absent from M_s = 1)
    assert np.min(np.abs(w1 - w0[0])) > 1e-6


def test_kramers_degeneracy():
    ints = synth.kramers_integrals(4, 41)
    dets = space.enumerate_dets(3, [8])
    w = np.linalg.eigvalsh(dense.hamiltonian(dets, ints.h, ints.g))
    assert np.allclose(w[0::2], w[1::2], atol=1e-10)


def test_davidson_matches_eigh():
    ints = rand_ints(10, 23)
    dets = space.enumerate_dets(4, [4, 6], [1, 1], [3, 3])
    H = dense.hamiltonian(dets, ints.h, ints.g)
    w, V = np.linalg.eigh(H)
    d = np.diag(H).real
    th, X, rn, it = davidson.davidson(lambda x: H @ x, d, k=3, tol=1e-9, m_max=12)
    assert np.allclose(th, w[:3], atol=1e-10)
    assert np.all(rn <= 1e-9)
    # traditional and compression-compatible forms reach the same energy
    th2, _, _, _ = davidson.davidson(lambda x: H @ x, d, k=1, tol=1e-9, eps=1e-3)
    assert abs(th2[0] - w[0]) < 1e-10


def test_config1_counts_and_ground_state():
    ints, sp, _ = synth.config("c1")
    hs, gs = spinfree.expand(ints.h, ints.g)
    dets = space.enumerate_dets(sp.n_elec, sp.sub, sp.lo, sp.hi)
    assert len(dets) == 4900 == math.comb(8, 4) ** 2
    H = dense.hamiltonian(dets, hs, gs, real=True)
    assert np.allclose(H, H.T, atol=1e-14)
    w = np.linalg.eigvalsh(H)
    th, _, rn, _ = davidson.davidson(lambda x: H @ x, np.diag(H), k=1, tol=1e-10, dtype=np.float64)
    assert abs(th[0] - w[0]) < 1e-10


def test_space_counts():
    assert len(space.enumerate_dets(3, [8])) == 56
    assert len(space.enumerate_dets(4, [4, 6], [1, 1], [3, 3])) == sum(
        math.comb(4, a) * math.comb(6, 4 - a) for a in (1, 2, 3) if 1 <= 4 - a <= 3)
    assert synth.CONFIGS["c2"]["space"].n_dets() == 735471
    assert synth.CONFIGS["c3p"]["space"].n_dets() == 1365867360
    assert synth.CONFIGS["c3lit"]["space"].n_dets() == 19255256592


def test_gap_theorem_paper_example():
    fx = json.load(open(os.path.join(HERE, "golden", "gap_theorem_hbrte.json")))
    b = bounds.gap_bound(fx["resid_norm"], fx["gap_estimate"])
    assert abs(b - 9.9245e-6) < 1e-9
    assert b <= fx["stated_bound"]
    assert bounds.gap_lower_bound(-1.0, -0.5, 0.1) == pytest.approx(0.4)


def test_gap_bound_holds_on_exact_spectrum():
    """Eq. gap with the rigorous gamma^- bounds the true Ritz error."""
    ints = rand_ints(9, 24)
    dets = space.enumerate_dets(3, [9])
    H = dense.hamiltonian(dets, ints.h, ints.g)
    w = np.linalg.eigvalsh(H)
    th, X, rn, _ = davidson.davidson(lambda x: H @ x, np.diag(H).real, k=2, tol=1e-4, max_iter=4)
    g_lo = bounds.gap_lower_bound(th[0], th[1], rn[1])
    if g_lo > 0:
        assert abs(th[0] - w[0]) <= bounds.gap_bound(rn[0], g_lo) + 1e-14


@pytest.mark.parametrize("n,sub,lo,hi", [
    (4, [4, 6], [1, 1], [3, 3]),
    (5, [4, 4, 4], [1, 1, 1], [2, 3, 2]),
    (4, [10], None, None),
])
def test_windowed_row_equals_listed_row(n, sub, lo, hi):
    """The list-free row of P H P (used on spaces too large to enumerate)
    equals the row taken over the explicit determinant list."""
    M = sum(sub)
    ints = synth.complex_integrals(M, 55)
    dets = space.enumerate_dets(n, sub, lo, hi)
    for row in (0, len(dets) // 3, len(dets) - 1):
        idx, v1 = csc.h_row(dets, ints.h, ints.g, row, e_core=0.7)
        bits, v2 = csc.h_row_window(sub, lo, hi, ints.h, ints.g, int(dets[row]), e_core=0.7)
        a = dict(zip(dets[idx].tolist(), v1))
        b = dict(zip(bits.tolist(), v2))
        assert a.keys() == b.keys()
        assert max(abs(a[k] - b[k]) for k in a) < 1e-14


def test_oracle_preconditioner_hand_values():
    """Eq. sparsePreconditioner on a hand-worked case: r = (1, 2, 3, 4, 1),
    H_ii = (0, 1, 2, 5, 2 - 1e-13), theta = 2: denominators (2, 1, 0, -3,
    1e-13), so s = (1/2, 2, 0, -4/3, 0) (the last two below the 1e-12 guard);
    ||s||^2 = 1/4 + 4 + 16/9 = 217/36, so eps = 0.3 keeps |s_i| >= 0.3
    sqrt(217)/6 = 0.7365: (0, 2, 0, -4/3, 0)."""
    from oracle import davidson as odav
    r = np.array([1.0, 2.0, 3.0, 4.0, 1.0])
    d = np.array([0.0, 1.0, 2.0, 5.0, 2.0 - 1e-13])
    s0 = odav.precondition(r, 2.0, d)
    assert np.allclose(s0, [0.5, 2.0, 0.0, -4.0 / 3.0, 0.0], rtol=0, atol=1e-15)
    s1 = odav.precondition(r, 2.0, d, eps=0.3)
    assert np.allclose(s1, [0.0, 2.0, 0.0, -4.0 / 3.0, 0.0], rtol=0, atol=1e-15)
    # just above and below the threshold of the first entry: 0.5 / sqrt(217/36)
    t = 0.5 / np.sqrt(217.0 / 36.0)
    assert odav.precondition(r, 2.0, d, eps=t * (1 - 1e-9))[0] == 0.5
    assert odav.precondition(r, 2.0, d, eps=t * (1 + 1e-9))[0] == 0.0
