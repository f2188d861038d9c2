"""GPU parity of the Davidson building blocks that the energies cannot see:
the diagonal formed on the fly (a wrong H_ii only slows convergence) and the
preconditioner of Eq. sparsePreconditioner, both against the CPU oracle,
element by element; and the eps > 0 solver against eps = 0.
"""
import numpy as np
import pytest

import synth
from oracle import csc, davidson as odav
from tests.gpu_util import Problem, rel_err

pytestmark = pytest.mark.gpu


def _diag_gpu(ctx, n):
    import torch
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.diagonal(d)
    torch.cuda.synchronize()
    return d


@pytest.mark.parametrize("name", ["T2", "T3", "T4", "T8", "T8fci", "c1", "c2"])
def test_diagonal_matches_oracle(name):
    """H_ii from the occupation bits (never stored by the solver) equals the
    oracle's Slater-Condon diagonal on every determinant."""
    print("case", name, flush=True)
    pb = Problem.named(name)
    ctx = pb.context()
    d = pb.from_device(_diag_gpu(ctx, len(pb.dets)))
    ref = csc.diag(pb.dets, pb.h, pb.g, e_core=pb.ints.e_core)
    assert np.max(np.abs(d - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_diagonal_config3p_sampled_rows():
    """40 spinors, 12|16|12, 11 electrons (1.37e9 determinants): H_ii on the
    first and last determinant of every category and on random ones, each
    determinant's bits taken from the library and its address checked
    against the documented layout."""
    import torch
    import paper_2505_20375_amd as stpci
    from tests import layout
    ints, sp, _ = synth.config("c3p")
    free, _tot = torch.cuda.mem_get_info()
    if free < 1.2 * sp.n_dets() * 8:
        pytest.skip("needs %.0f GB of free device memory" % (1.2 * sp.n_dets() * 8 / 1e9))
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    info = ctx.space_info()
    d = _diag_gpu(ctx, info.n_dets)
    rows = []
    for cat in range(info.n_cat):
        _, off, cnt = ctx.category(cat)
        rows += [off, off + cnt - 1, off + cnt // 2]
    rng = np.random.default_rng(11)
    rows = sorted(set(rows) | set(int(x) for x in rng.choice(info.n_dets, 200, replace=False)))
    bits = np.array([ctx.address_to_det(a) for a in rows], dtype=np.uint64)
    assert np.array_equal(layout.address_array(bits, sp.n_elec, sp.sub, sp.lo, sp.hi), np.array(rows))
    ref = csc.diag(bits, ints.h, ints.g)
    got = d[torch.tensor(rows, device="cuda")].cpu().numpy()
    del d
    torch.cuda.empty_cache()
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("name,eps", [("T4", 0.0), ("T4", 0.05), ("c1", 0.0), ("c1", 0.02), ("T8fci", 0.01),
                                      ("c2", 0.0), ("c2", 1e-3)])
def test_preconditioner_matches_oracle(name, eps):
    """Eq. sparsePreconditioner as the solver applies it, for three residuals
    at once, against the oracle's precondition(): s = r / (theta - H_ii) with
    the 1e-12 guard (one theta equal to a diagonal element, so the guard
    fires), then the eps ||s|| drop."""
    import torch
    print("case", name, eps, flush=True)
    pb = Problem.named(name)
    ctx = pb.context()
    n = len(pb.dets)
    diag = csc.diag(pb.dets, pb.h, pb.g, e_core=pb.ints.e_core)
    rng = np.random.default_rng(5)
    order = np.argsort(diag)
    thetas = [diag[order[0]] - 0.05, diag[order[min(3, n - 1)]], float(np.mean(diag))]
    rs = [pb.vector(40 + q) for q in range(3)]
    r_dev = torch.cat([pb.to_device(r) for r in rs])
    t_dev = torch.empty_like(r_dev)
    ctx.test_precond(r_dev, t_dev, thetas, eps)
    for q in range(3):
        got = pb.from_device(t_dev[q * n:(q + 1) * n])
        ref = odav.precondition(rs[q], thetas[q], diag, eps=eps)
        # entries within rounding of the drop threshold may go either way
        s = odav.precondition(rs[q], thetas[q], diag, eps=0.0)
        thr = eps * np.linalg.norm(s)
        near = np.abs(np.abs(s) - thr) <= 1e-10 * max(thr, 1e-300)
        ok = ~near
        # the library forms H_ii in its own summation order: a difference of
        # a few ulp of H_ii moves s_i by |s_i| |H_ii| ulp / |theta - H_ii|
        den = np.abs(thetas[q] - diag)
        cond = 1.0 + (np.abs(diag) + abs(thetas[q])) / np.maximum(den, 1e-300)
        bound = 1e-14 * np.abs(ref) * cond + 1e-15 * np.max(np.abs(ref))
        assert np.all(np.abs(got[ok] - ref[ok]) <= bound[ok])
        assert np.array_equal(got[ok] == 0, ref[ok] == 0)
        if eps > 0:
            assert np.count_nonzero(ref == 0) > np.count_nonzero(s == 0)   # the drop removed entries
    # the guard: theta equal to H_ii gives t_i = 0 there
    got1 = pb.from_device(t_dev[n:2 * n])
    assert got1[order[min(3, n - 1)]] == 0


@pytest.mark.parametrize("name,k,eps", [("T4", 2, 0.05), ("c1", 1, 0.02), ("T8", 3, 0.03)])
def test_davidson_with_eps_drop_matches_exact(name, k, eps):
    """Davidson with the compression-compatible preconditioner (eps > 0)
    converges to the same energies as exact diagonalisation and as the
    eps = 0 solver (the residual and sigma stay exact; only the expansion
    vectors are sparser)."""
    from oracle import dense
    pb = Problem.named(name)
    w = np.linalg.eigvalsh(dense.hamiltonian(pb.dets, pb.h, pb.g))[:k] + pb.ints.e_core
    ctx = pb.context()
    e0, r0, it0, _ = ctx.davidson(k=k, tol=1e-9, max_iter=300)
    e1, r1, it1, _ = ctx.davidson(k=k, tol=1e-9, max_iter=300, eps_drop=eps)
    assert np.max(r1) <= 1e-9
    assert np.max(np.abs(e1 - w)) <= 1e-9
    assert np.max(np.abs(e1 - e0)) <= 1e-9


@pytest.mark.parametrize("name,prec", [("T4", "fp32"), ("c2", "fp32"), ("c2", "bf16")])
def test_refine_tol_energy_stops_refinement(name, prec):
    """With a reduced-precision phase, refine_tol_energy > 0 ends the FP64
    refinement once every requested root's gap-theorem bound is below it
    (the run carries one extra root for the gap): the energy then lies within
    1e-8 Eh of the residual-converged solve, the reported bounds are below
    the tolerance."""
    import paper_2505_20375_amd as stpci
    code = {"fp32": stpci.FP32, "bf16": stpci.BF16}[prec]
    pb = Problem.named(name)
    ctx = pb.context()
    e_res, r_res, _, _ = ctx.davidson(k=1, tol=1e-9, max_iter=400, precision=code)
    e_en, r_en, _, st = ctx.davidson(k=1, tol=1e-9, max_iter=400, precision=code, refine_tol_energy=1e-9)
    gam, bnd = ctx.certificate()
    assert st == stpci.OK
    assert abs(e_en[0] - e_res[0]) <= 1e-8
    assert bnd[0] < 1e-9 or r_en[0] <= 1e-9


def test_invalid_solver_options_are_rejected():
    import paper_2505_20375_amd as stpci
    pb = Problem.named("T4")
    ctx = pb.context()
    for kw in (dict(eps_drop=-0.1), dict(eps_drop=1.5), dict(refine_tol_energy=-1.0),
               dict(refine_tol_energy=float("inf"))):
        with pytest.raises(stpci.StpciError):
            ctx.davidson(k=1, tol=1e-8, **kw)


@pytest.mark.parametrize("name,m,k,with_z", [("T4", 3, 1, False), ("T4", 7, 2, True), ("c1", 6, 5, True),
                                             ("T8fci", 1, 1, True), ("c2", 5, 2, True)])
def test_fused_ritz_pass_matches_oracle(name, m, k, with_z):
    """The solver's fused Rayleigh-Ritz pass (Ritz vectors, residuals'
    corrections by Eq. sparsePreconditioner before the eps drop, and the
    reductions the host reads) against numpy products and the oracle's
    precondition() on random basis vectors, coefficients and Ritz values
    (one equal to a diagonal element, so the guard fires), k up to 5 (two
    groups of four roots)."""
    import torch
    print("case", name, m, k, with_z, flush=True)
    pb = Problem.named(name)
    ctx = pb.context()
    n = len(pb.dets)
    diag = csc.diag(pb.dets, pb.h, pb.g, e_core=pb.ints.e_core)
    rng = np.random.default_rng(17)
    dt = np.complex128 if pb.cplx else np.float64

    def rnd(*shape):
        a = rng.standard_normal(shape)
        return a + 1j * rng.standard_normal(shape) if pb.cplx else a
    V, W = rnd(n, m), rnd(n, m)
    Y, Z = rnd(m, k), (rnd(m, k) if with_z else None)
    order = np.argsort(diag)
    theta = np.array([diag[order[0]] - 0.05, diag[order[min(3, n - 1)]], float(np.mean(diag)), 1.5, -2.0][:k])
    v_dev = torch.cat([pb.to_device(V[:, i].astype(dt)) for i in range(m)])
    w_dev = torch.cat([pb.to_device(W[:, i].astype(dt)) for i in range(m)])
    x_dev = torch.empty(k * n, dtype=v_dev.dtype, device="cuda")
    t_dev = torch.empty_like(x_dev)
    red = ctx.test_ritz(v_dev, w_dev, m, Y, Z, theta, x_dev, t_dev)
    X = V @ Y
    R = W @ Y - X * theta
    for j in range(k):
        x = pb.from_device(x_dev[j * n:(j + 1) * n])
        assert np.max(np.abs(x - X[:, j])) <= 1e-13 * np.max(np.abs(X[:, j]))
        t = pb.from_device(t_dev[j * n:(j + 1) * n])
        ref = odav.precondition(R[:, j], theta[j], diag, eps=0.0)
        den = np.abs(theta[j] - diag)
        cond = 1.0 + (np.abs(diag) + abs(theta[j])) / np.maximum(den, 1e-300)
        # r_j itself carries the rounding of two m-term sums
        bound = 1e-13 * (np.abs(ref) * cond + np.max(np.abs(R[:, j])) / np.maximum(den, 1e-12))
        assert np.all(np.abs(t - ref) <= bound)
        assert np.array_equal(t == 0, ref == 0)
        assert abs(red[j, 0] - np.linalg.norm(R[:, j]) ** 2) <= 1e-12 * np.linalg.norm(R[:, j]) ** 2
        assert abs(red[j, 1] - np.linalg.norm(ref) ** 2) <= 1e-11 * np.linalg.norm(ref) ** 2
        if with_z:
            dmax = np.max(np.abs(V @ Z[:, j]) ** 2)
            assert abs(red[j, 2] - dmax) <= 1e-12 * dmax
        else:
            assert red[j, 2] == 0
    if k >= 2:   # the guard: theta equal to H_ii gives t_i = 0 there
        assert pb.from_device(t_dev[n:2 * n])[order[min(3, n - 1)]] == 0
