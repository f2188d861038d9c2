"""Precision form: category-block contractions in FP32 (VALU) or BF16 (matrix
cores, FP32 accumulation), Davidson residual, orthogonalisation and subspace
problem in FP64, and FP64 refinement of the reduced-precision iterate.
Energies after refinement must agree with the all-FP64 result and with exact
diagonalisation within 1e-8 Eh; the sigma error against FP64 is bounded by
the rounding of the contraction type (FP32: 2^-24 relative per operand, the
bound 2e-6 allows the accumulation over up to a few hundred terms; BF16:
2^-9 per operand, bound 2e-2)."""
import numpy as np
import pytest

import synth
from oracle import dense
from tests.gpu_util import Problem, rel_err

pytestmark = pytest.mark.gpu


def _sigma(pb, c, prec):
    import torch
    import paper_2505_20375_amd as stpci
    ctx = pb.context()
    x = pb.to_device(c)
    out = torch.empty_like(x)
    ctx.sigma(x, out, precision=prec)
    torch.cuda.synchronize()
    return pb.from_device(out)


@pytest.mark.parametrize("name", ["T4", "c1", "c2"])
def test_fp32_sigma_error_is_single_precision(name):
    import paper_2505_20375_amd as stpci
    pb = Problem.named(name)
    c = pb.vector()
    s64 = _sigma(pb, c, stpci.FP64)
    s32 = _sigma(pb, c, stpci.FP32)
    err = rel_err(s32, s64)
    print("fp32 sigma relative error", name, err)
    assert 0 < err <= 2e-6
    if len(pb.dets) < 50000:
        assert rel_err(s64, pb.oracle_sigma(c)) <= 1e-12


@pytest.mark.parametrize("n,M,cplx,n_vec,kernel", [(5, 16, True, 2, "pair"), (6, 10, False, 3, "pair"),
                                                    (4, 12, True, 1, "pair_atomic"), (3, 8, True, 2, "pair"),
                                                    (4, 22, True, 2, "pair")])
def test_grouped_fp32_sigma(n, M, cplx, n_vec, kernel):
    """Spaces of one subspace: the grouped matrix-core kernel with the FP32
    table, right-hand side and accumulation (FP64 sums of the contributions)
    stays within single-precision error of the oracle, for one to three
    vectors and both scatter modes."""
    import torch
    import paper_2505_20375_amd as stpci
    print("case", n, M, cplx, n_vec, kernel, flush=True)
    ints = (synth.complex_integrals if cplx else synth.real_integrals)(M, 60 + n, rank=8, sigma_f=0.05)
    pb = Problem(ints, synth.SpaceSpec(n, [M]), seed=3)
    cs = [pb.vector(v) for v in range(1, n_vec + 1)]
    ctx = pb.context()
    ctx.set_sigma_kernel(kernel)
    x = torch.cat([pb.to_device(v) for v in cs])
    out = torch.empty_like(x)
    ctx.sigma(x, out, n_vec=n_vec, precision=stpci.FP32)
    torch.cuda.synchronize()
    assert ctx.sigma_kernel() in ("pair_grp", "pair_grp_atomic")
    nd = len(pb.dets)
    for i, c in enumerate(cs):
        err = rel_err(pb.from_device(out[i * nd:(i + 1) * nd]), pb.oracle_sigma(c))
        assert 0 < err <= 2e-6


@pytest.mark.parametrize("name,k", [("T4", 2), ("c1", 1)])
def test_mixed_precision_davidson_matches_exact(name, k):
    import paper_2505_20375_amd as stpci
    pb = Problem.named(name)
    w = np.linalg.eigvalsh(dense.hamiltonian(pb.dets, pb.h, pb.g, real=not pb.cplx))
    ctx = pb.context()
    e, r, it, st = ctx.davidson(k=k, tol=1e-8, precision=stpci.FP32)
    n64, n32 = ctx.dav_stats()
    assert n32 > 0
    assert np.max(np.abs(e - w[:k])) <= 1e-8


def test_mixed_precision_davidson_config2():
    """24 spinors, 8 electrons, 2 roots: the refined energies agree with the
    all-FP64 solve within 1e-8 Eh and most sigma products are FP32."""
    import paper_2505_20375_amd as stpci
    pb = Problem.named("c2")
    ctx = pb.context()
    e64, r64, it64, _ = ctx.davidson(k=2, tol=1e-6)
    n64_ref, _ = ctx.dav_stats()
    e32, r32, it32, _ = ctx.davidson(k=2, tol=1e-6, precision=stpci.FP32)
    n64, n32 = ctx.dav_stats()
    print("fp64 run: %d FP64 sigma vectors; mixed run: %d FP64 + %d FP32" % (n64_ref, n64, n32))
    assert np.max(np.abs(e32 - e64)) <= 1e-8
    assert np.all(r32 <= 1e-6)
    assert n32 > n64


@pytest.mark.parametrize("name", ["T4", "c1", "T8", "c2"])
def test_bf16_sigma_error_is_bfloat16_rounding(name):
    """The matrix-core form against the FP64 sigma: relative error of the
    order of bfloat16 rounding of integrals and coefficients (not zero: the
    reduced arithmetic really ran)."""
    import paper_2505_20375_amd as stpci
    pb = Problem.named(name)
    c = pb.vector()
    s64 = _sigma(pb, c, stpci.FP64)
    sbf = _sigma(pb, c, stpci.BF16)
    err = rel_err(sbf, s64)
    print("bf16 sigma relative error", name, err)
    assert 1e-6 < err <= 2e-2


def test_bf16_sigma_two_vectors_and_atomic_scatter():
    """Two vectors per pass (8 intermediates per product) and the device-atomic
    scatter give the same products as one vector with the stored scatter."""
    import torch
    import paper_2505_20375_amd as stpci
    pb = Problem.named("T4")
    c1, c2 = pb.vector(1), pb.vector(2)
    ref = []
    for kernel in ("pair", "pair_atomic"):
        ctx = pb.context()
        ctx.set_sigma_kernel(kernel)
        x = torch.cat([pb.to_device(c1), pb.to_device(c2)])
        out = torch.empty_like(x)
        ctx.sigma(x, out, n_vec=2, precision=stpci.BF16)
        one = torch.empty_like(x[:len(pb.dets)])
        ctx.sigma(x[:len(pb.dets)], one, n_vec=1, precision=stpci.BF16)
        torch.cuda.synchronize()
        n = len(pb.dets)
        ref.append((pb.from_device(out[:n]), pb.from_device(out[n:]), pb.from_device(one)))
    for a, b, o in ref:
        assert rel_err(a, o) <= 1e-6   # same bfloat16 products, FP32 sums in another order
        assert rel_err(b, pb.oracle_sigma(c2)) <= 2e-2
    assert rel_err(ref[0][0], ref[1][0]) <= 1e-6


@pytest.mark.parametrize("name,k", [("T4", 2), ("c1", 1)])
def test_bf16_davidson_matches_exact(name, k):
    import paper_2505_20375_amd as stpci
    pb = Problem.named(name)
    w = np.linalg.eigvalsh(dense.hamiltonian(pb.dets, pb.h, pb.g, real=not pb.cplx))
    ctx = pb.context()
    e, r, it, st = ctx.davidson(k=k, tol=1e-8, precision=stpci.BF16)
    assert ctx.dav_sigma_count(stpci.BF16) > 0
    assert np.max(np.abs(e - w[:k])) <= 1e-8
