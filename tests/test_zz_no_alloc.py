"""stpci_sigma_noalloc, the sigma entry point that allocates no device
memory (its store-and-reduce workspace is the library's static scratch
array), against stpci_sigma on the same inputs: two calls in a row, the
second with a smaller input, on every pair-kernel path that uses the
workspace, and the calls it must refuse.  Through the C ABI."""
import numpy as np
import pytest

import synth
from tests.gpu_util import Problem, rel_err

pytestmark = pytest.mark.gpu


def _both(pb, ctx, x, n_vec, prec):
    """(noalloc result, stpci_sigma result) on the device."""
    import torch
    a = torch.full_like(x, float("nan"))
    b = torch.full_like(x, float("nan"))
    ctx.sigma(x, b, n_vec=n_vec, precision=prec)      # builds the tables (and its own workspace)
    ctx.sigma_noalloc(x, a, n_vec=n_vec, precision=prec)
    torch.cuda.synchronize()
    return a, b


def _stack(pb, seeds):
    import torch
    return torch.cat([pb.to_device(pb.vector(s)) for s in seeds])


def _fci(m, n, seed):
    ints = synth.complex_integrals(m, seed, rank=8, sigma_f=0.05)
    return Problem(ints, synth.SpaceSpec(n, [m], [n], [n]), seed=seed)


@pytest.mark.parametrize("first,second,kernel", [
    ("fci22_7", "T8fci", "auto"),        # grouped matrix-core kernel: 170,544 then 70 determinants
    ("c1", "T4", "auto"),                # one intermediate per matrix-core product
    ("c1", "T4", "pair_valu"),           # vector-ALU pair kernel
])
def test_noalloc_matches_sigma_two_calls(first, second, kernel):
    """Each call equals stpci_sigma bit for bit (the same kernels, the
    store-and-reduce sums in a fixed order), the second call smaller than the
    first, so it runs over what the first left in the shared array; the
    small space is also checked against the oracle."""
    import paper_2505_20375_amd as stpci
    print("case", first, second, kernel, flush=True)
    assert stpci.sigma_noalloc_max_bytes() == 256 << 20
    for name, n_vec in ((first, 2), (second, 1)):
        pb = _fci(22, 7, 22) if name == "fci22_7" else Problem.named(name)
        ctx = pb.context()
        if kernel != "auto":
            ctx.set_sigma_kernel(kernel)
        x = _stack(pb, [pb.seed + v for v in range(n_vec)])
        a, b = _both(pb, ctx, x, n_vec, stpci.FP64)
        assert ctx.sigma_kernel() in ("pair_grp", "pair_mf64", "pair_valu")   # store-and-reduce paths
        assert not a.isnan().any()
        assert bool((a == b).all())
        if len(pb.dets) <= 5000:
            n = len(pb.dets)
            for v in range(n_vec):
                ref = pb.oracle_sigma(pb.vector(pb.seed + v))
                assert rel_err(pb.from_device(a[v * n:(v + 1) * n]), ref) <= 1e-12


def test_noalloc_same_context_smaller_second_call_and_fp32():
    """On one context: two vectors, then one; and the FP32 contraction once
    its FP32 tables exist (bitwise equal to stpci_sigma with FP32)."""
    import paper_2505_20375_amd as stpci
    pb = Problem.named("c1")
    ctx = pb.context()
    x2 = _stack(pb, [3, 4])
    a, b = _both(pb, ctx, x2, 2, stpci.FP64)
    assert bool((a == b).all())
    x1 = _stack(pb, [5])
    a, b = _both(pb, ctx, x1, 1, stpci.FP64)
    assert bool((a == b).all())
    a, b = _both(pb, ctx, x1, 1, stpci.FP32)
    assert bool((a == b).all())
    assert rel_err(pb.from_device(a), pb.oracle_sigma(pb.vector(5))) <= 2e-6


def test_noalloc_refuses_unbuilt_tables_and_oversized_workspace():
    """Without device tables (no earlier stpci_sigma / stpci_diagonal after
    the last set_space) it refuses instead of allocating; a space whose
    workspace exceeds the array is refused with the sizes named; FP32 before
    its tables exist is refused."""
    import torch
    import paper_2505_20375_amd as stpci
    pb = Problem.named("T4")
    ctx = pb.context()
    x = pb.to_device(pb.vector())
    y = torch.empty_like(x)
    with pytest.raises(stpci.StpciError, match="tables not built"):
        ctx.sigma_noalloc(x, y)
    d = torch.empty(len(pb.dets), dtype=torch.float64, device="cuda")
    ctx.diagonal(d)
    ctx.sigma_noalloc(x, y)           # the diagonal built the tables
    with pytest.raises(stpci.StpciError, match="FP32"):
        ctx.sigma_noalloc(x, y, precision=stpci.FP32)
    ctx.set_space(pb.sp.n_elec, pb.sp.sub, pb.sp.lo, pb.sp.hi)
    with pytest.raises(stpci.StpciError, match="tables not built"):
        ctx.sigma_noalloc(x, y)
    # 24 spinors, 8 electrons, one subspace: 735,471 x 28 x 2 x 16 bytes = 659 MB
    big = Problem.named("c2")
    cb = big.context()
    xb = big.to_device(big.vector())
    yb = torch.empty_like(xb)
    cb.sigma(xb, yb)
    torch.cuda.synchronize()
    assert cb.sigma_kernel() == "pair_grp"
    with pytest.raises(stpci.StpciError, match="exceeds the no-allocation scratch"):
        cb.sigma_noalloc(xb, yb)
