"""GPU tests of the step-wise Davidson calls (stpci_footprint_bytes,
stpci_dav_begin, stpci_dav_sigma_batched, stpci_dav_finish_step,
stpci_dav_result): a caller-driven loop over a mix of problems, each
problem's products launched in one batched call with the others, gives the
energies of stpci_davidson alone and of exact diagonalisation; the calls
refuse the wrong order."""
import numpy as np
import pytest

from tests.gpu_util import Problem
from tests.test_gpu_serving import exact, mix

pytestmark = pytest.mark.gpu


def test_caller_driven_batch_equals_solo_and_exact():
    import paper_2505_20375_amd as stpci
    cases = mix() + [(Problem.named("T8fci"), 2, 0)]     # one subspace: its own path
    ctxs, refs, solos = [], [], []
    for i, (pb, k, prec) in enumerate(cases):
        print("case", i, flush=True)
        refs.append(exact(pb, k))
        solo = pb.context()
        e, r, _, _ = solo.davidson(k=k, tol=1e-9, max_iter=300, precision=prec)
        solos.append(e)
        ctx = pb.context()
        fp = ctx.footprint_bytes(k=k, tol=1e-9, max_iter=300, precision=prec)
        assert fp > 0
        assert ctx.footprint_bytes(k=k, tol=1e-9, max_iter=300, precision=prec, max_subspace=48) >= fp
        ctx.dav_begin(k=k, tol=1e-9, max_iter=300, precision=prec, certify=True)
        ctxs.append(ctx)
    active = list(range(len(ctxs)))
    done_at = {}
    step = 0
    while active:
        stpci.dav_sigma_batched([ctxs[i] for i in active])
        still = []
        for i in active:
            if ctxs[i].dav_finish_step():
                done_at[i] = step
            else:
                still.append(i)
        active = still
        step += 1
        assert step < 2000
    for i, (pb, k, prec) in enumerate(cases):
        e, r, it, st = ctxs[i].dav_result()
        assert st == stpci.OK
        assert np.max(r) <= 1e-9
        assert np.max(np.abs(e - refs[i])) <= 1e-9
        assert np.max(np.abs(e - solos[i])) <= 1e-9
        gam, bnd = ctxs[i].certificate()     # certify = 1: every requested root has a bound
        fin = np.isfinite(bnd)               # (infinite where a neighbour is degenerate)
        assert not np.isnan(bnd).any()
        assert np.all(np.abs(e - refs[i])[fin] <= bnd[fin] + 1e-12)


def test_stepwise_call_order_is_checked():
    import torch
    import paper_2505_20375_amd as stpci
    pb = Problem.named("T4")
    ctx = pb.context()
    with pytest.raises(stpci.StpciError):
        ctx.dav_finish_step()                    # no run in progress
    with pytest.raises(stpci.StpciError):
        ctx.dav_result()                         # nothing finished
    ctx.dav_begin(k=2, tol=1e-9, max_iter=300)
    with pytest.raises(stpci.StpciError, match="not computed"):
        ctx.dav_finish_step()                    # products still pending
    with pytest.raises(stpci.StpciError):
        ctx.dav_result()
    with pytest.raises(stpci.StpciError, match="twice"):
        stpci.dav_sigma_batched([ctx, ctx])
    while True:
        stpci.dav_sigma_batched([ctx])
        if ctx.dav_finish_step():
            break
    e, r, it, st = ctx.dav_result()
    assert np.max(np.abs(e - exact(pb, 2))) <= 1e-9
    # a second batched call with nothing pending is a no-op, and the options are validated
    stpci.dav_sigma_batched([ctx])
    with pytest.raises(stpci.StpciError):
        ctx.dav_begin(k=1, tol=1e-9, eps_drop=2.0)
    assert ctx.footprint_bytes(k=0) == -1
    torch.cuda.synchronize()
