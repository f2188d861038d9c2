"""Spaces of many distributed active spaces at scale (two-electron terms that
span four distinct subspaces, thousands of categories): FP64 sigma on
sampled rows against the oracle's list-free rows.

  * 32 spinors as eight subspaces of 4, windows [0..4], 12 electrons:
    225,792,840 determinants in 23,940 categories (pair table 3.9 MB: one
    intermediate per matrix-core product, device atomics);
  * 40 spinors as four subspaces of 10, windows [1..4], 10 electrons:
    619,245,000 determinants in 44 categories (pair table 9.7 MB: the
    spectator-batched matrix-core kernel).
"""
import numpy as np
import pytest

import synth
from oracle import csc
from tests import layout

pytestmark = pytest.mark.gpu

SPACES = {
    "8x4": (synth.SpaceSpec(12, [4] * 8, [0] * 8, [4] * 8), 32, 225792840, 23940),
    "4x10": (synth.SpaceSpec(10, [10] * 4, [1] * 4, [4] * 4), 40, 619245000, 44),
}


@pytest.mark.parametrize("name", ["8x4", "4x10"])
def test_many_subspace_sigma_sampled_rows(name):
    import torch
    import paper_2505_20375_amd as stpci
    sp, M, n_expect, ncat_expect = SPACES[name]
    free, _tot = torch.cuda.mem_get_info()
    if free < 2.5 * n_expect * 16:
        pytest.skip("needs %.0f GB of free device memory" % (2.5 * n_expect * 16 / 1e9))
    ints = synth.complex_integrals(M, 4400 + M, rank=16, sigma_f=0.05)
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    info = ctx.space_info()
    assert info.n_dets == n_expect and info.n_cat == ncat_expect
    n = info.n_dets
    gen = torch.Generator(device="cuda").manual_seed(4500 + M)
    c = torch.randn(n, dtype=torch.complex128, device="cuda", generator=gen)
    c /= torch.linalg.vector_norm(c)
    out = torch.empty_like(c)
    print("case", name, n, "determinants", flush=True)
    ctx.sigma(c, out)
    torch.cuda.synchronize()
    print("kernel", ctx.sigma_kernel(), flush=True)
    rng = np.random.default_rng(4600 + M)
    cats = rng.choice(info.n_cat, min(info.n_cat, 100), replace=False)
    rows = []
    for cat in cats:
        _, off, cnt = ctx.category(int(cat))
        rows += [off, off + cnt - 1, int(off + rng.integers(0, cnt))]
    rows += [int(x) for x in rng.choice(n, 60, replace=False)]
    rows = np.array(sorted(set(rows)), dtype=np.int64)
    bits = np.array([ctx.address_to_det(int(a)) for a in rows], dtype=np.uint64)
    assert np.array_equal(layout.address_array(bits, sp.n_elec, sp.sub, sp.lo, sp.hi), rows)
    cols, vals, owner = [], [], []
    for i, b in enumerate(bits):
        kb, v = csc.h_row_window(sp.sub, sp.lo, sp.hi, ints.h, ints.g, int(b))
        cols.append(kb)
        vals.append(v)
        owner.append(np.full(len(kb), i))
    cols = layout.address_array(np.concatenate(cols), sp.n_elec, sp.sub, sp.lo, sp.hi)
    assert np.all(cols >= 0)
    vals, owner = np.concatenate(vals), np.concatenate(owner)
    cvals = c[torch.from_numpy(cols).to("cuda")].cpu().numpy()
    refs = np.zeros(len(rows), dtype=np.complex128)
    np.add.at(refs, owner, vals * cvals)
    got = out[torch.from_numpy(rows).to("cuda")].cpu().numpy()
    err = np.max(np.abs(got - refs)) / np.max(np.abs(refs))
    print("rows %d, max error %.2e" % (len(rows), err), flush=True)
    assert err <= 1e-12
