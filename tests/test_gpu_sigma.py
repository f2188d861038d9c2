"""GPU sigma parity: libstpci (HIP, through the C ABI) against the CPU oracle.

Bar: ||sigma_gpu - sigma_oracle|| <= 1e-12 ||sigma_oracle|| on the same seeded
vector, element by element after mapping both to the oracle's order.
"""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_util import Problem, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _run_sigma(pb, c_or, n_vec=1, kernel=None):
    import torch
    ctx = pb.context()
    if kernel:
        ctx.set_sigma_kernel(kernel)
    x = pb.to_device(c_or) if n_vec == 1 else torch.cat([pb.to_device(v) for v in c_or])
    out = torch.empty_like(x)
    ctx.sigma(x, out, n_vec=n_vec)
    torch.cuda.synchronize()
    if n_vec == 1:
        return pb.from_device(out)
    n = len(pb.dets)
    return [pb.from_device(out[i * n:(i + 1) * n]) for i in range(n_vec)]


@pytest.mark.parametrize("name", ["T2", "T3", "T4", "T8", "T8fci", "c1"])
def test_sigma_small_spaces(name):
    print("case", name, flush=True)
    pb = Problem.named(name)
    c = pb.vector()
    s_ref = pb.oracle_sigma(c)
    s_gpu = _run_sigma(pb, c)
    assert rel_err(s_gpu, s_ref) <= TOL


@pytest.mark.parametrize("sub,lo,hi,n", [
    ([16], None, None, 5),                     # one subspace, several thousand determinants
    ([8, 8], None, None, 5),                   # the same space as two open-window subspaces
    ([6, 5, 5], [1, 1, 1], [3, 3, 2], 5),      # windows: outside-window intermediates
    ([4, 4, 4, 4], [0, 1, 0, 1], [2, 2, 2, 2], 5),
    ([2] * 8, None, None, 6),                  # eight subspaces (the library's maximum), open windows
    ([2] * 8, [0, 1, 0, 1, 0, 1, 0, 1], [1, 2, 1, 2, 1, 2, 1, 2], 6),   # eight subspaces, windows
])
def test_sigma_medium_spaces(sub, lo, hi, n):
    print("case", sub, lo, hi, n, flush=True)
    ints = synth.complex_integrals(sum(sub), 77, rank=16, sigma_f=0.05)
    pb = Problem(ints, synth.SpaceSpec(n, sub, lo or [], hi or []), seed=7)
    c = pb.vector()
    assert rel_err(_run_sigma(pb, c), pb.oracle_sigma(c)) <= TOL


@pytest.mark.parametrize("n,sub,lo,hi", [
    (1, [8], None, None),                    # one electron: no pair intermediates
    (2, [8], None, None),                    # one pair intermediate per pair class (the empty determinant)
    (7, [8], None, None),                    # one hole
    (8, [8], None, None),                    # a single determinant (N = M)
    (1, [4, 4], [0, 0], [1, 1]),             # one electron in two subspaces
    (2, [4, 4], [1, 0], [2, 1]),             # windows leave one category pattern per subspace
    (7, [4, 4], [3, 3], [4, 4]),
])
def test_sigma_edge_electron_counts(n, sub, lo, hi):
    """Degenerate spaces at the ends of the electron count, with the default
    kernel choice (the pair form where it applies, N >= 2)."""
    print("case", n, sub, lo, hi, flush=True)
    ints = synth.complex_integrals(sum(sub), 41 + n, rank=8, sigma_f=0.05)
    pb = Problem(ints, synth.SpaceSpec(n, sub, lo or [], hi or []), seed=3)
    c = pb.vector()
    assert rel_err(_run_sigma(pb, c), pb.oracle_sigma(c)) <= TOL


def test_sigma_three_vectors():
    """An odd vector count above the kernel's two-vector width."""
    pb = Problem.named("T4")
    cs = [pb.vector(s) for s in (1, 2, 3)]
    out = _run_sigma(pb, cs, n_vec=3)
    for c, s in zip(cs, out):
        assert rel_err(s, pb.oracle_sigma(c)) <= TOL


def test_sigma_partition_invariance():
    """FCI as 1, 2 or 3 open-window subspaces gives the same sigma."""
    ints = synth.complex_integrals(12, 5)
    outs = []
    for sub in ([12], [6, 6], [4, 4, 4]):
        pb = Problem(ints, synth.SpaceSpec(4, sub), seed=3)
        outs.append(_run_sigma(pb, pb.vector()))
    assert rel_err(outs[1], outs[0]) <= TOL and rel_err(outs[2], outs[0]) <= TOL


def test_sigma_two_vectors():
    pb = Problem.named("T4")
    c1, c2 = pb.vector(1), pb.vector(2)
    s = _run_sigma(pb, [c1, c2], n_vec=2)
    assert rel_err(s[0], pb.oracle_sigma(c1)) <= TOL
    assert rel_err(s[1], pb.oracle_sigma(c2)) <= TOL


def test_sigma_real_spin_free():
    pb = Problem.named("c1")
    assert not pb.cplx
    c = pb.vector(11)
    assert rel_err(_run_sigma(pb, c), pb.oracle_sigma(c)) <= TOL


def test_compression_preservation():
    """A vector confined to one category yields sigma that vanishes exactly on
    every category more than two electron moves away (Methods: the categorical
    sigma build preserves categorical compression)."""
    ints = synth.complex_integrals(12, 9)
    sp = synth.SpaceSpec(6, [4, 4, 4])
    pb = Problem(ints, sp, seed=5)
    from tests import layout
    lib_dets = layout.layout_dets(6, [4, 4, 4])
    occ = np.array([[bin(int(b) >> (4 * k) & 0xF).count("1") for k in range(3)] for b in pb.dets])
    src = (4, 2, 0)
    c = pb.vector() * np.all(occ == src, axis=1)
    s = _run_sigma(pb, c)
    dist = np.abs(occ - np.array(src)).sum(axis=1) // 2
    assert np.all(s[dist > 2] == 0)
    assert np.any(s[dist <= 2] != 0)
    assert rel_err(s, pb.oracle_sigma(c)) <= TOL


def test_sigma_config2_full_partitions():
    """24 spinors, 8 electrons (735,471 determinants): the full sigma of the
    default kernel of each partition (one subspace: the grouped kernel; 12|12
    and 8|8|8 with open windows: the same space in other layouts) against the
    full oracle sigma, element by element."""
    import torch
    print("case c2 full, oracle sigma", flush=True)
    base = Problem.named("c2")
    c = base.vector()
    ref = base.oracle_sigma(c)
    for sub in ([24], [12, 12], [8, 8, 8]):
        pb = Problem(base.ints, synth.SpaceSpec(8, sub), seed=base.seed)
        ctx = pb.context()
        x = pb.to_device(c)
        out = torch.empty_like(x)
        ctx.sigma(x, out)
        torch.cuda.synchronize()
        err = rel_err(pb.from_device(out), ref)
        print("partition", sub, ctx.sigma_kernel(), "rel err %.2e" % err, flush=True)
        assert err <= TOL


@pytest.mark.parametrize("kernel", ["pair", "pair_atomic", "pair_mf64", "pair_valu", "tile", "rowtile"])
@pytest.mark.parametrize("name", ["T4", "c1"])
def test_every_kernel_matches_oracle(kernel, name):
    """Each sigma kernel (pair intermediates, one-move Hermitian tiles and the
    row-tiled one-move fallback) reproduces the oracle."""
    print("case", kernel, name, flush=True)
    pb = Problem.named(name)
    c = pb.vector()
    assert rel_err(_run_sigma(pb, c, kernel=kernel), pb.oracle_sigma(c)) <= TOL


@pytest.mark.parametrize("n,M,cplx,n_vec", [
    (3, 3, True, 1),      # one core (no electrons), three intermediates: a single partial item
    (3, 8, True, 2),      # one core, eight intermediates: two full items
    (4, 12, True, 3),     # three vectors: a two-vector launch and a one-vector launch
    (5, 16, False, 2),    # real integrals
    (6, 10, False, 1),
    (7, 8, True, 2),      # one hole: a single pair per intermediate
    (10, 14, True, 1),
    (4, 22, True, 2),     # 210 core pairs: the slice of eight would exceed 54 KB, four per item
    (4, 22, False, 3),
])
def test_grouped_pair_kernel(n, M, cplx, n_vec):
    """Spaces of one subspace: the grouped matrix-core kernel (eight, or
    four, intermediates sharing an (N-3)-electron core per table read)
    against the oracle, real and complex, one to three vectors."""
    import torch
    print("case", n, M, cplx, n_vec, flush=True)
    ints = (synth.complex_integrals if cplx else synth.real_integrals)(M, 50 + n, rank=8, sigma_f=0.05)
    pb = Problem(ints, synth.SpaceSpec(n, [M]), seed=3)
    cs = [pb.vector(s) for s in range(1, n_vec + 1)]
    ctx = pb.context()
    ctx.set_sigma_kernel("pair_grp")
    x = torch.cat([pb.to_device(v) for v in cs])
    out = torch.empty_like(x)
    ctx.sigma(x, out, n_vec=n_vec)
    torch.cuda.synchronize()
    assert ctx.sigma_kernel() == "pair_grp"
    nd = len(pb.dets)
    for i, c in enumerate(cs):
        assert rel_err(pb.from_device(out[i * nd:(i + 1) * nd]), pb.oracle_sigma(c)) <= TOL


@pytest.mark.parametrize("sub,lo,hi,n,n_vec,cplx", [
    ([4, 4, 4], [1, 1, 1], [2, 3, 2], 5, 1, True),      # T4-like: windows, outside-window intermediates
    ([4, 6], [1, 1], [3, 3], 4, 2, True),
    ([6, 5, 5], [1, 1, 1], [3, 3, 2], 5, 3, True),      # three vectors: a two-vector and a one-vector launch
    ([4, 4, 4, 4], [0, 1, 0, 1], [2, 2, 2, 2], 5, 2, True),
    ([2] * 8, None, None, 6, 1, True),                  # eight subspaces, open windows
    ([2] * 8, [0, 1, 0, 1, 0, 1, 0, 1], [1, 2, 1, 2, 1, 2, 1, 2], 6, 2, True),
    ([5, 9], None, None, 4, 1, True),                   # open windows: FCI as two subspaces
    ([3, 12], [0, 1], [3, 12], 6, 2, True),             # a last subspace of 12: groups of up to 462 members
    ([8, 6], [2, 1], [6, 4], 6, 2, False),              # real integrals
    ([6, 6], [0, 0], [6, 6], 3, 1, False),
    ([4, 4], [1, 0], [2, 1], 2, 2, True),               # two electrons
    ([4, 4], [3, 3], [4, 4], 7, 1, True),               # one hole
    ([4, 4], [4, 4], [4, 4], 8, 1, True),               # a single determinant
])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spectator_batched_kernel(sub, lo, hi, n, n_vec, cplx, prec):
    """Spaces of several subspaces: the spectator-batched matrix-core kernel
    (the pair intermediates of a category that share the strings of the
    leading subspaces contracted as one product over their padded pair list,
    contributions added with device atomics) against the oracle, real and
    complex, one to three vectors, degenerate electron counts; FP64 (parity
    bar) and its FP32 instance (FP32 table and tiles on the FP32 matrix
    cores, FP64 sums: single-precision bar)."""
    import torch
    import paper_2505_20375_amd as stpci
    print("case", sub, lo, hi, n, n_vec, cplx, prec, flush=True)
    M = sum(sub)
    ints = (synth.complex_integrals if cplx else synth.real_integrals)(M, 60 + n + M, rank=8, sigma_f=0.05)
    pb = Problem(ints, synth.SpaceSpec(n, sub, lo or [], hi or []), seed=3)
    cs = [pb.vector(s) for s in range(1, n_vec + 1)]
    ctx = pb.context()
    ctx.set_sigma_kernel("pair_sb")
    x = torch.cat([pb.to_device(v) for v in cs])
    out = torch.empty_like(x)
    ctx.sigma(x, out, n_vec=n_vec, precision=stpci.FP32 if prec == "fp32" else stpci.FP64)
    torch.cuda.synchronize()
    if n >= 2:
        assert ctx.sigma_kernel() == "pair_sb"
    nd = len(pb.dets)
    for i, c in enumerate(cs):
        assert rel_err(pb.from_device(out[i * nd:(i + 1) * nd]), pb.oracle_sigma(c)) <= (TOL if prec == "fp64"
                                                                                          else 2e-6)


def test_spectator_batched_kernel_core_energy_and_sparse():
    """The spectator-batched kernel with e_core != 0, and a vector confined to
    one category after a dense one (chunks whose gathered coefficients are all
    zero skip their products)."""
    import torch
    from oracle import csc
    ints = synth.complex_integrals(12, 9)
    ints.e_core = -1.75
    sp = synth.SpaceSpec(6, [4, 4, 4])
    pb = Problem(ints, sp, seed=5)
    occ = np.array([[bin(int(b) >> (4 * k) & 0xF).count("1") for k in range(3)] for b in pb.dets])
    sparse = pb.vector(8) * np.all(occ == (4, 2, 0), axis=1)
    dense = pb.vector(7)
    ctx = pb.context()
    ctx.set_sigma_kernel("pair_sb")
    xd, xs = pb.to_device(dense), pb.to_device(sparse)
    out = torch.empty_like(xd)
    ctx.sigma(xd, out)
    torch.cuda.synchronize()
    assert rel_err(pb.from_device(out), csc.sigma(pb.dets, pb.h, pb.g, dense, e_core=ints.e_core)) <= TOL
    ctx.sigma(xs, out)
    torch.cuda.synchronize()
    assert rel_err(pb.from_device(out), csc.sigma(pb.dets, pb.h, pb.g, sparse, e_core=ints.e_core)) <= TOL


def test_grouped_pair_kernel_atomic_and_sparse():
    """The grouped kernel with device atomics, and in store mode a vector
    confined to a few determinants after a dense one (items whose four
    intermediates see only zeros skip the products but must still overwrite
    their entries of the contribution workspace)."""
    import torch
    ints = synth.complex_integrals(12, 21, rank=8, sigma_f=0.05)
    pb = Problem(ints, synth.SpaceSpec(5, [12]), seed=3)
    dense = pb.vector(4)
    sparse = dense * (np.arange(len(dense)) % 97 == 0)
    ref_d, ref_s = pb.oracle_sigma(dense), pb.oracle_sigma(sparse)
    ctx = pb.context()
    ctx.set_sigma_kernel("pair_grp")
    xd, xs = pb.to_device(dense), pb.to_device(sparse)
    out = torch.empty_like(xd)
    ctx.sigma(xd, out)
    ctx.sigma(xs, out)
    torch.cuda.synchronize()
    assert ctx.sigma_kernel() == "pair_grp"
    assert rel_err(pb.from_device(out), ref_s) <= TOL
    ctx2 = pb.context()
    ctx2.set_sigma_kernel("pair_atomic")
    ctx2.sigma(xd, out)
    torch.cuda.synchronize()
    assert ctx2.sigma_kernel() == "pair_grp_atomic"
    assert rel_err(pb.from_device(out), ref_d) <= TOL


def test_grouped_pair_kernel_refuses_other_spaces():
    """Requesting the grouped kernel on a space of several subspaces is an error."""
    import torch
    pb = Problem.named("T4")
    ctx = pb.context()
    ctx.set_sigma_kernel("pair_grp")
    x = pb.to_device(pb.vector())
    with pytest.raises(Exception):
        ctx.sigma(x, torch.empty_like(x))


def test_default_kernel_is_pair():
    """The pair form is the default; with a pair table of at most 4 MB its FP64
    products run on the matrix cores; spaces of one subspace take the grouped
    matrix-core kernel; a larger table over several subspaces takes the
    spectator-batched matrix-core kernel (the vector-ALU kernel when that
    kernel's limits are exceeded)."""
    import torch
    pb = Problem.named("T4")
    ctx = pb.context()
    x = pb.to_device(pb.vector())
    ctx.sigma(x, torch.empty_like(x))
    torch.cuda.synchronize()
    assert ctx.sigma_kernel() == "pair_mf64"
    one = Problem.named("T8fci").context()      # one subspace: grouped intermediates
    y1 = torch.zeros(one.space_info().n_dets, dtype=torch.complex128, device="cuda")
    one.sigma(y1, torch.empty_like(y1))
    torch.cuda.synchronize()
    assert one.sigma_kernel() == "pair_grp"
    import paper_2505_20375_amd as stpci
    big = stpci.Context(0)            # 40 spinors: 780 pairs, a 9.7 MB complex table
    ints = synth.complex_integrals(40, 3, rank=4, sigma_f=0.05)
    big.set_integrals(ints.h, ints.g)
    big.set_space(4, [20, 20])
    n = big.space_info().n_dets
    y = torch.zeros(n, dtype=torch.complex128, device="cuda")
    big.sigma(y, torch.empty_like(y))
    torch.cuda.synchronize()
    assert big.sigma_kernel() == "pair_sb"


@pytest.mark.parametrize("kernel", ["pair", "pair_atomic", "pair_mf64", "pair_valu", "tile", "rowtile"])
def test_core_energy_term(kernel):
    """sigma includes e_core * c."""
    import torch
    from oracle import csc
    ints = synth.complex_integrals(10, 31)
    ints.e_core = -3.25
    pb = Problem(ints, synth.SpaceSpec(4, [4, 6], [1, 1], [3, 3]), seed=5)
    c = pb.vector()
    ref = csc.sigma(pb.dets, pb.h, pb.g, c, e_core=ints.e_core)
    assert rel_err(_run_sigma(pb, c, kernel=kernel), ref) <= TOL


def test_pair_store_mode_is_deterministic():
    """The store-and-reduce scatter sums every target's contributions in a
    fixed order: repeated sigma builds are bitwise equal."""
    import torch
    pb = Problem.named("T4")
    ctx = pb.context()
    x = pb.to_device(pb.vector())
    a, b = torch.empty_like(x), torch.empty_like(x)
    ctx.sigma(x, a)
    ctx.sigma(x, b)
    torch.cuda.synchronize()
    assert ctx.sigma_kernel() in ("pair_mf64", "pair_valu")
    assert torch.equal(a, b)
    ctx.set_sigma_kernel("pair_valu")
    ctx.sigma(x, a)
    ctx.sigma(x, b)
    torch.cuda.synchronize()
    assert ctx.sigma_kernel() == "pair_valu"
    assert torch.equal(a, b)


@pytest.mark.parametrize("kernel,prec", [("pair", "fp64"), ("pair_atomic", "fp64"), ("pair_valu", "fp64"), ("pair", "fp32"),
                                         ("pair", "bf16"), ("pair_atomic", "bf16")])
def test_sparse_vector_after_dense(kernel, prec):
    """Intermediates (BF16: batches of them) whose gathered coefficients are
    all zero skip the contraction; in store mode they must still overwrite
    their entries of the contribution workspace.  A dense sigma first fills
    the workspace, then a vector confined to one category (so that most
    intermediates see only zeros) must give the oracle's sigma."""
    import torch
    import paper_2505_20375_amd as stpci
    code = {"fp64": stpci.FP64, "fp32": stpci.FP32, "bf16": stpci.BF16}[prec]
    tol = {"fp64": TOL, "fp32": 2e-6, "bf16": 2e-2}[prec]
    ints = synth.complex_integrals(12, 9)
    sp = synth.SpaceSpec(6, [4, 4, 4])
    pb = Problem(ints, sp, seed=5)
    occ = np.array([[bin(int(b) >> (4 * k) & 0xF).count("1") for k in range(3)] for b in pb.dets])
    sparse = pb.vector(8) * np.all(occ == (4, 2, 0), axis=1)
    ctx = pb.context()
    ctx.set_sigma_kernel(kernel)
    xd, xs = pb.to_device(pb.vector(7)), pb.to_device(sparse)
    out = torch.empty_like(xd)
    ctx.sigma(xd, out, precision=code)
    ctx.sigma(xs, out, precision=code)
    torch.cuda.synchronize()
    assert rel_err(pb.from_device(out), pb.oracle_sigma(sparse)) <= tol


def test_sigma_config3p_sampled_rows():
    """Full-size STP-DAS space (40 spinors, 12|16|12, windows [2..6]|[4..10]|[2..6],
    11 electrons: 1,365,867,360 determinants in 10 categories, 21.9 GB per
    vector): one FP64, one FP32 and one BF16 sigma build on a seeded vector
    in the library layout, checked on 1000+ rows -- the first, middle and last
    determinant of every category and random rows of every category --
    against the oracle's list-free Slater-Condon rows, every column address
    taken from the documented layout (test module), not from the library."""
    import time
    import torch
    from oracle import csc
    from tests import layout
    ints, sp, _ = synth.config("c3p")
    free, _tot = torch.cuda.mem_get_info()
    n_expect = sp.n_dets()
    if free < 2.2 * n_expect * 16:
        pytest.skip("needs %.0f GB of free device memory" % (2.2 * n_expect * 16 / 1e9))
    import paper_2505_20375_amd as stpci
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    info = ctx.space_info()
    n = info.n_dets
    assert n == n_expect == 1365867360 and info.n_cat == 10
    gen = torch.Generator(device="cuda").manual_seed(3103)
    c = torch.randn(n, dtype=torch.complex128, device="cuda", generator=gen)
    c /= torch.linalg.vector_norm(c)
    out = torch.empty_like(c)
    rng = np.random.default_rng(3203)
    rows = []
    for cat in range(info.n_cat):
        _, off, cnt = ctx.category(cat)
        rows += [off, off + cnt // 2, off + cnt - 1]
        rows += [int(x) for x in off + rng.choice(cnt, 97, replace=False)]
    rows = np.array(sorted(set(rows)), dtype=np.int64)
    assert len(rows) >= 1000
    t0 = time.time()
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
    print("oracle rows: %d rows, %d couplings, %.1f s" % (len(rows), len(cols), time.time() - t0), flush=True)
    errs = {}
    # the FP64 build (parity bar 1e-12), then the FP32 (single-precision bar
    # 2e-6) and BF16 (bfloat16 rounding bar 2e-2) builds of the same vector
    bars = {"fp64": TOL, "fp32": 2e-6, "bf16": 2e-2}
    for prec, name in ((stpci.FP64, "fp64"), (stpci.FP32, "fp32"), (stpci.BF16, "bf16")):
        print("config 3' sigma (%s): %d determinants, kernel starting" % (name, n), flush=True)
        t0 = time.time()
        ctx.sigma(c, out, precision=prec)
        torch.cuda.synchronize()
        print("config 3' sigma (%s) done in %.1f s (kernel %s)" % (name, time.time() - t0, ctx.sigma_kernel()),
              flush=True)
        got = out[torch.from_numpy(rows).to("cuda")].cpu().numpy()
        errs[name] = np.linalg.norm(got - refs) / np.linalg.norm(refs)
        # every category on its own
        for cat in range(info.n_cat):
            _, off, cnt = ctx.category(cat)
            sel = (rows >= off) & (rows < off + cnt)
            e_cat = np.linalg.norm(got[sel] - refs[sel]) / np.linalg.norm(refs[sel])
            assert e_cat <= bars[name], (name, cat, e_cat)
        print("config 3' sampled-row relative error (%s): %.3g" % (name, errs[name]), flush=True)
    assert ctx.sigma_kernel() == "pair_sb"
    del c, out
    torch.cuda.empty_cache()
    for name, bar in bars.items():
        assert errs[name] <= bar, (name, errs[name])
    assert errs["fp32"] > 0
