"""GPU tests of the categorical compression (Results, categorical
compression; Methods, Alg. sigmaBuild): compression and expansion of dense
vectors with and without the eps drop, the exponential search on the
device, and sigma of compressed vectors against the oracle on small spaces
(sparse vectors, empty categories, the empty vector, e_core) and on sampled
rows of the 24-spinor and the 1.37e9-determinant spaces."""
import numpy as np
import pytest

import synth
from oracle import csc as ocsc
from tests.gpu_util import Problem, rel_err

pytestmark = pytest.mark.gpu


def _sparse(pb, density, seed, zero_cats=()):
    """Seeded vector in oracle order with about `density` nonzeros, and the
    categories listed set to zero (in library order)."""
    rng = np.random.default_rng(seed)
    x = pb.vector(seed)
    x[rng.random(len(x)) >= density] = 0
    if zero_cats:
        lib = pb.perm.to_lib(x)
        ctx = pb.context()
        for cat in zero_cats:
            _, off, cnt = ctx.category(cat)
            lib[off:off + cnt] = 0
        x = pb.perm.to_oracle(lib)
    return x


@pytest.mark.parametrize("name", ["T3", "T4", "T8", "c1"])
def test_compress_expand_roundtrip(name):
    """thresh = 0 keeps every nonzero: expanding gives the vector back; per
    category the addresses ascend and lie inside the block; thresh > 0
    keeps exactly the entries with |x_i| >= thresh."""
    import torch
    pb = Problem.named(name)
    ctx = pb.context()
    info = ctx.space_info()
    for density, thr in ((0.3, 0.0), (1.0, 0.0), (0.6, 0.02), (0.0, 0.0)):
        x = _sparse(pb, density, 7, zero_cats=(0,) if info.n_cat > 1 else ())
        xd = pb.to_device(x)
        cat_ptr, a, v = ctx.csc_compress(xd, thr)
        cp = cat_ptr.cpu().numpy()
        an = a.cpu().numpy().view(np.uint32)
        xl = pb.perm.to_lib(x)
        keep = (xl != 0) & (np.abs(xl) >= thr)
        assert cp[0] == 0 and cp[-1] == np.count_nonzero(keep) == len(an)
        for cat in range(info.n_cat):
            _, off, cnt = ctx.category(cat)
            seg = an[cp[cat]:cp[cat + 1]].astype(np.int64)
            assert np.all(np.diff(seg) > 0) and (len(seg) == 0 or (seg[0] >= 0 and seg[-1] < cnt))
            assert np.array_equal(seg, np.nonzero(keep[off:off + cnt])[0])
        out = torch.full_like(xd, 7.0)
        ctx.csc_expand(cat_ptr, a, v, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), np.where(keep, xl, 0))


def test_exponential_search_on_device():
    """The device search equals numpy.searchsorted from every start."""
    import torch
    import paper_2505_20375_amd as stpci
    rng = np.random.default_rng(3)
    for n in (1, 5, 300, 70001):
        a = np.sort(rng.integers(0, 3 * n, n).astype(np.uint32))
        m = 4096
        starts = rng.integers(0, n + 1, m)
        xs = rng.integers(0, 3 * n + 2, m).astype(np.uint32)
        ref = np.array([s + np.searchsorted(a[s:], x, "left") for s, x in zip(starts, xs)])
        ad = torch.from_numpy(a.view(np.int32)).cuda()
        sd = torch.from_numpy(starts.astype(np.int64)).cuda()
        xd = torch.from_numpy(xs.view(np.int32)).cuda()
        out = torch.empty(m, dtype=torch.int64, device="cuda")
        stpci.test_exp_search_dev(ad, sd, xd, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("name", ["T3", "T4", "T8", "T8fci", "c1"])
@pytest.mark.parametrize("density", [0.002, 0.05, 0.5, 1.0])
def test_sigma_of_compressed_vector_matches_oracle(name, density):
    """sigma of the compressed vector equals the oracle's sigma of the same
    (sparse) vector, relative 1e-12, with one category emptied."""
    import torch
    print("case", name, density, flush=True)
    pb = Problem.named(name)
    ctx = pb.context()
    info = ctx.space_info()
    x = _sparse(pb, density, 11, zero_cats=(info.n_cat - 1,) if info.n_cat > 1 else ())
    if not np.any(x):
        x[0] = 1.0
    cat_ptr, a, v = ctx.csc_compress(pb.to_device(x))
    out = torch.empty(len(pb.dets), dtype=torch.complex128 if pb.cplx else torch.float64, device="cuda")
    ctx.sigma_csc(cat_ptr, a, v, out)
    torch.cuda.synchronize()
    ref = pb.oracle_sigma(x)
    assert rel_err(pb.from_device(out), ref) <= 1e-12


def test_sigma_of_compressed_vector_edge_cases():
    """The empty vector gives sigma = 0 (sigma overwritten, not added to);
    e_core != 0 adds e_core c; a space of several subspaces and windows."""
    import torch
    ints = synth.complex_integrals(14, 33, rank=24, sigma_f=0.04)
    ints.e_core = -1.75
    pb = Problem(ints, synth.SpaceSpec(6, [4, 6, 4], [1, 2, 1], [2, 4, 2]), seed=2)
    ctx = pb.context()
    out = torch.full((len(pb.dets),), 3.0, dtype=torch.complex128, device="cuda")
    zero = pb.to_device(np.zeros(len(pb.dets), dtype=np.complex128))
    cat_ptr, a, v = ctx.csc_compress(zero)
    assert int(cat_ptr[-1]) == 0
    ctx.sigma_csc(cat_ptr, a, v, out)
    torch.cuda.synchronize()
    assert not torch.any(out != 0)
    x = _sparse(pb, 0.1, 5)
    cat_ptr, a, v = ctx.csc_compress(pb.to_device(x))
    ctx.sigma_csc(cat_ptr, a, v, out)
    torch.cuda.synchronize()
    ref = ocsc.sigma(pb.dets, pb.h, pb.g, x, e_core=ints.e_core)
    assert rel_err(pb.from_device(out), ref) <= 1e-12


def test_sigma_of_compressed_vector_config2_and_dense_agree():
    """24 spinors, 8 electrons (735,471 determinants), 0.1 % and 5 % of the
    coefficients nonzero: sigma of the compressed vector equals the dense
    sigma of the same vector (relative 1e-12) and the oracle on 300 rows."""
    import torch
    pb = Problem.named("c2")
    ctx = pb.context()
    rng = np.random.default_rng(9)
    rows = np.sort(rng.choice(len(pb.dets), 300, replace=False))
    for density in (1e-3, 5e-2):
        x = _sparse(pb, density, 13)
        xd = pb.to_device(x)
        cat_ptr, a, v = ctx.csc_compress(xd)
        out = torch.empty_like(xd)
        ctx.sigma_csc(cat_ptr, a, v, out)
        dense = torch.empty_like(xd)
        ctx.sigma(xd, dense)
        torch.cuda.synchronize()
        assert float(torch.linalg.vector_norm(out - dense) / torch.linalg.vector_norm(dense)) <= 1e-12
        got = pb.from_device(out)[rows]
        ref = pb.oracle_sigma(x, rows=rows)
        assert rel_err(got, ref) <= 1e-12


def test_sigma_of_compressed_vector_config3p_sampled_rows():
    """1.37e9-determinant space, 20,000 nonzero coefficients spread over the
    categories: sigma of the compressed vector checked on 300 rows reached
    from the nonzeros and 100 random rows against the oracle's list-free rows
    (only the nonzero columns contribute)."""
    import torch
    from tests import layout
    import paper_2505_20375_amd as stpci
    ints, sp, _ = synth.config("c3p")
    free, _tot = torch.cuda.mem_get_info()
    n_expect = sp.n_dets()
    if free < 2.5 * n_expect * 16:
        pytest.skip("needs %.0f GB of free device memory" % (2.5 * n_expect * 16 / 1e9))
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    n = ctx.space_info().n_dets
    rng = np.random.default_rng(21)
    nz = np.unique(rng.choice(n, 20000, replace=False))
    vals = rng.standard_normal(len(nz)) + 1j * rng.standard_normal(len(nz))
    x = torch.zeros(n, dtype=torch.complex128, device="cuda")
    x[torch.from_numpy(nz).cuda()] = torch.from_numpy(vals).cuda()
    cat_ptr, a, v = ctx.csc_compress(x)
    assert int(cat_ptr[-1]) == len(nz)
    out = torch.empty_like(x)
    ctx.sigma_csc(cat_ptr, a, v, out)
    torch.cuda.synchronize()
    del x
    # rows: 150 of the nonzeros' own rows, up to 150 other rows with a nonzero
    # sigma (found among 3e7 random positions) and 100 random rows
    probe = torch.from_numpy(np.unique(rng.integers(0, n, 30000000))).cuda()
    hit = probe[out[probe] != 0].cpu().numpy()
    del probe
    rows = np.unique(np.concatenate([rng.choice(nz, 150, replace=False), hit[:150],
                                     rng.choice(n, 100, replace=False)]))
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    cmap = dict(zip(nz.tolist(), vals.tolist()))
    refs = np.zeros(len(rows), dtype=np.complex128)
    for i, r in enumerate(rows):
        b = ctx.address_to_det(int(r))
        kb, hv = ocsc.h_row_window(sp.sub, sp.lo, sp.hi, ints.h, ints.g, int(b))
        cols = layout.address_array(np.asarray(kb, dtype=np.uint64), sp.n_elec, sp.sub, sp.lo, sp.hi)
        cv = np.array([cmap.get(int(cc), 0.0) for cc in cols])
        refs[i] = np.dot(hv, cv)
    assert np.count_nonzero(refs) >= 200
    assert np.max(np.abs(got - refs)) <= 1e-12 * max(1.0, np.max(np.abs(refs)))
