"""GPU parity on the edges of the method and of the kernel forms, element by
element against the oracle:

- the sliced smoother and residual kernels forced onto every level with 1, 2,
  4, 8 and 16 wavefronts per slice (the 3D 4 x 4-block case at split 1 is the
  kernel form that runs on the finest level of the 128^3 workload; coarse
  levels sort each colour's rows by length, which these cases reach);
- a strength threshold that drops weak edges (isolated nodes become singleton
  aggregates), another priority seed, a level cap, and the ratio stop that ends
  coarsening when a level would keep more than 90 % of its nodes;
- a block-1 pattern that is not structurally symmetric (one-sided entries):
  colours over the symmetrised pattern, as in the oracle;
- malformed device-resident input blocks, rejected before any kernel reads them.
"""
import numpy as np
import pytest

from gpu_util import assert_close, gpu_hierarchy, log, rel, torch_dev
from paper_2103_07537_amd.inputs import make_system

pytestmark = pytest.mark.gpu


def _vcycle_pair(s, hg, ho, seed):
    from oracle import amg
    r = np.random.default_rng(seed).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    return z.cpu().numpy(), amg.vcycle(ho, r)


def _assert_elementwise(zg, zo, tol):
    assert_close(zg, zo, tol)


SPLIT_CASES = {
    "3d-11-lognormal": lambda: make_system(11, 3, 2.0, seed=5, kappa="lognormal"),
    "2d-23-distinct": lambda: make_system(23, 2, 0.7, seed=3, blk1_scale=2.0, a10_scale=0.5),
}


@pytest.mark.parametrize("case", list(SPLIT_CASES))
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("split", [1, 2, 4, 8, 16])
def test_forced_slice_split_matches_oracle(case, precision, split, monkeypatch):
    from oracle import amg
    s = SPLIT_CASES[case]()
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60), n_vec=s.n_vec)
    monkeypatch.setenv("MBAMG_SLICE_SPLIT", str(split))
    monkeypatch.setenv("MBAMG_ROWS_FORM", "sliced")   # the sliced layout on every level
    log(f"case={case} precision={precision} split={split}")
    hg = gpu_hierarchy(s, max_coarse=60, precision=precision)
    assert hg.num_levels() == len(ho.levels) >= 3
    zg, zo = _vcycle_pair(s, hg, ho, 17)
    _assert_elementwise(zg, zo, 1e-12 if precision == 0 else 1e-5)
    # the operator apply reads the same sliced parts with the same split
    x = np.random.default_rng(18).standard_normal(s.n_dofs)
    w = torch_dev(np.zeros(s.n_dofs))
    hg.apply(torch_dev(x), w)
    ref = amg.apply_A(ho.levels[0], x)
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-14 * np.max(np.abs(ref)) * 10
    hg.close()


def test_forced_slice_split_rejects_other_values(monkeypatch):
    from paper_2103_07537_amd import mbamg
    s = make_system(8, 2, 0.5, seed=2)
    monkeypatch.setenv("MBAMG_SLICE_SPLIT", "3")
    with pytest.raises(mbamg.MbamgError):
        gpu_hierarchy(s, max_coarse=40)


EDGE_PARAMS = {
    "theta-0.05": dict(theta=0.05),
    "theta-0.1": dict(theta=0.1),
    "seed-12345": dict(seed=12345),
    "max-levels-2": dict(max_levels=2, max_coarse=1),
    "to-the-ratio-stop": dict(max_coarse=1),
}


@pytest.mark.parametrize("pkey", list(EDGE_PARAMS))
def test_parameter_edges_match_oracle(pkey):
    from oracle import amg
    kw = EDGE_PARAMS[pkey]
    s = make_system(11, 3, 2.0, seed=5, kappa="lognormal", sigma=2.0)
    ho = amg.setup(s.blocks, s.dofs, amg.Params(**kw), n_vec=s.n_vec)
    hg = gpu_hierarchy(s, **kw)
    L = len(ho.levels)
    log(f"params={pkey} levels={L} nodes={[lv.n for lv in ho.levels]}")
    assert hg.num_levels() == L
    singletons = 0
    for l in range(L - 1):
        agg = hg.aggregates(l)
        assert np.array_equal(agg, ho.levels[l].agg), f"aggregates differ on level {l}"
        singletons += int(np.sum(np.bincount(agg) == 1))
        for f in range(2):
            assert np.array_equal(hg.colours(l, f), ho.levels[l].colour[f])
    if pkey.startswith("theta"):
        assert singletons > 0          # weak edges dropped: isolated nodes are aggregates of their own
    if pkey == "max-levels-2":
        assert L == 2 and ho.levels[-1].n * 8 > 1
    if pkey == "to-the-ratio-stop":
        # coarsening ran until aggregation would keep more than 90 % of a level's nodes
        last = ho.levels[-1]
        _, n_agg = amg.aggregate(last.A[0][0], 0.0, 0, L - 1)
        assert n_agg > 0.9 * last.n and last.n * 8 > 1
    zg, zo = _vcycle_pair(s, hg, ho, 19)
    _assert_elementwise(zg, zo, 1e-12)
    hg.close()


def _one_sided_a11(s, pairs):
    """Add blocks A11[i, j] (no A11[j, i]) for the given node pairs."""
    from paper_2103_07537_amd.inputs import Bsr
    b = s.blocks[1][1]
    d = b.vals.shape[1]
    rows = [list(b.col_idx[b.row_ptr[i]:b.row_ptr[i + 1]]) for i in range(b.n_brows)]
    vals = [list(b.vals[b.row_ptr[i]:b.row_ptr[i + 1]]) for i in range(b.n_brows)]
    rng = np.random.default_rng(3)
    for i, j in pairs:
        assert j not in rows[i] and i not in rows[j]
        k = int(np.searchsorted(rows[i], j))
        rows[i].insert(k, j)
        vals[i].insert(k, 0.3 * rng.standard_normal((d, d)))
    rp = np.zeros(b.n_brows + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    s.blocks[1][1] = Bsr(b.n_brows, b.n_bcols, rp, np.array([c for r in rows for c in r], np.int32),
                         np.array([v for r in vals for v in r]))
    return s


def test_one_sided_block1_pattern_colours_symmetrised():
    from oracle import amg
    s = make_system(14, 2, 0.7, seed=8)
    s = _one_sided_a11(s, [(0, 2), (3, 40), (50, 52), (100, 130), (17, 19)])
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60), n_vec=s.n_vec)
    hg = gpu_hierarchy(s, max_coarse=60)
    assert hg.num_levels() == len(ho.levels) >= 2
    for l in range(len(ho.levels) - 1):
        col = hg.colours(l, 1)
        assert np.array_equal(col, ho.levels[l].colour[1]), f"block-1 colours differ on level {l}"
        # valid for the symmetrised pattern: no stored block in either direction joins two equal colours
        B = ho.levels[l].A[1][1]
        for i in range(B.n_rows):
            for j in B.ci[B.rp[i]:B.rp[i + 1]]:
                assert j == i or col[i] != col[j]
    zg, zo = _vcycle_pair(s, hg, ho, 23)
    _assert_elementwise(zg, zo, 1e-12)
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    xo, io = amg.gmres(ho, s.b, rtol=1e-8)
    assert info["converged"] and abs(info["iterations"] - io.iterations) <= 1
    hg.close()


@pytest.mark.parametrize("fault", ["column-out-of-range", "column-negative", "row-ptr-decreasing",
                                   "row-ptr-end", "columns-unsorted"])
def test_malformed_device_block_is_rejected(fault):
    import torch
    from paper_2103_07537_amd import mbamg
    s = make_system(9, 2, 0.5, seed=2)
    b = s.blocks[1][1]
    rp = b.row_ptr.copy()
    ci = b.col_idx.copy()
    if fault == "column-out-of-range":
        ci[5] = b.n_bcols + 3
    elif fault == "column-negative":
        ci[7] = -1
    elif fault == "row-ptr-decreasing":
        rp[4] = rp[5] + 1
    elif fault == "row-ptr-end":
        rp[-1] = rp[-1] - 1
    else:
        r0, r1 = rp[10], rp[11]
        ci[r0:r1] = ci[r0:r1][::-1].copy()
    s.blocks[1][1].row_ptr = rp
    s.blocks[1][1].col_idx = ci
    dev = mbamg.to_device(s)
    log(f"fault={fault}")
    with pytest.raises(mbamg.MbamgError) as e:
        mbamg.Hierarchy(dev, s.dofs, s.n_vec)
    assert e.value.code == -1
    torch.cuda.synchronize()
    # the library stays usable
    good = make_system(9, 2, 0.5, seed=2)
    h = mbamg.Hierarchy(mbamg.to_device(good), good.dofs, good.n_vec)
    z = torch_dev(np.zeros(good.n_dofs))
    h.vcycle(torch_dev(good.b), z)
    assert np.all(np.isfinite(z.cpu().numpy()))
    h.close()


def test_ratio_stop_on_the_finest_level_is_a_direct_solve():
    # every edge weak: each node is its own aggregate, aggregation would keep every node, so
    # the finest level is the coarsest (the colouring job it started is joined first) and the
    # V-cycle is the dense solve
    s = make_system(12, 2, 0.5, seed=6)
    hg = gpu_hierarchy(s, theta=1e12, max_coarse=10)
    assert hg.num_levels() == 1
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(s.b), z)
    ref = np.linalg.solve(s.to_scipy().toarray(), s.b)
    assert_close(z.cpu().numpy(), ref, 1e-11, "one-level V-cycle")
    hg.close()


def test_set_omega_equals_a_hierarchy_built_with_it():
    """Changing the smoother damping of a built hierarchy gives, bit for bit, the
    V-cycle of a hierarchy set up with that damping, and the oracle's; a damping
    that is not finite and positive is refused, there and at setup."""
    from oracle import amg
    from paper_2103_07537_amd import mbamg
    s = make_system(23, 2, 0.7, seed=3, blk1_scale=2.0, a10_scale=0.5)
    hg = gpu_hierarchy(s, max_coarse=60)
    hg.set_omega(0.55)
    fresh = gpu_hierarchy(s, max_coarse=60, omega=0.55)
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60, omega=0.55), n_vec=s.n_vec)
    r = np.random.default_rng(91).standard_normal(s.n_dofs)
    z1, z2 = torch_dev(np.zeros(s.n_dofs)), torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z1)
    fresh.vcycle(torch_dev(r), z2)
    assert np.array_equal(z1.cpu().numpy(), z2.cpu().numpy())
    assert_close(z1.cpu().numpy(), amg.vcycle(ho, r), 1e-12, "V-cycle after set_omega")
    for bad in (0.0, -0.5, float("nan"), float("inf")):
        with pytest.raises(mbamg.MbamgError) as e:
            hg.set_omega(bad)
        assert e.value.code == -1
    with pytest.raises(mbamg.MbamgError) as e:
        gpu_hierarchy(s, max_coarse=60, omega=float("inf"))
    assert e.value.code == -1
    hg.close()
    fresh.close()
