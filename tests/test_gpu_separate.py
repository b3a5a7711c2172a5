"""Separate aggregation per block on the GPU against the oracle (Sec. 4.3.1:
fields on different node sets, each block aggregated from its own diagonal
block), on the mixed systems whose block 1 lives on a grid twice as coarse
and on co-located blocks aggregated each on its own:
per-block aggregates and colours identical as integers on every level, the
Galerkin blocks with P00 != P11 element by element, V-cycles element by
element (FP64 1e-12, FP32 1e-5), and solves (iterations within +-1, solutions
within 1e-8 when the counts agree)."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import assert_close, gpu_hierarchy, log, rel, torch_dev
from paper_2103_07537_amd.inputs import make_mixed_system, make_system

pytestmark = pytest.mark.gpu

CASES = {
    "2d-41-mixed": lambda: make_mixed_system(41, 2, 0.8, seed=3, kappa="lognormal"),
    "2d-13-mixed": lambda: make_mixed_system(13, 2, 1.5, seed=7),
    "3d-15-mixed": lambda: make_mixed_system(15, 3, 0.6, seed=5, kappa="lognormal"),
    # co-located fields aggregated separately: the second strength graph and MIS-2
    # run on A11's own pattern and values over the same nodes
    "2d-23-colocated": lambda: make_system(23, 2, 0.7, seed=3, kappa="lognormal", blk1_scale=2.0, a10_scale=0.5),
}


def _pair(case, precision=0, **kw):
    from oracle import amg
    s = CASES[case]()
    log(f"case={case} N0={s.N} N1={s.N1} precision={precision}")
    ho = amg.setup(s.blocks, s.dofs, amg.Params(clone=False, max_coarse=60, **kw), n_vec=s.n_vec)
    hg = gpu_hierarchy(s, clone_aggregates=0, max_coarse=60, precision=precision, **kw)
    return s, ho, hg


@pytest.mark.parametrize("case", list(CASES))
def test_separate_setup_matches_oracle(case):
    s, ho, hg = _pair(case)
    L = len(ho.levels)
    assert hg.num_levels() == L >= 2
    for l, lev in enumerate(ho.levels):
        assert hg.block_nodes(l, 0) == lev.n and hg.block_nodes(l, 1) == lev.n1
        if l + 1 < L:
            assert np.array_equal(hg.aggregates(l, 0), lev.agg), f"block-0 aggregates differ on level {l}"
            assert np.array_equal(hg.aggregates(l, 1), lev.agg1), f"block-1 aggregates differ on level {l}"
            for f in range(2):
                assert np.array_equal(hg.colours(l, f), lev.colour[f]), f"colours differ on level {l}"
        if l == 0:
            continue
        prev = ho.levels[l - 1]
        for f in range(2):
            for g in range(2):
                rp, ci, v = hg.level_block(l, f, g)
                B = lev.A[f][g]
                assert np.array_equal(rp, B.rp) and np.array_equal(ci, B.ci), f"pattern ({f},{g}) level {l}"
                scale = (abs(prev.P[f]).T @ abs(prev.csr[f][g]) @ abs(prev.P[g])).toarray()
                got = sp.bsr_matrix((v, ci, rp), shape=scale.shape).toarray()
                assert np.all(np.abs(got - lev.csr[f][g].toarray()) <= 1e-13 * scale), f"({f},{g}) level {l}"
    hg.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_separate_vcycle_matches_oracle(case, precision):
    from oracle import amg
    s, ho, hg = _pair(case, precision)
    r = np.random.default_rng(41).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12 if precision == 0 else 1e-5)
    w = torch_dev(np.zeros(s.n_dofs))
    hg.apply(torch_dev(r), w)
    A = s.to_scipy()
    ref = A @ r
    assert np.max(np.abs(w.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    hg.close()


@pytest.mark.parametrize("case", ["2d-41-mixed", "3d-15-mixed", "2d-23-colocated"])
@pytest.mark.parametrize("precision", [0, 1])
def test_separate_solve_matches_oracle(case, precision):
    from oracle import amg
    s, ho, hg = _pair(case, precision)
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    xg = x.cpu().numpy()
    xo, io = amg.gmres(ho, s.b, rtol=1e-8)
    A = s.to_scipy()
    res = np.linalg.norm(s.b - A @ xg) / np.linalg.norm(s.b)
    log(f"  iterations gpu {info['iterations']} oracle {io.iterations}, true residual {res:.2e}, "
        f"difference {rel(xg, xo):.2e}")
    assert info["converged"] and io.converged and res <= 1e-8 * (1 + 1e-6)
    assert abs(info["iterations"] - io.iterations) <= 1
    if precision == 0 and info["iterations"] == io.iterations:
        assert rel(xg, xo) <= 1e-8
    hg.close()


def test_cloning_and_learned_forms_reject_what_they_cannot_build():
    from paper_2103_07537_amd import mbamg
    s = CASES["2d-13-mixed"]()
    with pytest.raises(mbamg.MbamgError) as e:
        gpu_hierarchy(s)                                  # cloning needs equal node counts
    assert e.value.code == -1
    with pytest.raises(mbamg.MbamgError):
        gpu_hierarchy(s, clone_aggregates=0, omega_p=0.5)
    with pytest.raises(mbamg.MbamgError):
        gpu_hierarchy(s, clone_aggregates=0, smoother=1)


@pytest.mark.parametrize("kw", [dict(max_levels=2), dict(theta=0.05, seed=9)], ids=["level-cap", "theta-seed"])
def test_separate_level_cap_threshold_and_seed_match_oracle(kw):
    from oracle import amg
    s, ho, hg = _pair("2d-41-mixed", **kw)
    assert hg.num_levels() == len(ho.levels)
    for l, lev in enumerate(ho.levels[:-1]):
        assert np.array_equal(hg.aggregates(l, 0), lev.agg)
        assert np.array_equal(hg.aggregates(l, 1), lev.agg1)
    r = np.random.default_rng(62).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12)
    hg.close()


def test_colocated_separate_aggregation_reproduces_cloning():
    """Co-located blocks whose strength graphs give the same aggregates (here
    A11 is a scaled copy of A00's structure): aggregating each block on its own
    builds the cloned hierarchy -- the same aggregates, coarse operators and
    V-cycle."""
    s = CASES["2d-23-colocated"]()
    hs = gpu_hierarchy(s, clone_aggregates=0, max_coarse=60)
    hc = gpu_hierarchy(s, max_coarse=60)
    assert hs.num_levels() == hc.num_levels() >= 3
    for l in range(hc.num_levels() - 1):
        assert np.array_equal(hs.aggregates(l, 0), hc.aggregates(l, 0))
        assert np.array_equal(hs.aggregates(l, 1), hc.aggregates(l, 0))
    for l in range(1, hc.num_levels()):
        for f in range(2):
            for g in range(2):
                rs, cs, vs = hs.level_block(l, f, g)
                rc, cc, vc = hc.level_block(l, f, g)
                assert np.array_equal(rs, rc) and np.array_equal(cs, cc)
                assert np.max(np.abs(vs - vc)) <= 1e-13 * np.max(np.abs(vc))
    r = np.random.default_rng(71).standard_normal(s.n_dofs)
    zs, zc = torch_dev(np.zeros(s.n_dofs)), torch_dev(np.zeros(s.n_dofs))
    hs.vcycle(torch_dev(r), zs)
    hc.vcycle(torch_dev(r), zc)
    assert_close(zs.cpu().numpy(), zc.cpu().numpy(), 1e-12, "separate against cloned V-cycle")
    hs.close()
    hc.close()
