"""Two blocks of 1, 2 and 3 dofs per node on the GPU against the oracle (the
generator gives 3 + 3 in 2D and 4 + 4 in 3D; these systems keep the first k
components of every node, a principal submatrix of the same system).  Every
form the two-block path builds for them: aggregates and colours identical as
integers, the Galerkin blocks element by element, the operator apply, the
FP64 and FP32 V-cycles element by element, GMRES solves, the full-node
smoother, and the smoothed prolongator with per-aggregate damping (weights
injected through the C-ABI callback)."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import assert_close, gpu_hierarchy, log, rel, torch_dev
from paper_2103_07537_amd.inputs import leading_components, make_system

pytestmark = pytest.mark.gpu

CASES = {
    "2d-23-k1": lambda: leading_components(make_system(23, 2, 0.7, seed=3, kappa="lognormal", blk1_scale=2.0,
                                                       a10_scale=0.5), 1),
    "2d-23-k2": lambda: leading_components(make_system(23, 2, 0.7, seed=3, kappa="lognormal", blk1_scale=2.0,
                                                       a10_scale=0.5), 2),
    "3d-11-k1": lambda: leading_components(make_system(11, 3, 2.0, seed=5, kappa="lognormal", blk1_scale=0.5,
                                                       a10_scale=1.5), 1),
    "3d-11-k2": lambda: leading_components(make_system(11, 3, 2.0, seed=5, kappa="lognormal", blk1_scale=0.5,
                                                       a10_scale=1.5), 2),
    "3d-11-k3": lambda: leading_components(make_system(11, 3, 2.0, seed=5, kappa="lognormal", blk1_scale=0.5,
                                                       a10_scale=1.5), 3),
}


def weights_fn(level, n_agg, F):
    k = np.arange(n_agg)
    return 0.1 + 0.6 * ((k * 37 + level) % 11) / 10.0, 0.5 + 0.5 * ((k * 13 + 3 * level) % 7) / 6.0


def _pair(case, **kw):
    from oracle import amg
    s = CASES[case]()
    okw = {k: v for k, v in kw.items() if k in amg.Params.__dataclass_fields__}
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60, **okw), n_vec=s.n_vec)
    hg = gpu_hierarchy(s, max_coarse=60, **kw)
    log(f"case={case} dofs={s.dofs} n_vec={s.n_vec} levels gpu {hg.num_levels()} oracle {len(ho.levels)} {kw}")
    assert hg.num_levels() == len(ho.levels) >= 3
    return s, ho, hg


@pytest.mark.parametrize("case", list(CASES))
def test_setup_matches_oracle(case):
    s, ho, hg = _pair(case)
    for l, lev in enumerate(ho.levels):
        assert hg.level_nodes(l) == lev.n
        if l + 1 < len(ho.levels):
            assert np.array_equal(hg.aggregates(l), lev.agg), f"aggregates differ on level {l}"
            for f in range(2):
                assert np.array_equal(hg.colours(l, f), lev.colour[f]), f"colours of block {f} on level {l}"
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
def test_apply_vcycle_and_solve_match_oracle(case, precision):
    from oracle import amg
    s, ho, hg = _pair(case, precision=precision)
    r = np.random.default_rng(61).standard_normal(s.n_dofs)
    w = torch_dev(np.zeros(s.n_dofs))
    hg.apply(torch_dev(r), w)
    assert rel(w.cpu().numpy(), amg.apply_A(ho.levels[0], r)) <= 1e-14
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12 if precision == 0 else 1e-5)
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    xo, io = amg.gmres(ho, s.b, rtol=1e-8)
    xg = x.cpu().numpy()
    res = np.linalg.norm(s.b - s.to_scipy() @ xg) / np.linalg.norm(s.b)
    log(f"  iterations gpu {info['iterations']} oracle {io.iterations}, true residual {res:.2e}")
    assert info["converged"] and io.converged and res <= 1e-8 * (1 + 1e-6)
    assert abs(info["iterations"] - io.iterations) <= 1
    if precision == 0 and info["iterations"] == io.iterations:
        assert rel(xg, xo) <= 1e-8
    hg.close()


@pytest.mark.parametrize("case", ["2d-23-k1", "2d-23-k2", "3d-11-k3"])
def test_full_node_smoother_matches_oracle(case):
    from oracle import amg
    s, ho, hg = _pair(case, smoother=1)
    r = np.random.default_rng(62).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12, "full-node V-cycle")
    hg.close()


@pytest.mark.parametrize("case", ["2d-23-k1", "3d-11-k2", "3d-11-k3"])
def test_weighted_form_matches_oracle(case):
    from oracle import amg
    s, ho, hg = _pair(case, weights=weights_fn, judge=0)
    wp, ws = hg.level_weights(0)
    assert np.array_equal(wp, weights_fn(0, ho.levels[0].n_agg, None)[0])
    r = np.random.default_rng(63).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12, "weighted V-cycle")
    hg.close()
