"""GPU parity of the full-node smoother (smoother = 1: damped nodal-block
Gauss-Seidel over the (d0+d1)-square node blocks, the fully coupled reference
the paper compares the blocked smoother with) against the oracle's `fc`."""
import dataclasses

import numpy as np
import pytest

from gpu_util import assert_close, gpu_hierarchy, log, oracle_params, rel, torch_dev
from paper_2103_07537_amd.inputs import make_system, workload

pytestmark = pytest.mark.gpu

CASES = {
    "2d-ragged-distinct": lambda: make_system(23, 2, 0.7, seed=3, blk1_scale=2.0, a10_scale=0.5),
    "3d-lognormal-distinct": lambda: make_system(11, 3, 2.0, seed=5, kappa="lognormal", blk1_scale=0.5,
                                                 a10_scale=1.5),
    "2d-64-lognormal": lambda: workload("2d-64-lognormal", seed=1000),
    # coupling inside each node: the full node blocks are no longer block diagonal
    "2d-node-coupling": lambda: make_system(23, 2, 0.7, seed=3, node_coupling=0.5),
    "3d-node-coupling": lambda: make_system(11, 3, 2.0, seed=5, kappa="lognormal", node_coupling=0.1),
}
PARAMS = {
    "default": dict(max_coarse=40),
    "sweeps": dict(max_coarse=40, bgs_sweeps=2, inner_sweeps=2, omega=0.6),
}


def weights_fn(level, n_agg, F):
    k = np.arange(n_agg)
    return 0.1 + 0.6 * ((k * 37 + level) % 11) / 10.0, 0.5 + 0.5 * ((k * 13 + 3 * level) % 7) / 6.0


def _pair(case, pkey, precision=0, weighted=False):
    from oracle import amg
    s = CASES[case]()
    kw = dict(PARAMS[pkey], smoother=1)
    okw = dict(weights=weights_fn) if weighted else {}
    ho = amg.setup(s.blocks, s.dofs, oracle_params(**kw, **okw), n_vec=s.n_vec)
    gkw = dict(weights=weights_fn, judge=0) if weighted else {}
    hg = gpu_hierarchy(s, precision=precision, **kw, **gkw)
    log(f"case={case} params={pkey} precision={precision} weighted={weighted} levels={hg.num_levels()}")
    assert hg.num_levels() == len(ho.levels) >= 3
    return s, ho, hg


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("pkey", list(PARAMS))
@pytest.mark.parametrize("precision", [0, 1])
def test_full_node_vcycle_matches_oracle(case, pkey, precision):
    from oracle import amg
    s, ho, hg = _pair(case, pkey, precision)
    r = np.random.default_rng(9).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12 if precision == 0 else 1e-5)
    hg.close()


def test_full_node_with_per_aggregate_damping_matches_oracle():
    from oracle import amg
    s, ho, hg = _pair("3d-lognormal-distinct", "default", weighted=True)
    r = np.random.default_rng(10).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12)
    hg.close()


@pytest.mark.parametrize("case", list(CASES))
def test_full_node_solve_matches_oracle(case):
    from oracle import amg
    s, ho, hg = _pair(case, "default")
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    xo, io = amg.gmres(ho, s.b, rtol=1e-8)
    log(f"  its gpu {info['iterations']} oracle {io.iterations}")
    assert info["converged"] and io.converged
    assert abs(info["iterations"] - io.iterations) <= 1
    assert rel(x.cpu().numpy(), xo) <= 1e-7
    hg.close()


def _with_extra_blocks(B, pairs):
    """B with zero blocks added at the (row, col) pairs (columns kept sorted)."""
    rows = np.repeat(np.arange(B.n_brows), np.diff(B.row_ptr))
    r = np.concatenate([rows, [i for i, _ in pairs]])
    c = np.concatenate([B.col_idx, [j for _, j in pairs]])
    v = np.concatenate([B.vals, np.zeros((len(pairs),) + B.vals.shape[1:])])
    order = np.lexsort((c, r))
    rp = np.zeros(B.n_brows + 1, dtype=B.row_ptr.dtype)
    np.add.at(rp, r[order] + 1, 1)
    return dataclasses.replace(B, row_ptr=np.cumsum(rp).astype(B.row_ptr.dtype),
                               col_idx=c[order].astype(B.col_idx.dtype), vals=v[order].copy())


def test_full_node_smoother_rejects_patterns_outside_a00():
    from paper_2103_07537_amd import mbamg
    s = make_system(10, 2, 0.5, seed=2)
    N = s.N
    # a long-range (zero) block pair in A11: its node graph is no longer A00's
    B2 = _with_extra_blocks(s.blocks[1][1], [(0, N - 1), (N - 1, 0)])
    blocks = [list(s.blocks[0]), [s.blocks[1][0], B2]]
    with pytest.raises(mbamg.MbamgError) as ei:
        mbamg.Hierarchy(blocks, s.dofs, s.n_vec, smoother=1, max_coarse=40)
    log(f"  error: {ei.value}")
    assert "full-node smoother" in str(ei.value)
    # the blocked smoother takes the same system
    h = mbamg.Hierarchy(blocks, s.dofs, s.n_vec, max_coarse=40)
    h.close()


def test_full_node_smoother_with_the_judge():
    # both builds of the judged learned form take the full-node smoother; the
    # learned one borrows level 0's aggregates and smoother blocks and builds
    # its own node inverses
    from oracle import amg
    s = CASES["3d-lognormal-distinct"]()
    hg = gpu_hierarchy(s, max_coarse=40, smoother=1, weights=weights_fn, judge=1)
    used = hg.info()["used_learned"]
    ho = amg.setup(s.blocks, s.dofs, oracle_params(max_coarse=40, smoother=1,
                                                   **(dict(weights=weights_fn) if used else {})),
                   n_vec=s.n_vec)
    r = np.random.default_rng(12).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    log(f"  used_learned={used}")
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12)
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    assert info["converged"]
    hg.close()


@pytest.mark.parametrize("case", ["2d-node-coupling", "3d-node-coupling"])
@pytest.mark.parametrize("precision", [0, 1])
def test_node_coupled_blocked_and_full_node_solves_match_oracle(case, precision):
    """With coupling inside the nodes the two smoothers differ: the blocked one
    sees the node's own coupling block only through Algorithm 1's block
    updates, the full-node one inverts it with the node.  Both V-cycles match
    the oracle element by element and both solves its iteration counts."""
    from oracle import amg
    s = CASES[case]()
    its = {}
    for sm in (0, 1):
        kw = dict(max_coarse=40, smoother=sm)
        ho = amg.setup(s.blocks, s.dofs, oracle_params(**kw), n_vec=s.n_vec)
        hg = gpu_hierarchy(s, precision=precision, **kw)
        r = np.random.default_rng(12).standard_normal(s.n_dofs)
        z = torch_dev(np.zeros(s.n_dofs))
        hg.vcycle(torch_dev(r), z)
        assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12 if precision == 0 else 1e-5,
                     f"{case} smoother {sm} V-cycle")
        x = torch_dev(np.zeros(s.n_dofs))
        info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
        xo, io = amg.gmres(ho, s.b, rtol=1e-8)
        its[sm] = (info["iterations"], io.iterations)
        assert info["converged"] and abs(info["iterations"] - io.iterations) <= 1
        hg.close()
    log(f"  {case} precision {precision}: blocked {its[0]}, full node {its[1]} (gpu, oracle)")
    assert its[1][1] < its[0][1]
