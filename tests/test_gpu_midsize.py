"""GPU against the oracle at the two mid-size benchmark configurations, where
the finest level takes the kernel forms of the large workloads (in 3D: 4 x 4
blocks, one wavefront per slice):

- 2D 256^2 nodes, 6 dofs/node, gamma 0.5 (393,216 unknowns), FP64: V-cycle
  element by element, and the GMRES(30) solve to rtol 1e-8 (iterations within
  +-1, solutions within 1e-8 when the counts agree), with the error against a
  tight (rtol 1e-12) oracle solution logged;
- 3D 64^3 nodes, 8 dofs/node, gamma 0.5 (2,097,152 unknowns): the FP64 V-cycle
  element by element (1e-12) and the FP32 one (1e-5), sampled-free: the whole
  vector, and the FP32-refined solve's true residual.
"""
import numpy as np
import pytest

from gpu_util import assert_close, gpu_hierarchy, log, rel, torch_dev
from paper_2103_07537_amd.inputs import workload

pytestmark = pytest.mark.gpu


def test_2d_256_vcycle_and_solve_match_oracle():
    from oracle import amg
    s = workload("2d-256", seed=1)
    log(f"2d-256: {s.n_dofs} unknowns")
    ho = amg.setup(s.blocks, s.dofs, amg.Params(), n_vec=s.n_vec)
    hg = gpu_hierarchy(s)
    assert hg.num_levels() == len(ho.levels)
    for l in range(len(ho.levels) - 1):
        assert np.array_equal(hg.aggregates(l), ho.levels[l].agg)
    r = np.random.default_rng(31).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12, "2d-256 FP64 V-cycle")
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    xg = x.cpu().numpy()
    xo, io = amg.gmres(ho, s.b, rtol=1e-8)
    log(f"  iterations gpu {info['iterations']} oracle {io.iterations}; "
        f"solution difference {rel(xg, xo):.2e}")
    assert info["converged"] and io.converged
    assert abs(info["iterations"] - io.iterations) <= 1
    if info["iterations"] == io.iterations:
        assert rel(xg, xo) <= 1e-8
    xt, it = amg.gmres(ho, s.b, rtol=1e-12)
    log(f"  error vs the oracle's rtol 1e-12 solution: gpu {rel(xg, xt):.2e}, oracle rtol 1e-8 {rel(xo, xt):.2e}")
    hg.close()


def test_3d_64_vcycles_match_oracle():
    from oracle import amg
    s = workload("3d-64", seed=1)
    log(f"3d-64: {s.n_dofs} unknowns")
    ho = amg.setup(s.blocks, s.dofs, amg.Params(), n_vec=s.n_vec)
    r = np.random.default_rng(32).standard_normal(s.n_dofs)
    zo = amg.vcycle(ho, r)
    for precision, tol in [(0, 1e-12), (1, 1e-5)]:
        hg = gpu_hierarchy(s, precision=precision)
        assert hg.num_levels() == len(ho.levels)
        z = torch_dev(np.zeros(s.n_dofs))
        hg.vcycle(torch_dev(r), z)
        assert_close(z.cpu().numpy(), zo, tol, f"3d-64 {'FP64' if precision == 0 else 'FP32'} V-cycle")
        if precision == 1:
            x = torch_dev(np.zeros(s.n_dofs))
            info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
            A = s.to_scipy()
            res = np.linalg.norm(s.b - A @ x.cpu().numpy()) / np.linalg.norm(s.b)
            log(f"  FP32-refined solve: {info['iterations']} iterations, true residual {res:.2e}")
            assert info["converged"] and res <= 1e-8 * (1 + 1e-6)
        hg.close()
