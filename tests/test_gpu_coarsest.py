"""The coarsest-level direct solve at the sizes where the blocked Gauss-Jordan
inverse changes its panel shape (threads, rows per thread, panel width), with
ragged last panels and a matrix smaller than one panel.  One level, so the
V-cycle is the dense solve itself; compared with LAPACK's LU solve."""
import numpy as np
import pytest

from gpu_util import gpu_hierarchy, log, rel, torch_dev
from paper_2103_07537_amd.inputs import make_system

pytestmark = pytest.mark.gpu


# 2D grids, 6 unknowns per node: n = 6 m^2 = 24 (one partial panel), 216, 486,
# 1014, 1944, 2904, 4056, 7776, 8214 -- one or two sizes in every panel shape
@pytest.mark.parametrize("m", [2, 6, 9, 13, 18, 22, 26, 36, 37])
def test_coarsest_solve_matches_lu(m):
    s = make_system(m, 2, 0.5, seed=m)
    log(f"  m={m}: {s.n_dofs} unknowns")
    hg = gpu_hierarchy(s, max_coarse=10 ** 6)
    assert hg.num_levels() == 1
    r = np.random.default_rng(m).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    A = s.to_scipy().toarray()
    zc = z.cpu().numpy()
    ref = np.linalg.solve(A, r)
    res = np.linalg.norm(r - A @ zc) / np.linalg.norm(r)
    err = rel(zc, ref)
    log(f"    residual {res:.2e}, vs LU {err:.2e}")
    # even the correctly rounded inverse leaves a residual of about cond(A) times
    # the unit roundoff (cond up to about 1e5 here), so the residual bound only
    # catches gross errors; the forward error against LU is the tight check
    assert res <= 1e-9
    assert err <= 1e-11
