"""Error paths of the C-ABI on the GPU: each bad input returns its status code
(raised as MbamgError by the binding) and leaves the library usable.  The
failing conditions are made on the host; no kernel is made to fault."""
import dataclasses

import numpy as np
import pytest

from gpu_util import gpu_hierarchy, log, rel, torch_dev
from paper_2103_07537_amd.inputs import make_system

pytestmark = pytest.mark.gpu

E_INVALID, E_SINGULAR = -1, -4


def _small():
    return make_system(6, 2, 0.5, seed=11)


def _still_works():
    from oracle import amg
    s = _small()
    hg = gpu_hierarchy(s, max_coarse=60)
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60))
    r = np.random.default_rng(0).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert rel(z.cpu().numpy(), amg.vcycle(ho, r)) <= 1e-12


def test_singular_coarsest_matrix_is_reported():
    """All values zero and one level: the Gauss-Jordan inverse finds no pivot."""
    from paper_2103_07537_amd import mbamg
    s = _small()
    zero = [[dataclasses.replace(B, vals=np.zeros_like(B.vals)) for B in row] for row in s.blocks]
    with pytest.raises(mbamg.MbamgError) as e:
        mbamg.Hierarchy(zero, s.dofs, s.n_vec, max_coarse=10 ** 6)
    log(f"  {e.value}")
    assert e.value.code == E_SINGULAR
    _still_works()


def test_singular_nodal_block_is_reported():
    """A zero diagonal block on the smoothed level: the nodal inverse fails."""
    from paper_2103_07537_amd import mbamg
    s = _small()
    A00 = s.blocks[0][0]
    vals = A00.vals.copy()
    rows = np.repeat(np.arange(A00.n_brows), np.diff(A00.row_ptr))
    vals[(rows == 3) & (A00.col_idx == 3)] = 0.0
    blocks = [[dataclasses.replace(A00, vals=vals), s.blocks[0][1]], s.blocks[1]]
    with pytest.raises(mbamg.MbamgError) as e:
        mbamg.Hierarchy(blocks, s.dofs, s.n_vec, max_coarse=60)
    log(f"  {e.value}")
    assert e.value.code == E_SINGULAR
    _still_works()


@pytest.mark.parametrize("bad", [dict(restart=40), dict(omega=0.0), dict(max_levels=0), dict(omega_p=-1.0)])
def test_invalid_parameters_are_rejected(bad):
    from paper_2103_07537_amd import mbamg
    s = _small()
    with pytest.raises(mbamg.MbamgError) as e:
        gpu_hierarchy(s, **bad)
    log(f"  {bad}: {e.value}")
    assert e.value.code == E_INVALID


def test_block_shape_mismatch_is_rejected():
    """Field map says 2 dofs per node for block 0, the blocks carry 3."""
    from paper_2103_07537_amd import mbamg
    s = _small()
    with pytest.raises(mbamg.MbamgError) as e:
        mbamg.Hierarchy(s.blocks, (2, 3), (1, 2))
    log(f"  {e.value}")
    assert e.value.code == E_INVALID
    _still_works()


def test_singular_nodal_block_with_judge_is_reported():
    """The same error while the fixed and learned hierarchies are built at the
    same time on two host threads: reported once, and nothing is left running."""
    from paper_2103_07537_amd import mbamg
    s = _small()
    A00 = s.blocks[0][0]
    vals = A00.vals.copy()
    rows = np.repeat(np.arange(A00.n_brows), np.diff(A00.row_ptr))
    vals[(rows == 3) & (A00.col_idx == 3)] = 0.0
    blocks = [[dataclasses.replace(A00, vals=vals), s.blocks[0][1]], s.blocks[1]]

    def weights(level, n_agg, F):
        return np.full(n_agg, 0.5), np.full(n_agg, 0.8)

    with pytest.raises(mbamg.MbamgError) as e:
        mbamg.Hierarchy(blocks, s.dofs, s.n_vec, max_coarse=60, weights=weights, judge=1)
    log(f"  {e.value}")
    assert e.value.code == E_SINGULAR
    _still_works()


def test_empty_system_is_rejected():
    """No nodes: setup returns the invalid-input code before any device work."""
    from paper_2103_07537_amd import mbamg
    from paper_2103_07537_amd.inputs import Bsr
    s = _small()
    empty = [[Bsr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32),
                  np.zeros((0, s.dofs[f], s.dofs[g]))) for g in range(2)] for f in range(2)]
    with pytest.raises(mbamg.MbamgError) as e:
        mbamg.Hierarchy(empty, s.dofs, s.n_vec)
    log(f"  {e.value}")
    assert e.value.code == E_INVALID
    _still_works()


def test_zero_rhs_and_converged_initial_guess():
    """b = 0 gives x = 0 without an iteration whatever x held; an initial guess
    that already meets the tolerance (dense LU's solution) is returned after no
    iteration, unchanged up to the colour-order round trip (exact)."""
    s = _small()
    hg = gpu_hierarchy(s, max_coarse=60)
    assert hg.num_levels() >= 2
    x = torch_dev(np.random.default_rng(1).standard_normal(s.n_dofs))
    info = hg.solve(torch_dev(np.zeros(s.n_dofs)), x, rtol=1e-8)
    assert info["converged"] and info["iterations"] == 0
    assert not np.any(x.cpu().numpy())
    xs = np.linalg.solve(s.to_scipy().toarray(), s.b)
    x = torch_dev(xs)
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    log(f"  exact guess: its={info['iterations']} rel={info['rel_residual']:.2e}")
    assert info["converged"] and info["iterations"] == 0
    assert np.array_equal(x.cpu().numpy(), xs)
    hg.close()
