"""Input generator: sizes, determinism and well-posedness (CPU only)."""
import numpy as np
import pytest

from paper_2103_07537_amd.inputs import make_system, workload


def _structural(s):
    return sum(int((b.vals != 0).sum()) for row in s.blocks for b in row)


@pytest.mark.parametrize("n,dim", [(32, 2), (7, 2), (5, 3), (12, 3)])
def test_sizes_match_stencil_counts(n, dim):
    s = make_system(n, dim, 0.5, seed=1)
    N = n ** dim
    assert s.N == N and s.dofs == (dim + 1, dim + 1)
    pairs = 2 * dim * n ** (dim - 1) * (n - 1)          # directed neighbour pairs
    assert s.blocks[0][0].nnzb == N + pairs
    assert s.blocks[0][1].nnzb == pairs
    per_pair = 14 if dim == 2 else 18
    assert _structural(s) == (2 * (dim + 1)) * N + per_pair * pairs - 0 * N
    for row in s.blocks:
        for b in row:
            for i in range(0, N, max(1, N // 50)):
                c = b.col_idx[b.row_ptr[i]:b.row_ptr[i + 1]]
                assert np.all(np.diff(c) > 0)


def test_benchmark_sizes():
    s = workload("2d-256")
    assert s.n_dofs == 393216 and s.blocks[0][0].nnzb == 326656 and s.blocks[0][1].nnzb == 261120


def test_deterministic_and_seed_dependent():
    a = make_system(6, 3, 2.0, seed=4, kappa="lognormal")
    b = make_system(6, 3, 2.0, seed=4, kappa="lognormal")
    c = make_system(6, 3, 2.0, seed=5, kappa="lognormal")
    assert np.array_equal(a.b, b.b) and np.array_equal(a.blocks[0][0].vals, b.blocks[0][0].vals)
    assert not np.array_equal(a.b, c.b)
    assert not np.array_equal(a.blocks[0][0].vals, c.blocks[0][0].vals)


@pytest.mark.parametrize("kw", [dict(n=5, dim=2, gamma=5.0, kappa="lognormal"),
                                dict(n=3, dim=3, gamma=2.0, kappa="lognormal"),
                                dict(n=6, dim=2, gamma=0.5)])
def test_positive_real(kw):
    s = make_system(seed=2, **kw)
    A = s.to_scipy().toarray()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    Z = s.blocks[0][1].to_scipy().toarray()
    assert np.array_equal(Z, -Z.T)
    assert np.abs(s.b).max() <= 1.0


def test_coupling_field_is_normalised():
    s = make_system(8, 2, 1.0, seed=3)
    h = 1.0 / 9
    Z = s.blocks[0][1].vals
    assert np.abs(Z).max() == pytest.approx(1.0 / (2 * h), rel=1e-12)


def test_study_table_marks_unconverged_points():
    from paper_2103_07537_amd import studies
    rows = [dict(params=dict(precision=1, omega=0.8), iterations=12, converged=True, setup_ms=1.0, solve_ms=2.0,
                 total_ms=3.0, ms_per_iteration=0.1667),
            dict(params=dict(precision=1, omega=1.1), iterations=1000, converged=False, setup_ms=1.0,
                 solve_ms=9.0, total_ms=10.0, ms_per_iteration=0.009)]
    t = studies.table(rows).splitlines()
    assert t[2].startswith("| omega=0.8 | 12 |") and "precision" not in t[2]
    assert "1000 (not converged)" in t[3]


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 3)])
def test_leading_components_is_the_principal_submatrix(dim, k):
    """The k-component system is the rows and columns of the first k components
    of every node of both blocks, and its right-hand side is b's same entries."""
    from paper_2103_07537_amd.inputs import leading_components
    s = make_system(5, dim, 0.6, seed=4, kappa="lognormal", a10_scale=0.5)
    t = leading_components(s, k)
    d = s.dofs[0]
    keep = np.array([node * d + c for node in range(2 * s.N) for c in range(k)])
    A = s.to_scipy().toarray()
    assert t.dofs == (k, k) and t.n_dofs == 2 * s.N * k
    assert np.array_equal(t.to_scipy().toarray(), A[np.ix_(keep, keep)])
    assert np.array_equal(t.b, s.b[keep])
    with pytest.raises(ValueError):
        leading_components(s, d + 1)
