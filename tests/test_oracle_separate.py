"""Pins for the oracle's separate per-block aggregation (Sec. 4.3.1: fields on
different node sets get an AMG setup of their own per block), on the mixed
system whose block 1 lives on a grid twice as coarse as block 0's.  Each pin
compares with something other than the oracle: partitions, the near-null
space, dense triple products with the assembled block-diagonal P (P00 != P11),
a dense two-grid cycle, dense LU, and the cloned hierarchy where both blocks'
graphs coincide.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg
from paper_2103_07537_amd.inputs import make_mixed_system, make_system
from test_oracle_pins import _gs_matrix

SEP = amg.Params(clone=False, max_coarse=40)


def _mixed(si=0):
    return [make_mixed_system(13, 2, 0.8, seed=3, kappa="lognormal"),
            make_mixed_system(7, 3, 0.6, seed=5, kappa="lognormal")][si]


def test_generator_blocks_and_positive_real():
    s = _mixed(0)
    assert (s.N, s.N1) == (13 ** 2, 6 ** 2) and s.n_dofs == s.b.shape[0]
    A = s.to_scipy().toarray()
    assert A.shape == (s.n_dofs, s.n_dofs)
    # the coupling part is skew: A10 = -A01^T
    Z = s.blocks[0][1].to_scipy().toarray()
    assert np.array_equal(s.blocks[1][0].to_scipy().toarray(), -Z.T)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0


@pytest.mark.parametrize("si", [0, 1])
def test_each_block_is_partitioned_by_its_own_aggregates(si):
    s = _mixed(si)
    h = amg.setup(s.blocks, s.dofs, SEP)
    assert len(h.levels) >= 3
    for l, lev in enumerate(h.levels[:-1]):
        nxt = h.levels[l + 1]
        for agg, n_agg, n, nc in [(lev.agg, lev.n_agg, lev.n, nxt.n), (lev.agg1, lev.n_agg1, lev.n1, nxt.n1)]:
            assert agg.shape == (n,) and agg.min() >= 0 and agg.max() == n_agg - 1 == nc - 1
            assert np.all(np.bincount(agg, minlength=n_agg) >= 1)
    lev = h.levels[0]
    assert lev.n != lev.n1 and lev.n_agg != lev.n_agg1


def test_tentative_prolongators_reproduce_each_blocks_near_null_space():
    s = _mixed(0)
    h = amg.setup(s.blocks, s.dofs, SEP)
    B = [np.ones(s.N * s.dofs[0]), np.ones(s.N1 * s.dofs[1])]
    for l, lev in enumerate(h.levels[:-1]):
        for f in range(2):
            P = lev.P[f]
            # the coarse near-null space is the aggregate norms: P B_c = B_f up to rounding
            d = lev.dofs[f]
            agg = lev.agg if f == 0 else lev.agg1
            n_agg = lev.n_agg if f == 0 else lev.n_agg1
            norms = np.sqrt(np.bincount(np.repeat(agg, d) * d + np.tile(np.arange(d), len(agg)),
                                        weights=B[f] ** 2, minlength=n_agg * d))
            assert np.allclose(P @ norms, B[f], rtol=1e-15, atol=1e-15)
            # orthonormal columns
            PtP = (P.T @ P).toarray()
            assert np.allclose(PtP, np.eye(PtP.shape[0]), atol=1e-14)
            B[f] = norms


@pytest.mark.parametrize("si", [0, 1])
def test_galerkin_blocks_equal_the_dense_triple_product(si):
    s = _mixed(si)
    h = amg.setup(s.blocks, s.dofs, SEP)
    for l in range(len(h.levels) - 1):
        lev, nxt = h.levels[l], h.levels[l + 1]
        Af = sp.bmat([[lev.csr[0][0], lev.csr[0][1]], [lev.csr[1][0], lev.csr[1][1]]]).toarray()
        P = sp.block_diag([lev.P[0], lev.P[1]]).toarray()
        ref = P.T @ Af @ P
        scale = np.abs(P).T @ np.abs(Af) @ np.abs(P)
        got = sp.bmat([[nxt.csr[0][0], nxt.csr[0][1]], [nxt.csr[1][0], nxt.csr[1][1]]]).toarray()
        assert got.shape == ref.shape
        assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-300)


def test_two_grid_vcycle_dense():
    s = _mixed(0)
    p = amg.Params(clone=False, max_levels=2, max_coarse=1, omega=0.7)
    h = amg.setup(s.blocks, s.dofs, p)
    assert len(h.levels) == 2
    lev = h.levels[0]
    A = [[lev.csr[f][g].toarray() for g in range(2)] for f in range(2)]
    Afull = np.block(A)
    M = [np.linalg.inv(_gs_matrix(A[f][f], lev.colour[f], lev.dofs[f])) for f in range(2)]
    n0 = A[0][0].shape[0]
    w = p.omega

    def smooth(x, b):
        x0, x1 = x[:n0], x[n0:]
        x0 = x0 + w * M[0] @ (b[:n0] - A[0][0] @ x0 - A[0][1] @ x1)
        x1 = x1 + w * M[1] @ (b[n0:] - A[1][0] @ x0 - A[1][1] @ x1)
        return np.concatenate([x0, x1])

    P = sp.block_diag([lev.P[0], lev.P[1]]).toarray()
    Ac = P.T @ Afull @ P
    b = s.b
    x = smooth(np.zeros_like(b), b)
    x = x + P @ np.linalg.solve(Ac, P.T @ (b - Afull @ x))
    x = smooth(x, b)
    assert np.allclose(amg.vcycle(h, b), x, rtol=1e-11, atol=1e-11 * np.abs(x).max())


@pytest.mark.parametrize("si", [0, 1])
def test_gmres_matches_dense_lu(si):
    s = _mixed(si)
    h = amg.setup(s.blocks, s.dofs, SEP)
    x, info = amg.gmres(h, s.b, rtol=1e-12)
    assert info.converged
    xr = np.linalg.solve(s.to_scipy().toarray(), s.b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


def test_separate_equals_cloned_when_both_graphs_coincide():
    # A11 = A00 (same values, same pattern): block 1's own aggregation is block 0's, so
    # the separate setup builds the cloned hierarchy and the V-cycles agree to rounding
    s = make_system(12, 2, 0.7, seed=6)
    assert s.blocks[1][1] is s.blocks[0][0]
    hc = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=40))
    hs = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=40, clone=False))
    assert len(hc.levels) == len(hs.levels)
    for a, b in zip(hc.levels[:-1], hs.levels[:-1]):
        assert np.array_equal(a.agg, b.agg) and np.array_equal(b.agg, b.agg1)
    r = np.random.default_rng(2).standard_normal(s.n_dofs)
    zc, zs = amg.vcycle(hc, r), amg.vcycle(hs, r)
    assert np.linalg.norm(zc - zs) <= 1e-14 * np.linalg.norm(zc)


def test_cloning_rejects_fields_on_different_node_sets():
    s = _mixed(0)
    with pytest.raises(ValueError):
        amg.setup(s.blocks, s.dofs, amg.Params())
