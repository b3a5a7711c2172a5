"""Pins for the oracle of block systems with more than two blocks (the
n_b x n_b form of eq. block-prec-form, here the 4 x 4 split of Sec. 2.1 into
u, p, b, r).  Each check compares with something other than the n-block code:
the field split as a permutation of the 2 x 2 system, the two-block oracle
when n_b = 2, Algorithm 1 over four blocks in closed form with dense matrices,
a dense two-grid cycle, the dense triple product, and dense LU.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg, nblock
from paper_2103_07537_amd.inputs import make_system, split_fields
from test_oracle_pins import _gs_matrix


def _systems():
    return [make_system(9, 2, 0.8, seed=3, kappa="lognormal", blk1_scale=1.6, a10_scale=0.7),
            make_system(5, 3, 0.6, seed=5, kappa="lognormal")]


def _perm(s):
    N, d, dim = s.N, s.dofs[0], s.dim
    vec = lambda off: off + (np.arange(N)[:, None] * d + np.arange(dim)[None, :]).reshape(-1)
    return np.concatenate([vec(0), np.arange(N) * d + dim, vec(N * d), N * d + np.arange(N) * d + dim])


@pytest.mark.parametrize("si", [0, 1])
def test_field_split_is_a_permutation_of_the_two_block_system(si):
    s = _systems()[si]
    t = split_fields(s)
    assert t.dofs == (s.dim, 1, s.dim, 1) and t.n_dofs == s.n_dofs
    q = _perm(s)
    assert abs(s.to_scipy()[q][:, q] - t.to_scipy()).max() == 0.0
    assert np.array_equal(s.b[q], t.b)
    # no stored block of a sub-block is entirely zero
    for row in t.blocks:
        for B in row:
            assert B.vals.shape[0] == B.col_idx.shape[0]
            assert np.all(np.any(B.vals != 0.0, axis=(1, 2)))


def test_two_blocks_reproduce_the_two_block_oracle():
    s = _systems()[0]
    p = amg.Params(max_coarse=40)
    h2 = amg.setup(s.blocks, s.dofs, p)
    hn = nblock.setup(s.blocks, s.dofs, p)
    assert [lv.n for lv in h2.levels] == [lv.n for lv in hn.levels]
    r = np.random.default_rng(1).standard_normal(s.n_dofs)
    z2, zn = amg.vcycle(h2, r), nblock.vcycle(hn, r)
    assert np.linalg.norm(z2 - zn) <= 1e-14 * np.linalg.norm(z2)


@pytest.mark.parametrize("si", [0, 1])
def test_algorithm1_over_four_blocks_closed_form(si):
    # one sweep from a nonzero iterate: x_f += omega M_f (b_f - sum_g A_fg x_g), blocks in order,
    # M_f^-1 the colour-ordered block lower triangle of A_ff
    t = split_fields(_systems()[si])
    p = amg.Params(max_coarse=1, max_levels=2, omega=0.7)
    h = nblock.setup(t.blocks, t.dofs, p)
    lev = h.levels[0]
    A = [[lev.csr[f][g].toarray() for g in range(4)] for f in range(4)]
    M = [np.linalg.inv(_gs_matrix(A[f][f], lev.colour[f], lev.dofs[f])) for f in range(4)]
    rng = np.random.default_rng(2)
    b = [rng.standard_normal(A[f][f].shape[0]) for f in range(4)]
    x = [rng.standard_normal(A[f][f].shape[0]) for f in range(4)]
    ref = [xi.copy() for xi in x]
    for f in range(4):
        ref[f] = ref[f] + 0.7 * M[f] @ (b[f] - sum(A[f][g] @ ref[g] for g in range(4)))
    got = nblock.bgs(lev, x, b, p)
    for f in range(4):
        assert np.allclose(got[f], ref[f], rtol=1e-12, atol=1e-12 * np.abs(ref[f]).max())


@pytest.mark.parametrize("si", [0, 1])
def test_galerkin_blocks_equal_the_dense_triple_product(si):
    t = split_fields(_systems()[si])
    h = nblock.setup(t.blocks, t.dofs, amg.Params(max_coarse=20))
    assert len(h.levels) >= 3
    for l in range(len(h.levels) - 1):
        lev, nxt = h.levels[l], h.levels[l + 1]
        Af = sp.bmat(lev.csr).toarray()
        P = sp.block_diag(lev.P).toarray()
        ref = P.T @ Af @ P
        scale = np.abs(P).T @ np.abs(Af) @ np.abs(P)
        got = sp.bmat(nxt.csr).toarray()
        assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-300)


def test_two_grid_vcycle_dense():
    t = split_fields(_systems()[0])
    p = amg.Params(max_levels=2, max_coarse=1, omega=0.7)
    h = nblock.setup(t.blocks, t.dofs, p)
    assert len(h.levels) == 2
    lev = h.levels[0]
    A = [[lev.csr[f][g].toarray() for g in range(4)] for f in range(4)]
    Afull = np.block(A)
    M = [np.linalg.inv(_gs_matrix(A[f][f], lev.colour[f], lev.dofs[f])) for f in range(4)]
    o = lev.offsets()

    def smooth(x, b):
        xs = [x[o[f]:o[f + 1]].copy() for f in range(4)]
        for f in range(4):
            xs[f] = xs[f] + 0.7 * M[f] @ (b[o[f]:o[f + 1]] - sum(A[f][g] @ xs[g] for g in range(4)))
        return np.concatenate(xs)

    P = sp.block_diag(lev.P).toarray()
    Ac = P.T @ Afull @ P
    b = t.b
    x = smooth(np.zeros_like(b), b)
    x = x + P @ np.linalg.solve(Ac, P.T @ (b - Afull @ x))
    x = smooth(x, b)
    assert np.allclose(nblock.vcycle(h, b), x, rtol=1e-11, atol=1e-11 * np.abs(x).max())


@pytest.mark.parametrize("si", [0, 1])
def test_gmres_matches_dense_lu(si):
    t = split_fields(_systems()[si])
    h = nblock.setup(t.blocks, t.dofs, amg.Params(max_coarse=20))
    x, info = nblock.gmres(h, t.b, rtol=1e-12)
    assert info.converged
    xr = np.linalg.solve(t.to_scipy().toarray(), t.b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
