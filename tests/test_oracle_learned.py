"""Pins for the learned form's oracle pieces: smoothed prolongator, generic
ordered Galerkin product, features, the network's gradient and bfloat16
rounding.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg, learned
from paper_2103_07537_amd.inputs import make_system, workload


def _sys():
    return make_system(7, 2, 0.8, seed=4, kappa="lognormal", blk1_scale=1.7, a10_scale=0.6)


def _bsr(b):
    return amg.BsrM(b.n_brows, b.n_bcols, b.row_ptr, b.col_idx, b.vals)


def test_zero_weights_reproduce_the_fixed_method_exactly():
    s = workload("2d-64-lognormal", seed=1001)
    h0 = amg.setup(s.blocks, s.dofs, amg.Params())
    hw = amg.setup(s.blocks, s.dofs, amg.Params(weights=lambda l, n, F: (np.zeros(n), np.full(n, 0.8))))
    r = np.random.default_rng(0).standard_normal(s.n_dofs)
    assert np.array_equal(amg.vcycle(h0, r), amg.vcycle(hw, r))


def test_uniform_weight_is_textbook_smoothed_aggregation():
    s = _sys()
    A = _bsr(s.blocks[0][0])
    agg, nagg = amg.aggregate(A, 0.0, 0, 0)
    mp, mi = amg.members(agg, nagg)
    q, _ = amg.tentative(np.ones((s.N, 3)), agg, mp, mi)
    w = 0.55
    P = amg.sa_prolongator(A, 2, agg, q, np.full(nagg, w), nagg).csr().toarray()
    Ad = A.csr().toarray()
    Ph = amg.prolongator(q, agg, nagg).toarray()
    vec = np.tile(np.array([1.0, 1.0, 0.0]), s.N)
    Avv = np.diag(vec) @ Ad @ np.diag(vec)
    ref = Ph - w * np.diag(np.where(vec > 0, 1.0 / np.diag(Ad), 0.0)) @ Avv @ Ph
    assert np.abs(P - ref).max() <= 1e-14 * np.abs(ref).max()


def test_generic_product_matches_the_piecewise_constant_stages_bitwise():
    s = _sys()
    A00 = _bsr(s.blocks[0][0])
    agg, nagg = amg.aggregate(A00, 0.0, 0, 0)
    mp, mi = amg.members(agg, nagg)
    q, _ = amg.tentative(np.ones((s.N, 3)), agg, mp, mi)
    Pb = amg.tentative_bsr(q, agg, nagg)
    for f, g in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        A = _bsr(s.blocks[f][g])
        ref = amg.galerkin(A, agg, mp, mi, nagg, q, q)
        got = amg.spgemm(amg.transpose(Pb), amg.spgemm(A, Pb))
        assert np.array_equal(ref.rp, got.rp) and np.array_equal(ref.ci, got.ci)
        assert np.array_equal(ref.val, got.val)


def test_smoothed_galerkin_equals_dense_triple_product():
    s = _sys()
    rng = np.random.default_rng(3)
    h = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=1,
                                               weights=lambda l, n, F: (rng.uniform(0.1, 0.8, n),
                                                                        rng.uniform(0.5, 1.0, n))))
    assert len(h.levels) >= 2
    for l in range(len(h.levels) - 1):
        lev, nxt = h.levels[l], h.levels[l + 1]
        for f in range(2):
            for g in range(2):
                Pf, Pg = lev.P[f].toarray(), lev.P[g].toarray()
                Af = lev.csr[f][g].toarray()
                scale = np.abs(Pf).T @ np.abs(Af) @ np.abs(Pg)
                assert np.all(np.abs(Pf.T @ Af @ Pg - nxt.csr[f][g].toarray()) <= 1e-13 * scale + 1e-300)


def test_per_node_damping_matches_closed_form():
    s = _sys()
    ws = np.random.default_rng(5).uniform(0.4, 1.2, 64)
    h = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=1,
                                               weights=lambda l, n, F: (np.zeros(n), ws[:n])))
    lev = h.levels[0]
    A = [[lev.csr[f][g].toarray() for g in range(2)] for f in range(2)]
    from test_oracle_pins import _gs_matrix
    M = [np.linalg.inv(_gs_matrix(A[f][f], lev.colour[f], 3)) for f in range(2)]
    W = np.repeat(ws[lev.agg], 3)
    b0, b1 = np.random.default_rng(1).standard_normal((2, s.N * 3))
    z0, z1 = amg.bgs(lev, np.zeros_like(b0), np.zeros_like(b1), b0, b1, h.params)
    r0 = W * (M[0] @ b0)
    assert np.allclose(z0, r0, rtol=1e-12, atol=1e-12)
    assert np.allclose(z1, W * (M[1] @ (b1 - A[1][0] @ r0)), rtol=1e-12, atol=1e-12)


def test_network_gradient_matches_central_differences():
    th = learned.init_params(3)
    th[4992:5122] = np.random.default_rng(9).standard_normal(130) * 0.3   # non-trivial output layer
    X = np.random.default_rng(1).standard_normal((40, 12))
    T = np.stack([np.random.default_rng(2).uniform(0, 0.8, 40), np.random.default_rng(3).uniform(0.3, 1.3, 40)], 1)
    L, g = learned.loss_grad(th, X, T)
    for k in [0, 100, 700, 770, 900, 4000, 4930, 5000, 5121]:
        e = np.zeros_like(th)
        e[k] = 1e-6
        fd = (learned.loss_grad(th + e, X, T)[0] - learned.loss_grad(th - e, X, T)[0]) / 2e-6
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9), k


def test_outputs_stay_in_their_ranges():
    th = learned.init_params(0)
    th[4992:5122] = np.random.default_rng(4).standard_normal(130)
    out, _ = learned.forward(th, np.random.default_rng(0).standard_normal((200, 12)))
    assert np.all(out[:, 0] > 0) and np.all(out[:, 0] < 5 / 6)
    assert np.all(out[:, 1] > 0.3) and np.all(out[:, 1] < 1.3)
    # saturated logits reach the closed ends of the ranges, never beyond
    with np.errstate(over="ignore"):
        out, _ = learned.forward(th * 50, np.random.default_rng(0).standard_normal((200, 12)) * 10)
    assert np.all(out[:, 0] >= 0) and np.all(out[:, 0] <= 5 / 6)
    assert np.all(out[:, 1] >= 0.3) and np.all(out[:, 1] <= 1.3)


def test_bf16_rounding_table():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e38])
    # 3.0e38 lies between 2^127 * (1 + 97/128) and 2^127 * (1 + 98/128), nearer the latter
    ref = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 2.0 ** 127 * (1 + 98 / 128)])
    assert np.array_equal(learned.bf16(x), ref)


def test_features_properties_and_brute_force():
    s = _sys()
    h = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=1, weights=lambda l, n, F: (np.zeros(n), np.ones(n))))
    lev = h.levels[0]
    F = lev.features
    n, nagg, agg = lev.n, lev.n_agg, lev.agg
    size = np.bincount(agg)
    assert F.shape == (nagg, 12)
    assert abs(np.sum(size * F[:, 0])) < 1e-10
    assert F[:, 4].mean() == pytest.approx(1.0)
    assert np.all(F[:, 5] >= 0) and np.all(F[:, 5] <= 1) and np.all(F[:, 1] >= 0) and np.all(F[:, 2] >= 0)
    assert np.all(F[:, 11] == 0.0)
    # brute force from the definitions, loops over nodes and blocks
    A00 = lev.A[0][0].csr().toarray()
    A01 = lev.A[0][1].csr().toarray()
    d = 3
    blk = lambda M, i, j: M[i * d:(i + 1) * d, j * d:(j + 1) * d]
    dv = np.array([np.mean(np.diag(blk(A00, i, i))[:2]) for i in range(n)])
    for k in range(nagg):
        mem = [i for i in range(n) if agg[i] == k]
        ld = np.log(dv[mem])
        assert F[k, 0] == pytest.approx(ld.mean() - np.log(dv).mean(), abs=1e-12)
        assert F[k, 1] == pytest.approx(ld.std(), abs=1e-12)
        num = sum(np.sum(blk(A01, i, j) ** 2) for i in mem for j in range(n))
        den = sum(np.sum(blk(A00, i, j) ** 2) for i in mem for j in range(n))
        assert F[k, 6] == pytest.approx(np.sqrt(num / den), rel=1e-12)
        off = [sum(np.mean(np.abs(np.diag(blk(A00, i, j))[:2])) for j in range(n) if j != i) for i in mem]
        assert F[k, 8] == pytest.approx(np.mean(np.array(off) / dv[mem]), rel=1e-12)
