"""Oracle for the learned form -- TEST INFRASTRUCTURE ONLY.

Plain FP64 NumPy: the 12 per-aggregate algebraic features and the
12 -> 64 -> 64 -> 2 network (ReLU hidden layers) that maps them to a
prolongator-smoothing weight omega_P in (0, 5/6) and a smoother damping
omega_S in (0.3, 1.3) per aggregate, with its loss gradient.  An optional
emulation rounds inputs, weights and hidden activations to bfloat16 the way
the GPU kernels feed the matrix cores, keeping every sum in FP64.

Parameter packing (5122 FP32 values): W1[64][12], b1[64], W2[64][64], b2[64],
W3[2][64], b3[2].
"""
from __future__ import annotations

import numpy as np

N_FEAT = 12
HID = 64
N_OUT = 2
OFF = {"W1": 0, "b1": 768, "W2": 832, "b2": 4928, "W3": 4992, "b3": 5120}
N_PARAMS = 5122
OMEGA_P_MAX = 5.0 / 6.0      # (2/3) * 1.25
OMEGA_S_MIN = 0.3
OMEGA_S_SPAN = 1.0


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    return (t[0:768].reshape(64, 12), t[768:832], t[832:4928].reshape(64, 64), t[4928:4992],
            t[4992:5120].reshape(2, 64), t[5120:5122])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(theta, X, emulate=False):
    """Returns (out[n,2] = (omega_P, omega_S), cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    X = r(X)
    z1 = X @ r(W1).T + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(W2).T + b2
    h2 = r(np.maximum(z2, 0.0))
    o = h2 @ r(W3).T + b3
    s = sigmoid(o)
    out = np.stack([OMEGA_P_MAX * s[:, 0], OMEGA_S_MIN + OMEGA_S_SPAN * s[:, 1]], axis=1)
    return out, (X, z1, h1, z2, h2, o, s)


def loss_grad(theta, X, T, emulate=False):
    """L = mean over rows of sum_c (out_c - T_c)^2 and its gradient (5122)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    out, (Xr, z1, h1, z2, h2, o, s) = forward(theta, X, emulate)
    n = X.shape[0]
    diff = out - T
    loss = float(np.sum(diff * diff) / n)
    scale = np.array([OMEGA_P_MAX, OMEGA_S_SPAN])
    # with emulation the backward signals enter the matrix products as bfloat16
    # while the bias gradients sum the unrounded values, as on the GPU
    do = (2.0 / n) * diff * scale * s * (1.0 - s)
    gW3 = r(do).T @ h2
    gb3 = do.sum(axis=0)
    dh2 = r(do) @ r(W3)
    dz2 = dh2 * (h2 > 0)
    gW2 = r(dz2).T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = r(dz2) @ r(W2)
    dz1 = dh1 * (h1 > 0)
    gW1 = r(dz1).T @ Xr
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def init_params(seed=0):
    """He-normal hidden layers, small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 12)) * np.sqrt(2.0 / 12)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    W3 = rng.standard_normal((2, 64)) * 0.01
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.zeros(2)])


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------

def features(lev, n_vec, level: int) -> np.ndarray:
    """Twelve algebraic features per aggregate of one level (FP64).

    With dv(i) the mean vector-diagonal entry of A00's diagonal block at node i
    and c_ij the mean |vector-vector diagonal entry| of the off-diagonal block
    A00[i,j]:
      1 mean log dv over the aggregate minus the level's mean log dv
      2 standard deviation of log dv in the aggregate
      3 max - min of log dv in the aggregate
      4 log(max c / min c) over pairs inside the aggregate (0 if none)
      5 aggregate size / mean aggregate size
      6 share of the members' off-diagonal vector weight sum c that leaves the aggregate
      7 ||A01 rows|| / ||A00 rows|| (Frobenius over the members' rows)
      8 ||A10 rows|| / ||A11 rows||
      9 mean over members of sum_j c_ij / dv(i) (A00)
     10 the same for A11
     11 mean over members of sum_j ||A00[i,j][vector, scalar]||^2 / (dv(i) * |A00[i,i][scalar, scalar]|)
     12 level / 4
    """
    n, nagg = lev.n, lev.n_agg
    agg = lev.agg
    nv0, nv1 = n_vec
    A00, A01, A10, A11 = lev.A[0][0], lev.A[0][1], lev.A[1][0], lev.A[1][1]

    def per_row(A, nv):
        rows = np.repeat(np.arange(A.n_rows), np.diff(A.rp))
        dg = rows == A.ci
        vv = np.abs(A.val[:, np.arange(nv), np.arange(nv)])          # (nnzb, nv)
        c = vv.mean(axis=1)
        dv = np.zeros(A.n_rows)
        dv[rows[dg]] = A.val[dg][:, np.arange(nv), np.arange(nv)].mean(axis=1)
        off_sum = np.bincount(rows[~dg], weights=c[~dg], minlength=A.n_rows)
        out_sum = np.bincount(rows[~dg], weights=np.where(agg[A.ci[~dg]] != agg[rows[~dg]], c[~dg], 0.0),
                              minlength=A.n_rows)
        fro2 = np.bincount(rows, weights=np.sum(A.val.reshape(A.val.shape[0], -1) ** 2, axis=1),
                           minlength=A.n_rows)
        return rows, dg, c, dv, off_sum, out_sum, fro2

    rows0, dg0, c0, dv0, off0, out0, fro00 = per_row(A00, nv0)
    rows1, dg1, c1, dv1, off1, _, fro11 = per_row(A11, nv1)
    fro01 = np.bincount(np.repeat(np.arange(n), np.diff(A01.rp)),
                        weights=np.sum(A01.val.reshape(A01.val.shape[0], -1) ** 2, axis=1), minlength=n)
    fro10 = np.bincount(np.repeat(np.arange(n), np.diff(A10.rp)),
                        weights=np.sum(A10.val.reshape(A10.val.shape[0], -1) ** 2, axis=1), minlength=n)
    ld = np.log(dv0)
    mu = ld.mean()
    size = np.bincount(agg, minlength=nagg).astype(np.float64)
    F = np.zeros((nagg, 12))
    mean_ld = np.bincount(agg, weights=ld, minlength=nagg) / size
    F[:, 0] = mean_ld - mu
    var = np.bincount(agg, weights=(ld - mean_ld[agg]) ** 2, minlength=nagg) / size
    F[:, 1] = np.sqrt(np.maximum(var, 0.0))
    mx = np.full(nagg, -np.inf)
    mn = np.full(nagg, np.inf)
    np.maximum.at(mx, agg, ld)
    np.minimum.at(mn, agg, ld)
    F[:, 2] = mx - mn
    # internal pairs
    inside = (~dg0) & (agg[A00.ci] == agg[rows0])
    cmax = np.full(nagg, -np.inf)
    cmin = np.full(nagg, np.inf)
    np.maximum.at(cmax, agg[rows0[inside]], c0[inside])
    np.minimum.at(cmin, agg[rows0[inside]], c0[inside])
    ok = np.isfinite(cmax) & (cmin > 0)
    F[:, 3] = np.where(ok, np.log(np.where(ok, cmax, 1.0)) - np.log(np.where(ok, cmin, 1.0)), 0.0)
    F[:, 4] = size / (n / nagg)
    tot = np.bincount(agg, weights=off0, minlength=nagg)
    outw = np.bincount(agg, weights=out0, minlength=nagg)
    F[:, 5] = np.where(tot > 0, outw / np.where(tot > 0, tot, 1.0), 0.0)
    a00 = np.bincount(agg, weights=fro00, minlength=nagg)
    a01 = np.bincount(agg, weights=fro01, minlength=nagg)
    a10 = np.bincount(agg, weights=fro10, minlength=nagg)
    a11 = np.bincount(agg, weights=fro11, minlength=nagg)
    F[:, 6] = np.sqrt(a01) / np.sqrt(a00)
    F[:, 7] = np.sqrt(a10) / np.sqrt(a11)
    F[:, 8] = np.bincount(agg, weights=off0 / dv0, minlength=nagg) / size
    F[:, 9] = np.bincount(agg, weights=off1 / dv1, minlength=nagg) / size
    d0 = A00.val.shape[1]
    if d0 > nv0:
        g2 = np.sum(A00.val[:, :nv0, nv0:] ** 2, axis=(1, 2))
        gsum = np.bincount(rows0, weights=g2, minlength=n)
        cpp = np.zeros(n)
        cpp[rows0[dg0]] = np.abs(A00.val[dg0][:, nv0, nv0])
        F[:, 10] = np.bincount(agg, weights=gsum / np.maximum(dv0 * cpp, 1e-300), minlength=nagg) / size
    F[:, 11] = level / 4.0
    return F
