"""Oracle for the monolithic blocked AMG hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded FP64 reference.  Only ``tests/``, the smoke check
and the benchmark's CPU-baseline leg may import it; the GPU library never
does, and the two share no code.  The sequential integer steps and the
ordered Galerkin sums live in ``seq.c`` (plain loops); everything else is
NumPy/SciPy written to follow the paper's definitions:

* V-cycle ``MGV`` exactly as the multigrid algorithm figure of Sec. 3
  (pre-smooth, residual, restrict, recurse from a zero guess, prolongate,
  post-smooth; direct solve on the last level).
* Coarse operators by the Galerkin product of Sec. 3 with R = P^T and block
  diagonal transfers P = diag(P00, P11) (Sec. 4.3.1, eq. blocktransfers).
* Aggregates built from the graph of A00 and cloned for block 1 (Sec. 4.3.1,
  the aggregate-cloning figure), piecewise-constant interpolation for each
  solution component over each aggregate.
* Smoother: the damped block Gauss-Seidel of Algorithm 1 (Sec. 4.3.2); the
  approximate sub-block solves are multicolour nodal-block Gauss-Seidel sweeps
  started from zero.
* Outer solver: restarted GMRES with right preconditioning, modified
  Gram-Schmidt and Givens rotations (Saad, Iterative Methods, Alg. 6.9/9.5).

Readings of points the paper leaves open are listed with the project's design
notes; each function below names the one it relies on.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle_seq.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile seq.c (plain C, one thread, no FP contraction)."""
    src = os.path.join(_HERE, "seq.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared",
                               "-fPIC", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        lib.or_aggregate.argtypes = [ctypes.c_int, i32p, i32p, f64p, u64p, i32p, i32p]
        lib.or_aggregate.restype = ctypes.c_int
        lib.or_colour.argtypes = [ctypes.c_int, i32p, i32p, i32p]
        lib.or_colour.restype = ctypes.c_int
        lib.or_rap_stage1.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, i32p, f64p,
                                      i32p, f64p, i32p, i32p, f64p]
        lib.or_rap_stage1.restype = ctypes.c_int64
        lib.or_rap_stage2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, i32p, i32p,
                                      i32p, f64p, f64p, i32p, i32p, f64p]
        lib.or_rap_stage2.restype = ctypes.c_int64
        lib.or_spgemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, i32p, f64p,
                                  i32p, i32p, f64p, ctypes.c_int64, i32p, i32p, f64p]
        lib.or_spgemm.restype = ctypes.c_int64
        lib.or_sa_prolongator.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, i32p, f64p, i32p, f64p,
                                          f64p, i32p, i32p, f64p]
        lib.or_sa_prolongator.restype = ctypes.c_int64
        _lib = lib
    return _lib


# ----------------------------------------------------------------------------
# parameters and containers
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    omega: float = 0.8          # BGS damping (Algorithm 1)
    bgs_sweeps: int = 1         # Algorithm 1 sweeps, pre and post
    inner_sweeps: int = 1       # multicolour GS sweeps per sub-block solve
    theta: float = 0.0          # strength threshold
    max_levels: int = 10
    max_coarse: int = 2500      # dofs
    seed: int = 0               # aggregation priority seed
    omega_p: float = 0.0        # uniform prolongator-smoothing weight (0: piecewise constant P)
    weights: object = None      # callable(level, n_agg, features) -> (omega_p[n_agg], omega_s[n_agg])
    smoother: int = 0           # 0: block Gauss-Seidel over the two blocks (Algorithm 1);
                                # 1: nodal-block Gauss-Seidel over the full node blocks (FC-AMG analogue)
    clone: bool = True          # block 1 reuses block 0's aggregates (Sec. 4.3.1, the cloning figure);
                                # False: each block is aggregated from its own diagonal block's graph,
                                # the separate AMG setup per block for fields on different node sets


@dataclasses.dataclass
class BsrM:
    """Square-node BSR block: row_ptr, col_idx, vals[nnzb, br, bc]."""
    n_rows: int
    n_cols: int
    rp: np.ndarray
    ci: np.ndarray
    val: np.ndarray

    def csr(self):
        br, bc = self.val.shape[1], self.val.shape[2]
        return sp.bsr_matrix((self.val, self.ci, self.rp),
                             shape=(self.n_rows * br, self.n_cols * bc)).tocsr()


@dataclasses.dataclass
class Level:
    n: int                      # nodes of block 0
    dofs: tuple
    A: list                     # 2x2 BsrM
    csr: list                   # 2x2 scipy CSR
    agg: np.ndarray = None      # node -> aggregate (None on the last level)
    n_agg: int = 0
    m_ptr: np.ndarray = None    # aggregate members, increasing node order
    m_idx: np.ndarray = None
    q: list = None              # per block, tentative-P weights (n, d_f)
    P: list = None              # per block, scalar CSR (n*d_f, n_agg*d_f)
    colour: list = None         # per block
    n_colours: list = None
    dinv: list = None           # per block (n, d, d)
    gs: list = None             # per block: list over colours of (rows, off-diag rows, Dinv)
    fc: list = None             # full node blocks: list over colours of (rows, off-node-block rows, Dinv)
    fc_colour: np.ndarray = None
    omega_s: np.ndarray = None  # per-node smoother damping (None: Params.omega)
    omega_p: np.ndarray = None  # per-aggregate prolongator-smoothing weights used for P
    features: np.ndarray = None
    n1: int = -1                # nodes of block 1 (-1: n, co-located fields)
    agg1: np.ndarray = None     # block 1's aggregates when it is aggregated separately
    n_agg1: int = 0

    def __post_init__(self):
        if self.n1 < 0:
            self.n1 = self.n

    def nodes(self, f: int) -> int:
        return self.n if f == 0 else self.n1

    def n_dofs(self) -> int:
        return self.n * self.dofs[0] + self.n1 * self.dofs[1]


@dataclasses.dataclass
class Hierarchy:
    levels: list
    params: Params
    coarse_lu: tuple = None
    coarse_n: int = 0


# ----------------------------------------------------------------------------
# setup pieces
# ----------------------------------------------------------------------------

def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def priority_keys(n: int, seed: int, level: int) -> np.ndarray:
    """Node priority (hash, index) packed in 64 bits; larger is picked first.

    hash = top 32 bits of the SplitMix64 finaliser of
    i + 0x9E3779B97F4A7C15 * (seed*1024 + level + 1) (mod 2^64).
    """
    mult = (0x9E3779B97F4A7C15 * (seed * 1024 + level + 1)) & ((1 << 64) - 1)
    with np.errstate(over="ignore"):
        z = np.arange(n, dtype=np.uint64) + np.uint64(mult)
        h = _mix64(z) >> np.uint64(32)
    return (h << np.uint64(32)) | np.arange(n, dtype=np.uint64)


def block_sq_norms(val: np.ndarray) -> np.ndarray:
    """Squared Frobenius norm of each block, summed in row-major order."""
    v = val.reshape(val.shape[0], -1)
    acc = v[:, 0] * v[:, 0]
    for k in range(1, v.shape[1]):
        acc = acc + v[:, k] * v[:, k]
    return acc


def strength_graph(A: BsrM, theta: float):
    """Strong-connection node graph of a square block matrix.

    Amalgamation (Sec. 4.4: the node graph G(A) of the sub-block): edge (i,j),
    i != j, carries w2 = max(||A_ij||_F^2, ||A_ji||_F^2) and is strong iff
    w2 > 0 and w2^2 >= theta^4 * ||A_ii||_F^2 * ||A_jj||_F^2.
    Returns CSR (ptr, idx, w2) with sorted, symmetric rows.
    """
    n = A.n_rows
    n2 = block_sq_norms(A.val)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.rp))
    cols = A.ci.astype(np.int64)
    dmask = rows == cols
    dn2 = np.zeros(n)
    dn2[rows[dmask]] = n2[dmask]
    off = ~dmask
    W = sp.csr_matrix((n2[off], (rows[off], cols[off])), shape=(n, n))
    W = W.maximum(W.T.tocsr()).tocsr()
    W.sort_indices()
    coo = W.tocoo()
    w2 = coo.data
    t4 = (theta * theta) * (theta * theta)
    keep = (w2 > 0.0) & (w2 * w2 >= t4 * (dn2[coo.row] * dn2[coo.col]))
    S = sp.csr_matrix((w2[keep], (coo.row[keep], coo.col[keep])), shape=(n, n))
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


def aggregate(A00: BsrM, theta: float, seed: int, level: int):
    """Aggregates from the strong graph of A00 (greedy MIS-2 + two phases)."""
    lib = _load()
    ptr, idx, w2 = strength_graph(A00, theta)
    keys = priority_keys(A00.n_rows, seed, level)
    agg = np.zeros(A00.n_rows, dtype=np.int32)
    nagg = np.zeros(1, dtype=np.int32)
    rc = lib.or_aggregate(A00.n_rows, ptr, idx, np.ascontiguousarray(w2), keys, agg, nagg)
    if rc != 0:
        raise RuntimeError("aggregation left a node unattached")
    return agg, int(nagg[0])


def members(agg: np.ndarray, n_agg: int):
    order = np.argsort(agg, kind="stable").astype(np.int32)
    counts = np.bincount(agg, minlength=n_agg)
    ptr = np.zeros(n_agg + 1, dtype=np.int32)
    np.cumsum(counts, out=ptr[1:])
    return ptr, order


def tentative(B: np.ndarray, agg: np.ndarray, m_ptr: np.ndarray, m_idx: np.ndarray):
    """Piecewise-constant interpolation per component (Sec. 4.3.1).

    Column norms of the near-null space over each aggregate, summed over the
    members in increasing order: q[i,c] = B[i,c] / ||B[A_k, c]||_2 and the
    coarse near-null space is B_c[k,c] = ||B[A_k, c]||_2.
    """
    n_agg = m_ptr.shape[0] - 1
    d = B.shape[1]
    sizes = np.diff(m_ptr)
    acc = np.zeros((n_agg, d))
    for p in range(int(sizes.max()) if n_agg else 0):
        has = sizes > p
        node = m_idx[m_ptr[:-1][has] + p]
        acc[has] = acc[has] + B[node] * B[node]
    norms = np.sqrt(acc)
    q = B / norms[agg]
    return q, norms


def prolongator(q: np.ndarray, agg: np.ndarray, n_agg: int):
    n, d = q.shape
    rows = np.arange(n * d)
    cols = (agg[:, None].astype(np.int64) * d + np.arange(d)[None, :]).reshape(-1)
    return sp.csr_matrix((q.reshape(-1), (rows, cols)), shape=(n * d, n_agg * d))


def galerkin(A: BsrM, agg, m_ptr, m_idx, n_agg, q_row, q_col) -> BsrM:
    """A_c = P_f^T A_fg P_g as (P^T (A P)) with ordered sums (seq.c)."""
    lib = _load()
    br, bc = A.val.shape[1], A.val.shape[2]
    n = A.n_rows
    cap = max(A.ci.shape[0], 1)
    t_rp = np.zeros(n + 1, dtype=np.int32)
    t_ci = np.zeros(cap, dtype=np.int32)
    t_val = np.zeros(cap * br * bc)
    nt = lib.or_rap_stage1(n, br, bc, A.rp, A.ci, np.ascontiguousarray(A.val.reshape(-1)),
                           agg, np.ascontiguousarray(q_col.reshape(-1)), t_rp, t_ci, t_val)
    c_rp = np.zeros(n_agg + 1, dtype=np.int32)
    c_ci = np.zeros(max(nt, 1), dtype=np.int32)
    c_val = np.zeros(max(nt, 1) * br * bc)
    nc = lib.or_rap_stage2(n_agg, br, bc, m_ptr, m_idx, t_rp, t_ci, t_val,
                           np.ascontiguousarray(q_row.reshape(-1)), c_rp, c_ci, c_val)
    return BsrM(n_agg, n_agg, c_rp, c_ci[:nc].copy(), c_val[:nc * br * bc].reshape(nc, br, bc).copy())


def colouring(A: BsrM):
    """First-fit greedy colours in increasing node order over the symmetrised pattern."""
    lib = _load()
    n = A.n_rows
    rows = np.repeat(np.arange(n), np.diff(A.rp))
    M = sp.csr_matrix((np.ones(rows.shape[0]), (rows, A.ci)), shape=(n, n))
    M = (M + M.T).tocsr()
    M.sort_indices()
    col = np.zeros(n, dtype=np.int32)
    nc = lib.or_colour(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), col)
    return col, nc


def diag_blocks(A: BsrM) -> np.ndarray:
    br = A.val.shape[1]
    out = np.zeros((A.n_rows, br, br))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.rp))
    m = rows == A.ci
    out[rows[m]] = A.val[m]
    return out


def _prepare_gs(lev: Level, f: int):
    """Per colour: dof rows, the off-diagonal rows of A_ff, and the block-diagonal D^-1."""
    d = lev.dofs[f]
    Aff = lev.csr[f][f]
    D = diag_blocks(lev.A[f][f])
    Dsp = sp.block_diag(list(D), format="csr") if lev.n else sp.csr_matrix((0, 0))
    Aoff = (Aff - Dsp).tocsr()
    out = []
    for c in range(lev.n_colours[f]):
        nodes = np.nonzero(lev.colour[f] == c)[0]
        rows = (nodes[:, None] * d + np.arange(d)[None, :]).reshape(-1)
        Dc = sp.block_diag(list(lev.dinv[f][nodes]), format="csr")
        out.append((rows, Aoff[rows, :].tocsr(), Dc))
    return out


def _node_dofs(lev: Level, nodes: np.ndarray) -> np.ndarray:
    """Indices of the nodes' dofs in the full vector [field 0 | field 1], node
    by node (field 0's dofs, then field 1's)."""
    d0, d1 = lev.dofs
    nodes = np.asarray(nodes)
    i0 = nodes[:, None] * d0 + np.arange(d0)[None, :]
    i1 = lev.n * d0 + nodes[:, None] * d1 + np.arange(d1)[None, :]
    return np.concatenate([i0, i1], axis=1).reshape(-1)


def fc_colouring(lev: Level):
    """First-fit greedy colours in increasing node order over the union of the
    four blocks' node graphs (symmetrised): nodes of one colour share no block
    of any A_fg."""
    n = lev.n
    rows, cols = [], []
    for f in range(2):
        for g in range(2):
            A = lev.A[f][g]
            rows.append(np.repeat(np.arange(n), np.diff(A.rp)))
            cols.append(np.asarray(A.ci))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    M = sp.csr_matrix((np.ones(r.shape[0]), (r, c)), shape=(n, n))
    M = (M + M.T).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    col = np.zeros(n, dtype=np.int32)
    nc = _load().or_colour(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), col)
    return col, nc


def node_blocks(lev: Level) -> np.ndarray:
    """Full node-diagonal blocks D_i = [[A00_ii, A01_ii], [A10_ii, A11_ii]]."""
    d0, d1 = lev.dofs
    D = np.zeros((lev.n, d0 + d1, d0 + d1))
    for f, (a, b) in enumerate(((0, d0), (d0, d0 + d1))):
        for g, (c, e) in enumerate(((0, d0), (d0, d0 + d1))):
            A = lev.A[f][g]
            rows = np.repeat(np.arange(lev.n), np.diff(A.rp))
            m = rows == A.ci
            D[rows[m], a:b, c:e] = A.val[m]
    return D


def _prepare_fc(lev: Level):
    """Per colour of the full node graph: the dofs of its nodes, the rows of
    the full operator without the node-diagonal blocks, and the inverses of
    the full node blocks (block diagonal over the colour's nodes)."""
    Afull = sp.bmat([[lev.csr[0][0], lev.csr[0][1]], [lev.csr[1][0], lev.csr[1][1]]]).tocsr()
    D = node_blocks(lev)
    m = D.shape[1]
    idx = _node_dofs(lev, np.arange(lev.n)).reshape(lev.n, m)
    r = np.repeat(idx[:, :, None], m, axis=2).reshape(-1)
    c = np.repeat(idx[:, None, :], m, axis=1).reshape(-1)
    Dsp = sp.csr_matrix((D.reshape(-1), (r, c)), shape=Afull.shape)
    Aoff = (Afull - Dsp).tocsr()
    Dinv = np.linalg.inv(D)
    col, nc = fc_colouring(lev)
    out = []
    for k in range(nc):
        nodes = np.nonzero(col == k)[0]
        rows = _node_dofs(lev, nodes)
        out.append((rows, Aoff[rows, :].tocsr(), sp.block_diag(list(Dinv[nodes]), format="csr")))
    return col, out


def spgemm(A: BsrM, B: BsrM) -> BsrM:
    """A B with the ordered sums of seq.c (columns of each row increasing)."""
    lib = _load()
    br, bm = A.val.shape[1], A.val.shape[2]
    bc = B.val.shape[2]
    cap = max(1, sum(int(B.rp[j + 1] - B.rp[j]) for j in A.ci)) if A.ci.shape[0] else 1
    c_rp = np.zeros(A.n_rows + 1, dtype=np.int32)
    c_ci = np.zeros(cap, dtype=np.int32)
    c_val = np.zeros(cap * br * bc)
    nz = lib.or_spgemm(A.n_rows, br, bm, bc, A.rp, A.ci, np.ascontiguousarray(A.val.reshape(-1)), B.rp, B.ci,
                       np.ascontiguousarray(B.val.reshape(-1)), cap, c_rp, c_ci, c_val)
    assert nz >= 0
    return BsrM(A.n_rows, B.n_cols, c_rp, c_ci[:nz].copy(), c_val[:nz * br * bc].reshape(nz, br, bc).copy())


def transpose(P: BsrM) -> BsrM:
    """Block transpose; rows of the result list their columns in increasing order."""
    rows = np.repeat(np.arange(P.n_rows), np.diff(P.rp))
    order = np.lexsort((rows, P.ci))
    cnt = np.bincount(P.ci, minlength=P.n_cols)
    rp = np.zeros(P.n_cols + 1, dtype=np.int32)
    np.cumsum(cnt, out=rp[1:])
    return BsrM(P.n_cols, P.n_rows, rp, rows[order].astype(np.int32),
                np.ascontiguousarray(P.val[order].transpose(0, 2, 1)))


def sa_prolongator(A: BsrM, nv: int, agg: np.ndarray, q: np.ndarray, w: np.ndarray, n_agg: int) -> BsrM:
    """P = Phat - D_vv^-1 A_vv Phat W on the vector components (seq.c)."""
    lib = _load()
    d = A.val.shape[1]
    cap = max(A.ci.shape[0], 1)
    p_rp = np.zeros(A.n_rows + 1, dtype=np.int32)
    p_ci = np.zeros(cap, dtype=np.int32)
    p_val = np.zeros(cap * d * d)
    nz = lib.or_sa_prolongator(A.n_rows, d, nv, A.rp, A.ci, np.ascontiguousarray(A.val.reshape(-1)), agg,
                               np.ascontiguousarray(q.reshape(-1)), np.ascontiguousarray(w, dtype=np.float64),
                               p_rp, p_ci, p_val)
    return BsrM(A.n_rows, n_agg, p_rp, p_ci[:nz].copy(), p_val[:nz * d * d].reshape(nz, d, d).copy())


def tentative_bsr(q: np.ndarray, agg: np.ndarray, n_agg: int) -> BsrM:
    n, d = q.shape
    val = np.zeros((n, d, d))
    val[:, np.arange(d), np.arange(d)] = q
    return BsrM(n, n_agg, np.arange(n + 1, dtype=np.int32), agg.astype(np.int32), val)


def setup(blocks, dofs, params: Params | None = None, n_vec=None) -> Hierarchy:
    """Build the hierarchy.  ``blocks`` is [[A00, A01], [A10, A11]], each an
    object with n_brows, n_bcols, row_ptr, col_idx, vals (the generator's Bsr).

    Coarsening stops when a level has at most max_coarse dofs, when max_levels
    levels exist, or when the next level would keep more than 90% of the nodes.
    """
    p = params or Params()
    n_vec = tuple(n_vec) if n_vec is not None else (dofs[0] - 1, dofs[1] - 1)
    A = [[BsrM(b.n_brows, b.n_bcols, np.asarray(b.row_ptr, np.int32), np.asarray(b.col_idx, np.int32),
               np.asarray(b.vals, np.float64)) for b in row] for row in blocks]
    n = A[0][0].n_rows
    n1 = A[1][1].n_rows
    if p.clone and n1 != n:
        raise ValueError("cloned aggregation needs co-located fields (equal node counts)")
    if not p.clone:
        return _setup_separate(A, dofs, p, n_vec)
    levels = []
    B = [np.ones((n, dofs[0])), np.ones((n, dofs[1]))]
    lvl = 0
    while True:
        lev = Level(n=n, dofs=tuple(dofs), A=A, csr=[[A[f][g].csr() for g in range(2)] for f in range(2)])
        levels.append(lev)
        ndof = n * sum(dofs)
        if ndof <= p.max_coarse or len(levels) >= p.max_levels:
            break
        agg, n_agg = aggregate(A[0][0], p.theta, p.seed, lvl)
        if n_agg > 0.9 * n:
            break
        m_ptr, m_idx = members(agg, n_agg)
        q, Bc = [], []
        for f in range(2):
            qf, bc = tentative(B[f], agg, m_ptr, m_idx)        # block 1 reuses block 0's aggregates
            q.append(qf)
            Bc.append(bc)
        lev.agg, lev.n_agg, lev.m_ptr, lev.m_idx, lev.q = agg, n_agg, m_ptr, m_idx, q
        wp = None
        if p.weights is not None:
            from oracle import learned
            lev.features = learned.features(lev, n_vec, lvl)
            wp, ws = p.weights(lvl, n_agg, lev.features)
            wp = np.asarray(wp, dtype=np.float64)
            lev.omega_s = np.asarray(ws, dtype=np.float64)[agg]
        elif p.omega_p != 0.0:
            wp = np.full(n_agg, float(p.omega_p))
        if wp is None:
            lev.P = [prolongator(q[f], agg, n_agg) for f in range(2)]
            A = [[galerkin(A[f][g], agg, m_ptr, m_idx, n_agg, q[f], q[g]) for g in range(2)] for f in range(2)]
        else:
            lev.omega_p = wp
            Pb = [sa_prolongator(A[f][f], n_vec[f], agg, q[f], wp, n_agg) for f in range(2)]
            lev.P = [Pb[f].csr() for f in range(2)]
            PT = [transpose(Pb[f]) for f in range(2)]
            A = [[spgemm(PT[f], spgemm(A[f][g], Pb[g])) for g in range(2)] for f in range(2)]
        B = Bc
        n = n_agg
        lvl += 1
    return _finish(levels, p)


def _setup_separate(A, dofs, p: Params, n_vec) -> Hierarchy:
    """Hierarchy with each block aggregated from the graph of its own diagonal
    block (Sec. 4.3.1: fields that do not share nodes get a separate AMG setup
    per block): aggregates, tentative P_ff and near-null space per block, the
    transfer P = diag(P00, P11) with P00 != P11, and the Galerkin products of
    all four blocks as P_f^T (A_fg P_g).  Coarsening stops when the level has
    at most max_coarse dofs, at max_levels levels, or when the two blocks'
    aggregates together keep more than 90 % of the level's nodes."""
    if p.weights is not None or p.omega_p != 0.0 or p.smoother != 0:
        raise ValueError("separate aggregation is built for the fixed form with the blocked smoother")
    n = [A[0][0].n_rows, A[1][1].n_rows]
    B = [np.ones((n[0], dofs[0])), np.ones((n[1], dofs[1]))]
    levels = []
    lvl = 0
    while True:
        lev = Level(n=n[0], n1=n[1], dofs=tuple(dofs), A=A,
                    csr=[[A[f][g].csr() for g in range(2)] for f in range(2)])
        levels.append(lev)
        if n[0] * dofs[0] + n[1] * dofs[1] <= p.max_coarse or len(levels) >= p.max_levels:
            break
        aggs = [aggregate(A[f][f], p.theta, p.seed, lvl) for f in range(2)]
        if aggs[0][1] + aggs[1][1] > 0.9 * (n[0] + n[1]):
            break
        Pb, q, Bc = [], [], []
        for f in range(2):
            agg, n_agg = aggs[f]
            m_ptr, m_idx = members(agg, n_agg)
            qf, bc = tentative(B[f], agg, m_ptr, m_idx)
            q.append(qf)
            Bc.append(bc)
            Pb.append(tentative_bsr(qf, agg, n_agg))
        lev.agg, lev.n_agg = aggs[0]
        lev.agg1, lev.n_agg1 = aggs[1]
        lev.m_ptr, lev.m_idx = members(*aggs[0])
        lev.q = q
        lev.P = [Pb[f].csr() for f in range(2)]
        PT = [transpose(Pb[f]) for f in range(2)]
        A = [[spgemm(PT[f], spgemm(A[f][g], Pb[g])) for g in range(2)] for f in range(2)]
        B = Bc
        n = [aggs[0][1], aggs[1][1]]
        lvl += 1
    return _finish(levels, p)


def _finish(levels, p: Params) -> Hierarchy:
    """Smoother data on every level but the last, and the last level's LU."""
    for lev in levels[:-1]:
        lev.colour, lev.n_colours, lev.dinv, lev.gs = [], [], [], []
        for f in range(2):
            col, nc = colouring(lev.A[f][f])
            lev.colour.append(col)
            lev.n_colours.append(nc)
            D = diag_blocks(lev.A[f][f])
            lev.dinv.append(np.linalg.inv(D))
        for f in range(2):
            lev.gs.append(_prepare_gs(lev, f))
        if p.smoother == 1:
            lev.fc_colour, lev.fc = _prepare_fc(lev)
    last = levels[-1]
    Ad = sp.bmat([[last.csr[0][0], last.csr[0][1]], [last.csr[1][0], last.csr[1][1]]]).toarray()
    h = Hierarchy(levels=levels, params=p)
    h.coarse_lu = sla.lu_factor(Ad)
    h.coarse_n = Ad.shape[0]
    return h


# ----------------------------------------------------------------------------
# solve phase
# ----------------------------------------------------------------------------

def _split(lev: Level, v: np.ndarray):
    n0 = lev.n * lev.dofs[0]
    return v[:n0], v[n0:]


def inner_gs(lev: Level, f: int, r: np.ndarray, sweeps: int) -> np.ndarray:
    """Approximate solve of A_ff e = r: multicolour nodal-block Gauss-Seidel
    from e = 0, colours in increasing order; node i of colour c takes
    e_i = D_i^-1 (r_i - sum_{j != i} A_ff[i,j] e_j)."""
    e = np.zeros_like(r)
    for _ in range(sweeps):
        for rows, Aoff_c, Dc in lev.gs[f]:
            e[rows] = Dc @ (r[rows] - Aoff_c @ e)
    return e


def bgs(lev: Level, x0: np.ndarray, x1: np.ndarray, b0, b1, p: Params, omega=None):
    """Damped block Gauss-Seidel, Algorithm 1, starting from the incoming iterate.

    ``omega`` may be a per-node array (one damping per node of the level)."""
    w = p.omega if omega is None else omega
    d0, d1 = lev.dofs
    x0 = x0.copy()
    x1 = x1.copy()
    if omega is None and lev.omega_s is not None:
        w = lev.omega_s
    for _ in range(p.bgs_sweeps):
        r0 = b0 - lev.csr[0][0] @ x0 - lev.csr[0][1] @ x1
        e0 = inner_gs(lev, 0, r0, p.inner_sweeps)
        x0 = x0 + (np.repeat(w, d0) if np.ndim(w) else w) * e0
        r1 = b1 - lev.csr[1][0] @ x0 - lev.csr[1][1] @ x1      # uses the updated x0
        e1 = inner_gs(lev, 1, r1, p.inner_sweeps)
        x1 = x1 + (np.repeat(w, d1) if np.ndim(w) else w) * e1
    return x0, x1


def fc(lev: Level, x0: np.ndarray, x1: np.ndarray, b0, b1, p: Params, omega=None):
    """Damped nodal-block Gauss-Seidel over the full node blocks, the FC-AMG
    analogue the paper compares the blocked smoother with: per sweep
    r = b - A x, then the correction e from zero by multicolour sweeps over the
    full node graph, node i of colour c taking
    e_i = D_i^-1 (r_i - sum_{j != i} A[i, j] e_j) with the (d0+d1)-square node
    blocks of the whole operator, then x += omega e (both fields at once)."""
    w = p.omega if omega is None else omega
    if omega is None and lev.omega_s is not None:
        w = lev.omega_s
    d0, d1 = lev.dofs
    x = np.concatenate([x0, x1])
    b = np.concatenate([b0, b1])
    wv = np.concatenate([np.repeat(w, d0), np.repeat(w, d1)]) if np.ndim(w) else w
    for _ in range(p.bgs_sweeps):
        r = b - apply_A(lev, x)
        e = np.zeros_like(r)
        for _ in range(p.inner_sweeps):
            for rows, Aoff_c, Dc in lev.fc:
                e[rows] = Dc @ (r[rows] - Aoff_c @ e)
        x = x + wv * e
    return _split(lev, x)


def smooth(lev: Level, x0, x1, b0, b1, p: Params):
    """The level's smoother: Algorithm 1 (p.smoother = 0) or the full-node form (1)."""
    return fc(lev, x0, x1, b0, b1, p) if p.smoother == 1 else bgs(lev, x0, x1, b0, b1, p)


def apply_A(lev: Level, x: np.ndarray) -> np.ndarray:
    x0, x1 = _split(lev, x)
    return np.concatenate([lev.csr[0][0] @ x0 + lev.csr[0][1] @ x1,
                           lev.csr[1][0] @ x0 + lev.csr[1][1] @ x1])


def apply_rows(blocks, dofs, x: np.ndarray, nodes: np.ndarray, absolute: bool = False) -> np.ndarray:
    """(A x) on the given nodes' rows of both fields, straight from the
    definition of the 2x2 block system (Sec. 4.2, eq. 2x2system): for node i
    of field f, sum over g and over the blocks A_fg[i, j] of row i of
    A_fg[i, j] x_g[j].  With ``absolute`` the same sums of |A| |x| (the scale
    of the rounding error of any evaluation order).  Returns an array
    (len(nodes), dofs[0] + dofs[1])."""
    N = blocks[0][0].n_brows
    xs = [x[:N * dofs[0]].reshape(N, dofs[0]), x[N * dofs[0]:].reshape(N, dofs[1])]
    out = np.zeros((len(nodes), dofs[0] + dofs[1]))
    for k, i in enumerate(np.asarray(nodes)):
        for f in range(2):
            acc = np.zeros(dofs[f])
            for g in range(2):
                B = blocks[f][g]
                for p in range(B.row_ptr[i], B.row_ptr[i + 1]):
                    if absolute:
                        acc += np.abs(B.vals[p]) @ np.abs(xs[g][B.col_idx[p]])
                    else:
                        acc += B.vals[p] @ xs[g][B.col_idx[p]]
            out[k, (0 if f == 0 else dofs[0]):(dofs[0] if f == 0 else dofs[0] + dofs[1])] = acc
    return out


def mgv(h: Hierarchy, lvl: int, b: np.ndarray) -> np.ndarray:
    """One V-cycle from a zero initial guess (Sec. 3, the MGV figure)."""
    lev = h.levels[lvl]
    if lvl == len(h.levels) - 1:
        return sla.lu_solve(h.coarse_lu, b)
    b0, b1 = _split(lev, b)
    z = np.zeros(lev.n * lev.dofs[0])
    x0, x1 = smooth(lev, z, np.zeros(lev.n1 * lev.dofs[1]), b0, b1, h.params)
    u = np.concatenate([x0, x1])
    r = b - apply_A(lev, u)
    r0, r1 = _split(lev, r)
    bc = np.concatenate([lev.P[0].T @ r0, lev.P[1].T @ r1])
    uc = mgv(h, lvl + 1, bc)
    nxt = h.levels[lvl + 1]
    nc0 = nxt.n * nxt.dofs[0]
    x0 = x0 + lev.P[0] @ uc[:nc0]
    x1 = x1 + lev.P[1] @ uc[nc0:]
    x0, x1 = smooth(lev, x0, x1, b0, b1, h.params)
    return np.concatenate([x0, x1])


def vcycle(h: Hierarchy, r: np.ndarray) -> np.ndarray:
    """z = M^-1 r, one V-cycle on the finest level."""
    return mgv(h, 0, np.asarray(r, dtype=np.float64))


@dataclasses.dataclass
class SolveInfo:
    iterations: int
    converged: bool
    rel_residual: float
    history: list


def gmres(h, b: np.ndarray, rtol: float = 1e-8, restart: int = 30,
          max_iters: int = 1000, precond=None, operator=None) -> tuple:
    """Restarted GMRES, right preconditioned by one V-cycle, x0 = 0.

    Stops when the recurrence residual |g_{j+1}| <= rtol*||b||, then confirms
    with the true residual and restarts if that test fails.  ``precond`` and
    ``operator`` replace the V-cycle and the operator apply of ``h`` (which may
    then be None).
    """
    M = precond or (lambda v: vcycle(h, v))
    A = operator or (lambda v: apply_A(h.levels[0], v))
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    its = 0
    hist = []
    if bnorm == 0.0:
        return x, SolveInfo(0, True, 0.0, hist)
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            return x, SolveInfo(its, True, beta / bnorm, hist)
        if its >= max_iters:
            return x, SolveInfo(its, False, beta / bnorm, hist)
        m = restart
        V = np.zeros((m + 1, b.shape[0]))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = A(M(V[j]))
            for i in range(j + 1):                   # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                       # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or its >= max_iters:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + M(V[:k].T @ y)


def seeded_vector(n: int, seed: int) -> np.ndarray:
    """Start vector of the convergence probe: 2 u - 1 with u the top 53 bits of
    the SplitMix64 output finaliser of i + 0x9E3779B97F4A7C15 * (seed + 1)."""
    mult = (0x9E3779B97F4A7C15 * (seed + 1)) & ((1 << 64) - 1)
    with np.errstate(over="ignore"):
        z = _mix64(np.arange(n, dtype=np.uint64) + np.uint64(mult))
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0


def probe(h: Hierarchy, iters: int = 10, seed: int = 12345) -> float:
    """Asymptotic factor of the stationary iteration e <- e - M A e:
    (||e_iters|| / ||e_{iters-4}||)^(1/4)."""
    lev = h.levels[0]
    e = seeded_vector(lev.n_dofs(), seed)
    n4 = nk = 0.0
    for k in range(1, iters + 1):
        e = e - vcycle(h, apply_A(lev, e))
        if k == iters - 4:
            n4 = np.linalg.norm(e)
        if k == iters:
            nk = np.linalg.norm(e)
    return (nk / n4) ** 0.25
