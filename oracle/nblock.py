"""Oracle for block systems of more than two blocks -- TEST INFRASTRUCTURE ONLY.

The general n_b x n_b block form of the problem (Sec. 4.1, eq.
block-prec-form), here with the four co-located fields of the 4 x 4 split of
Sec. 2.1 as the case in view.  Plain FP64 NumPy/SciPy on the sequential
primitives of ``amg`` (aggregation, tentative interpolation, ordered Galerkin
sums, colouring), written to follow the paper:

* aggregates from the strong graph of A_00 (the first field's diagonal
  block), cloned to every block (Sec. 4.3.1), and a piecewise-constant P_f per
  block over them, P = diag(P_00, ..., P_(n_b-1)(n_b-1)) (eq. blocktransfers);
* coarse operators A^c_fg = P_f^T A_fg P_g for all n_b^2 pairs (Sec. 3);
* smoother: Algorithm 1 (Sec. 4.3.2) over n_b blocks -- for f = 0, 1, ...:
  r_f = b_f - sum_g A_fg x_g with the blocks before f already updated in this
  sweep, e_f from multicolour nodal-block Gauss-Seidel on A_ff from zero,
  x_f += omega e_f;
* the V-cycle of the MGV figure (Sec. 3) with a direct solve on the last level.

Coarsening stops at max_coarse dofs, max_levels levels, or when aggregation
would keep more than 90 % of the nodes (as for two blocks).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import amg


@dataclasses.dataclass
class NLevel:
    n: int                  # nodes (every field on every node)
    dofs: tuple             # dofs per node of each block
    A: list                 # n_b x n_b BsrM (entries with no stored block have nnz 0)
    csr: list
    agg: np.ndarray = None
    n_agg: int = 0
    P: list = None          # per block, scalar CSR
    colour: list = None
    gs: list = None         # per block: list over colours of (rows, off-diagonal rows of A_ff, D^-1)

    @property
    def nb(self) -> int:
        return len(self.dofs)

    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([self.n * d for d in self.dofs])])


@dataclasses.dataclass
class NHierarchy:
    levels: list
    params: amg.Params
    coarse_lu: tuple = None


def _bsr(b) -> amg.BsrM:
    vals = np.asarray(b.vals, np.float64)
    return amg.BsrM(b.n_brows, b.n_bcols, np.asarray(b.row_ptr, np.int32), np.asarray(b.col_idx, np.int32), vals)


def _prepare_gs(lev: NLevel, f: int):
    d = lev.dofs[f]
    Aff = lev.csr[f][f]
    D = amg.diag_blocks(lev.A[f][f])
    Dsp = sp.block_diag(list(D), format="csr")
    Aoff = (Aff - Dsp).tocsr()
    Dinv = np.linalg.inv(D)
    out = []
    for c in range(int(lev.colour[f].max()) + 1):
        nodes = np.nonzero(lev.colour[f] == c)[0]
        rows = (nodes[:, None] * d + np.arange(d)[None, :]).reshape(-1)
        out.append((rows, Aoff[rows, :].tocsr(), sp.block_diag(list(Dinv[nodes]), format="csr")))
    return out


def setup(blocks, dofs, params: amg.Params | None = None) -> NHierarchy:
    """``blocks``: n_b x n_b generator blocks (n_brows = n_bcols = nodes;
    a block with nnzb 0 is a zero block)."""
    p = params or amg.Params()
    if p.weights is not None or p.omega_p != 0.0 or p.smoother != 0 or not p.clone:
        raise ValueError("the n_b-block oracle builds the fixed form with cloned aggregates")
    nb = len(dofs)
    A = [[_bsr(blocks[f][g]) for g in range(nb)] for f in range(nb)]
    n = A[0][0].n_rows
    B = [np.ones((n, d)) for d in dofs]
    levels = []
    lvl = 0
    while True:
        lev = NLevel(n=n, dofs=tuple(dofs), A=A, csr=[[A[f][g].csr() for g in range(nb)] for f in range(nb)])
        levels.append(lev)
        if n * sum(dofs) <= p.max_coarse or len(levels) >= p.max_levels:
            break
        agg, n_agg = amg.aggregate(A[0][0], p.theta, p.seed, lvl)
        if n_agg > 0.9 * n:
            break
        m_ptr, m_idx = amg.members(agg, n_agg)
        q, Bc = [], []
        for f in range(nb):
            qf, bc = amg.tentative(B[f], agg, m_ptr, m_idx)
            q.append(qf)
            Bc.append(bc)
        lev.agg, lev.n_agg = agg, n_agg
        lev.P = [amg.prolongator(q[f], agg, n_agg) for f in range(nb)]
        A = [[amg.galerkin(A[f][g], agg, m_ptr, m_idx, n_agg, q[f], q[g]) for g in range(nb)] for f in range(nb)]
        B = Bc
        n = n_agg
        lvl += 1
    for lev in levels[:-1]:
        lev.colour = [amg.colouring(lev.A[f][f])[0] for f in range(nb)]
        lev.gs = [_prepare_gs(lev, f) for f in range(nb)]
    last = levels[-1]
    Ad = sp.bmat(last.csr).toarray()
    return NHierarchy(levels=levels, params=p, coarse_lu=sla.lu_factor(Ad))


def split(lev: NLevel, v: np.ndarray) -> list:
    o = lev.offsets()
    return [v[o[f]:o[f + 1]] for f in range(lev.nb)]


def apply_A(lev: NLevel, x: np.ndarray) -> np.ndarray:
    xs = split(lev, x)
    return np.concatenate([sum(lev.csr[f][g] @ xs[g] for g in range(lev.nb)) for f in range(lev.nb)])


def bgs(lev: NLevel, x: list, b: list, p: amg.Params) -> list:
    """Algorithm 1 over the level's n_b blocks from the incoming iterate."""
    x = [xi.copy() for xi in x]
    for _ in range(p.bgs_sweeps):
        for f in range(lev.nb):
            r = b[f] - sum(lev.csr[f][g] @ x[g] for g in range(lev.nb))
            e = np.zeros_like(r)
            for _ in range(p.inner_sweeps):
                for rows, Aoff_c, Dc in lev.gs[f]:
                    e[rows] = Dc @ (r[rows] - Aoff_c @ e)
            x[f] = x[f] + p.omega * e
    return x


def mgv(h: NHierarchy, lvl: int, b: np.ndarray) -> np.ndarray:
    lev = h.levels[lvl]
    if lvl == len(h.levels) - 1:
        return sla.lu_solve(h.coarse_lu, b)
    bs = split(lev, b)
    x = bgs(lev, [np.zeros_like(bi) for bi in bs], bs, h.params)
    r = b - apply_A(lev, np.concatenate(x))
    rs = split(lev, r)
    uc = mgv(h, lvl + 1, np.concatenate([lev.P[f].T @ rs[f] for f in range(lev.nb)]))
    ucs = split(h.levels[lvl + 1], uc)
    x = [x[f] + lev.P[f] @ ucs[f] for f in range(lev.nb)]
    x = bgs(lev, x, bs, h.params)
    return np.concatenate(x)


def vcycle(h: NHierarchy, r: np.ndarray) -> np.ndarray:
    return mgv(h, 0, np.asarray(r, dtype=np.float64))


def gmres(h: NHierarchy, b: np.ndarray, rtol: float = 1e-8, restart: int = 30, max_iters: int = 1000):
    return amg.gmres(None, b, rtol=rtol, restart=restart, max_iters=max_iters,
                     precond=lambda v: vcycle(h, v), operator=lambda v: apply_A(h.levels[0], v))
