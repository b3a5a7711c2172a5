"""Seeded synthetic two-field block systems (inputs only, no multigrid arithmetic).

The paper's matrices come from a stabilised finite-element resistive-MHD code
that is not available, so the workloads are synthetic stand-ins with the same
algebraic structure: co-located multi-field nodes (Sec. 4.3.1: all fields on
the same nodal mesh) grouped into a 2x2 block system (Sec. 4.2, eq. 2x2system)
whose diagonal blocks are saddle-point systems (velocity/pressure and
magnetic-field/multiplier) and whose off-diagonal blocks couple the two
physics (Sec. 2.1, the 4x4 block Jacobian).

Per block f, node i carries ``dim`` vector dofs and one scalar dof, so a node
block is (dim+1) x (dim+1):

* vector-vector: -div(kappa grad) + reaction, 5/7-point stencil per component,
  edge coefficient = harmonic mean of the nodal kappas, Dirichlet edges use
  kappa_i with a zero outside value;
* vector-scalar: central-difference gradient G;
* scalar-vector: central-difference divergence D = -G^T;
* scalar-scalar: tau * (2*dim on the diagonal, -1 per in-grid neighbour).

Coupling A01 (u rows x b columns) and A10 (b rows x u columns) are the
nearest-neighbour skew operator Z[(i,a),(j,a)] = gamma*g(m_ij)*s_ij/(2h) on the
vector components only, so the symmetric part of the whole matrix is
block-diagonal and positive definite (the system is positive-real).

Random numbers come from a counter-based SplitMix64 (Steele, Lea & Flood,
2014): value(seed, stream, index) is the output of a SplitMix64 sequence whose
start is derived from (seed, stream), taken at position index+1. Streams:
1 = smooth coupling field g, 2 = lognormal kappa, 3 = right-hand side.

Every array is returned in the layout the C-ABI takes: BSR with int32 row
pointers and sorted int32 column indices, FP64 blocks row-major, and vectors
blocked as [x0; x1] with x_f[node*d_f + component].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM_MUL = 0xD1B54A32D192ED03
_MASK64 = (1 << 64) - 1


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser on a uint64 array (wrapping arithmetic)."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _MASK64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _MASK64
    z ^= z >> 31
    return z


def rng_u64(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Counter-based SplitMix64 draw for each entry of ``index`` (int64 >= 0)."""
    base = _mix64_int((seed & _MASK64) ^ ((stream * _STREAM_MUL) & _MASK64))
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64(base) + (idx + np.uint64(1)) * _GAMMA
    return _mix64(ctr)


def rng_uniform(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Uniform [0, 1) from the top 53 bits."""
    return (rng_u64(seed, stream, index) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def rng_normal(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Standard normal by Box-Muller on uniforms at counters 2*index, 2*index+1."""
    idx = np.asarray(index, dtype=np.int64)
    u1 = rng_uniform(seed, stream, 2 * idx)
    u2 = rng_uniform(seed, stream, 2 * idx + 1)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


@dataclasses.dataclass
class Bsr:
    """Block-sparse rows: row_ptr[n_brows+1], col_idx[nnzb], vals[nnzb, br, bc]."""
    n_brows: int
    n_bcols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray

    @property
    def br(self) -> int:
        return int(self.vals.shape[1])

    @property
    def bc(self) -> int:
        return int(self.vals.shape[2])

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.bsr_matrix((self.vals, self.col_idx, self.row_ptr),
                             shape=(self.n_brows * self.br, self.n_bcols * self.bc)).tocsr()


@dataclasses.dataclass
class BlockSystem:
    """A 2x2 block system A x = b: block 0 on N nodes, block 1 on N1 nodes
    (N1 = N when the fields are co-located)."""
    dim: int
    n: int
    N: int
    dofs: tuple          # dofs per node of each block
    n_vec: tuple         # leading vector components per block
    blocks: list         # [[A00, A01], [A10, A11]] as Bsr
    b: np.ndarray        # [b0; b1]
    params: dict
    N1: int = -1         # nodes of block 1 (-1: N)

    def __post_init__(self):
        if self.N1 < 0:
            self.N1 = self.N

    @property
    def nodes(self) -> tuple:
        return (self.N, self.N1)

    @property
    def co_located(self) -> bool:
        return self.N1 == self.N

    @property
    def n_dofs(self) -> int:
        return self.N * self.dofs[0] + self.N1 * self.dofs[1]

    def to_scipy(self):
        """Monolithic scalar CSR in the blocked [x0; x1] ordering."""
        import scipy.sparse as sp
        return sp.bmat([[self.blocks[0][0].to_scipy(), self.blocks[0][1].to_scipy()],
                        [self.blocks[1][0].to_scipy(), self.blocks[1][1].to_scipy()]],
                       format="csr")


def _offsets(n: int, dim: int):
    """Neighbour slots ordered by column offset: (axis, sign) with sign=0 for the node itself."""
    slots = []
    for axis in reversed(range(dim)):
        slots.append((axis, -1))
    slots.append((None, 0))
    for axis in range(dim):
        slots.append((axis, +1))
    return slots


def _coupling_field(n: int, dim: int, seed: int, h: float):
    """Smooth random field g on the edge midpoints, scaled so max |g| = 1.

    g~(x) = sum over k in {1..4}^dim of a_k prod_a cos(pi k_a x_a + phi_{k,a}),
    a_k ~ N(0,1)/|k|^2, phi ~ U[0, 2pi).  Returns, for each axis e, an array of
    shape (n,)*dim whose entry at node i is g at the midpoint of edge (i, i+e_e)
    (the last layer along e is unused).
    """
    modes = np.array(np.meshgrid(*([np.arange(1, 5)] * dim), indexing="ij")).reshape(dim, -1).T
    nm = modes.shape[0]
    amp = rng_normal(seed, 1, np.arange(nm)) / np.sum(modes.astype(np.float64) ** 2, axis=1)
    phase = 2.0 * math.pi * rng_uniform(seed, 1, 1_000_000 + np.arange(nm * dim)).reshape(nm, dim)
    node_x = (np.arange(n) + 1.0) * h
    mid_x = (np.arange(n) + 1.5) * h
    out = []
    for e in range(dim):
        g = np.zeros((n,) * dim)
        for m in range(nm):
            term = None
            for a in range(dim):
                xs = mid_x if a == e else node_x
                c = np.cos(math.pi * modes[m, a] * xs + phase[m, a])
                shape = [1] * dim
                shape[dim - 1 - a] = n          # node index = ix + n*iy (+ n^2*iz): x is the last array axis
                c = c.reshape(shape)
                term = c if term is None else term * c
            g += amp[m] * term
        out.append(g)
    # normalise over in-grid edges only
    gmax = 0.0
    for e in range(dim):
        sl = [slice(None)] * dim
        sl[dim - 1 - e] = slice(0, n - 1)
        gmax = max(gmax, float(np.max(np.abs(out[e][tuple(sl)]))))
    return [g / gmax for g in out]


def make_system(n: int, dim: int, gamma: float, *, seed: int = 1, kappa: str = "const",
                sigma: float = 1.0, tau: float = 1.0, reaction: float = 1.0,
                blk1_scale: float = 1.0, a10_scale: float = 1.0, node_coupling: float = 0.0) -> BlockSystem:
    """Build the seeded 2x2 block system on an n^dim grid of interior nodes.

    ``blk1_scale`` scales the vector Laplacian of block 1 and ``a10_scale``
    scales A10 relative to A01; both default to 1 (the workload reading) and
    exist so tests can tell the four blocks apart.

    ``node_coupling`` = c > 0 adds a coupling inside every node between the
    two blocks' vector components (a cross-product-like term, as the u x B
    terms of the MHD Jacobian couple fields at one point):
    Z[(i,a),(i,b)] = c w_i (2 dim / h^2) K[a][b] with K the skew matrix
    [[0, 1], [-1, 0]] (2D) or [[0, 1, -1], [-1, 0, 1], [1, -1, 0]] (3D) and
    w_i ~ U[0.5, 1) (stream 4), so c measures the term against the vector
    Laplacian's diagonal; Z stays skew, so A stays positive-real.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    h = 1.0 / (n + 1)
    N = n ** dim
    d = dim + 1
    idx = np.arange(N, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for a in range(dim):
        coords.append(rem % n)
        rem //= n
    strides = [n ** a for a in range(dim)]

    if kappa == "const":
        kap = np.ones(N)
    elif kappa == "lognormal":
        kap = np.exp(sigma * rng_normal(seed, 2, idx))
    else:
        raise ValueError(kappa)
    gfield = [g.reshape(-1) for g in _coupling_field(n, dim, seed, h)] if gamma != 0.0 else None

    slots = _offsets(n, dim)
    ns = len(slots)
    valid = np.zeros((N, ns), dtype=bool)
    cols = np.zeros((N, ns), dtype=np.int64)
    kedge = np.zeros((N, ns))          # edge kappa for neighbour slots
    sgn = np.zeros(ns)
    gz = np.zeros((N, ns))             # coupling value per neighbour slot
    diag_lap = np.zeros(N)             # sum of edge kappas, including Dirichlet edges
    nbr_count = np.zeros(N)
    for s, (axis, sign) in enumerate(slots):
        if sign == 0:
            valid[:, s] = True
            cols[:, s] = idx
            continue
        ci = coords[axis] + sign
        inside = (ci >= 0) & (ci < n)
        j = idx + sign * strides[axis]
        valid[:, s] = inside
        cols[:, s] = np.where(inside, j, idx)
        kj = kap[np.where(inside, j, idx)]
        ke = np.where(inside, 2.0 * kap * kj / (kap + kj), kap)
        kedge[:, s] = np.where(inside, ke, 0.0)
        diag_lap += ke
        nbr_count += inside
        sgn[s] = sign
        if gfield is not None:
            # midpoint of edge (i, j): stored at the lower endpoint along the axis
            lower = np.where(sign > 0, idx, np.where(inside, j, idx))
            gz[:, s] = np.where(inside, gfield[axis][lower], 0.0)

    inv_h2 = 1.0 / (h * h)
    inv_2h = 1.0 / (2.0 * h)

    def saddle_block(lap_scale: float) -> Bsr:
        v = np.zeros((N, ns, d, d))
        for s, (axis, sign) in enumerate(slots):
            if sign == 0:
                for a in range(dim):
                    v[:, s, a, a] = lap_scale * diag_lap * inv_h2 + reaction
                v[:, s, dim, dim] = tau * 2.0 * dim
            else:
                m = valid[:, s]
                for a in range(dim):
                    v[:, s, a, a] = -lap_scale * kedge[:, s] * inv_h2
                v[:, s, axis, dim] = np.where(m, sign * inv_2h, 0.0)
                v[:, s, dim, axis] = np.where(m, sign * inv_2h, 0.0)
                v[:, s, dim, dim] = np.where(m, -tau, 0.0)
        return _compress(N, valid, cols, v)

    skew = np.array([[0.0, 1.0], [-1.0, 0.0]]) if dim == 2 else \
        np.array([[0.0, 1.0, -1.0], [-1.0, 0.0, 1.0], [1.0, -1.0, 0.0]])
    wnode = 0.5 + 0.5 * rng_uniform(seed, 4, idx) if node_coupling != 0.0 else None

    def coupling_block(scale: float) -> Bsr:
        nb = [s for s, (axis, sign) in enumerate(slots) if sign != 0 or node_coupling != 0.0]
        v = np.zeros((N, len(nb), d, d))
        for t, s in enumerate(nb):
            if slots[s][1] == 0:
                c = scale * node_coupling * (2.0 * dim) * inv_h2 * wnode
                v[:, t, :dim, :dim] = c[:, None, None] * skew
                continue
            z = scale * gamma * gz[:, s] * sgn[s] * inv_2h
            for a in range(dim):
                v[:, t, a, a] = z
        return _compress(N, valid[:, nb], cols[:, nb], v)

    A00 = saddle_block(1.0)
    A11 = A00 if blk1_scale == 1.0 else saddle_block(blk1_scale)
    A01 = coupling_block(1.0)
    A10 = A01 if a10_scale == 1.0 else coupling_block(a10_scale)
    b = 2.0 * rng_uniform(seed, 3, np.arange(2 * N * d)) - 1.0
    params = dict(n=n, dim=dim, gamma=gamma, seed=seed, kappa=kappa, sigma=sigma, tau=tau,
                  reaction=reaction, blk1_scale=blk1_scale, a10_scale=a10_scale, node_coupling=node_coupling)
    return BlockSystem(dim=dim, n=n, N=N, dofs=(d, d), n_vec=(dim, dim),
                       blocks=[[A00, A01], [A10, A11]], b=b, params=params)


def make_mixed_system(n: int, dim: int, gamma: float, *, seed: int = 1, kappa: str = "const",
                      sigma: float = 1.0, tau: float = 1.0, reaction: float = 1.0) -> BlockSystem:
    """The same two saddle blocks with block 1 on a grid twice as coarse, the
    synthetic counterpart of a mixed discretisation whose fields live on
    different node sets (block 0 on the finer nodes, block 1 on the coarser).

    n must be odd: block 0 has n^dim interior nodes with spacing h = 1/(n+1),
    block 1 has m^dim with m = (n-1)/2 and spacing 2h; coarse node J sits on
    fine node 2J+1 along each axis.  kappa is drawn on the fine nodes and read
    at the coincident ones for block 1.  Coupling: block-0 vector component a
    at fine node i couples to block-1 component a at the coarse nodes of the
    (multi)linear interpolation stencil of x_i, Z[(i,a),(J,a)] =
    gamma g(i) phi_J(x_i) / (2h) with g the smooth seeded field of the
    co-located generator; A01 = Z and A10 = -Z^T, so the coupling part of A is
    skew and its symmetric part is the two saddle blocks' (A is positive-real).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n % 2 != 1 or n < 3:
        raise ValueError("the mixed system needs an odd n >= 3")
    m = (n - 1) // 2
    fine = make_system(n, dim, gamma, seed=seed, kappa=kappa, sigma=sigma, tau=tau, reaction=reaction)
    h = 1.0 / (n + 1)
    N, N1 = n ** dim, m ** dim
    d = dim + 1
    # block 1: the saddle block on the coarse grid with kappa read at the coincident fine nodes
    cidx = np.arange(N1, dtype=np.int64)
    ccoords, rem = [], cidx.copy()
    for a in range(dim):
        ccoords.append(rem % m)
        rem //= m
    fine_of_coarse = sum((2 * ccoords[a] + 1) * n ** a for a in range(dim))
    if kappa == "const":
        kap_f = np.ones(N)
    else:
        kap_f = np.exp(sigma * rng_normal(seed, 2, np.arange(N, dtype=np.int64)))
    coarse = _saddle_on_grid(m, dim, kap_f[fine_of_coarse], tau, reaction)
    # coupling: fine node i, coarse nodes of its interpolation stencil
    idx = np.arange(N, dtype=np.int64)
    coords, rem = [], idx.copy()
    for a in range(dim):
        coords.append(rem % n)
        rem //= n
    per_axis = []            # per axis: list of (coarse index, weight) candidates for each fine index
    for a in range(dim):
        ia = coords[a]
        odd = ia % 2 == 1
        j_lo = np.where(odd, (ia - 1) // 2, ia // 2 - 1)
        j_hi = np.where(odd, (ia - 1) // 2, ia // 2)
        w = np.where(odd, 1.0, 0.5)
        per_axis.append([(j_lo, w, np.ones(N, bool)), (j_hi, w, ~odd)])
    gfield = _coupling_field(n, dim, seed, h)[0].reshape(-1) if gamma != 0.0 else np.zeros(N)
    rows, cols, wts = [], [], []
    import itertools
    for choice in itertools.product(range(2), repeat=dim):
        J = np.zeros(N, dtype=np.int64)
        wgt = np.ones(N)
        ok = np.ones(N, bool)
        for a, c in enumerate(choice):
            j, w, use = per_axis[a][c]
            ok &= use & (j >= 0) & (j < m)
            J += np.clip(j, 0, m - 1) * m ** a
            wgt *= w
        rows.append(idx[ok])
        cols.append(J[ok])
        wts.append(wgt[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    wts = np.concatenate(wts)
    order = np.lexsort((cols, rows))
    rows, cols, wts = rows[order], cols[order], wts[order]
    zval = gamma * gfield[rows] * wts / (2.0 * h)
    vals = np.zeros((rows.shape[0], d, d))
    for a in range(dim):
        vals[:, a, a] = zval
    rp = np.zeros(N + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    A01 = Bsr(n_brows=N, n_bcols=N1, row_ptr=rp, col_idx=cols.astype(np.int32), vals=vals)
    A10 = _negative_transpose(A01)
    b = 2.0 * rng_uniform(seed, 3, np.arange(N * d + N1 * d)) - 1.0
    params = dict(n=n, dim=dim, gamma=gamma, seed=seed, kappa=kappa, sigma=sigma, tau=tau, reaction=reaction,
                  mixed=True)
    return BlockSystem(dim=dim, n=n, N=N, dofs=(d, d), n_vec=(dim, dim),
                       blocks=[[fine.blocks[0][0], A01], [A10, coarse]], b=b, params=params, N1=N1)


@dataclasses.dataclass
class NBlockSystem:
    """A block system of n_b co-located fields: blocks[f][g] couples field f's
    dofs (dofs[f] per node) to field g's; b = [b_0; ...; b_(n_b-1)], each
    segment node-major."""
    dim: int
    n: int
    N: int
    dofs: tuple
    n_vec: tuple
    blocks: list
    b: np.ndarray
    params: dict

    @property
    def n_dofs(self) -> int:
        return self.N * sum(self.dofs)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.bmat([[blk.to_scipy() for blk in row] for row in self.blocks], format="csr")


def leading_components(s: BlockSystem, k: int) -> BlockSystem:
    """The 2 x 2 system restricted to the first k components of every node of
    both blocks (a principal submatrix, so positive real when s is): two
    blocks of k dofs per node, for 1 <= k <= the blocks' dofs.  Every stored
    node block is kept (possibly zero), so the block patterns do not change."""
    if not s.co_located or s.dofs[0] != s.dofs[1] or not 1 <= k <= s.dofs[0]:
        raise ValueError("co-located blocks with at least k dofs per node")
    blocks = [[Bsr(n_brows=B.n_brows, n_bcols=B.n_bcols, row_ptr=B.row_ptr.copy(), col_idx=B.col_idx.copy(),
                   vals=np.ascontiguousarray(B.vals[:, :k, :k])) for B in row] for row in s.blocks]
    d = s.dofs[0]
    b0 = s.b[:s.N * d].reshape(s.N, d)[:, :k]
    b1 = s.b[s.N * d:].reshape(s.N, d)[:, :k]
    return BlockSystem(dim=s.dim, n=s.n, N=s.N, dofs=(k, k), n_vec=(min(s.n_vec[0], k), min(s.n_vec[1], k)),
                       blocks=blocks, b=np.concatenate([b0.reshape(-1), b1.reshape(-1)]),
                       params=dict(s.params, components=k))


def split_fields(s: BlockSystem, split_second: bool = True) -> NBlockSystem:
    """The 4 x 4 field split of a co-located 2 x 2 system: each block's vector
    and scalar components become fields of their own -- (u, p, b, r), with
    dim, 1, dim and 1 dofs per node (split_second False: (u, p, [b, r]), three
    fields).  A block between two fields stores a node pair only where its
    sub-block has a nonzero entry; a field pair with no such entry is a zero
    block."""
    if not s.co_located:
        raise ValueError("the field split needs co-located blocks")
    dim = s.dim
    comps = [(0, list(range(dim))), (0, [dim])]
    comps += [(1, list(range(dim))), (1, [dim])] if split_second else [(1, list(range(dim + 1)))]
    blocks = []
    for F, rsel in comps:
        row = []
        for G, csel in comps:
            B = s.blocks[F][G]
            sub = B.vals[:, rsel, :][:, :, csel]
            keep = np.any(sub != 0.0, axis=(1, 2))
            rows = np.repeat(np.arange(B.n_brows), np.diff(B.row_ptr))[keep]
            rp = np.zeros(B.n_brows + 1, dtype=np.int32)
            np.add.at(rp, rows + 1, 1)
            rp = np.cumsum(rp).astype(np.int32)
            vals = np.ascontiguousarray(sub[keep])
            if vals.shape[0] == 0:
                vals = np.zeros((0, len(rsel), len(csel)))
            row.append(Bsr(n_brows=B.n_brows, n_bcols=B.n_bcols, row_ptr=rp,
                           col_idx=np.ascontiguousarray(B.col_idx[keep]).astype(np.int32), vals=vals))
        blocks.append(row)
    N = s.N
    d0 = s.dofs[0]
    b0 = s.b[:N * d0].reshape(N, d0)
    b1 = s.b[N * d0:].reshape(N, s.dofs[1])
    if split_second:
        b = np.concatenate([b0[:, :dim].reshape(-1), b0[:, dim], b1[:, :dim].reshape(-1), b1[:, dim]])
        dofs, n_vec, name = (dim, 1, dim, 1), (dim, 0, dim, 0), "u,p,b,r"
    else:
        b = np.concatenate([b0[:, :dim].reshape(-1), b0[:, dim], b1.reshape(-1)])
        dofs, n_vec, name = (dim, 1, dim + 1), (dim, 0, dim), "u,p,br"
    return NBlockSystem(dim=dim, n=s.n, N=N, dofs=dofs, n_vec=n_vec, blocks=blocks, b=b,
                        params=dict(s.params, split=name))


def _saddle_on_grid(n: int, dim: int, kap: np.ndarray, tau: float, reaction: float) -> Bsr:
    """The saddle block of make_system on an n^dim grid (spacing 1/(n+1)) for
    given nodal kappa values."""
    h = 1.0 / (n + 1)
    N = n ** dim
    d = dim + 1
    idx = np.arange(N, dtype=np.int64)
    coords, rem = [], idx.copy()
    for a in range(dim):
        coords.append(rem % n)
        rem //= n
    strides = [n ** a for a in range(dim)]
    slots = _offsets(n, dim)
    ns = len(slots)
    valid = np.zeros((N, ns), dtype=bool)
    cols = np.zeros((N, ns), dtype=np.int64)
    kedge = np.zeros((N, ns))
    diag_lap = np.zeros(N)
    for s, (axis, sign) in enumerate(slots):
        if sign == 0:
            valid[:, s] = True
            cols[:, s] = idx
            continue
        ci = coords[axis] + sign
        inside = (ci >= 0) & (ci < n)
        j = idx + sign * strides[axis]
        valid[:, s] = inside
        cols[:, s] = np.where(inside, j, idx)
        kj = kap[np.where(inside, j, idx)]
        ke = np.where(inside, 2.0 * kap * kj / (kap + kj), kap)
        kedge[:, s] = np.where(inside, ke, 0.0)
        diag_lap += ke
    inv_h2, inv_2h = 1.0 / (h * h), 1.0 / (2.0 * h)
    v = np.zeros((N, ns, d, d))
    for s, (axis, sign) in enumerate(slots):
        if sign == 0:
            for a in range(dim):
                v[:, s, a, a] = diag_lap * inv_h2 + reaction
            v[:, s, dim, dim] = tau * 2.0 * dim
        else:
            mk = valid[:, s]
            for a in range(dim):
                v[:, s, a, a] = -kedge[:, s] * inv_h2
            v[:, s, axis, dim] = np.where(mk, sign * inv_2h, 0.0)
            v[:, s, dim, axis] = np.where(mk, sign * inv_2h, 0.0)
            v[:, s, dim, dim] = np.where(mk, -tau, 0.0)
    return _compress(N, valid, cols, v)


def _negative_transpose(A: Bsr) -> Bsr:
    """-A^T of a BSR block (blocks transposed, columns sorted within rows)."""
    rows = np.repeat(np.arange(A.n_brows), np.diff(A.row_ptr))
    cols = A.col_idx.astype(np.int64)
    order = np.lexsort((rows, cols))
    rp = np.zeros(A.n_bcols + 1, dtype=np.int64)
    np.add.at(rp, cols + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = -np.transpose(A.vals[order], (0, 2, 1)).copy()
    return Bsr(n_brows=A.n_bcols, n_bcols=A.n_brows, row_ptr=rp, col_idx=rows[order].astype(np.int32), vals=vals)


def _compress(N: int, valid: np.ndarray, cols: np.ndarray, v: np.ndarray) -> Bsr:
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int32)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid].astype(np.int32)
    vals = np.ascontiguousarray(v[valid])
    return Bsr(n_brows=N, n_bcols=N, row_ptr=row_ptr, col_idx=col_idx, vals=vals)


# Named workloads (sizes and coefficients of the five benchmark configurations).
WORKLOADS = {
    "2d-32": dict(n=32, dim=2, gamma=0.1, kappa="const"),
    "2d-256": dict(n=256, dim=2, gamma=0.5, kappa="const"),
    "3d-64": dict(n=64, dim=3, gamma=0.5, kappa="const"),
    "2d-512-lognormal": dict(n=512, dim=2, gamma=5.0, kappa="lognormal", sigma=1.0),
    "2d-64-lognormal": dict(n=64, dim=2, gamma=5.0, kappa="lognormal", sigma=1.0),
    "3d-128-lognormal": dict(n=128, dim=3, gamma=2.0, kappa="lognormal", sigma=1.0),
}


def workload(name: str, seed: int = 1, **over) -> BlockSystem:
    kw = dict(WORKLOADS[name])
    kw.update(over)
    return make_system(seed=seed, **kw)
