// Solve-phase kernels for gfx950: one 64-lane wavefront per slice of 64
// block rows, one lane per block row.  Matrix values are stored slot-major and
// lane-contiguous, so every value load of a wavefront is one contiguous
// 256 B (FP32) or 512 B (FP64) segment; only block entries that are nonzero
// somewhere in the slice are stored, which keeps the streamed bytes close to
// the structural nonzeros.  All loops over slots and mask bits are
// wave-uniform (scalar branches).
#include "solve_kernels.h"
#include "dpp.h"

#include <algorithm>
#include <climits>
#include <utility>

namespace mbamg {

constexpr int WPB = 4;          // waves per block when a slice has at most 4 waves

// P waves share each slice; a block holds max(P, WPB) waves
template <int P>
constexpr int waves_per_block() { return P > WPB ? P : WPB; }
constexpr int CHUNK = 2;        // slots whose loads are issued together

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of slices so neighbour gathers stay in its own L2.
__device__ __forceinline__ int xcd_block(int padded_blocks) {
    const int per = padded_blocks >> 3;
    const int bid = blockIdx.x;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// grid for nslices slices with P waves per slice (4/P slices per 256-thread block)
static inline unsigned xcd_grid(int nslices, int P) {
    int blocks = (int)ceil_div(nslices, std::max(WPB, P) / P);
    return (unsigned)(ceil_div(blocks, 8) * 8);
}

template <class T, int BS>
__device__ __forceinline__ void load_masked(const T* __restrict__ p, uint32_t m, T (&v)[BS]) {
    int g = 0;
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        if (m & (1u << k)) {
            v[k] = p[(int64_t)g * WAVE];
            ++g;
        } else {
            v[k] = T(0);
        }
    }
}

template <class T, int D>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&v)[D]) {
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = p[c];
}

template <>
__device__ __forceinline__ void load_vec<double, 4>(const double* __restrict__ p, double (&v)[4]) {
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

template <>
__device__ __forceinline__ void load_vec<float, 4>(const float* __restrict__ p, float (&v)[4]) {
    float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

template <>
__device__ __forceinline__ void load_vec<double, 2>(const double* __restrict__ p, double (&v)[2]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    v[0] = a.x; v[1] = a.y;
}

template <class T, int D>
__device__ __forceinline__ void store_vec(T* __restrict__ p, const T (&v)[D]) {
#pragma unroll
    for (int c = 0; c < D; ++c) p[c] = v[c];
}

template <>
__device__ __forceinline__ void store_vec<double, 4>(double* __restrict__ p, const double (&v)[4]) {
    double2* q = reinterpret_cast<double2*>(p);
    q[0] = make_double2(v[0], v[1]);
    q[1] = make_double2(v[2], v[3]);
}

template <>
__device__ __forceinline__ void store_vec<float, 4>(float* __restrict__ p, const float (&v)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

// acc[r] -= sum_c A[r,c] * x_col(c) over the slots part, part+P, part+2P, ...
// of one slice.  MODE 0: x from xa.  MODE 1: columns below cstart from xa
// (already updated this sweep), others from xb.  MODE 2: columns below cstart
// from xa, others contribute 0.
// When P waves share a slice (coarse levels: few wide slices, so each wave's
// chain of dependent loads is what the launch waits for), the column indices,
// masks and value offsets of the next chunk are fetched while the current
// chunk's values and gathers are in flight, and FP32 chunks are 4 slots wide.
template <class T, int P>
constexpr int sell_chunk() { return P >= 4 && sizeof(T) == 4 ? 4 : CHUNK; }

// Column indices, masks and value offsets of one chunk of slots.
template <int CH>
struct SlotChunk {
    int j[CH];
    uint32_t m[CH];
    int64_t vg[CH];
};

// the chunk of slots t0, t0 + P, ... of slice s (slots past the width: empty)
template <class T, int P, int CH>
__device__ __forceinline__ void fetch_chunk(const SellView<T>& A, int s, int lane, int t0, SlotChunk<CH>& c) {
    const int w = A.width[s];
    const int64_t cb = A.coff[s];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int tt = t0 + u * P;
        const bool live = tt < w;
        c.m[u] = live ? A.mask[cb + tt] : 0u;
        c.vg[u] = live ? A.voff[cb + tt] : 0;
        c.j[u] = live ? A.col[(cb + tt) * WAVE + lane] : -1;
    }
}

// SKIPD: the slot holding column `self` (the row's own node) is left out.
// pre (split slices only): the first chunk, fetched by the caller ahead of time.
template <class T, int BR, int BC, int MODE, int P, bool SKIPD = false>
__device__ __forceinline__ void sell_sub(const SellView<T>& A, int s, int lane, int part, const T* __restrict__ xa,
                                         const T* __restrict__ xb, int cstart, T (&acc)[BR], int self = -1,
                                         const SlotChunk<sell_chunk<T, P>()>* pre = nullptr) {
    constexpr int CH = sell_chunk<T, P>();
    constexpr bool PF = P >= 4;
    const int w = A.width[s];
    const int64_t cb = A.coff[s];
    int j[CH];
    uint32_t m[CH];
    int64_t vg[CH];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int tt = t0 + u * P;
            const bool live = tt < w;
            m[u] = live ? A.mask[cb + tt] : 0u;
            vg[u] = live ? A.voff[cb + tt] : 0;
            j[u] = live ? A.col[(cb + tt) * WAVE + lane] : -1;
        }
    };
    if (PF) {
        if (pre) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                j[u] = pre->j[u];
                m[u] = pre->m[u];
                vg[u] = pre->vg[u];
            }
        } else {
            fetch(part);
        }
    }
    for (int t = part; t < w; t += P * CH) {
        if (!PF) fetch(t);
        int jc[CH];
        uint32_t mc[CH];
        int64_t gc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            jc[u] = j[u];
            mc[u] = m[u];
            gc[u] = vg[u];
        }
        if (PF) fetch(t + P * CH);
        T v[CH][BR * BC];
#pragma unroll
        for (int u = 0; u < CH; ++u) load_masked<T, BR * BC>(A.val + gc[u] * WAVE + lane, mc[u], v[u]);
        T xj[CH][BC];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int jj = jc[u];
            const T* src = nullptr;
            if (MODE == 0) src = xa;
            else if (MODE == 1) src = jj < cstart ? xa : xb;
            else src = jj < cstart ? xa : nullptr;
            if (jj >= 0 && src && !(SKIPD && jj == self)) load_vec<T, BC>(src + (int64_t)jj * BC, xj[u]);
            else {
#pragma unroll
                for (int c = 0; c < BC; ++c) xj[u][c] = T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int r = 0; r < BR; ++r)
#pragma unroll
                for (int c = 0; c < BC; ++c) acc[r] -= v[u][r * BC + c] * xj[u][c];
    }
}

// Sum the P partial accumulators of one slice through LDS in a fixed order;
// the result is valid in the slice's part-0 wave.
template <class T, int D, int P>
__device__ __forceinline__ void combine_parts(T (&acc)[D], int wave, int part, int lane) {
    if constexpr (P > 1) {
        __shared__ T red[waves_per_block<P>()][WAVE][D];
#pragma unroll
        for (int r = 0; r < D; ++r) red[wave][lane][r] = acc[r];
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int p = 1; p < P; ++p)
#pragma unroll
                for (int r = 0; r < D; ++r) acc[r] += red[wave + p][lane][r];
        }
    }
}

// One colour of the multicolour nodal-block Gauss-Seidel sub-solve of block f
// inside Algorithm 1: for each row i of the colour
//   t_i  = D_i^-1 (b_i - sum_{j != i} A_ff[i,j] t_j - (A_fg x_g)_i)
//   xn_i = x_i + omega (t_i - x_i)
// where t_j is the updated value for rows of earlier colours and x_j otherwise;
// t_i - x_i is the sub-solve's correction e_i for the residual b - A x.
template <class T, int D, bool ZX, bool CPL, int P>
__global__ __launch_bounds__(waves_per_block<P>() * WAVE) void k_gs(GsArgs<T> a, int padded_blocks) {
    const int wave = wave_id();
    const int part = wave % P;
    const int sidx = xcd_block(padded_blocks) * (waves_per_block<P>() / P) + wave / P;
    const bool valid = sidx < a.s_count;
    if (P == 1 && !valid) return;
    const int s = a.s_begin + (valid ? sidx : 0);
    const int lane = threadIdx.x & (WAVE - 1);
    const int row0 = a.sl.row0[s], nrow = a.sl.nrow[s];
    const bool act = valid && lane < nrow;
    const int row = row0 + (lane < nrow ? lane : 0);
    T acc[D];
    if (part == 0) load_vec<T, D>(a.b + (int64_t)row * D, acc);
    else {
#pragma unroll
        for (int r = 0; r < D; ++r) acc[r] = T(0);
    }
    // small levels (split slices): the row's own data, and the coupling part's first slots,
    // are fetched before the sums, so their latency overlaps the sums' instead of following
    T dv[D * D], xo[D];
    T w = a.omega;
    constexpr int CH = sell_chunk<T, P>();
    SlotChunk<CH> cpre;
    if (P > 1 && valid) {
        if (part == 0) {
            load_masked<T, D * D>(a.dinv.val + a.dinv.voff[a.dinv.coff[s]] * WAVE + lane,
                                  a.dinv.mask[a.dinv.coff[s]], dv);
            if (!ZX) load_vec<T, D>(a.x + (int64_t)row * D, xo);
            if (a.w_row) w = a.w_row[row];
        }
        if (CPL && P >= 4) fetch_chunk<T, P, CH>(a.cpl, s, lane, part, cpre);
    }
    if (valid) {
        if (!a.skip_off) {
            if (ZX) sell_sub<T, D, D, 2, P>(a.off, s, lane, part, a.t, nullptr, a.cstart, acc);
            else sell_sub<T, D, D, 1, P>(a.off, s, lane, part, a.t, a.x, a.cstart, acc);
        }
        if (CPL) sell_sub<T, D, D, 0, P>(a.cpl, s, lane, part, a.xg, nullptr, 0, acc, -1, P >= 4 ? &cpre : nullptr);
    }
    combine_parts<T, D, P>(acc, wave, part, lane);
    if (part != 0 || !valid) return;
    if (P == 1)
        load_masked<T, D * D>(a.dinv.val + a.dinv.voff[a.dinv.coff[s]] * WAVE + lane, a.dinv.mask[a.dinv.coff[s]],
                              dv);
    T tn[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T sum = T(0);
#pragma unroll
        for (int c = 0; c < D; ++c) sum += dv[r * D + c] * acc[c];
        tn[r] = sum;
    }
    if (!act) return;
    if (P == 1 && a.w_row) w = a.w_row[row];
    T xn[D];
    if (ZX) {
#pragma unroll
        for (int r = 0; r < D; ++r) xn[r] = w * tn[r];
    } else {
        if (P == 1) load_vec<T, D>(a.x + (int64_t)row * D, xo);
#pragma unroll
        for (int r = 0; r < D; ++r) xn[r] = xo[r] + w * (tn[r] - xo[r]);
    }
    store_vec<T, D>(a.t + (int64_t)row * D, tn);
    store_vec<T, D>(a.xn + (int64_t)row * D, xn);
}

// One colour of the nodal-block Gauss-Seidel over the full node blocks (the
// FC-AMG comparison smoother): for each node i of the colour, both blocks' rows
//   t_i  = D_i^-1 (b_i - sum_{j != i} A[i,j] t_j / x_j)   (D_i: the full node block)
//   xn_i = x_i + omega (t_i - x_i)
// with the sums over A_ff's off-diagonal blocks and A_fg's blocks other than
// the node's own, t_j for rows of earlier colours and x_j otherwise.
template <class T, int D, bool ZX, int P>
__global__ __launch_bounds__(waves_per_block<P>() * WAVE) void k_gs_fc(GsFcArgs<T> a, int padded_blocks) {
    constexpr int M = 2 * D;
    const int wave = wave_id();
    const int part = wave % P;
    const int sidx = xcd_block(padded_blocks) * (waves_per_block<P>() / P) + wave / P;
    const bool valid = sidx < a.s_count;
    if (P == 1 && !valid) return;
    const int s = a.s_begin + (valid ? sidx : 0);
    const int lane = threadIdx.x & (WAVE - 1);
    const int row0 = a.sl.row0[s], nrow = a.sl.nrow[s];
    const bool act = valid && lane < nrow;
    const int row = row0 + (lane < nrow ? lane : 0);
    T acc0[D], acc1[D];
    if (part == 0) {
        load_vec<T, D>(a.b[0] + (int64_t)row * D, acc0);
        load_vec<T, D>(a.b[1] + (int64_t)row * D, acc1);
    } else {
#pragma unroll
        for (int r = 0; r < D; ++r) acc0[r] = acc1[r] = T(0);
    }
    if (valid && !a.skip_off) {
        constexpr int MODE = ZX ? 2 : 1;
        sell_sub<T, D, D, MODE, P>(a.off[0], s, lane, part, a.t[0], a.x[0], a.cstart, acc0);
        sell_sub<T, D, D, MODE, P, true>(a.cpl[0], s, lane, part, a.t[1], a.x[1], a.cstart, acc0, row);
        sell_sub<T, D, D, MODE, P>(a.off[1], s, lane, part, a.t[1], a.x[1], a.cstart, acc1);
        sell_sub<T, D, D, MODE, P, true>(a.cpl[1], s, lane, part, a.t[0], a.x[0], a.cstart, acc1, row);
    }
    T acc[M];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        acc[r] = acc0[r];
        acc[D + r] = acc1[r];
    }
    combine_parts<T, M, P>(acc, wave, part, lane);
    if (part != 0 || !valid) return;
    // the node inverse: only the slice's nonzero entries are stored
    const uint64_t dm = a.dmask[s];
    const T* dv = a.dinv + (int64_t)a.doff[s] * WAVE + lane;
    T inv[M * M];
    int g = 0;
#pragma unroll
    for (int k = 0; k < M * M; ++k) {
        if ((dm >> k) & 1) {
            inv[k] = dv[(int64_t)g * WAVE];
            ++g;
        } else {
            inv[k] = T(0);
        }
    }
    T tn[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        T sum = T(0);
#pragma unroll
        for (int c = 0; c < M; ++c) sum += inv[r * M + c] * acc[c];
        tn[r] = sum;
    }
    if (!act) return;
    const T w = a.w_row ? a.w_row[row] : a.omega;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        T tf[D], xn[D];
#pragma unroll
        for (int r = 0; r < D; ++r) tf[r] = tn[f * D + r];
        if (ZX) {
#pragma unroll
            for (int r = 0; r < D; ++r) xn[r] = w * tf[r];
        } else {
            T xo[D];
            load_vec<T, D>(a.x[f] + (int64_t)row * D, xo);
#pragma unroll
            for (int r = 0; r < D; ++r) xn[r] = xo[r] + w * (tf[r] - xo[r]);
        }
        store_vec<T, D>(a.t[f] + (int64_t)row * D, tf);
        store_vec<T, D>(a.xn[f] + (int64_t)row * D, xn);
    }
}

// ---------------------------------------------------------------------------
// Row-form kernels for coarse levels: one wavefront per row, lanes over the
// row's blocks, partial sums combined across the wavefront.
// ---------------------------------------------------------------------------
// a dense block of N values, with 16-byte loads where the size allows (blocks
// are stored back to back, so a block of 4 or 16 entries is 16-byte aligned)
template <class T, int N>
__device__ __forceinline__ void load_block(const T* __restrict__ p, T (&v)[N]) {
    if constexpr (sizeof(T) == 4 && N % 4 == 0) {
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const float4 q = reinterpret_cast<const float4*>(p)[k];
            v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
        }
    } else if constexpr (sizeof(T) == 8 && N % 2 == 0) {
#pragma unroll
        for (int k = 0; k < N / 2; ++k) {
            const double2 q = reinterpret_cast<const double2*>(p)[k];
            v[2 * k] = q.x; v[2 * k + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = p[k];
    }
}

template <class T, int D, int DG, int MODE, bool SKIP_DIAG>
__device__ __forceinline__ void row_sub(const RowView<T>& A, int row, int lane, const T* __restrict__ xa,
                                        const T* __restrict__ xb, int cstart, T (&acc)[D]) {
    const int e = A.rp[row + 1];
    for (int p = A.rp[row] + lane; p < e; p += WAVE) {
        const int j = A.col[p];
        if (SKIP_DIAG && j == row) continue;
        const T* src;
        if (MODE == 0) src = xa;
        else if (MODE == 1) src = j < cstart ? xa : xb;
        else src = j < cstart ? xa : nullptr;
        if (!src) continue;
        T xj[DG];
        load_vec<T, DG>(src + (int64_t)j * DG, xj);
        T blk[D * DG];
        load_block<T, D * DG>(A.val + (int64_t)p * D * DG, blk);
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < DG; ++c) acc[r] -= blk[r * DG + c] * xj[c];
    }
}

// The same sums with the row's values read back to back: in a pass over the
// row, lane u reads the u-th 16-byte piece (one block row of a float block,
// half of a double one), so one load instruction covers 1 KiB with no gaps.
// Every lane keeps one block-row position (the row's first block starts a
// piece group), so its partial sum belongs to one component r.
// With RP wavefronts on one row, wavefront `part` takes every RP-th pass.
template <class T, int D, int MODE, bool SKIP_DIAG, int RP = 1>
__device__ __forceinline__ void row_sub_c(const RowView<T>& A, int row, int lane, const T* __restrict__ xa,
                                          const T* __restrict__ xb, int cstart, T (&acc)[D], int wpart = 0) {
    constexpr int V = 16 / (int)sizeof(T);   // values per piece
    static_assert(D % V == 0, "block rows split into 16-byte pieces");
    constexpr int LR = D / V;                // pieces per block row
    constexpr int LB = D * LR;               // pieces per block
    static_assert(WAVE % LB == 0, "a pass keeps every lane on one block-row position");
    constexpr int UNROLL = 4;
    const int part = lane % LB;
    const int r = part / LR, c0 = (part % LR) * V;
    const int64_t u0 = (int64_t)A.rp[row] * LB, u1 = (int64_t)A.rp[row + 1] * LB;
    T sum = T(0);
    for (int64_t ub = u0 + (int64_t)wpart * WAVE; ub < u1; ub += UNROLL * RP * WAVE) {
        T av[UNROLL][V], xv[UNROLL][V];
        bool ok[UNROLL];
#pragma unroll
        for (int h = 0; h < UNROLL; ++h) {
            const int64_t u = ub + (int64_t)h * RP * WAVE + lane;
            ok[h] = u < u1;
            const int64_t uc = ok[h] ? u : u0 + part;   // in range: the row's first block
            const int j = A.col[uc / LB];
            if (SKIP_DIAG && j == row) ok[h] = false;
            const T* src = xa;
            if (MODE == 1 && j >= cstart) src = xb;
            if (MODE == 2 && j >= cstart) ok[h] = false;
            load_vec<T, V>(A.val + uc * V, av[h]);
            load_vec<T, V>(src + (int64_t)j * D + c0, xv[h]);
        }
#pragma unroll
        for (int h = 0; h < UNROLL; ++h) {
            T s = T(0);
#pragma unroll
            for (int c = 0; c < V; ++c) s += av[h][c] * xv[h][c];
            sum += ok[h] ? s : T(0);
        }
    }
#pragma unroll
    for (int rr = 0; rr < D; ++rr) acc[rr] -= rr == r ? sum : T(0);
}

// Sum over the wavefront, valid in lane WAVE - 1, per component.
template <class T, int D>
__device__ __forceinline__ void wave_sum_vec(T (&acc)[D]) {
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = group_sum<64>(acc[r]);
}

// Sum of the RP wavefronts' partial sums of one row (each valid in its lane
// WAVE - 1), in wavefront order, left in wavefront 0's lane WAVE - 1.
template <class T, int D, int RP>
__device__ __forceinline__ void combine_row_parts(T (&acc)[D], int wpart, int lane) {
    if constexpr (RP > 1) {
        __shared__ T red[RP][D];
        if (lane == WAVE - 1)
#pragma unroll
            for (int r = 0; r < D; ++r) red[wpart][r] = acc[r];
        __syncthreads();
        if (wpart == 0 && lane == WAVE - 1) {
#pragma unroll
            for (int r = 0; r < D; ++r) {
                T v = red[0][r];
#pragma unroll
                for (int q = 1; q < RP; ++q) v += red[q][r];
                acc[r] = v;
            }
        }
    }
}

// One colour of the block row's Gauss-Seidel sub-solve (the arithmetic of k_gs).
// RP = 1: one wavefront per row; RP = 4: the four wavefronts of a workgroup
// share one long row (4 x 4 blocks only).
template <class T, int D, bool ZX, bool CPL, int RP>
__global__ __launch_bounds__(256) void k_gs_rows(GsRowArgs<T> a) {
    static_assert(RP == 1 || (RP == WPB && D == 4), "rows shared by the workgroup's wavefronts: 4 x 4 blocks");
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpart = RP > 1 ? wave_id() : 0;
    const int w = RP > 1 ? (int)blockIdx.x : (int)blockIdx.x * WPB + wave_id();
    if (w >= a.r_count) return;   // whole wavefronts (the whole workgroup when RP > 1)
    const int row = a.r_begin + w;
    // the row's own data first: its latency overlaps the row sums'
    T bb[D], dv[D * D], xo[D];
    if (wpart == 0) {
        load_vec<T, D>(a.b + (int64_t)row * D, bb);
        load_block<T, D * D>(a.dinv + (int64_t)row * D * D, dv);
        if (!ZX) load_vec<T, D>(a.x + (int64_t)row * D, xo);
    }
    const T wgt = a.w_row ? a.w_row[row] : a.omega;
    T acc[D];
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = T(0);
    if constexpr (D == 4) {
        if (!a.skip_off) {
            if (ZX) row_sub_c<T, D, 2, true, RP>(a.aff, row, lane, a.t, nullptr, a.cstart, acc, wpart);
            else row_sub_c<T, D, 1, true, RP>(a.aff, row, lane, a.t, a.x, a.cstart, acc, wpart);
        }
        if (CPL) row_sub_c<T, D, 0, false, RP>(a.afg, row, lane, a.xg, nullptr, 0, acc, wpart);
    } else {
        if (!a.skip_off) {
            if (ZX) row_sub<T, D, D, 2, true>(a.aff, row, lane, a.t, nullptr, a.cstart, acc);
            else row_sub<T, D, D, 1, true>(a.aff, row, lane, a.t, a.x, a.cstart, acc);
        }
        if (CPL) row_sub<T, D, D, 0, false>(a.afg, row, lane, a.xg, nullptr, 0, acc);
    }
    wave_sum_vec<T, D>(acc);
    combine_row_parts<T, D, RP>(acc, wpart, lane);
    if (wpart != 0 || lane != WAVE - 1) return;
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] += bb[r];
    T tn[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T sum = T(0);
#pragma unroll
        for (int c = 0; c < D; ++c) sum += dv[r * D + c] * acc[c];
        tn[r] = sum;
    }
    T xn[D];
    if (ZX) {
#pragma unroll
        for (int r = 0; r < D; ++r) xn[r] = wgt * tn[r];
    } else {
#pragma unroll
        for (int r = 0; r < D; ++r) xn[r] = xo[r] + wgt * (tn[r] - xo[r]);
    }
    store_vec<T, D>(a.t + (int64_t)row * D, tn);
    store_vec<T, D>(a.xn + (int64_t)row * D, xn);
}

// r = b - A x (or w = A x when b is NULL), rows of block 0 then block 1
template <class T, int D>
__global__ __launch_bounds__(256) void k_resid_rows(ResidRowArgs<T> a) {
    const int lane = threadIdx.x & (WAVE - 1);
    int row = blockIdx.x * WPB + wave_id();
    int f = 0;
    if (row >= a.n[0]) {
        row -= a.n[0];
        f = 1;
        if (row >= a.n[1]) return;   // whole wavefront
    }
    const int g = 1 - f;
    T bb[D];   // fetched first: its latency overlaps the row sums'
    if (a.b[f]) load_vec<T, D>(a.b[f] + (int64_t)row * D, bb);
    T acc[D];
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = T(0);
    if constexpr (D == 4) {
        row_sub_c<T, D, 0, false>(a.aff[f], row, lane, a.x[f], nullptr, 0, acc);
        row_sub_c<T, D, 0, false>(a.afg[f], row, lane, a.x[g], nullptr, 0, acc);
    } else {
        row_sub<T, D, D, 0, false>(a.aff[f], row, lane, a.x[f], nullptr, 0, acc);
        row_sub<T, D, D, 0, false>(a.afg[f], row, lane, a.x[g], nullptr, 0, acc);
    }
    wave_sum_vec<T, D>(acc);
    if (lane != WAVE - 1) return;
    T out[D];
    if (a.b[f]) {
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = bb[r] + acc[r];
    } else {
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = -acc[r];
    }
    store_vec<T, D>(a.r[f] + (int64_t)row * D, out);
}

// y = A x (or y += A x when accumulating) for a transfer in row form: one
// wavefront per row, the row's blocks read as in the row-form smoother.
template <class T, int D>
__global__ __launch_bounds__(256) void k_xfer_rows(XferRowArgs<T> a) {
    const int lane = threadIdx.x & (WAVE - 1);
    int row = blockIdx.x * WPB + wave_id();
    int f = 0;
    if (row >= a.n[0]) {
        row -= a.n[0];
        f = 1;
        if (row >= a.n[1]) return;   // whole wavefront
    }
    T acc[D];
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = T(0);
    if constexpr (D == 4) row_sub_c<T, D, 0, false>(a.A[f], row, lane, a.x[f], nullptr, 0, acc);
    else row_sub<T, D, D, 0, false>(a.A[f], row, lane, a.x[f], nullptr, 0, acc);
    wave_sum_vec<T, D>(acc);
    if (lane != WAVE - 1) return;
    const int orow = a.out_row[f] ? a.out_row[f][row] : row;
    T out[D];
    if (a.accumulate) {
        T y[D];
        load_vec<T, D>(a.y[f] + (int64_t)orow * D, y);
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = y[r] - acc[r];
    } else {
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = -acc[r];
    }
    store_vec<T, D>(a.y[f] + (int64_t)orow * D, out);
}

template <class T>
void launch_xfer_rows(int d, const XferRowArgs<T>& a, hipStream_t s) {
    const int64_t total = (int64_t)a.n[0] + a.n[1];
    if (total <= 0) return;
    const unsigned grid = (unsigned)ceil_div(total, WPB);
    switch (d) {
        case 1: k_xfer_rows<T, 1><<<grid, 256, 0, s>>>(a); break;
        case 2: k_xfer_rows<T, 2><<<grid, 256, 0, s>>>(a); break;
        case 3: k_xfer_rows<T, 3><<<grid, 256, 0, s>>>(a); break;
        case 4: k_xfer_rows<T, 4><<<grid, 256, 0, s>>>(a); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}
template void launch_xfer_rows<double>(int, const XferRowArgs<double>&, hipStream_t);
template void launch_xfer_rows<float>(int, const XferRowArgs<float>&, hipStream_t);

// y += sign * A x for one block A_fg of any block shape (br, bc <= 4) in row
// form (rows in block f's colour order, columns in block g's): one thread per
// row, the row's blocks in their stored order.  Used where a system has more
// than two blocks, whose couplings are folded into the right-hand sides.
template <class T>
__global__ __launch_bounds__(256) void k_rows_acc(int n, int br, int bc, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const T* __restrict__ val,
                                                  const T* __restrict__ x, T* __restrict__ y, T sign) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const int bs = br * bc;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int64_t j = col[p];
        const T* v = val + (int64_t)p * bs;
        T xj[4];
        for (int c = 0; c < bc; ++c) xj[c] = x[j * bc + c];
        for (int r = 0; r < br; ++r)
            for (int c = 0; c < bc; ++c) acc[r] += v[r * bc + c] * xj[c];
    }
    for (int r = 0; r < br; ++r) y[(int64_t)i * br + r] += sign * acc[r];
}

template <class T>
void launch_rows_acc(int n, int br, int bc, const RowView<T>& A, const T* x, T* y, T sign, hipStream_t s) {
    if (n <= 0) return;
    MB_CHECK(br >= 1 && br <= 4 && bc >= 1 && bc <= 4, MBAMG_E_INVALID, "row blocks of at most 4 x 4");
    k_rows_acc<T><<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, br, bc, A.rp, A.col, A.val, x, y, sign);
    MB_LAUNCH_CHECK();
}
template void launch_rows_acc<double>(int, int, int, const RowView<double>&, const double*, double*, double,
                                      hipStream_t);

// r = b - A x (or w = A x when b is NULL) for both block rows in one launch.
template <class T, int D, int P>
__global__ __launch_bounds__(waves_per_block<P>() * WAVE) void k_resid(ResidArgs<T> a, int padded_blocks) {
    const int wave = wave_id();
    const int part = wave % P;
    int sidx = xcd_block(padded_blocks) * (waves_per_block<P>() / P) + wave / P;
    int f = 0;
    bool valid = true;
    if (sidx >= a.s_count[0]) {
        sidx -= a.s_count[0];
        f = 1;
        if (sidx >= a.s_count[1]) valid = false;
    }
    if (P == 1 && !valid) return;
    if (!valid) {   // padding wave of a split slice: read any existing slice, write nothing
        f = a.s_count[0] > 0 ? 0 : 1;
        sidx = 0;
    } else if (a.order[f]) {
        sidx = a.order[f][sidx];
    }
    const int g = 1 - f;
    const int lane = threadIdx.x & (WAVE - 1);
    const int row0 = a.sl[f].row0[sidx], nrow = a.sl[f].nrow[sidx];
    const bool act = valid && lane < nrow;
    const int row = row0 + (lane < nrow ? lane : 0);
    T acc[D];
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = T(0);
    if (valid) {
        sell_sub<T, D, D, 0, P>(a.diag[f], sidx, lane, part, a.x[f], nullptr, 0, acc);
        sell_sub<T, D, D, 0, P>(a.off[f], sidx, lane, part, a.x[f], nullptr, 0, acc);
        sell_sub<T, D, D, 0, P>(a.cpl[f], sidx, lane, part, a.x[g], nullptr, 0, acc);
    }
    combine_parts<T, D, P>(acc, wave, part, lane);
    if (part != 0 || !act) return;
    T out[D];
    if (a.b[f]) {
        T bb[D];
        load_vec<T, D>(a.b[f] + (int64_t)row * D, bb);
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = bb[r] + acc[r];
    } else {
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = -acc[r];
    }
    store_vec<T, D>(a.r[f] + (int64_t)row * D, out);
}

// y = A x (or y += A x) for both blocks in one launch: the smoothed
// prolongator (rows of the fine level) and its transpose (rows of the coarse
// level) in masked sliced-ELL form.
template <class T, int D, int P>
__global__ __launch_bounds__(waves_per_block<P>() * WAVE) void k_xfer(XferArgs<T> a, int padded_blocks) {
    const int wave = wave_id();
    const int part = wave % P;
    int sidx = xcd_block(padded_blocks) * (waves_per_block<P>() / P) + wave / P;
    int f = 0;
    bool valid = true;
    if (sidx >= a.s_count[0]) {
        sidx -= a.s_count[0];
        f = 1;
        if (sidx >= a.s_count[1]) valid = false;
    }
    if (P == 1 && !valid) return;
    if (!valid) {   // padding wave of a split slice: read any existing slice, write nothing
        f = a.s_count[0] > 0 ? 0 : 1;
        sidx = 0;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const int row0 = a.sl[f].row0[sidx], nrow = a.sl[f].nrow[sidx];
    const int row = row0 + (lane < nrow ? lane : 0);
    T acc[D];
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = T(0);
    if (valid) sell_sub<T, D, D, 0, P>(a.A[f], sidx, lane, part, a.x[f], nullptr, 0, acc);
    combine_parts<T, D, P>(acc, wave, part, lane);
    if (part != 0 || !valid || lane >= nrow) return;
    const int orow = a.out_row[f] ? a.out_row[f][row] : row;
    T out[D];
    if (a.accumulate) {
        T y[D];
        load_vec<T, D>(a.y[f] + (int64_t)orow * D, y);
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = y[r] - acc[r];
    } else {
#pragma unroll
        for (int r = 0; r < D; ++r) out[r] = -acc[r];
    }
    store_vec<T, D>(a.y[f] + (int64_t)orow * D, out);
}

// Sum over aligned groups of G lanes, valid in each group's last lane, per component.
template <class T, int D, int G>
__device__ __forceinline__ void group_sum_vec(T (&acc)[D]) {
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = group_sum<G>(acc[r]);
}

// coarse b_k = sum over members i of aggregate k of q_i .* r_i (per component):
// G lanes per coarse row, the members strided over them (their rows are
// scattered over the fine vector, so many are fetched at once; the weights q
// are stored in member-list order, so only r is gathered)
template <class T, int D, int G>
__global__ __launch_bounds__(256) void k_restrict(TransferArgs<T> a, int padded_blocks) {
    // consecutive coarse rows (neighbouring aggregates, which share fine rows' cache lines)
    // go to the same XCD
    const int64_t t = (int64_t)xcd_block(padded_blocks) * blockDim.x + threadIdx.x;
    int k = (int)(t / G);
    const int gl = (int)(t % G);
    int f = 0;
    if (k >= a.n_rows[0]) {
        k -= a.n_rows[0];
        f = 1;
        if (k >= a.n_rows[1]) return;   // whole groups
    }
    if (a.order[f]) k = a.order[f][k];
    const int32_t* mp = a.map[f];
    const int32_t* mi = a.idx[f];
    T acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = T(0);
    for (int m = mp[k] + gl; m < mp[k + 1]; m += G) {
        const int64_t i = mi[m];
        T q[D], r[D];
        load_vec<T, D>(a.q[f] + (int64_t)m * D, q);
        load_vec<T, D>(a.in[f] + i * D, r);
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] += q[c] * r[c];
    }
    group_sum_vec<T, D, G>(acc);
    if (gl == G - 1) store_vec<T, D>(a.out[f] + (int64_t)k * D, acc);
}

// x_i += q_i .* x_c[agg(i)] (per component)
template <class T, int D>
__global__ void k_prolong(TransferArgs<T> a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int f = 0;
    if (i >= a.n_rows[0]) {
        i -= a.n_rows[0];
        f = 1;
        if (i >= a.n_rows[1]) return;
    }
    const int64_t k = a.map[f][i];
    T q[D], xc[D], x[D];
    load_vec<T, D>(a.q[f] + (int64_t)i * D, q);
    load_vec<T, D>(a.in[f] + k * D, xc);
    load_vec<T, D>(a.out[f] + (int64_t)i * D, x);
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] += q[c] * xc[c];
    store_vec<T, D>(a.out[f] + (int64_t)i * D, x);
}

// y = inv * x with the inverse in FP64 (one wavefront per row)
template <class T>
__global__ __launch_bounds__(256) void k_coarse(int n, const double* __restrict__ inv, const T* __restrict__ x,
                                                T* __restrict__ y) {
    const int row = blockIdx.x * WPB + (threadIdx.x >> 6);
    const int lane = threadIdx.x & (WAVE - 1);
    if (row >= n) return;
    const double* a = inv + (int64_t)row * n;
    double s = 0.0;
    for (int c = lane; c < n; c += WAVE) s += a[c] * (double)x[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
    if (lane == 0) y[row] = (T)s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class T, int D, int P>
static void gs_dispatch(bool zx, bool cpl, const GsArgs<T>& a, hipStream_t s) {
    unsigned grid = xcd_grid(a.s_count, P);
    int pb = (int)grid;
    constexpr int TPB = waves_per_block<P>() * WAVE;
    if (zx) {
        if (cpl) k_gs<T, D, true, true, P><<<grid, TPB, 0, s>>>(a, pb);
        else k_gs<T, D, true, false, P><<<grid, TPB, 0, s>>>(a, pb);
    } else {
        if (cpl) k_gs<T, D, false, true, P><<<grid, TPB, 0, s>>>(a, pb);
        else k_gs<T, D, false, false, P><<<grid, TPB, 0, s>>>(a, pb);
    }
}

template <class T, int D>
static void gs_dispatch_p(int P, bool zx, bool cpl, const GsArgs<T>& a, hipStream_t s) {
    switch (P) {
        case 1: gs_dispatch<T, D, 1>(zx, cpl, a, s); break;
        case 2: gs_dispatch<T, D, 2>(zx, cpl, a, s); break;
        case 4: gs_dispatch<T, D, 4>(zx, cpl, a, s); break;
        case 8: gs_dispatch<T, D, 8>(zx, cpl, a, s); break;
        case 16: gs_dispatch<T, D, 16>(zx, cpl, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "slot split must be 1, 2, 4, 8 or 16");
    }
}

template <class T>
void launch_gs(int d, int P, bool zero_x, bool has_cpl, const GsArgs<T>& a, hipStream_t s) {
    if (a.s_count <= 0) return;
    switch (d) {
        case 1: gs_dispatch_p<T, 1>(P, zero_x, has_cpl, a, s); break;
        case 2: gs_dispatch_p<T, 2>(P, zero_x, has_cpl, a, s); break;
        case 3: gs_dispatch_p<T, 3>(P, zero_x, has_cpl, a, s); break;
        case 4: gs_dispatch_p<T, 4>(P, zero_x, has_cpl, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}

template <class T, int D, int P>
static void gs_fc_dispatch(bool zx, const GsFcArgs<T>& a, hipStream_t s) {
    const unsigned grid = xcd_grid(a.s_count, P);
    constexpr int TPB = waves_per_block<P>() * WAVE;
    if (zx) k_gs_fc<T, D, true, P><<<grid, TPB, 0, s>>>(a, (int)grid);
    else k_gs_fc<T, D, false, P><<<grid, TPB, 0, s>>>(a, (int)grid);
}

template <class T, int D>
static void gs_fc_dispatch_p(int P, bool zx, const GsFcArgs<T>& a, hipStream_t s) {
    switch (P) {
        case 1: gs_fc_dispatch<T, D, 1>(zx, a, s); break;
        case 2: gs_fc_dispatch<T, D, 2>(zx, a, s); break;
        case 4: gs_fc_dispatch<T, D, 4>(zx, a, s); break;
        case 8: gs_fc_dispatch<T, D, 8>(zx, a, s); break;
        case 16: gs_fc_dispatch<T, D, 16>(zx, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "slot split must be 1, 2, 4, 8 or 16");
    }
}

template <class T>
void launch_gs_fc(int d, int P, bool zero_x, const GsFcArgs<T>& a, hipStream_t s) {
    if (a.s_count <= 0) return;
    switch (d) {
        case 1: gs_fc_dispatch_p<T, 1>(P, zero_x, a, s); break;
        case 2: gs_fc_dispatch_p<T, 2>(P, zero_x, a, s); break;
        case 3: gs_fc_dispatch_p<T, 3>(P, zero_x, a, s); break;
        case 4: gs_fc_dispatch_p<T, 4>(P, zero_x, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}

template <class T, int D, int RP>
static void gs_rows_dispatch(bool zx, bool cpl, const GsRowArgs<T>& a, hipStream_t s) {
    const unsigned grid = (unsigned)ceil_div(a.r_count, WPB / RP);
    if (zx) {
        if (cpl) k_gs_rows<T, D, true, true, RP><<<grid, 256, 0, s>>>(a);
        else k_gs_rows<T, D, true, false, RP><<<grid, 256, 0, s>>>(a);
    } else {
        if (cpl) k_gs_rows<T, D, false, true, RP><<<grid, 256, 0, s>>>(a);
        else k_gs_rows<T, D, false, false, RP><<<grid, 256, 0, s>>>(a);
    }
}

template <class T>
void launch_gs_rows(int d, int rp, bool zero_x, bool has_cpl, const GsRowArgs<T>& a, hipStream_t s) {
    if (a.r_count <= 0) return;
    MB_CHECK(rp == 1 || (rp == WPB && d == 4), MBAMG_E_INVALID, "row split must be 1, or 4 with 4 x 4 blocks");
    switch (d) {
        case 1: gs_rows_dispatch<T, 1, 1>(zero_x, has_cpl, a, s); break;
        case 2: gs_rows_dispatch<T, 2, 1>(zero_x, has_cpl, a, s); break;
        case 3: gs_rows_dispatch<T, 3, 1>(zero_x, has_cpl, a, s); break;
        case 4:
            if (rp == WPB) gs_rows_dispatch<T, 4, WPB>(zero_x, has_cpl, a, s);
            else gs_rows_dispatch<T, 4, 1>(zero_x, has_cpl, a, s);
            break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}
template void launch_gs_rows<double>(int, int, bool, bool, const GsRowArgs<double>&, hipStream_t);
template void launch_gs_rows<float>(int, int, bool, bool, const GsRowArgs<float>&, hipStream_t);

template <class T>
void launch_resid_rows(int d, const ResidRowArgs<T>& a, hipStream_t s) {
    const int total = a.n[0] + a.n[1];
    if (total <= 0) return;
    const unsigned grid = (unsigned)ceil_div(total, WPB);
    switch (d) {
        case 1: k_resid_rows<T, 1><<<grid, 256, 0, s>>>(a); break;
        case 2: k_resid_rows<T, 2><<<grid, 256, 0, s>>>(a); break;
        case 3: k_resid_rows<T, 3><<<grid, 256, 0, s>>>(a); break;
        case 4: k_resid_rows<T, 4><<<grid, 256, 0, s>>>(a); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}
template void launch_resid_rows<double>(int, const ResidRowArgs<double>&, hipStream_t);
template void launch_resid_rows<float>(int, const ResidRowArgs<float>&, hipStream_t);

template <class T, int D>
static void resid_dispatch(int P, const ResidArgs<T>& a, hipStream_t s) {
    const int total = a.s_count[0] + a.s_count[1];
    unsigned grid = xcd_grid(total, P);
    int pb = (int)grid;
    switch (P) {
        case 1: k_resid<T, D, 1><<<grid, 256, 0, s>>>(a, pb); break;
        case 2: k_resid<T, D, 2><<<grid, 256, 0, s>>>(a, pb); break;
        case 4: k_resid<T, D, 4><<<grid, 256, 0, s>>>(a, pb); break;
        case 8: k_resid<T, D, 8><<<grid, 512, 0, s>>>(a, pb); break;
        case 16: k_resid<T, D, 16><<<grid, 1024, 0, s>>>(a, pb); break;
        default: throw Error(MBAMG_E_INVALID, "slot split must be 1, 2, 4, 8 or 16");
    }
}

template <class T>
void launch_resid(int d, int P, const ResidArgs<T>& a, hipStream_t s) {
    if (a.s_count[0] + a.s_count[1] <= 0) return;
    switch (d) {
        case 1: resid_dispatch<T, 1>(P, a, s); break;
        case 2: resid_dispatch<T, 2>(P, a, s); break;
        case 3: resid_dispatch<T, 3>(P, a, s); break;
        case 4: resid_dispatch<T, 4>(P, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}

template <class T, int D>
static void xfer_dispatch(int P, const XferArgs<T>& a, hipStream_t s) {
    const int total = a.s_count[0] + a.s_count[1];
    unsigned grid = xcd_grid(total, P);
    int pb = (int)grid;
    switch (P) {
        case 1: k_xfer<T, D, 1><<<grid, 256, 0, s>>>(a, pb); break;
        case 2: k_xfer<T, D, 2><<<grid, 256, 0, s>>>(a, pb); break;
        case 4: k_xfer<T, D, 4><<<grid, 256, 0, s>>>(a, pb); break;
        case 8: k_xfer<T, D, 8><<<grid, 512, 0, s>>>(a, pb); break;
        case 16: k_xfer<T, D, 16><<<grid, 1024, 0, s>>>(a, pb); break;
        default: throw Error(MBAMG_E_INVALID, "slot split must be 1, 2, 4, 8 or 16");
    }
}

template <class T>
void launch_xfer(int d, int P, const XferArgs<T>& a, hipStream_t s) {
    if (a.s_count[0] + a.s_count[1] <= 0) return;
    switch (d) {
        case 1: xfer_dispatch<T, 1>(P, a, s); break;
        case 2: xfer_dispatch<T, 2>(P, a, s); break;
        case 3: xfer_dispatch<T, 3>(P, a, s); break;
        case 4: xfer_dispatch<T, 4>(P, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}
template void launch_xfer<double>(int, int, const XferArgs<double>&, hipStream_t);
template void launch_xfer<float>(int, int, const XferArgs<float>&, hipStream_t);

template <class T, int D>
static void restrict_dispatch(int64_t total, int G, const TransferArgs<T>& a, hipStream_t s) {
    const unsigned grid = (unsigned)(ceil_div(ceil_div(total * G, 256), 8) * 8);
    const int pb = (int)grid;
    switch (G) {
        case 4: k_restrict<T, D, 4><<<grid, 256, 0, s>>>(a, pb); break;
        case 8: k_restrict<T, D, 8><<<grid, 256, 0, s>>>(a, pb); break;
        case 16: k_restrict<T, D, 16><<<grid, 256, 0, s>>>(a, pb); break;
        default: k_restrict<T, D, 64><<<grid, 256, 0, s>>>(a, pb); break;
    }
}

template <class T>
void launch_restrict(int d, const TransferArgs<T>& a, int G, hipStream_t s) {
    const int64_t total = (int64_t)a.n_rows[0] + a.n_rows[1];
    if (total <= 0) return;
    MB_CHECK(G == 4 || G == 8 || G == 16 || G == 64, MBAMG_E_INVALID, "restriction group of 4, 8, 16 or 64 lanes");
    switch (d) {
        case 1: restrict_dispatch<T, 1>(total, G, a, s); break;
        case 2: restrict_dispatch<T, 2>(total, G, a, s); break;
        case 3: restrict_dispatch<T, 3>(total, G, a, s); break;
        case 4: restrict_dispatch<T, 4>(total, G, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}

template <class T>
void launch_prolong(int d, const TransferArgs<T>& a, hipStream_t s) {
    const int total = a.n_rows[0] + a.n_rows[1];
    if (total <= 0) return;
    unsigned grid = (unsigned)ceil_div(total, 256);
    switch (d) {
        case 1: k_prolong<T, 1><<<grid, 256, 0, s>>>(a); break;
        case 2: k_prolong<T, 2><<<grid, 256, 0, s>>>(a); break;
        case 3: k_prolong<T, 3><<<grid, 256, 0, s>>>(a); break;
        case 4: k_prolong<T, 4><<<grid, 256, 0, s>>>(a); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}

template <class T>
void launch_coarse(int n, const double* inv, const T* x, T* y, hipStream_t s) {
    if (n <= 0) return;
    k_coarse<T><<<(unsigned)ceil_div(n, WPB), 256, 0, s>>>(n, inv, x, y);
    MB_LAUNCH_CHECK();
}

template void launch_gs<double>(int, int, bool, bool, const GsArgs<double>&, hipStream_t);
template void launch_gs_fc<double>(int, int, bool, const GsFcArgs<double>&, hipStream_t);
template void launch_gs_fc<float>(int, int, bool, const GsFcArgs<float>&, hipStream_t);
template void launch_gs<float>(int, int, bool, bool, const GsArgs<float>&, hipStream_t);
template void launch_resid<double>(int, int, const ResidArgs<double>&, hipStream_t);
template void launch_resid<float>(int, int, const ResidArgs<float>&, hipStream_t);
template void launch_restrict<double>(int, const TransferArgs<double>&, int, hipStream_t);
template void launch_restrict<float>(int, const TransferArgs<float>&, int, hipStream_t);
template void launch_prolong<double>(int, const TransferArgs<double>&, hipStream_t);
template void launch_prolong<float>(int, const TransferArgs<float>&, hipStream_t);
template void launch_coarse<double>(int, const double*, const double*, double*, hipStream_t);
template void launch_coarse<float>(int, const double*, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// Krylov kernels: fixed grid, per-block partial sums, one-block final sums
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double r = sh[0] + sh[1] + sh[2] + sh[3];
    return r;
}

// Dot pass: partial[q][block] = sum V_q . w over this block's elements (q < NQ),
// partial[NQ][block] = sum w . w.  NQ is the exact count (one instance per
// count: guarded loads would cost a branch each and registers for the
// predicates); all loads of one element are issued before any use.
template <int NQ>
__global__ __launch_bounds__(256) void k_orth(int64_t n, const double* __restrict__ V, int64_t ldv,
                                              const double* __restrict__ w, double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    double nn = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double v[NQ > 0 ? NQ : 1];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = V[q * ldv + e];
        const double u = w[e];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += v[q] * u;
        nn += u * u;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double r = block_sum(acc[q], sh);
        if (threadIdx.x == 0) partial[(int64_t)q * KBLOCKS + blockIdx.x] = r;
    }
    const double r = block_sum(nn, sh);
    if (threadIdx.x == 0) partial[(int64_t)NQ * KBLOCKS + blockIdx.x] = r;
}

// Update pass of classical Gram-Schmidt with delayed reorthogonalisation
// (DCGS2: Swirydowicz, Langou, Ananthan, Yang & Thomas 2020; Bielich et al.
// 2022).  Q_0..Q_{NQ-1} are final orthonormal basis vectors, u the candidate for
// Q_NQ (projected once), w the operator applied to the preconditioned u, and
// coef holds a = Q^T u (found by the previous update pass), b = Q^T w, 1/nu with
// nu = |u - Q a|, and c_j = (u . w - a . b) / nu.  Per element:
//   q  = (u - sum_k a_k Q_k) / nu            (the reorthogonalised candidate, over u)
//   un = (w - sum_k b_k Q_k - c_j q) / nu     (the next candidate, projected once)
// and the dots a' = [Q q]^T un and |un|^2 for the next step:
// partial[k] = Q_k . un (k < NQ), partial[NQ] = q . un, partial[NQ + 1] = un . un.
// NQ is the exact count, as in k_orth.
template <int NQ>
__global__ __launch_bounds__(256) void k_dcgs_update(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ coef, double* u,
                                                     const double* __restrict__ w, double* __restrict__ out,
                                                     double* __restrict__ partial) {
    __shared__ double sh[4];
    __shared__ double cab[2 * (NQ > 0 ? NQ : 1)];
    if (threadIdx.x < NQ) {
        cab[threadIdx.x] = coef[KC_A + threadIdx.x];
        cab[NQ + threadIdx.x] = coef[KC_B + threadIdx.x];
    }
    const double inv_nu = coef[KC_INV_NU];
    const double cj = coef[KC_CJ];
    __syncthreads();
    double acc[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;
    double accq = 0.0, nn = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double v[NQ > 0 ? NQ : 1];
#pragma unroll
        for (int k = 0; k < NQ; ++k) v[k] = V[k * ldv + e];
        double q = u[e];
        double un = w[e];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            q -= cab[k] * v[k];
            un -= cab[NQ + k] * v[k];
        }
        q *= inv_nu;
        un = (un - cj * q) * inv_nu;
        u[e] = q;
        out[e] = un;
#pragma unroll
        for (int k = 0; k < NQ; ++k) acc[k] += v[k] * un;
        accq += q * un;
        nn += un * un;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const double r = block_sum(acc[k], sh);
        if (threadIdx.x == 0) partial[(int64_t)k * KBLOCKS + blockIdx.x] = r;
    }
    double r = block_sum(accq, sh);
    if (threadIdx.x == 0) partial[(int64_t)NQ * KBLOCKS + blockIdx.x] = r;
    r = block_sum(nn, sh);
    if (threadIdx.x == 0) partial[(int64_t)(NQ + 1) * KBLOCKS + blockIdx.x] = r;
}

// Final sums in a fixed order, one wavefront per slot: lane l adds the blocks
// l, l + 64, ... in turn, then a butterfly over the wavefront.  r_q for q = 0..nq:
// d[q] = r_q (q < nq), *nu = r_nq; with coef, the delayed-reorthogonalisation
// coefficients b (r_q, q < nq - 1) and c_j (see launch_orth_reduce).
__global__ __launch_bounds__(1024) void k_orth_reduce(const double* __restrict__ partial, int nb, int nq,
                                                      double* __restrict__ d, double* __restrict__ nu,
                                                      double* __restrict__ coef) {
    __shared__ double res[KMAXQ];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (WAVE - 1);
    for (int q = wave; q <= nq; q += (int)(blockDim.x >> 6)) {
        // all of a lane's loads issued before the first add (KBLOCKS / WAVE of them)
        static_assert(KBLOCKS % WAVE == 0, "whole rounds of block partials");
        double t[KBLOCKS / WAVE];
#pragma unroll
        for (int u = 0; u < KBLOCKS / WAVE; ++u) {
            const int b = lane + u * WAVE;
            t[u] = b < nb ? partial[(int64_t)q * KBLOCKS + b] : 0.0;
        }
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < KBLOCKS / WAVE; ++u) v += t[u];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
        if (lane == 0) res[q] = v;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (d != nullptr && t < nq) d[t] = res[t];
    if (nu != nullptr && t == 0) *nu = res[nq];
    if (coef != nullptr) {
        if (t < nq - 1) coef[KC_B + t] = res[t];
        if (t == 0) {
            double ab = 0.0;
            for (int k = 0; k < nq - 1; ++k) ab += coef[KC_A + k] * res[k];
            coef[KC_CJ] = (res[nq - 1] - ab) * coef[KC_INV_NU];
        }
    }
}

template <class TZ>
__global__ void k_combine(int64_t n, int k, const TZ* __restrict__ Z, int64_t ldz, const double* __restrict__ y,
                          double* __restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double s = x[e];
        for (int q = 0; q < k; ++q) s += y[q] * (double)Z[q * ldz + e];
        x[e] = s;
    }
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = a * x[e] + b * y[e];
}

// dst[p*d + c] = src[perm[p]*d + c]
__global__ void k_gather(int n_rows, int d, const int32_t* __restrict__ perm, const double* __restrict__ src,
                         double* __restrict__ dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rows * d) return;
    int64_t p = t / d;
    int c = (int)(t - p * d);
    dst[t] = src[(int64_t)perm[p] * d + c];
}

__global__ void k_scatter(int n_rows, int d, const int32_t* __restrict__ perm, const double* __restrict__ src,
                          double* __restrict__ dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rows * d) return;
    int64_t p = t / d;
    int c = (int)(t - p * d);
    dst[(int64_t)perm[p] * d + c] = src[t];
}

__global__ void k_c64to32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        b[e] = (float)a[e];
}

__global__ void k_c32to64(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        b[e] = (double)a[e];
}

// seeded start vector in [-1, 1): SplitMix64 output finaliser of (i + seed * golden ratio)
__global__ void k_seeded(int64_t n, uint64_t seed, double* v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = (uint64_t)e + 0x9E3779B97F4A7C15ull * (seed + 1);
        z ^= z >> 30;
        z *= 0xBF58476D1CE4E5B9ull;
        z ^= z >> 27;
        z *= 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[e] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
    }
}

int krylov_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(KBLOCKS, ceil_div(n, 1024))); }

static unsigned stream_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n, 256)));
}

// one instance per basis size 0..32
template <template <int> class L, int... Q>
static void by_count(int nq, std::integer_sequence<int, Q...>, const typename L<0>::Args& a) {
    ((nq == Q ? (L<Q>::run(a), 0) : 0), ...);
}

struct OrthArgs {
    int64_t n;
    const double* V;
    int64_t ldv;
    const double* w;
    double* partial;
    int nblocks;
    hipStream_t s;
};
template <int Q>
struct OrthLaunch {
    using Args = OrthArgs;
    static void run(const OrthArgs& a) { k_orth<Q><<<a.nblocks, 256, 0, a.s>>>(a.n, a.V, a.ldv, a.w, a.partial); }
};

struct DcgsArgs {
    int64_t n;
    const double* V;
    int64_t ldv;
    const double* coef;
    double* u;
    const double* w;
    double* out;
    double* partial;
    int nblocks;
    hipStream_t s;
};
template <int Q>
struct DcgsLaunch {
    using Args = DcgsArgs;
    static void run(const DcgsArgs& a) {
        k_dcgs_update<Q><<<a.nblocks, 256, 0, a.s>>>(a.n, a.V, a.ldv, a.coef, a.u, a.w, a.out, a.partial);
    }
};

void launch_orth(int64_t n, int nq, const double* V, int64_t ldv, const double* w, double* partial, int nblocks,
                 hipStream_t s) {
    MB_CHECK(nq >= 0 && nq <= KMAXQ - 1 && nq <= 32 && nblocks >= 1 && nblocks <= KBLOCKS, MBAMG_E_INVALID,
             "too many Krylov vectors");
    by_count<OrthLaunch>(nq, std::make_integer_sequence<int, 33>{}, OrthArgs{n, V, ldv, w, partial, nblocks, s});
    MB_LAUNCH_CHECK();
}

void launch_dcgs_update(int64_t n, int nq, const double* V, int64_t ldv, const double* coef, double* u,
                        const double* w, double* out, double* partial, int nblocks, hipStream_t s) {
    MB_CHECK(nq >= 0 && nq <= KMAXQ - 2 && nq <= 31 && nblocks >= 1 && nblocks <= KBLOCKS, MBAMG_E_INVALID,
             "too many Krylov vectors");
    by_count<DcgsLaunch>(nq, std::make_integer_sequence<int, 32>{},
                         DcgsArgs{n, V, ldv, coef, u, w, out, partial, nblocks, s});
    MB_LAUNCH_CHECK();
}

void launch_orth_reduce(const double* partial, int nblocks, int nq, double* d, double* nu, double* coef,
                        hipStream_t s) {
    MB_CHECK(nq >= 0 && nq <= KMAXQ - 1 && nblocks >= 1 && nblocks <= KBLOCKS && (coef == nullptr || nq >= 1),
             MBAMG_E_INVALID, "invalid Krylov reduction");
    k_orth_reduce<<<1, 1024, 0, s>>>(partial, nblocks, nq, d, nu, coef);
    MB_LAUNCH_CHECK();
}

void launch_combine(int64_t n, int k, const double* Z, int64_t ldz, const double* y, double* x, hipStream_t s) {
    if (k <= 0) return;
    k_combine<double><<<stream_grid(n), 256, 0, s>>>(n, k, Z, ldz, y, x);
    MB_LAUNCH_CHECK();
}

void launch_combine32(int64_t n, int k, const float* Z, int64_t ldz, const double* y, double* x, hipStream_t s) {
    if (k <= 0) return;
    k_combine<float><<<stream_grid(n), 256, 0, s>>>(n, k, Z, ldz, y, x);
    MB_LAUNCH_CHECK();
}

void launch_seeded(int64_t n, uint64_t seed, double* v, hipStream_t s) {
    k_seeded<<<stream_grid(n), 256, 0, s>>>(n, seed, v);
    MB_LAUNCH_CHECK();
}

void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
    k_axpby<<<stream_grid(n), 256, 0, s>>>(n, a, x, b, y);
    MB_LAUNCH_CHECK();
}

void launch_gather(int n_rows, int d, const int32_t* perm, const double* src, double* dst, hipStream_t s) {
    int64_t n = (int64_t)n_rows * d;
    if (n == 0) return;
    MB_CHECK(perm && src && dst, MBAMG_E_INVALID, "gather: NULL pointer");
    k_gather<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n_rows, d, perm, src, dst);
    MB_LAUNCH_CHECK();
}

void launch_scatter(int n_rows, int d, const int32_t* perm, const double* src, double* dst, hipStream_t s) {
    int64_t n = (int64_t)n_rows * d;
    if (n == 0) return;
    MB_CHECK(perm && src && dst, MBAMG_E_INVALID, "scatter: NULL pointer");
    k_scatter<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n_rows, d, perm, src, dst);
    MB_LAUNCH_CHECK();
}

void launch_cast64to32(int64_t n, const double* a, float* b, hipStream_t s) {
    if (n == 0) return;
    k_c64to32<<<stream_grid(n), 256, 0, s>>>(n, a, b);
    MB_LAUNCH_CHECK();
}

void launch_cast32to64(int64_t n, const float* a, double* b, hipStream_t s) {
    if (n == 0) return;
    k_c32to64<<<stream_grid(n), 256, 0, s>>>(n, a, b);
    MB_LAUNCH_CHECK();
}

}  // namespace mbamg
