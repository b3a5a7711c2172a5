// Setup-phase kernels: strength graph, distance-2 aggregation, tentative
// prolongator, Galerkin products, nodal block inverses, packing into the
// smoother's sliced format and the coarsest-level inverse.
//
// This translation unit is compiled with -ffp-contract=off: every product and
// sum is one IEEE rounding in the order written, so the squared block norms,
// aggregate norms and Galerkin sums come out bit-identical to a sequential
// evaluation in the same order.  That keeps the aggregates of coarse levels
// (which compare those numbers) reproducible.
#include "setup_kernels.h"

#include <utility>
#include <cstdlib>
#include <cstring>

namespace mbamg {

// ----------------------------------------------------------------------------
// scan (exclusive, int32 in, int32 out): per-block sums, one-block scan of the
// block sums, then per-block local scans.  1024 items per block.
// ----------------------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_BLOCK = SCAN_T * SCAN_ITEMS;

__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int incl = sh[t];
    *total = sh[SCAN_T - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_blocksum(const int32_t* in, int64_t n, int32_t* bsum) {
    __shared__ int sh[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    int total;
    block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void k_scan_sums(int32_t* bsum, int nb, int32_t* grand) {
    __shared__ int sh[SCAN_T];
    int carry = 0;
    for (int base = 0; base < nb; base += SCAN_T) {
        int i = base + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, sh, &total);
        if (i < nb) bsum[i] = ex + carry;
        carry += total;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void k_scan_final(const int32_t* in, int64_t n, const int32_t* bsum, int32_t* out) {
    __shared__ int sh[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, sh, &total) + bsum[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

// out[i] = sum_{k<i} in[k] for i in [0, n]; out has n+1 entries.  Returns the total.
int scan_exclusive(const int32_t* in, int64_t n, int32_t* out, hipStream_t s) {
    int nb = (int)std::max<int64_t>(1, ceil_div(n, SCAN_BLOCK));
    DevBuf<int32_t> bsum(nb);
    k_scan_blocksum<<<nb, SCAN_T, 0, s>>>(in, n, bsum.p);
    MB_LAUNCH_CHECK();
    k_scan_sums<<<1, SCAN_T, 0, s>>>(bsum.p, nb, out + n);
    MB_LAUNCH_CHECK();
    k_scan_final<<<nb, SCAN_T, 0, s>>>(in, n, bsum.p, out);
    MB_LAUNCH_CHECK();
    int32_t total = 0;
    MB_HIP(hipMemcpyAsync(&total, out + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    return total;
}

// ----------------------------------------------------------------------------
// strength graph
// ----------------------------------------------------------------------------
// Kernel-form overrides for tests: every form computes the same sums in the
// same order, so a hierarchy must come out bit-identical under each.
//   MBAMG_SA_FORM     = thread | wave | generic   (smoothed prolongator)
//   MBAMG_SPGEMM_FORM = block | chunk2 | chunk4 | entry | fused
//                                                  (numeric Galerkin product: thread per
//                                                   output block with 1, 2 or 4 lookups
//                                                   in flight, lane per entry, or one
//                                                   launch for every group of pairs)
//   MBAMG_SORT_FORM   = thread | wave              (aggregate member lists)
//   MBAMG_SYM_FORM    = thread | wave              (product pattern)
//   MBAMG_ROWS_FORM   = rows | sliced              (coarse-level smoother layout;
//                                                   changes the summation order)
const char* form_override(const char* var) {
    const char* v = std::getenv(var);
    return (v && *v) ? v : nullptr;
}

__device__ inline int find_col(const int32_t* ci, int lo, int hi, int key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int c = ci[mid];
        if (c == key) return mid;
        if (c < key) lo = mid + 1; else hi = mid;
    }
    return -1;
}

__global__ void k_block_sqnorm(const double* val, int64_t nnzb, int bs, double* n2) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnzb) return;
    const double* v = val + p * bs;
    double acc = v[0] * v[0];
    for (int k = 1; k < bs; ++k) acc = acc + v[k] * v[k];
    n2[p] = acc;
}

// pass 0: count strong neighbours per row; pass 1: write them.
__global__ void k_strength(int n, const int32_t* rp, const int32_t* ci, const double* n2, double t4,
                           int pass, int32_t* cnt, const int32_t* sptr, int32_t* sidx, double* sw2,
                           int32_t* asym) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = rp[i], e = rp[i + 1];
    int pd = find_col(ci, b, e, i);
    double dn2i = pd >= 0 ? n2[pd] : 0.0;
    int c = 0;
    int out = pass ? sptr[i] : 0;
    for (int p = b; p < e; ++p) {
        int j = ci[p];
        if (j == i) continue;
        int q = find_col(ci, rp[j], rp[j + 1], i);
        if (q < 0) { if (pass == 0) atomicAdd(asym, 1); continue; }
        double a = n2[p], t = n2[q];
        double w2 = a > t ? a : t;
        int pj = find_col(ci, rp[j], rp[j + 1], j);
        double dn2j = pj >= 0 ? n2[pj] : 0.0;
        bool strong = (w2 > 0.0) && (w2 * w2 >= t4 * (dn2i * dn2j));
        if (!strong) continue;
        if (pass) { sidx[out + c] = j; sw2[out + c] = w2; }
        ++c;
    }
    if (!pass) cnt[i] = c;
}

// ----------------------------------------------------------------------------
// distance-2 maximal independent set with fixed priorities
// ----------------------------------------------------------------------------
__device__ inline uint64_t splitmix_final(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

__global__ void k_keys(int n, uint64_t mult, uint64_t* key, int8_t* state) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t h = splitmix_final((uint64_t)i + mult) >> 32;
    key[i] = (h << 32) | (uint64_t)(uint32_t)i;
    state[i] = 0;
}

// best1[i] = undecided node of largest key in {i} U N(i), or -1
__global__ void k_mis_a(int n, const int32_t* sp, const int32_t* si, const uint64_t* key, const int8_t* state,
                        int32_t* best1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int best = state[i] == 0 ? i : -1;
    for (int p = sp[i]; p < sp[i + 1]; ++p) {
        int j = si[p];
        if (state[j] == 0 && (best < 0 || key[j] > key[best])) best = j;
    }
    best1[i] = best;
}

// undecided i becomes a root when it has the largest key among undecided nodes within two hops
__global__ void k_mis_b(int n, const int32_t* sp, const int32_t* si, const uint64_t* key, const int32_t* best1,
                        int8_t* state) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || state[i] != 0) return;
    int best = best1[i];
    for (int p = sp[i]; p < sp[i + 1]; ++p) {
        int c = best1[si[p]];
        if (c >= 0 && (best < 0 || key[c] > key[best])) best = c;
    }
    if (best == i) state[i] = 1;
}

__global__ void k_mis_c(int n, const int32_t* sp, const int32_t* si, const int8_t* state, int8_t* near1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int8_t f = state[i] == 1;
    for (int p = sp[i]; p < sp[i + 1] && !f; ++p) f = state[si[p]] == 1;
    near1[i] = f;
}

__global__ void k_mis_d(int n, const int32_t* sp, const int32_t* si, const int8_t* near1, int8_t* state,
                        int32_t* undecided) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || state[i] != 0) return;
    int8_t f = near1[i];
    for (int p = sp[i]; p < sp[i + 1] && !f; ++p) f = near1[si[p]];
    if (f) state[i] = 2;
    else atomicAdd(undecided, 1);
}

__global__ void k_is_root(int n, const int8_t* state, int32_t* flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = state[i] == 1;
}

__global__ void k_phase1(int n, const int32_t* sp, const int32_t* si, const int8_t* state, const int32_t* rootscan,
                         int32_t* phase1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || state[i] != 1) return;
    int id = rootscan[i];
    phase1[i] = id;
    for (int p = sp[i]; p < sp[i + 1]; ++p) phase1[si[p]] = id;   // root neighbourhoods are disjoint
}

__global__ void k_phase2(int n, const int32_t* sp, const int32_t* si, const double* sw2, const int32_t* phase1,
                         int32_t* agg, int32_t* fail) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a1 = phase1[i];
    if (a1 >= 0) { agg[i] = a1; return; }
    int best = -1;
    double bw = 0.0;
    for (int p = sp[i]; p < sp[i + 1]; ++p) {
        int a = phase1[si[p]];
        if (a < 0) continue;
        double w = sw2[p];
        if (best < 0 || w > bw || (w == bw && a < best)) { best = a; bw = w; }
    }
    if (best < 0) { atomicAdd(fail, 1); best = 0; }
    agg[i] = best;
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_count_members(int n, const int32_t* agg, int32_t* cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[agg[i]], 1);
}

__global__ void k_place_members(int n, const int32_t* agg, const int32_t* mptr, int32_t* cursor, int32_t* midx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int k = agg[i];
    int slot = atomicAdd(&cursor[k], 1);
    midx[mptr[k] + slot] = i;
}

__global__ void k_sort_members(int nagg, const int32_t* mptr, int32_t* midx) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nagg) return;
    int b = mptr[k], e = mptr[k + 1];
    for (int a = b + 1; a < e; ++a) {
        int v = midx[a];
        int c = a - 1;
        while (c >= b && midx[c] > v) { midx[c + 1] = midx[c]; --c; }
        midx[c + 1] = v;
    }
}

// the same with one wavefront per aggregate (large aggregates on coarse
// levels): members ranked in LDS; longer lists than the LDS copy holds take
// the one-lane insertion sort
constexpr int SORT_LDS = 2048;
__global__ __launch_bounds__(WAVE) void k_sort_members_w(int nagg, const int32_t* mptr, int32_t* midx) {
    __shared__ int32_t v[SORT_LDS];
    const int k = blockIdx.x, lane = threadIdx.x;
    const int b = mptr[k], e = mptr[k + 1], m = e - b;
    if (m > SORT_LDS) {
        if (lane == 0)
            for (int a = b + 1; a < e; ++a) {
                const int x = midx[a];
                int c = a - 1;
                while (c >= b && midx[c] > x) {
                    midx[c + 1] = midx[c];
                    --c;
                }
                midx[c + 1] = x;
            }
        return;
    }
    for (int t = lane; t < m; t += WAVE) v[t] = midx[b + t];
    __syncthreads();
    for (int t = lane; t < m; t += WAVE) {
        const int key = v[t];
        int r = 0;
        for (int u = 0; u < m; ++u) r += v[u] < key;
        midx[b + r] = key;
    }
}

// ----------------------------------------------------------------------------
// tentative prolongator: q = B / ||B over the aggregate||, per component
// ----------------------------------------------------------------------------
// one thread per (aggregate, component); each sum over the members in order
__global__ void k_tentative(int nagg, int d, const int32_t* mptr, const int32_t* midx, const double* B,
                            double* q, double* Bc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nagg * d) return;
    const int k = (int)(t / d), c = (int)(t % d);
    int b = mptr[k], e = mptr[k + 1];
    {
        double acc = 0.0;
        for (int m = b; m < e; ++m) {
            double v = B[(int64_t)midx[m] * d + c];
            acc = acc + v * v;
        }
        double nrm = sqrt(acc);
        Bc[(int64_t)k * d + c] = nrm;
        for (int m = b; m < e; ++m) {
            int64_t o = (int64_t)midx[m] * d + c;
            q[o] = B[o] / nrm;
        }
    }
}

// the tentative prolongator as a block matrix: row i holds one block, in
// column agg(i), equal to diag(q_i)
__global__ void k_tentative_bsr(int n, int d, const int32_t* agg, const double* q, int32_t* rp, int32_t* ci,
                                double* val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    rp[i] = i;
    if (i == n) return;
    ci[i] = agg[i];
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) val[(int64_t)i * d * d + r * d + c] = r == c ? q[(int64_t)i * d + r] : 0.0;
}

__global__ void k_fill_f64(double* a, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}


// ----------------------------------------------------------------------------
// nodal block inverses: LU with partial pivoting of the diagonal block, d <= 8
// ----------------------------------------------------------------------------
// x = a^-1 for a d x d block (d <= 8, row-major) by LU with partial pivoting,
// the identity's columns solved one by one; false (a overwritten) when a
// pivot is zero
__device__ bool lu_inverse(double (&a)[64], int d, double (&x)[64]) {
    int piv[8];
    for (int k = 0; k < d; ++k) {
        int p = k;
        double m = fabs(a[k * d + k]);
        for (int r = k + 1; r < d; ++r)
            if (fabs(a[r * d + k]) > m) { m = fabs(a[r * d + k]); p = r; }
        piv[k] = p;
        if (m == 0.0) return false;
        if (p != k)
            for (int c = 0; c < d; ++c) { double t = a[k * d + c]; a[k * d + c] = a[p * d + c]; a[p * d + c] = t; }
        for (int r = k + 1; r < d; ++r) {
            double l = a[r * d + k] / a[k * d + k];
            a[r * d + k] = l;
            for (int c = k + 1; c < d; ++c) a[r * d + c] = a[r * d + c] - l * a[k * d + c];
        }
    }
    for (int col = 0; col < d; ++col) {
        double y[8];
        for (int r = 0; r < d; ++r) y[r] = r == col ? 1.0 : 0.0;
        for (int k = 0; k < d; ++k) { double t = y[k]; y[k] = y[piv[k]]; y[piv[k]] = t; }
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < r; ++c) y[r] = y[r] - a[r * d + c] * y[c];
        for (int r = d - 1; r >= 0; --r) {
            for (int c = r + 1; c < d; ++c) y[r] = y[r] - a[r * d + c] * y[c];
            y[r] = y[r] / a[r * d + r];
        }
        for (int r = 0; r < d; ++r) x[r * d + col] = y[r];
    }
    return true;
}

__global__ void k_dinv(int n, int d, const int32_t* rp, const int32_t* ci, const double* val, double* dinv,
                       int32_t* singular) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[64], x[64];
    const int bs = d * d;
    int pd = find_col(ci, rp[i], rp[i + 1], i);
    for (int k = 0; k < bs; ++k) a[k] = pd >= 0 ? val[(int64_t)pd * bs + k] : 0.0;
    if (!lu_inverse(a, d, x)) {
        atomicAdd(singular, 1);
        for (int k = 0; k < bs; ++k) dinv[(int64_t)i * bs + k] = 0.0;
        return;
    }
    for (int k = 0; k < bs; ++k) dinv[(int64_t)i * bs + k] = x[k];
}

// Inverse of the full node block D_i = [[A00_ii, A01_ii], [A10_ii, A11_ii]]
// (m = d0 + d1 <= 8, row-major) of every node
struct NodeBlocks {
    const int32_t* rp[4];
    const int32_t* ci[4];
    const double* val[4];
};
__global__ void k_node_inv(int n, int d0, int d1, NodeBlocks B, double* inv, int32_t* singular) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = d0 + d1;
    double a[64], x[64];
    for (int k = 0; k < m * m; ++k) a[k] = 0.0;
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g) {
            const int q = f * 2 + g;
            if (!B.rp[q]) continue;
            const int br = f ? d1 : d0, bc = g ? d1 : d0;
            const int pd = find_col(B.ci[q], B.rp[q][i], B.rp[q][i + 1], i);
            if (pd < 0) continue;
            for (int r = 0; r < br; ++r)
                for (int c = 0; c < bc; ++c)
                    a[(f * d0 + r) * m + g * d0 + c] = B.val[q][(int64_t)pd * br * bc + r * bc + c];
        }
    if (!lu_inverse(a, m, x)) {
        atomicAdd(singular, 1);
        for (int k = 0; k < m * m; ++k) inv[(int64_t)i * m * m + k] = 0.0;
        return;
    }
    for (int k = 0; k < m * m; ++k) inv[(int64_t)i * m * m + k] = x[k];
}

// Masked slice-major layout of the node inverses for the smoother: per slice,
// bit k of mask[s] is set when entry k is nonzero for some row of the slice;
// the set entries follow each other as groups of 64 values (one per lane) from
// group off[s].  One wavefront per slice: the mask and its group count.
__global__ void k_node_inv_mask(int n_slices, int mm, const int32_t* row0, const int32_t* nrow, const int32_t* perm,
                                const double* in, uint64_t* mask, int32_t* cnt) {
    const int s = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    if (s >= n_slices) return;   // whole wavefronts
    const int lane = threadIdx.x & (WAVE - 1);
    const bool live = lane < nrow[s];
    const int64_t base = live ? (int64_t)perm[row0[s] + lane] * mm : 0;
    uint64_t m = 0;
    for (int k = 0; k < mm; ++k)
        if (__ballot(live && in[base + k] != 0.0) != 0) m |= (uint64_t)1 << k;
    if (lane == 0) {
        mask[s] = m;
        cnt[s] = __popcll(m);
    }
}

template <class T>
__global__ void k_node_inv_pack(int n_slices, int mm, const int32_t* row0, const int32_t* nrow, const int32_t* perm,
                                const double* in, const uint64_t* mask, const int32_t* off, T* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_slices * mm * WAVE) return;
    const int lane = (int)(t % WAVE);
    const int64_t sk = t / WAVE;
    const int s = (int)(sk / mm), k = (int)(sk % mm);
    const uint64_t m = mask[s];
    if (!((m >> k) & 1)) return;
    const int g = __popcll(m & (((uint64_t)1 << k) - 1));
    out[((int64_t)off[s] + g) * WAVE + lane] =
        lane < nrow[s] ? (T)in[(int64_t)perm[row0[s] + lane] * mm + k] : T(0);
}

// flag (initially 1) is cleared when a block of B lies outside A's pattern
__global__ void k_subpattern(int n, const int32_t* __restrict__ rpa, const int32_t* __restrict__ cia,
                             const int32_t* __restrict__ rpb, const int32_t* __restrict__ cib, int32_t* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int p = rpb[i]; p < rpb[i + 1]; ++p)
        if (find_col(cia, rpa[i], rpa[i + 1], cib[p]) < 0) {
            atomicAnd(flag, 0);
            return;
        }
}

// ----------------------------------------------------------------------------
// packing into masked slices: src[slot*64 + lane] is the source block index
// (-1 for padding); mask bit k of a slot is set when entry k is nonzero in any
// lane's block.
// ----------------------------------------------------------------------------
// One wavefront per slot (one lane per row): the slot's mask is the OR of the
// lanes' nonzero patterns and slot_nz the sum of their nonzero counts.
// One wavefront per slot of 64 rows; the 64 source blocks (bs <= 16 entries,
// src < 0: padding) are read 4 at a time, 16 lanes per block, so every load
// is a contiguous block.  mask = entries nonzero in any row of the slot,
// slot_nz = nonzero entries over the slot.
__global__ __launch_bounds__(256) void k_sell_mask(int64_t n_slots, int bs, const int64_t* __restrict__ src,
                                                   const double* __restrict__ val, uint32_t* mask,
                                                   uint32_t* slot_nz) {
    const int64_t slot = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (slot >= n_slots) return;   // whole wavefronts
    const int lane = threadIdx.x & (WAVE - 1), k = lane & 15, sub = lane >> 4;
    uint32_t m = 0, nz = 0;
    for (int it = 0; it < WAVE / 4; ++it) {
        const int64_t sb = src[slot * WAVE + it * 4 + sub];
        const bool on = sb >= 0 && k < bs && val[sb * bs + k] != 0.0;
        const uint64_t bal = __ballot(on);
        nz += (uint32_t)__popcll(bal);
        m |= (uint32_t)((bal | (bal >> 16) | (bal >> 32) | (bal >> 48)) & 0xFFFFu);
    }
    if (lane == 0) {
        mask[slot] = m;
        slot_nz[slot] = nz;
    }
}

// The slot's blocks are staged through LDS (read as in k_sell_mask) and
// written entry by entry of the mask, 64 rows per entry.
__global__ __launch_bounds__(256) void k_sell_fill(int64_t n_slots, int bs, const int64_t* __restrict__ src,
                                                   const double* __restrict__ val, const uint32_t* __restrict__ mask,
                                                   const int64_t* __restrict__ slot_voff, double* out) {
    __shared__ double tile[256 / WAVE][WAVE][17];
    const int64_t slot = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (slot >= n_slots) return;   // whole wavefronts; no block-wide barrier below
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1), k = lane & 15, sub = lane >> 4;
    for (int it = 0; it < WAVE / 4; ++it) {
        const int row = it * 4 + sub;
        const int64_t sb = src[slot * WAVE + row];
        tile[w][row][k] = (sb >= 0 && k < bs) ? val[sb * bs + k] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t m = mask[slot];
    int64_t g = slot_voff[slot];
    for (int e = 0; e < bs; ++e) {
        if (!(m & (1u << e))) continue;
        out[g * WAVE + lane] = tile[w][lane][e];
        ++g;
    }
}

__global__ void k_cast_f64_f32(const double* a, float* b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ----------------------------------------------------------------------------
// smoothed prolongator, block transpose and the generic ordered block product
// ----------------------------------------------------------------------------
// P = Phat - D_vv^-1 A_vv Phat W on the vector components.  Row i lists agg(i)
// and the aggregates k of its columns with w[k] != 0, in increasing order.
// Vector entry (a,c) of block (i,k): s = sum over the row's columns j in
// increasing order with agg(j) = k of A[i,j][a][c] * q[j,c];
// P = base - w[k] * (s / A[i,i][a][a]) with base = q[i,a] on (k = agg(i), c = a).
// Smoothed prolongator row i: the distinct kept aggregates l of row i in
// increasing order; block (i,l) = [l == agg(i)] diag(q_i) - w_l D_i^-1 sum over
// the row's entries p with agg(col p) == l, in increasing p, of A_p diag(q_col).
// Any row length, one thread, no local storage.
__device__ void sa_row_generic(int i, int d, int nv, const int32_t* rp, const int32_t* ci, const double* val,
                               const int32_t* agg, const double* q, const double* w, int pass, int32_t* cnt,
                               const int32_t* prp, int32_t* pci, double* pval) {
    const int b = rp[i], e = rp[i + 1], bs = d * d, ai = agg[i];
    int pd = find_col(ci, b, e, i);
    int prev = -1, out = pass ? prp[i] : 0, c = 0;
    while (true) {
        int l = INT_MAX;
        for (int p = b; p < e; ++p) {
            int a = agg[ci[p]];
            if (a != ai && w[a] == 0.0) continue;
            if (a > prev && a < l) l = a;
        }
        if (l == INT_MAX) break;
        if (pass) {
            double* blk = pval + (int64_t)(out + c) * bs;
            pci[out + c] = l;
            for (int ra = 0; ra < d; ++ra)
                for (int cc = 0; cc < d; ++cc) {
                    double base = (l == ai && cc == ra) ? q[(int64_t)i * d + ra] : 0.0;
                    if (ra < nv && cc < nv) {
                        double acc = 0.0;
                        for (int p = b; p < e; ++p) {
                            int j = ci[p];
                            if (agg[j] != l) continue;
                            double term = val[(int64_t)p * bs + ra * d + cc] * q[(int64_t)j * d + cc];
                            acc = acc + term;
                        }
                        // a missing diagonal block gives inf here; the nodal inverses report it as singular
                        double dg = pd >= 0 ? val[(int64_t)pd * bs + ra * d + ra] : 0.0;
                        double t = acc / dg;
                        double u = w[l] * t;
                        blk[ra * d + cc] = base - u;
                    } else {
                        blk[ra * d + cc] = base;
                    }
                }
        }
        ++c;
        prev = l;
    }
    if (!pass) cnt[i] = c;
}

// One thread per row: rows of at most SA_REG entries keep their columns and
// aggregates in registers and read each block of A once; longer rows take
// the generic form.  Same sums in the same order.
constexpr int SA_REG = 16;
template <int D>
__global__ __launch_bounds__(128) void k_sa_prolong_t(int n, int nv, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const double* __restrict__ val, const int32_t* __restrict__ agg,
                               const double* __restrict__ q, const double* __restrict__ w, int pass, int32_t* cnt,
                               const int32_t* prp, int32_t* pci, double* pval, int generic_only) {
    constexpr int BS = D * D;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = rp[i], e = rp[i + 1], ai = agg[i];
    if (e - b > SA_REG || generic_only) {
        sa_row_generic(i, D, nv, rp, ci, val, agg, q, w, pass, cnt, prp, pci, pval);
        return;
    }
    int jj[SA_REG], ag[SA_REG];   // ag = INT_MAX: no entry, or an aggregate that is not kept
#pragma unroll
    for (int u = 0; u < SA_REG; ++u) {
        jj[u] = 0;
        ag[u] = INT_MAX;
        if (b + u < e) {
            jj[u] = ci[b + u];
            const int a = agg[jj[u]];
            if (a == ai || w[a] != 0.0) ag[u] = a;
        }
    }
    double dg[D];
    if (pass) {
        const int pd = find_col(ci, b, e, i);
#pragma unroll
        for (int r = 0; r < D; ++r) dg[r] = pd >= 0 ? val[(int64_t)pd * BS + r * D + r] : 0.0;
    }
    int prev = -1, c = 0;
    const int out = pass ? prp[i] : 0;
    while (true) {
        int l = INT_MAX;
#pragma unroll
        for (int u = 0; u < SA_REG; ++u)
            if (ag[u] > prev && ag[u] < l) l = ag[u];
        if (l == INT_MAX) break;
        if (pass) {
            double acc[BS];
#pragma unroll
            for (int x = 0; x < BS; ++x) acc[x] = 0.0;
#pragma unroll
            for (int u = 0; u < SA_REG; ++u) {
                if (ag[u] != l) continue;
                const double* vb = val + (int64_t)(b + u) * BS;
                double qj[D];
#pragma unroll
                for (int cc = 0; cc < D; ++cc) qj[cc] = q[(int64_t)jj[u] * D + cc];
#pragma unroll
                for (int x = 0; x < BS; ++x) {
                    const double term = vb[x] * qj[x % D];
                    acc[x] = acc[x] + term;
                }
            }
            double* blk = pval + (int64_t)(out + c) * BS;
            pci[out + c] = l;
            const double wl = w[l];
#pragma unroll
            for (int ra = 0; ra < D; ++ra)
#pragma unroll
                for (int cc = 0; cc < D; ++cc) {
                    const double base = (l == ai && cc == ra) ? q[(int64_t)i * D + ra] : 0.0;
                    if (ra < nv && cc < nv) {
                        const double t = acc[ra * D + cc] / dg[ra];
                        const double u = wl * t;
                        blk[ra * D + cc] = base - u;
                    } else {
                        blk[ra * D + cc] = base;
                    }
                }
        }
        ++c;
        prev = l;
    }
    if (!pass) cnt[i] = c;
}

__global__ void k_count_cols(int n, const int32_t* rp, const int32_t* ci, int32_t* cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void k_place_cols(int n, const int32_t* rp, const int32_t* ci, const int32_t* trp, int32_t* cursor,
                             int32_t* trow, int32_t* tsrc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int c = ci[p];
        int slot = trp[c] + atomicAdd(&cursor[c], 1);
        trow[slot] = i;
        tsrc[slot] = p;
    }
}

// C = A B.  Row i of C lists the distinct columns reached through row i of A,
// in increasing order; entry (r,c) of block (i,l) sums A[i,j][r][m]*B[j,l][m][c]
// over the columns j of row i in increasing order and, for each, m increasing.
__global__ void k_spgemm(int n, int br, int bm, int bc, const int32_t* arp, const int32_t* aci, const double* aval,
                         const int32_t* brp, const int32_t* bci, const double* bval, int pass, int32_t* cnt,
                         const int32_t* crp, int32_t* cci, double* cval) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ab = arp[i], ae = arp[i + 1];
    int prev = -1, out = pass ? crp[i] : 0, c = 0;
    while (true) {
        int l = INT_MAX;
        for (int p = ab; p < ae; ++p) {
            int j = aci[p];
            for (int q = brp[j]; q < brp[j + 1]; ++q) {
                int col = bci[q];
                if (col > prev) {
                    if (col < l) l = col;
                    break;     // columns of B's row increase: the first above prev is the smallest
                }
            }
        }
        if (l == INT_MAX) break;
        if (pass) {
            double acc[16];
            for (int e = 0; e < br * bc; ++e) acc[e] = 0.0;
            for (int p = ab; p < ae; ++p) {
                int j = aci[p];
                int q = find_col(bci, brp[j], brp[j + 1], l);
                if (q < 0) continue;
                const double* a = aval + (int64_t)p * br * bm;
                const double* bb = bval + (int64_t)q * bm * bc;
                for (int r = 0; r < br; ++r)
                    for (int cc = 0; cc < bc; ++cc)
                        for (int m = 0; m < bm; ++m) {
                            double term = a[r * bm + m] * bb[m * bc + cc];
                            acc[r * bc + cc] = acc[r * bc + cc] + term;
                        }
            }
            cci[out + c] = l;
            double* dst = cval + (int64_t)(out + c) * br * bc;
            for (int e = 0; e < br * bc; ++e) dst[e] = acc[e];
        }
        ++c;
        prev = l;
    }
    if (!pass) cnt[i] = c;
}

// ----------------------------------------------------------------------------
// Wave-per-row forms of the products above.  One 64-lane wavefront (one
// workgroup) owns one output row: its distinct output columns are gathered in
// an LDS hash set and ranked into increasing order.  Values are computed with
// the same summation order as the thread-per-row kernels (over the row's
// columns in increasing order, m increasing), so the results are
// bit-identical.  Rows with more than KS_MAX distinct columns raise an
// overflow flag and the host reruns that product with the thread-per-row
// kernels.
// ----------------------------------------------------------------------------
constexpr int KS_LOG = 10;
constexpr int KS_TABLE = 1 << KS_LOG;   // hash slots (at most half full)
constexpr int KS_MAX = KS_TABLE / 2;    // distinct columns per row

struct KeySet {
    int32_t table[KS_TABLE];
    int32_t keys[KS_MAX];
    int32_t sorted[KS_MAX];
    int32_t count;
    int32_t overflow;
    int32_t tlog;
};

// a table of 2^tlog slots, sized so that `cand` insertions fill at most half
__device__ inline void ks_clear(KeySet& S, int lane, int64_t cand) {
    int tlog = 6;
    while (tlog < KS_LOG && ((int64_t)1 << (tlog - 1)) < cand) ++tlog;
    for (int t = lane; t < (1 << tlog); t += WAVE) S.table[t] = -1;
    if (lane == 0) {
        S.count = 0;
        S.overflow = 0;
        S.tlog = tlog;
    }
    __syncthreads();
}

__device__ inline void ks_insert(KeySet& S, int key) {
    const int tlog = S.tlog;
    const uint32_t mask = (1u << tlog) - 1;
    uint32_t h = ((uint32_t)key * 2654435761u) >> (32 - tlog);
    for (int probe = 0; probe <= (int)mask; ++probe) {
        const int prev = atomicCAS(&S.table[h], -1, key);
        if (prev == -1) {
            const int idx = atomicAdd(&S.count, 1);
            if (idx < (1 << (tlog - 1))) S.keys[idx] = key;
            else S.overflow = 1;
            return;
        }
        if (prev == key) return;
        h = (h + 1) & mask;
    }
    S.overflow = 1;
}

// number of distinct keys after the inserts, or -1 on overflow (call after a barrier)
__device__ inline int ks_count(const KeySet& S) { return (S.overflow || S.count > KS_MAX) ? -1 : S.count; }

// sorted[0..K) = keys in increasing order (keys are distinct)
__device__ inline void ks_sort(KeySet& S, int lane, int K) {
    for (int t = lane; t < K; t += WAVE) {
        const int key = S.keys[t];
        int r = 0;
        for (int u = 0; u < K; ++u) r += S.keys[u] < key;
        S.sorted[r] = key;
    }
    __syncthreads();
}

// Pattern of C = A B, one thread per row: the row's distinct columns kept
// sorted in registers (at most SYM_REG; more sets *overflow and the caller
// takes the wavefront form).  Pass 0 counts, pass 1 writes.
constexpr int SYM_REG = 32;
__global__ __launch_bounds__(128) void k_spgemm_sym_t(int n, const int32_t* __restrict__ arp,
                                                      const int32_t* __restrict__ aci,
                                                      const int32_t* __restrict__ brp,
                                                      const int32_t* __restrict__ bci, int pass, int32_t* cnt,
                                                      const int32_t* crp, int32_t* cci, int32_t* overflow) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cols[SYM_REG];
#pragma unroll
    for (int u = 0; u < SYM_REG; ++u) cols[u] = INT_MAX;
    int k = 0;
    for (int p = arp[i]; p < arp[i + 1]; ++p) {
        const int j = aci[p];
        for (int q = brp[j]; q < brp[j + 1]; ++q) {
            const int c = bci[q];
            int pos = 0;
            bool present = false;
#pragma unroll
            for (int u = 0; u < SYM_REG; ++u) {
                pos += cols[u] < c;
                present |= cols[u] == c;
            }
            if (present) continue;
            if (k == SYM_REG) {
                atomicOr(overflow, 1);
                return;
            }
#pragma unroll
            for (int u = SYM_REG - 1; u > 0; --u)
                if (u > pos) cols[u] = cols[u - 1];
#pragma unroll
            for (int u = 0; u < SYM_REG; ++u)
                if (u == pos) cols[u] = c;
            ++k;
        }
    }
    if (!pass) {
        cnt[i] = k;
        return;
    }
    const int out = crp[i];
#pragma unroll
    for (int u = 0; u < SYM_REG; ++u)
        if (u < k) cci[out + u] = cols[u];
}

// Pattern of C = A B: pass 0 counts each row's distinct columns, pass 1
// writes them in increasing order.  The candidates (the columns of the B rows
// named by the row of A) are enumerated flat: for up to 64 entries of the A
// row at a time, every lane fetches one entry's B row range, a wavefront scan
// of the range lengths places them end to end, and each lane then takes every
// 64th candidate, so the loads of all the B rows are in flight together.
__global__ __launch_bounds__(WAVE) void k_spgemm_sym(const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                                     const int32_t* __restrict__ brp, const int32_t* __restrict__ bci,
                                                     int pass, int32_t* cnt, const int32_t* crp, int32_t* cci,
                                                     int32_t* overflow) {
    __shared__ KeySet S;
    __shared__ int32_t s_start[WAVE], s_base[WAVE];
    const int i = blockIdx.x, lane = threadIdx.x;
    const int ab = arp[i], ae = arp[i + 1];
    int64_t cand = 0;
    for (int c0 = ab; c0 < ae; c0 += WAVE) {
        const int p = c0 + lane;
        int len = 0;
        if (p < ae) {
            const int j = aci[p];
            len = brp[j + 1] - brp[j];
        }
        for (int off = WAVE / 2; off > 0; off >>= 1) len += __shfl_xor(len, off);
        cand += len;
    }
    ks_clear(S, lane, cand);
    for (int c0 = ab; c0 < ae; c0 += WAVE) {
        const int p = c0 + lane;
        int b0 = 0, len = 0;
        if (p < ae) {
            const int j = aci[p];
            b0 = brp[j];
            len = brp[j + 1] - b0;
        }
        int incl = len;   // inclusive scan of the lengths over the lanes
        for (int off = 1; off < WAVE; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        const int total = __shfl(incl, WAVE - 1);
        s_start[lane] = incl - len;
        s_base[lane] = b0;
        __syncthreads();
        for (int t = lane; t < total; t += WAVE) {
            // the entry whose range holds candidate t: the last one starting at or before t
            int lo = 0, hi = WAVE - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_start[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            ks_insert(S, bci[s_base[lo] + (t - s_start[lo])]);
        }
        __syncthreads();
    }
    const int K = ks_count(S);
    if (K < 0) {
        if (lane == 0) {
            atomicOr(overflow, 1);
            if (!pass) cnt[i] = 0;
        }
        return;
    }
    if (!pass) {
        if (lane == 0) cnt[i] = K;
        return;
    }
    ks_sort(S, lane, K);
    const int out = crp[i];
    for (int t = lane; t < K; t += WAVE) cci[out + t] = S.sorted[t];
}

__global__ void k_row_of(int n, const int32_t* __restrict__ rp, int32_t* __restrict__ row) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) row[p] = i;
}

// Values of C = A B on a known pattern, one thread per output block (i, l):
// the sum over the columns j of row i of A in increasing order and, for each,
// m increasing -- the order of the thread-per-row kernel.
// find_col for the short sorted rows of the product's right operand: up to
// 16 columns are loaded at once (no chain of dependent loads), longer rows
// are searched by bisection
__device__ __forceinline__ int find_col_short(const int32_t* __restrict__ ci, int lo, int hi, int key) {
    const int len = hi - lo;
    if (len > 16) return find_col(ci, lo, hi, key);
    int c[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) c[u] = u < len ? ci[lo + u] : -1;
    int pos = -1;
#pragma unroll
    for (int u = 0; u < 16; ++u)
        if (c[u] == key) pos = lo + u;
    return pos;
}

// Numeric product, one thread per output block (i, l): the sum over the row
// entries p of A_i whose B row holds column l, in row order, each block
// product's terms in m order.  The lookups of CH consecutive row entries are
// issued together (their column, row-range and column loads do not wait on
// each other).
template <int BR, int BM, int BC, int CH>
__global__ __launch_bounds__(128) void k_spgemm_num_c(int64_t nnz, const int32_t* __restrict__ arp,
                                                      const int32_t* __restrict__ aci,
                                                      const double* __restrict__ aval,
                                                      const int32_t* __restrict__ brp,
                                                      const int32_t* __restrict__ bci,
                                                      const double* __restrict__ bval,
                                                      const int32_t* __restrict__ crow,
                                                      const int32_t* __restrict__ cci, double* __restrict__ cval) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int i = crow[k], l = cci[k];
    double acc[BR * BC];
#pragma unroll
    for (int e = 0; e < BR * BC; ++e) acc[e] = 0.0;
    const int p0 = arp[i], p1 = arp[i + 1];
    for (int pb = p0; pb < p1; pb += CH) {
        int j[CH], lo[CH], hi[CH], q[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) j[u] = pb + u < p1 ? aci[pb + u] : -1;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            lo[u] = j[u] >= 0 ? brp[j[u]] : 0;
            hi[u] = j[u] >= 0 ? brp[j[u] + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) q[u] = find_col_short(bci, lo[u], hi[u], l);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (q[u] < 0) continue;
            const int64_t p = pb + u;
            double a[BR * BM], bb[BM * BC];
#pragma unroll
            for (int e = 0; e < BR * BM; ++e) a[e] = aval[p * BR * BM + e];
#pragma unroll
            for (int e = 0; e < BM * BC; ++e) bb[e] = bval[(int64_t)q[u] * BM * BC + e];
#pragma unroll
            for (int r = 0; r < BR; ++r)
#pragma unroll
                for (int cc = 0; cc < BC; ++cc)
#pragma unroll
                    for (int m = 0; m < BM; ++m) {
                        double term = a[r * BM + m] * bb[m * BC + cc];
                        acc[r * BC + cc] = acc[r * BC + cc] + term;
                    }
        }
    }
    double* dst = cval + k * BR * BC;
#pragma unroll
    for (int e = 0; e < BR * BC; ++e) dst[e] = acc[e];
}

// K products C_k = A_k B_k with one pattern (A_k share one, B_k share one):
// every output block's column lookups are done once for all K; each entry's
// sum runs in the same order as one product alone.
template <int K>
struct SpgemmVals {
    const double* a[K];
    const double* b[K];
    double* c[K];
};
template <int BR, int BM, int BC, int K, int CH>
__global__ __launch_bounds__(128) void k_spgemm_num_k(int64_t nnz, const int32_t* __restrict__ arp,
                                                      const int32_t* __restrict__ aci,
                                                      const int32_t* __restrict__ brp,
                                                      const int32_t* __restrict__ bci,
                                                      const int32_t* __restrict__ crow,
                                                      const int32_t* __restrict__ cci, SpgemmVals<K> v) {
    const int64_t kk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= nnz) return;
    const int i = crow[kk], l = cci[kk];
    double acc[K][BR * BC];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int e = 0; e < BR * BC; ++e) acc[k][e] = 0.0;
    const int p0 = arp[i], p1 = arp[i + 1];
    for (int pb = p0; pb < p1; pb += CH) {
        // the lookups of CH row entries are issued together, as in k_spgemm_num_c
        int j[CH], lo[CH], hi[CH], q[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) j[u] = pb + u < p1 ? aci[pb + u] : -1;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            lo[u] = j[u] >= 0 ? brp[j[u]] : 0;
            hi[u] = j[u] >= 0 ? brp[j[u] + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) q[u] = find_col_short(bci, lo[u], hi[u], l);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (q[u] < 0) continue;
            const int64_t p = pb + u;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                double a[BR * BM], bb[BM * BC];
#pragma unroll
                for (int e = 0; e < BR * BM; ++e) a[e] = v.a[k][p * BR * BM + e];
#pragma unroll
                for (int e = 0; e < BM * BC; ++e) bb[e] = v.b[k][(int64_t)q[u] * BM * BC + e];
#pragma unroll
                for (int r = 0; r < BR; ++r)
#pragma unroll
                    for (int cc = 0; cc < BC; ++cc)
#pragma unroll
                        for (int m = 0; m < BM; ++m) {
                            const double term = a[r * BM + m] * bb[m * BC + cc];
                            acc[k][r * BC + cc] = acc[k][r * BC + cc] + term;
                        }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double* dst = v.c[k] + kk * BR * BC;
#pragma unroll
        for (int e = 0; e < BR * BC; ++e) dst[e] = acc[k][e];
    }
}

// one output block by a group of 16 lanes, lane `ent` holding entry `ent`:
// the group looks up 16 consecutive row entries at once (one per lane), then
// every lane adds their terms in row order, so each entry's sum runs in the
// same order as in the one-thread-per-block kernels
template <int BR, int BM, int BC, int K>
__device__ __forceinline__ void entry_sums(const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                           const int32_t* __restrict__ brp, const int32_t* __restrict__ bci,
                                           int i, int l, int ent, const double* const (&a)[K],
                                           const double* const (&b)[K], double (&acc)[K]) {
    static_assert(BR * BC <= 16, "at most 16 entries per output block");
    const bool live = ent < BR * BC;
    const int r = live ? ent / BC : 0, cc = live ? ent % BC : 0;
    const int p0 = arp[i], p1 = arp[i + 1];
    for (int pb = p0; pb < p1; pb += 16) {
        int q = -1;
        if (pb + ent < p1) {
            const int j = aci[pb + ent];
            q = find_col_short(bci, brp[j], brp[j + 1], l);
        }
        const int cnt = min(16, p1 - pb);
#pragma unroll 4
        for (int t = 0; t < cnt; ++t) {
            const int qt = __shfl(q, t, 16);
            const bool hit = qt >= 0 && live;
            const int64_t p = pb + t, qs = hit ? qt : 0;
#pragma unroll
            for (int u = 0; u < K; ++u) {
                double s = acc[u];
#pragma unroll
                for (int m = 0; m < BM; ++m) {
                    const double term = a[u][p * BR * BM + r * BM + m] * b[u][qs * BM * BC + m * BC + cc];
                    s = s + term;
                }
                acc[u] = hit ? s : acc[u];
            }
        }
    }
}

// K products as in k_spgemm_num_k, 16 lanes per output block (small outputs):
// each column lookup serves all K products
template <int BR, int BM, int BC, int K>
__global__ __launch_bounds__(256) void k_spgemm_num_ek(int64_t nnz, const int32_t* __restrict__ arp,
                                                       const int32_t* __restrict__ aci,
                                                       const int32_t* __restrict__ brp,
                                                       const int32_t* __restrict__ bci,
                                                       const int32_t* __restrict__ crow,
                                                       const int32_t* __restrict__ cci, SpgemmVals<K> v) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = tid / 16;
    const int ent = (int)(tid % 16);
    if (k >= nnz) return;   // whole groups of 16
    double acc[K];
#pragma unroll
    for (int u = 0; u < K; ++u) acc[u] = 0.0;
    entry_sums<BR, BM, BC, K>(arp, aci, brp, bci, crow[k], cci[k], ent, v.a, v.b, acc);
    if (ent < BR * BC)
#pragma unroll
        for (int u = 0; u < K; ++u) v.c[u][k * BR * BC + ent] = acc[u];
}

// one product with 16 lanes per output block, for outputs too small to fill
// the GPU one block per thread
template <int BR, int BM, int BC>
__global__ __launch_bounds__(256) void k_spgemm_num_e(int64_t nnz, const int32_t* __restrict__ arp,
                                                      const int32_t* __restrict__ aci,
                                                      const double* __restrict__ aval,
                                                      const int32_t* __restrict__ brp,
                                                      const int32_t* __restrict__ bci,
                                                      const double* __restrict__ bval,
                                                      const int32_t* __restrict__ crow,
                                                      const int32_t* __restrict__ cci, double* __restrict__ cval) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = tid / 16;
    const int ent = (int)(tid % 16);
    if (k >= nnz) return;   // whole groups of 16
    const double* const a[1] = {aval};
    const double* const b[1] = {bval};
    double acc[1] = {0.0};
    entry_sums<BR, BM, BC, 1>(arp, aci, brp, bci, crow[k], cci[k], ent, a, b, acc);
    if (ent < BR * BC) cval[k * BR * BC + ent] = acc[0];
}

// the same for any block shape with at most 16 entries per output block
__global__ void k_spgemm_num_any(int64_t nnz, int br, int bm, int bc, const int32_t* __restrict__ arp,
                                 const int32_t* __restrict__ aci, const double* __restrict__ aval,
                                 const int32_t* __restrict__ brp, const int32_t* __restrict__ bci,
                                 const double* __restrict__ bval, const int32_t* __restrict__ crow,
                                 const int32_t* __restrict__ cci, double* __restrict__ cval) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int i = crow[k], l = cci[k];
    double acc[16];
    for (int e = 0; e < br * bc; ++e) acc[e] = 0.0;
    for (int p = arp[i]; p < arp[i + 1]; ++p) {
        const int j = aci[p];
        const int q = find_col(bci, brp[j], brp[j + 1], l);
        if (q < 0) continue;
        const double* a = aval + (int64_t)p * br * bm;
        const double* bb = bval + (int64_t)q * bm * bc;
        for (int r = 0; r < br; ++r)
            for (int cc = 0; cc < bc; ++cc)
                for (int m = 0; m < bm; ++m) {
                    double term = a[r * bm + m] * bb[m * bc + cc];
                    acc[r * bc + cc] = acc[r * bc + cc] + term;
                }
    }
    double* dst = cval + k * br * bc;
    for (int e = 0; e < br * bc; ++e) dst[e] = acc[e];
}

// Structure check of a BSR block that arrived in device memory (host input is
// checked on the host): bad[0] row_ptr[0] != 0 or row_ptr[n_rows] != nnzb,
// bad[1] a row whose range is negative, decreasing or beyond nnzb, bad[2] a
// column outside [0, n_cols), bad[3] columns not strictly increasing within a
// row.  One thread per row; a row's columns are read only once its range is
// known to lie inside [0, nnzb), so no read leaves the arrays.
__global__ void k_check_bsr(int n_rows, int n_cols, int64_t nnzb, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ ci, int32_t* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    if (i == 0 && rp[0] != 0) bad[0] = 1;
    if (i == n_rows - 1 && (int64_t)rp[n_rows] != nnzb) bad[0] = 1;
    const int a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || (int64_t)b > nnzb) {
        bad[1] = 1;
        return;
    }
    for (int p = a; p < b; ++p) {
        const int j = ci[p];
        if (j < 0 || j >= n_cols) {
            bad[2] = 1;
            return;
        }
        if (p > a && j <= ci[p - 1]) {
            bad[3] = 1;
            return;
        }
    }
}

void check_bsr_device(int n_rows, int n_cols, int64_t nnzb, const int32_t* rp, const int32_t* ci, hipStream_t s) {
    if (n_rows <= 0) return;
    DevBuf<int32_t> bad(4);
    MB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t) * 4, s));
    k_check_bsr<<<(unsigned)ceil_div(n_rows, 256), 256, 0, s>>>(n_rows, n_cols, nnzb, rp, ci, bad.p);
    MB_LAUNCH_CHECK();
    const std::vector<int32_t> f = bad.download(s, 4);
    MB_CHECK(!f[0], MBAMG_E_INVALID, "row_ptr inconsistent with nnzb");
    MB_CHECK(!f[1], MBAMG_E_INVALID, "row_ptr not monotone");
    MB_CHECK(!f[2], MBAMG_E_INVALID, "column index out of range");
    MB_CHECK(!f[3], MBAMG_E_INVALID, "column indices must be strictly increasing within a row");
}

// flag (initially 1) is cleared when two index arrays of equal length differ
// anywhere: row pointers and then columns, one element per thread (grid-stride,
// coalesced), one atomic per wavefront that found a difference
__global__ void k_same_pattern(int64_t n_rp, int64_t n_ci, const int32_t* __restrict__ rpa,
                               const int32_t* __restrict__ cia, const int32_t* __restrict__ rpb,
                               const int32_t* __restrict__ cib, int32_t* flag) {
    bool diff = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_rp + n_ci; t += stride)
        diff |= t < n_rp ? rpa[t] != rpb[t] : cia[t - n_rp] != cib[t - n_rp];
    if (__ballot(diff) != 0 && (threadIdx.x & (WAVE - 1)) == 0) atomicAnd(flag, 0);
}

// One wavefront per row (long rows, at most SA_WROW entries and KS_MAX
// distinct aggregates, else *overflow is set): the distinct kept aggregates
// are collected and sorted in LDS, every entry is tagged with its output
// block, and 16 lanes per output block (one per entry) sum over the row's
// entries in increasing order -- the sums of the generic form, in its order.
constexpr int SA_WROW = 1024;
template <int D>
__global__ __launch_bounds__(WAVE) void k_sa_prolong_w(int nv, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                       const int32_t* __restrict__ agg, const double* __restrict__ q,
                                                       const double* __restrict__ w, int pass, int32_t* cnt,
                                                       const int32_t* prp, int32_t* pci, double* pval,
                                                       int32_t* overflow) {
    constexpr int BS = D * D;
    __shared__ KeySet S;
    __shared__ int32_t slot[SA_WROW], sj[SA_WROW];
    const int i = blockIdx.x, lane = threadIdx.x;
    const int b = rp[i], e = rp[i + 1], ai = agg[i], len = e - b;
    if (len > SA_WROW) {
        if (lane == 0) {
            atomicOr(overflow, 1);
            if (!pass) cnt[i] = 0;
        }
        return;
    }
    ks_clear(S, lane, len);
    for (int p = lane; p < len; p += WAVE) {
        const int j = ci[b + p];
        const int a = agg[j];
        const bool keep = a == ai || w[a] != 0.0;
        if (keep) ks_insert(S, a);
        sj[p] = j;
        slot[p] = keep ? a : -1;
    }
    __syncthreads();
    const int K = ks_count(S);
    if (K < 0) {
        if (lane == 0) {
            atomicOr(overflow, 1);
            if (!pass) cnt[i] = 0;
        }
        return;
    }
    if (!pass) {
        if (lane == 0) cnt[i] = K;
        return;
    }
    ks_sort(S, lane, K);
    // output block of each entry: the rank of its aggregate among the sorted ones
    for (int p = lane; p < len; p += WAVE) {
        const int a = slot[p];
        if (a < 0) continue;
        int lo = 0, hi = K - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (S.sorted[mid] < a) lo = mid + 1;
            else hi = mid;
        }
        slot[p] = lo;
    }
    __syncthreads();
    const int pd = find_col(ci, b, e, i);
    const int out = prp[i];
    const int sub = lane / 16, ent = lane % 16, ra = ent / D, cc = ent % D;
    const bool live = ent < BS;
    const double dg = (live && pd >= 0) ? val[(int64_t)pd * BS + ra * D + ra] : 0.0;
    for (int t0 = 0; t0 < K; t0 += WAVE / 16) {
        const int t = t0 + sub;
        double acc = 0.0;
        for (int p = 0; p < len; ++p) {
            if (slot[p] != t || !live) continue;
            const double term = val[(int64_t)(b + p) * BS + ent] * q[(int64_t)sj[p] * D + cc];
            acc = acc + term;
        }
        if (t < K && live) {
            const int l = S.sorted[t];
            const double base = (l == ai && cc == ra) ? q[(int64_t)i * D + ra] : 0.0;
            double r = base;
            if (ra < nv && cc < nv) {
                const double tq = acc / dg;
                const double u = w[l] * tq;
                r = base - u;
            }
            pval[(int64_t)(out + t) * BS + ent] = r;
            if (ent == 0) pci[out + t] = l;
        }
    }
}

// transposed row k: entries placed in arbitrary order (trow = source row,
// tsrc = source block) are ranked by source row (distinct within a row) and
// written in increasing order with the blocks transposed
__global__ __launch_bounds__(WAVE) void k_transpose_rank(int br, int bc, const int32_t* __restrict__ trp,
                                                         const int32_t* __restrict__ trow,
                                                         const int32_t* __restrict__ tsrc,
                                                         const double* __restrict__ val, int32_t* __restrict__ tci,
                                                         double* __restrict__ tval) {
    constexpr int TR_LDS = 1024;
    __shared__ int32_t rows[TR_LDS], dst[TR_LDS];
    const int k = blockIdx.x, lane = threadIdx.x;
    const int b = trp[k], e = trp[k + 1], len = e - b, bs = br * bc;
    if (len > TR_LDS) {   // long rows: ranks from global memory, one lane per entry
        for (int a = b + lane; a < e; a += WAVE) {
            const int r = trow[a];
            int rank = 0;
            for (int u = b; u < e; ++u) rank += trow[u] < r;
            const int dp = b + rank;
            tci[dp] = r;
            const double* src = val + (int64_t)tsrc[a] * bs;
            double* out = tval + (int64_t)dp * bs;
            for (int r2 = 0; r2 < br; ++r2)
                for (int c = 0; c < bc; ++c) out[c * br + r2] = src[r2 * bc + c];
        }
        return;
    }
    // the row's source rows in LDS, ranked there; then the blocks are copied
    // 16 lanes per block (bs <= 16), each a contiguous read and write
    for (int u = lane; u < len; u += WAVE) rows[u] = trow[b + u];
    for (int a = lane; a < len; a += WAVE) {
        const int r = rows[a];
        int rank = 0;
        for (int u = 0; u < len; ++u) rank += rows[u] < r;
        dst[a] = rank;
        tci[b + rank] = r;
    }
    for (int t = lane; t < len * 16; t += WAVE) {
        const int a = t >> 4, ent = t & 15;
        if (ent >= bs) continue;
        const int r2 = ent / bc, c = ent % bc;
        tval[(int64_t)(b + dst[a]) * bs + c * br + r2] = val[(int64_t)tsrc[b + a] * bs + ent];
    }
}

// ----------------------------------------------------------------------------
// building the sliced smoother format on the device.  kind: 0 off-diagonal
// blocks of A_ff, 1 all blocks of A_fg, 2 the diagonal block, 3 one entry per
// node (the node index itself, for the nodal inverses).
// ----------------------------------------------------------------------------
__device__ inline bool part_selects(int kind, int node, int col) {
    return kind == 1 || (kind == 0 && col != node) || (kind == 2 && col == node);
}

__global__ void k_part_rowlen(int n, int kind, const int32_t* perm, const int32_t* rp, const int32_t* ci,
                              int32_t* rowlen) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (kind == 3) { rowlen[p] = 1; return; }
    int node = perm[p], c = 0;
    for (int q = rp[node]; q < rp[node + 1]; ++q) c += part_selects(kind, node, ci[q]);
    rowlen[p] = c;
}

__global__ void k_part_width(int ns, int kind, const int32_t* row0, const int32_t* nrow, const int32_t* rowlen,
                             int32_t* width) {
    int sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= ns) return;
    int w = 0;
    for (int l = 0; l < nrow[sl]; ++l) w = max(w, rowlen[row0[sl] + l]);
    width[sl] = (kind >= 2) ? 1 : w;
}

// one thread per (slice, lane): column (in the column block's colour order) and
// source index of each slot, -1 for padding
__global__ void k_part_fill_index(int ns, int kind, const int32_t* row0, const int32_t* nrow, const int32_t* width,
                                  const int32_t* coff, const int32_t* perm, const int32_t* rp, const int32_t* ci,
                                  const int32_t* col_iperm, int32_t* col, int64_t* src, int32_t* slot_blocks) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ns * WAVE) return;
    int sl = (int)(t / WAVE), lane = (int)(t % WAVE);
    int w = width[sl];
    int64_t base = coff[sl];
    int k = 0;
    if (lane < nrow[sl]) {
        int p = row0[sl] + lane;
        int node = perm[p];
        if (kind == 3) {
            col[base * WAVE + lane] = p;
            src[base * WAVE + lane] = node;
            k = 1;
        } else {
            for (int q = rp[node]; q < rp[node + 1] && k < w; ++q) {
                int j = ci[q];
                if (!part_selects(kind, node, j)) continue;
                col[(base + k) * WAVE + lane] = col_iperm[j];
                src[(base + k) * WAVE + lane] = q;
                ++k;
            }
        }
    }
    const int placed = k;
    for (; k < w; ++k) {
        col[(base + k) * WAVE + lane] = -1;
        src[(base + k) * WAVE + lane] = -1;
    }
    // blocks per slot: the slots of a slice belong to its wavefront alone
    for (int kk = 0; kk < w; ++kk) {
        const int c = (int)__popcll(__ballot(kk < placed));
        if (lane == 0) slot_blocks[base + kk] = c;
    }
}

__global__ void k_popcount(int64_t n, const uint32_t* mask, int32_t* cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = __popc(mask[i]);
}

__global__ void k_i32_to_i64(int64_t n, const int32_t* a, int64_t* b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// transfer maps between colour orders: aggp[p] = ciperm[agg[perm[p]]]
__global__ void k_map_agg(int n, const int32_t* perm, const int32_t* agg, const int32_t* ciperm, int32_t* aggp) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) aggp[p] = ciperm[agg[perm[p]]];
}

__global__ void k_map_count(int nc, const int32_t* cperm, const int32_t* mptr, int32_t* cnt) {
    int kp = blockIdx.x * blockDim.x + threadIdx.x;
    if (kp < nc) { int k = cperm[kp]; cnt[kp] = mptr[k + 1] - mptr[k]; }
}

__global__ void k_map_members(int nc, const int32_t* cperm, const int32_t* mptr, const int32_t* midx,
                              const int32_t* iperm, const int32_t* optr, int32_t* oidx) {
    int kp = blockIdx.x * blockDim.x + threadIdx.x;
    if (kp >= nc) return;
    int k = cperm[kp], o = optr[kp];
    for (int m = mptr[k]; m < mptr[k + 1]; ++m) oidx[o++] = iperm[midx[m]];
}

// ----------------------------------------------------------------------------
// coarsest level: dense assembly and Gauss-Jordan inverse with partial pivoting
// ----------------------------------------------------------------------------
__global__ void k_dense_scatter(int n_rows, int br, int bc, const int32_t* rp, const int32_t* ci, const double* val,
                                int64_t row_off, int64_t col_off, int64_t ld, double* M) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int j = ci[p];
        for (int r = 0; r < br; ++r)
            for (int c = 0; c < bc; ++c)
                M[(row_off + (int64_t)i * br + r) * ld + col_off + (int64_t)j * bc + c] =
                    val[((int64_t)p * br + r) * bc + c];
    }
}

// ----------------------------------------------------------------------------
// Coarsest inverse: blocked Gauss-Jordan with partial (row) pivoting.
//
// One Gauss-Jordan step on column k with pivot row p and piv = M[p][k] trades
// rows p and k, scales the new row k by 1/piv (1/piv in column k), and
// subtracts M[r][k] times it from every other row r (which then holds
// -M[r][k]/piv in column k).  Panels of B columns: one workgroup holds the
// panel's n x B entries in registers and runs its B steps on them alone,
// recording for every row the row whose data it now holds (rowsrc).  The
// panel then holds the columns in which the composite transformation T of its
// steps differs from the identity, so every other column x (the inverse built
// so far on the left, the untouched matrix on the right) becomes
//   T P x = P x + (G - E) (P x)[panel rows],   (P x)[r] = x[rowsrc[r]],
// G the panel and E the panel's columns of the identity: one tiled rank-B
// update, written to the other half of a ping-pong pair so that reads of
// x[rowsrc[r]] never see updated values.  The product of the row interchanges
// (ord) is carried along; the columns of the result are finally scattered to
// ord, which undoes the column interchanges that in-place Gauss-Jordan
// inversion leaves (Quintana-Orti, Quintana-Orti, van de Geijn & Remon, "A
// note on parallel matrix inversion", SIAM J. Sci. Comput. 22, 2001).
// ----------------------------------------------------------------------------
constexpr int GJ_TILE = 64;

// larger magnitude wins, ties to the smaller position
__device__ __forceinline__ void gj_take(double& best, int& bi, double ob, int oi) {
    if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
    }
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void gj_dpp_take(double& best, int& bi) {
    const int lo = __double2loint(best), hi = __double2hiint(best);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    const int oi = __builtin_amdgcn_update_dpp(bi, bi, CTRL, ROWS, 0xF, false);
    gj_take(best, bi, __hiloint2double(ohi, olo), oi);
}
// arg-max over the wave, returned to every lane: exchanges inside quads and
// half-rows and rows of 16 lanes, then row broadcasts carry the total to lane 63
__device__ __forceinline__ void gj_wave_argmax(double& best, int& bi) {
    gj_dpp_take<0xB1, 0xF>(best, bi);    // quad_perm [1,0,3,2]
    gj_dpp_take<0x4E, 0xF>(best, bi);    // quad_perm [2,3,0,1]
    gj_dpp_take<0x141, 0xF>(best, bi);   // row_half_mirror
    gj_dpp_take<0x140, 0xF>(best, bi);   // row_mirror
    gj_dpp_take<0x142, 0xA>(best, bi);   // row_bcast:15 into rows 1 and 3
    gj_dpp_take<0x143, 0xC>(best, bi);   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(best), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(best), 63);
    bi = __builtin_amdgcn_readlane(bi, 63);
    best = __hiloint2double(hi, lo);
}

// Panel [k0, k0 + b), b <= B; thread t of T owns rows t + j * T, j < R, in
// registers.  Rows are never moved inside the panel: lab[j] is the position
// that the thread's j-th row holds in the row order so far, and a row
// interchange exchanges two labels.  The columns sit in a rotating frame so
// that the step loop indexes registers with constants: at step kk, v[j][c]
// holds panel column (c + kk) mod B, the pivot column is v[j][0].  Global
// memory is read and written in coalesced order and redistributed through
// LDS one slot (T rows) at a time.  Each row ends at position lab[j];
// rowsrc[position] = the row it came from.
template <int T, int R, int B>
__global__ __launch_bounds__(T) void k_gj_panel(double* M, int n, int k0, int b, int32_t* rowsrc, int32_t* singular) {
    __shared__ double stage[T][B + 1];
    __shared__ int slab[T];
    __shared__ double wbest[T / WAVE];
    __shared__ int widx[T / WAVE];
    __shared__ double rowk[B];
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    double v[R][B];
    int lab[R];
    {
        // every load in flight at once
        double u[R][B];
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int e = t + q * T, rr = e / B, c = e % B, r = j * T + rr;
                u[j][q] = (r < n && c < b) ? M[(int64_t)r * n + k0 + c] : 0.0;
            }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            lab[j] = t + j * T;
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int e = t + q * T;
                stage[e / B][e % B] = u[j][q];
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < B; ++c) v[j][c] = stage[t][c];
            __syncthreads();
        }
    }
    for (int kk = 0; kk < b; ++kk) {
        const int k = k0 + kk;
        // pivot: largest magnitude in column k at position k or below, ties to the smaller position
        double best = -1.0;
        int bi = INT_MAX;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const double a = fabs(v[j][0]);
            if (lab[j] >= k && lab[j] < n && (a > best || (a == best && lab[j] < bi))) {
                best = a;
                bi = lab[j];
            }
        }
        gj_wave_argmax(best, bi);
        if (lane == 0) {
            wbest[wv] = best;
            widx[wv] = bi;
        }
        __syncthreads();
        best = wbest[0];
        bi = widx[0];
#pragma unroll
        for (int w = 1; w < T / WAVE; ++w) gj_take(best, bi, wbest[w], widx[w]);
        // no finite candidate (NaN after an earlier zero pivot): keep a valid row
        const int lp = bi == INT_MAX ? k : bi;
        if (t == 0 && (!(best > 0.0) || bi == INT_MAX)) atomicAdd(singular, 1);
        // the owner of the pivot row publishes the new row k (rotated frame)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (__any(lab[j] == lp) && lab[j] == lp) {
                const double inv = 1.0 / v[j][0];
                rowk[0] = inv;
#pragma unroll
                for (int c = 1; c < B; ++c) rowk[c] = v[j][c] * inv;
            }
        }
        __syncthreads();
        // eliminate column k from every row and rotate the frame by one
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool piv = lab[j] == lp;
            const double f = v[j][0];
#pragma unroll
            for (int c = 1; c < B; ++c) v[j][c - 1] = fma(-f, rowk[c], v[j][c]);
            v[j][B - 1] = -f * rowk[0];
            // one lane of one wave holds the pivot row: the others skip its copy
            if (__any(piv)) {
#pragma unroll
                for (int c = 1; c < B; ++c) v[j][c - 1] = piv ? rowk[c] : v[j][c - 1];
                v[j][B - 1] = piv ? rowk[0] : v[j][B - 1];
            }
            lab[j] = piv ? k : (lab[j] == k ? lp : lab[j]);
        }
    }
    // after b steps, frame column c holds panel column (c + b) mod B
#pragma unroll
    for (int j = 0; j < R; ++j) {
#pragma unroll
        for (int c = 0; c < B; ++c) stage[t][c] = v[j][c];
        slab[t] = lab[j];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int e = t + q * T, rr = e / B, c = e % B, r = j * T + rr;
            const int pc = (c + b) % B;
            if (r < n && pc < b) M[(int64_t)slab[rr] * n + k0 + pc] = stage[rr][c];
        }
        if (t + j * T < n) rowsrc[lab[j]] = t + j * T;
        __syncthreads();
    }
}

// Out = P In + (G - E) (P In)[panel rows] outside the panel, Out = In inside it;
// GJ_TILE x GJ_TILE tiles, 256 threads, each thread one column and 16 rows.
// Column-tile 0 also carries the row order: ord_out[r] = ord_in[rowsrc[r]]
// (ord_in null: the identity).
template <int B>
__global__ __launch_bounds__(256) void k_gj_update(const double* __restrict__ Min, double* __restrict__ Mout, int n,
                                                   int k0, int b, const int32_t* __restrict__ rowsrc,
                                                   const int32_t* __restrict__ ord_in, int32_t* __restrict__ ord_out) {
    __shared__ double G[B][GJ_TILE];
    __shared__ int rsrc[GJ_TILE];
    const int t = threadIdx.x, tx = t % GJ_TILE, ty = t / GJ_TILE;
    const int row0 = blockIdx.y * GJ_TILE;
    const int c = blockIdx.x * GJ_TILE + tx;
    for (int e = t; e < GJ_TILE * B; e += 256) {
        const int rr = e / B, q = e % B;
        const int r = row0 + rr;
        double g = 0.0;
        if (r < n && q < b) g = Min[(int64_t)r * n + k0 + q] - (r == k0 + q ? 1.0 : 0.0);
        G[q][rr] = g;
    }
    if (t < GJ_TILE) {
        const int r = row0 + t;
        const int sr = r < n ? rowsrc[r] : 0;
        rsrc[t] = sr;
        if (blockIdx.x == 0 && r < n) ord_out[r] = ord_in ? ord_in[sr] : sr;
    }
    __syncthreads();
    if (c >= n) return;
    const bool in_panel = c >= k0 && c < k0 + b;
    double x[B];
#pragma unroll
    for (int q = 0; q < B; ++q) x[q] = (q < b && !in_panel) ? Min[(int64_t)rowsrc[k0 + q] * n + c] : 0.0;
#pragma unroll 4
    for (int i = 0; i < GJ_TILE / 4; ++i) {
        const int rr = ty * (GJ_TILE / 4) + i;
        const int r = row0 + rr;
        if (r >= n) break;
        double out;
        if (in_panel) {
            out = Min[(int64_t)r * n + c];
        } else {
            out = Min[(int64_t)rsrc[rr] * n + c];
#pragma unroll
            for (int q = 0; q < B; ++q) out = fma(G[q][rr], x[q], out);
        }
        Mout[(int64_t)r * n + c] = out;
    }
}

// inv[:, ord[i]] = X[:, i]
__global__ void k_gj_extract(const double* X, int n, const int32_t* ord, double* inv) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int r = (int)(t / n), i = (int)(t % n);
    inv[(int64_t)r * n + ord[i]] = X[t];
}

// ----------------------------------------------------------------------------
// host wrappers
// ----------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int threads = 256) {
    return (unsigned)std::max<int64_t>(1, ceil_div(n, threads));
}

Strength build_strength(const SetupBsr& A, double theta, hipStream_t s) {
    MB_CHECK(A.br == A.bc, MBAMG_E_INVALID, "A00 blocks must be square");
    Strength S;
    S.n = A.n_rows;
    const int n = A.n_rows;
    DevBuf<double> n2(std::max<int64_t>(A.nnzb, 1));
    k_block_sqnorm<<<grid_for(A.nnzb), 256, 0, s>>>(A.val.p, A.nnzb, A.br * A.bc, n2.p);
    MB_LAUNCH_CHECK();
    double t4 = (theta * theta) * (theta * theta);
    DevBuf<int32_t> cnt(std::max(n, 1)), asym(1);
    MB_HIP(hipMemsetAsync(asym.p, 0, sizeof(int32_t), s));
    k_strength<<<grid_for(n), 256, 0, s>>>(n, A.rp.p, A.ci.p, n2.p, t4, 0, cnt.p, nullptr, nullptr, nullptr,
                                           asym.p);
    MB_LAUNCH_CHECK();
    int32_t h_asym = 0;
    MB_HIP(hipMemcpyAsync(&h_asym, asym.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    S.ptr.alloc(n + 1);
    int nnz = scan_exclusive(cnt.p, n, S.ptr.p, s);   // synchronises
    MB_CHECK(h_asym == 0, MBAMG_E_INVALID, "the node pattern of A00 must be structurally symmetric");
    S.nnz = nnz;
    S.idx.alloc(std::max(nnz, 1));
    S.w2.alloc(std::max(nnz, 1));
    k_strength<<<grid_for(n), 256, 0, s>>>(n, A.rp.p, A.ci.p, n2.p, t4, 1, nullptr, S.ptr.p, S.idx.p, S.w2.p,
                                           asym.p);
    MB_LAUNCH_CHECK();
    return S;
}

Aggregates build_aggregates(const Strength& S, uint64_t seed, int level, hipStream_t s) {
    const int n = S.n;
    Aggregates G;
    G.n = n;
    DevBuf<uint64_t> key(std::max(n, 1));
    DevBuf<int8_t> state(std::max(n, 1)), near1(std::max(n, 1));
    DevBuf<int32_t> best1(std::max(n, 1)), counter(1);
    uint64_t mult = 0x9E3779B97F4A7C15ull * (seed * 1024ull + (uint64_t)level + 1ull);
    k_keys<<<grid_for(n), 256, 0, s>>>(n, mult, key.p, state.p);
    MB_LAUNCH_CHECK();
    int rounds = 0;
    while (true) {
        MB_CHECK(rounds < 100000, MBAMG_E_INVALID, "aggregation did not terminate");
        k_mis_a<<<grid_for(n), 256, 0, s>>>(n, S.ptr.p, S.idx.p, key.p, state.p, best1.p);
        k_mis_b<<<grid_for(n), 256, 0, s>>>(n, S.ptr.p, S.idx.p, key.p, best1.p, state.p);
        k_mis_c<<<grid_for(n), 256, 0, s>>>(n, S.ptr.p, S.idx.p, state.p, near1.p);
        MB_HIP(hipMemsetAsync(counter.p, 0, sizeof(int32_t), s));
        k_mis_d<<<grid_for(n), 256, 0, s>>>(n, S.ptr.p, S.idx.p, near1.p, state.p, counter.p);
        MB_LAUNCH_CHECK();
        int32_t und = 0;
        MB_HIP(hipMemcpyAsync(&und, counter.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MB_HIP(hipStreamSynchronize(s));
        ++rounds;
        if (und == 0) break;
    }
    G.mis_rounds = rounds;
    DevBuf<int32_t> flag(std::max(n, 1)), rootscan(n + 1);
    k_is_root<<<grid_for(n), 256, 0, s>>>(n, state.p, flag.p);
    MB_LAUNCH_CHECK();
    G.n_agg = scan_exclusive(flag.p, n, rootscan.p, s);
    DevBuf<int32_t> phase1(std::max(n, 1)), fail(1);
    k_fill_i32<<<grid_for(n), 256, 0, s>>>(phase1.p, n, -1);
    k_phase1<<<grid_for(n), 256, 0, s>>>(n, S.ptr.p, S.idx.p, state.p, rootscan.p, phase1.p);
    MB_HIP(hipMemsetAsync(fail.p, 0, sizeof(int32_t), s));
    G.agg.alloc(std::max(n, 1));
    k_phase2<<<grid_for(n), 256, 0, s>>>(n, S.ptr.p, S.idx.p, S.w2.p, phase1.p, G.agg.p, fail.p);
    MB_LAUNCH_CHECK();
    int32_t h_fail = 0;
    MB_HIP(hipMemcpyAsync(&h_fail, fail.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    // members, increasing node order within each aggregate
    const int na = G.n_agg;
    DevBuf<int32_t> cnt(std::max(na, 1)), cursor(std::max(na, 1));
    MB_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * std::max(na, 1), s));
    MB_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int32_t) * std::max(na, 1), s));
    k_count_members<<<grid_for(n), 256, 0, s>>>(n, G.agg.p, cnt.p);
    MB_LAUNCH_CHECK();
    G.mptr.alloc(na + 1);
    scan_exclusive(cnt.p, na, G.mptr.p, s);
    MB_CHECK(h_fail == 0, MBAMG_E_INVALID, "aggregation left a node unattached");
    G.midx.alloc(std::max(n, 1));
    k_place_members<<<grid_for(n), 256, 0, s>>>(n, G.agg.p, G.mptr.p, cursor.p, G.midx.p);
    bool wave_sort = n >= 16 * (int64_t)na;
    if (const char* f = form_override("MBAMG_SORT_FORM")) wave_sort = std::strcmp(f, "wave") == 0;
    if (na > 0 && wave_sort) k_sort_members_w<<<na, WAVE, 0, s>>>(na, G.mptr.p, G.midx.p);
    else k_sort_members<<<grid_for(na), 256, 0, s>>>(na, G.mptr.p, G.midx.p);
    MB_LAUNCH_CHECK();
    return G;
}

void build_tentative(const Aggregates& G, int d, const double* B, double* q, double* Bc, hipStream_t s) {
    k_tentative<<<grid_for((int64_t)G.n_agg * d), 256, 0, s>>>(G.n_agg, d, G.mptr.p, G.midx.p, B, q, Bc);
    MB_LAUNCH_CHECK();
}

void fill_ones(double* a, int64_t n, hipStream_t s) { fill_value(a, n, 1.0, s); }

void fill_value(double* a, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    k_fill_f64<<<grid_for(n), 256, 0, s>>>(a, n, v);
    MB_LAUNCH_CHECK();
}

SetupBsr tentative_bsr(const Aggregates& G, int d, const double* q, hipStream_t s) {
    const int n = G.n;
    SetupBsr P;
    P.n_rows = n;
    P.n_cols = G.n_agg;
    P.br = P.bc = d;
    P.nnzb = n;
    P.rp.alloc(n + 1);
    P.ci.alloc(std::max(n, 1));
    P.val.alloc(std::max<int64_t>((int64_t)n * d * d, 1));
    k_tentative_bsr<<<grid_for(n + 1), 256, 0, s>>>(n, d, G.agg.p, q, P.rp.p, P.ci.p, P.val.p);
    MB_LAUNCH_CHECK();
    return P;
}

void build_dinv(const SetupBsr& A, double* dinv, hipStream_t s) {
    MB_CHECK(A.br == A.bc && A.br <= 8, MBAMG_E_INVALID, "diagonal blocks must be square with at most 8 dofs");
    DevBuf<int32_t> sing(1);
    MB_HIP(hipMemsetAsync(sing.p, 0, sizeof(int32_t), s));
    k_dinv<<<grid_for(A.n_rows, 64), 64, 0, s>>>(A.n_rows, A.br, A.rp.p, A.ci.p, A.val.p, dinv, sing.p);
    MB_LAUNCH_CHECK();
    int32_t h = 0;
    MB_HIP(hipMemcpyAsync(&h, sing.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    MB_CHECK(h == 0, MBAMG_E_SINGULAR, "a nodal diagonal block is singular");
}

void build_node_inverses(const SetupBsr (&A)[2][2], int n_slices, const int32_t* row0, const int32_t* nrow,
                         const int32_t* perm, DevBuf<uint64_t>& mask, DevBuf<int32_t>& off, DevBuf<double>& inv64,
                         DevBuf<float>* inv32, hipStream_t s) {
    const int n = A[0][0].n_rows, d0 = A[0][0].br, d1 = A[1][1].br, m = d0 + d1;
    MB_CHECK(m <= 8, MBAMG_E_INVALID, "full node blocks of at most 8 dofs");
    NodeBlocks B{};
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g) {
            const SetupBsr& X = A[f][g];
            const int q = f * 2 + g;
            B.rp[q] = X.nnzb ? X.rp.p : nullptr;
            B.ci[q] = X.ci.p;
            B.val[q] = X.val.p;
        }
    DevBuf<double> nat((size_t)std::max(n, 1) * m * m);
    DevBuf<int32_t> sing(1);
    MB_HIP(hipMemsetAsync(sing.p, 0, sizeof(int32_t), s));
    k_node_inv<<<grid_for(n, 64), 64, 0, s>>>(n, d0, d1, B, nat.p, sing.p);
    MB_LAUNCH_CHECK();
    mask.alloc((size_t)std::max(n_slices, 1));
    off.alloc((size_t)n_slices + 1);
    DevBuf<int32_t> cnt((size_t)std::max(n_slices, 1));
    if (n_slices) k_node_inv_mask<<<grid_for((int64_t)n_slices * WAVE), 256, 0, s>>>(n_slices, m * m, row0, nrow, perm,
                                                                                      nat.p, mask.p, cnt.p);
    MB_LAUNCH_CHECK();
    const int64_t groups = scan_exclusive(cnt.p, n_slices, off.p, s);
    const int64_t total = (int64_t)n_slices * m * m * WAVE;
    inv64.alloc((size_t)std::max<int64_t>(groups * WAVE, 1));
    if (total) k_node_inv_pack<double><<<grid_for(total), 256, 0, s>>>(n_slices, m * m, row0, nrow, perm, nat.p,
                                                                       mask.p, off.p, inv64.p);
    if (inv32) {
        inv32->alloc((size_t)std::max<int64_t>(groups * WAVE, 1));
        if (total) k_node_inv_pack<float><<<grid_for(total), 256, 0, s>>>(n_slices, m * m, row0, nrow, perm, nat.p,
                                                                          mask.p, off.p, inv32->p);
    }
    MB_LAUNCH_CHECK();
    int32_t h = 0;
    MB_HIP(hipMemcpyAsync(&h, sing.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    MB_CHECK(h == 0, MBAMG_E_SINGULAR, "a full node block is singular");
}

bool within_pattern(const SetupBsr& A, const SetupBsr& B, hipStream_t s) {
    if (B.nnzb == 0) return true;
    DevBuf<int32_t> flag(1);
    const std::vector<int32_t> one(1, 1);
    flag.upload(one, s);
    k_subpattern<<<grid_for(B.n_rows), 256, 0, s>>>(B.n_rows, A.rp.p, A.ci.p, B.rp.p, B.ci.p, flag.p);
    MB_LAUNCH_CHECK();
    return flag.download(s, 1)[0] != 0;
}

void sell_masks(int64_t n_slots, int bs, const int64_t* src, const double* val, uint32_t* mask, uint32_t* slot_nz,
                hipStream_t s) {
    MB_CHECK(bs >= 1 && bs <= 16, MBAMG_E_INVALID, "sliced format: blocks of at most 16 entries");
    MB_HIP(hipMemsetAsync(mask, 0, sizeof(uint32_t) * std::max<int64_t>(n_slots, 1), s));
    if (n_slots == 0) return;
    k_sell_mask<<<grid_for(n_slots * WAVE), 256, 0, s>>>(n_slots, bs, src, val, mask, slot_nz);
    MB_LAUNCH_CHECK();
}

void sell_fill(int64_t n_slots, int bs, const int64_t* src, const double* val, const uint32_t* mask,
               const int64_t* slot_voff, double* out, hipStream_t s) {
    if (n_slots == 0) return;
    k_sell_fill<<<grid_for(n_slots * WAVE), 256, 0, s>>>(n_slots, bs, src, val, mask, slot_voff, out);
    MB_LAUNCH_CHECK();
}

void cast_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
    if (n == 0) return;
    k_cast_f64_f32<<<grid_for(n), 256, 0, s>>>(a, b, n);
    MB_LAUNCH_CHECK();
}

template <int D>
static void sa_launch(const SetupBsr& A, int nv, const Aggregates& G, const double* q, const double* w, bool wave,
                      bool generic, int pass, int32_t* cnt, SetupBsr* P, int32_t* ovf, hipStream_t s) {
    const int n = A.n_rows;
    int32_t* prp = P ? P->rp.p : nullptr;
    int32_t* pci = P ? P->ci.p : nullptr;
    double* pval = P ? P->val.p : nullptr;
    if (wave)
        k_sa_prolong_w<D><<<n, WAVE, 0, s>>>(nv, A.rp.p, A.ci.p, A.val.p, G.agg.p, q, w, pass, cnt, prp, pci, pval,
                                             ovf);
    else
        k_sa_prolong_t<D><<<grid_for(n, 128), 128, 0, s>>>(n, nv, A.rp.p, A.ci.p, A.val.p, G.agg.p, q, w, pass, cnt,
                                                            prp, pci, pval, generic ? 1 : 0);
    MB_LAUNCH_CHECK();
}

static void sa_dispatch(int d, const SetupBsr& A, int nv, const Aggregates& G, const double* q, const double* w,
                        bool wave, bool generic, int pass, int32_t* cnt, SetupBsr* P, int32_t* ovf, hipStream_t s) {
    switch (d) {
        case 1: sa_launch<1>(A, nv, G, q, w, wave, generic, pass, cnt, P, ovf, s); break;
        case 2: sa_launch<2>(A, nv, G, q, w, wave, generic, pass, cnt, P, ovf, s); break;
        case 3: sa_launch<3>(A, nv, G, q, w, wave, generic, pass, cnt, P, ovf, s); break;
        default: sa_launch<4>(A, nv, G, q, w, wave, generic, pass, cnt, P, ovf, s); break;
    }
}

SetupBsr sa_prolongator(const SetupBsr& A, int nv, const Aggregates& G, const double* q, const double* w,
                        hipStream_t s) {
    MB_CHECK(A.br == A.bc && A.br >= 1 && A.br <= 4, MBAMG_E_INVALID,
             "smoothed prolongator needs square blocks of at most 4");
    const int n = A.n_rows, d = A.br;
    SetupBsr P;
    P.n_rows = n;
    P.n_cols = G.n_agg;
    P.br = P.bc = d;
    DevBuf<int32_t> cnt(std::max(n, 1)), ovf(1);
    MB_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int32_t), s));
    // short rows: one thread per row; long rows: one wavefront per row, or
    // one thread per row when some row does not fit the wavefront form
    bool wave = n > 0 && A.nnzb > (int64_t)16 * n;
    bool generic = false;
    if (const char* f = form_override("MBAMG_SA_FORM")) {
        wave = n > 0 && std::strcmp(f, "wave") == 0;
        generic = std::strcmp(f, "generic") == 0;
    }
    if (wave) {
        sa_dispatch(d, A, nv, G, q, w, true, false, 0, cnt.p, nullptr, ovf.p, s);
        wave = ovf.download(s, 1)[0] == 0;
    }
    if (n > 0 && !wave) sa_dispatch(d, A, nv, G, q, w, false, generic, 0, cnt.p, nullptr, ovf.p, s);
    P.rp.alloc(n + 1);
    P.nnzb = scan_exclusive(cnt.p, n, P.rp.p, s);
    P.ci.alloc(std::max<int64_t>(P.nnzb, 1));
    P.val.alloc(std::max<int64_t>(P.nnzb * d * d, 1));
    if (n > 0) sa_dispatch(d, A, nv, G, q, w, wave, generic, 1, nullptr, &P, ovf.p, s);
    return P;
}

SetupBsr block_transpose(const SetupBsr& P, hipStream_t s) {
    MB_CHECK(P.br * P.bc <= 16, MBAMG_E_INVALID, "block transpose: blocks of at most 16 entries");
    const int n = P.n_rows, nc = P.n_cols;
    SetupBsr T;
    T.n_rows = nc;
    T.n_cols = n;
    T.br = P.bc;
    T.bc = P.br;
    T.nnzb = P.nnzb;
    DevBuf<int32_t> cnt(std::max(nc, 1)), cursor(std::max(nc, 1));
    MB_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * std::max(nc, 1), s));
    MB_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int32_t) * std::max(nc, 1), s));
    k_count_cols<<<grid_for(n), 256, 0, s>>>(n, P.rp.p, P.ci.p, cnt.p);
    MB_LAUNCH_CHECK();
    T.rp.alloc(nc + 1);
    scan_exclusive(cnt.p, nc, T.rp.p, s);
    T.ci.alloc(std::max<int64_t>(P.nnzb, 1));
    DevBuf<int32_t> src(std::max<int64_t>(P.nnzb, 1));
    k_place_cols<<<grid_for(n), 256, 0, s>>>(n, P.rp.p, P.ci.p, T.rp.p, cursor.p, T.ci.p, src.p);
    T.val.alloc(std::max<int64_t>(P.nnzb * P.br * P.bc, 1));
    if (nc > 0) {
        DevBuf<int32_t> sorted_ci(std::max<int64_t>(P.nnzb, 1));
        k_transpose_rank<<<nc, WAVE, 0, s>>>(P.br, P.bc, T.rp.p, T.ci.p, src.p, P.val.p, sorted_ci.p, T.val.p);
        MB_LAUNCH_CHECK();
        MB_HIP(hipStreamSynchronize(s));
        T.ci = std::move(sorted_ci);
    }
    MB_HIP(hipStreamSynchronize(s));
    return T;
}

__global__ void k_rows_count(int n, const int32_t* perm, const int32_t* rp, int32_t* cnt) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int node = perm[p];
    cnt[p] = rp[node + 1] - rp[node];
}

// one wavefront per row: the row's blocks are contiguous at both ends
__global__ __launch_bounds__(256) void k_rows_fill(int n, int bs, const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                   const double* __restrict__ val,
                                                   const int32_t* __restrict__ col_iperm,
                                                   const int32_t* __restrict__ rrp, int32_t* __restrict__ rcol,
                                                   double* __restrict__ rval) {
    const int p = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    if (p >= n) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int node = perm[p];
    const int k0 = rp[node], len = rp[node + 1] - k0;
    const int q0 = rrp[p];
    for (int u = lane; u < len; u += WAVE) rcol[q0 + u] = col_iperm[ci[k0 + u]];
    const int64_t nv = (int64_t)len * bs;
    const double* a = val + (int64_t)k0 * bs;
    double* b = rval + (int64_t)q0 * bs;
    for (int64_t u = lane; u < nv; u += WAVE) b[u] = a[u];
}

__global__ void k_gather_blocks(int n, int bs, const int32_t* perm, const double* src, double* dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * bs) return;
    const int p = (int)(t / bs), e = (int)(t % bs);
    dst[t] = src[(int64_t)perm[p] * bs + e];
}

void build_rows(RowPart& R, int n, const int32_t* perm, const SetupBsr& A, const int32_t* col_iperm, bool want32,
                hipStream_t s) {
    R.br = A.br;
    R.bc = A.bc;
    const int bs = A.br * A.bc;
    R.rp.alloc(n + 1);
    if (A.nnzb == 0 || n == 0) {
        MB_HIP(hipMemsetAsync(R.rp.p, 0, sizeof(int32_t) * (n + 1), s));
        R.nnzb = 0;
        R.col.alloc(1);
        R.v64.alloc(1);
        if (want32) R.v32.alloc(1);
        return;
    }
    DevBuf<int32_t> cnt(n);
    k_rows_count<<<grid_for(n), 256, 0, s>>>(n, perm, A.rp.p, cnt.p);
    MB_LAUNCH_CHECK();
    R.nnzb = scan_exclusive(cnt.p, n, R.rp.p, s);
    R.col.alloc(std::max<int64_t>(R.nnzb, 1));
    R.v64.alloc(std::max<int64_t>(R.nnzb * bs, 1));
    k_rows_fill<<<grid_for((int64_t)n * WAVE), 256, 0, s>>>(n, bs, perm, A.rp.p, A.ci.p, A.val.p, col_iperm, R.rp.p,
                                                           R.col.p, R.v64.p);
    MB_LAUNCH_CHECK();
    if (want32) {
        R.v32.alloc(std::max<int64_t>(R.nnzb * bs, 1));
        cast_to_f32(R.v64.p, R.v32.p, R.nnzb * bs, s);
    }
    MB_HIP(hipStreamSynchronize(s));   // cnt is released on return
}

// Per row (colour order p, node perm[p]) of a block row: nonzero entries and
// blocks of A_ff's off-diagonal blocks, of A_fg, of D^-1 and of A_ff's
// diagonal block -- the counts the sliced parts would record.
__global__ __launch_bounds__(256) void k_row_stats(int n, const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ frp, const int32_t* __restrict__ fci,
                                                   const double* __restrict__ fval, int fbs,
                                                   const int32_t* __restrict__ grp, const double* __restrict__ gval,
                                                   int gbs, const double* __restrict__ dinv,
                                                   int32_t* __restrict__ out) {
    // one wavefront per row: lanes over the row's values (contiguous), counts by ballot
    const int p = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    if (p >= n) return;   // whole wavefronts
    const int lane = threadIdx.x & (WAVE - 1);
    const int node = perm[p];
    int off_nz = 0, diag_nz = 0, diag_bl = 0, cpl_nz = 0, dinv_nz = 0;
    const int f0 = frp[node], flen = frp[node + 1] - f0;
    for (int u0 = 0; u0 < flen * fbs; u0 += WAVE) {
        const int u = u0 + lane;
        bool nz = false, diag = false;
        if (u < flen * fbs) {
            nz = fval[(int64_t)f0 * fbs + u] != 0.0;
            diag = fci[f0 + u / fbs] == node;
        }
        diag_nz += (int)__popcll(__ballot(nz && diag));
        off_nz += (int)__popcll(__ballot(nz && !diag));
    }
    for (int q = lane; q < flen; q += WAVE) diag_bl += fci[f0 + q] == node;
    for (int off = WAVE / 2; off > 0; off >>= 1) diag_bl += __shfl_xor(diag_bl, off);
    int glen = 0;
    if (grp) {
        const int g0 = grp[node];
        glen = grp[node + 1] - g0;
        for (int u0 = 0; u0 < glen * gbs; u0 += WAVE) {
            const int u = u0 + lane;
            const bool nz = u < glen * gbs && gval[(int64_t)g0 * gbs + u] != 0.0;
            cpl_nz += (int)__popcll(__ballot(nz));
        }
    }
    for (int u0 = 0; u0 < fbs; u0 += WAVE)
        dinv_nz += (int)__popcll(__ballot(u0 + lane < fbs && dinv[(int64_t)node * fbs + u0 + lane] != 0.0));
    if (lane != 0) return;
    int32_t* o = out + (int64_t)p * 7;
    o[0] = off_nz;
    o[1] = flen - diag_bl;
    o[2] = cpl_nz;
    o[3] = glen;
    o[4] = dinv_nz;
    o[5] = diag_nz;
    o[6] = diag_bl;
}

std::vector<int64_t> row_colour_stats(int n, const int32_t* perm, const SetupBsr& Aff, const SetupBsr& Afg,
                                      const double* dinv, const std::vector<int>& colour_row, hipStream_t s) {
    const int nc = (int)colour_row.size() - 1;
    std::vector<int64_t> sums((size_t)std::max(nc, 0) * 7, 0);
    if (n == 0) return sums;
    DevBuf<int32_t> per((size_t)n * 7);
    k_row_stats<<<grid_for((int64_t)n * WAVE), 256, 0, s>>>(n, perm, Aff.rp.p, Aff.ci.p, Aff.val.p,
                                                            Aff.br * Aff.bc, Afg.nnzb ? Afg.rp.p : nullptr,
                                                            Afg.val.p, Afg.br * Afg.bc, dinv, per.p);
    MB_LAUNCH_CHECK();
    const std::vector<int32_t> h = per.download(s, (size_t)n * 7);
    for (int c = 0; c < nc; ++c)
        for (int p = colour_row[c]; p < colour_row[c + 1]; ++p)
            for (int k = 0; k < 7; ++k) sums[(size_t)c * 7 + k] += h[(size_t)p * 7 + k];
    return sums;
}

void gather_blocks(int n, int bs, const int32_t* perm, const double* src, double* dst, hipStream_t s) {
    if (n == 0) return;
    k_gather_blocks<<<grid_for((int64_t)n * bs), 256, 0, s>>>(n, bs, perm, src, dst);
    MB_LAUNCH_CHECK();
}

bool same_pattern(const SetupBsr& X, const SetupBsr& Y, hipStream_t s) {
    if (X.n_rows != Y.n_rows || X.n_cols != Y.n_cols || X.nnzb != Y.nnzb) return false;
    if (X.n_rows == 0 || X.nnzb == 0) return true;
    DevBuf<int32_t> flag(1);
    const std::vector<int32_t> one(1, 1);
    flag.upload(one, s);
    const int64_t total = (int64_t)X.n_rows + 1 + X.nnzb;
    k_same_pattern<<<(unsigned)std::min<int64_t>(4096, ceil_div(total, 256)), 256, 0, s>>>(
        (int64_t)X.n_rows + 1, X.nnzb, X.rp.p, X.ci.p, Y.rp.p, Y.ci.p, flag.p);
    MB_LAUNCH_CHECK();
    return flag.download(s, 1)[0] != 0;
}

// outputs with fewer blocks than this take one lane per output entry (above
// it, one thread per block is faster: the lanes of a block repeat its
// column searches)
constexpr int64_t SPGEMM_ENTRY_MAX = (int64_t)1 << 15;

template <int BR, int BM, int BC>
static void num_chunked(int chunk, unsigned g, int64_t z, const SetupBsr& A, const SetupBsr& B, SetupBsr& C,
                        const int32_t* crow, hipStream_t s) {
    if (chunk == 1)
        k_spgemm_num_c<BR, BM, BC, 1><<<g, 128, 0, s>>>(z, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p, B.val.p, crow,
                                                        C.ci.p, C.val.p);
    else if (chunk == 2)
        k_spgemm_num_c<BR, BM, BC, 2><<<g, 128, 0, s>>>(z, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p, B.val.p, crow,
                                                        C.ci.p, C.val.p);
    else
        k_spgemm_num_c<BR, BM, BC, 4><<<g, 128, 0, s>>>(z, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p, B.val.p, crow,
                                                        C.ci.p, C.val.p);
}

static void spgemm_values(const SetupBsr& A, const SetupBsr& B, SetupBsr& C, const int32_t* crow, hipStream_t s) {
    if (C.nnzb == 0) return;
    const unsigned g = grid_for(C.nnzb, 128);
    const int64_t z = C.nnzb;
    bool entry = z < SPGEMM_ENTRY_MAX;
    int chunk = 4;   // measured: lookups of 4 row entries at once beat 1 and 2
    if (const char* f = form_override("MBAMG_SPGEMM_FORM")) {
        entry = std::strcmp(f, "entry") == 0;
        chunk = std::strcmp(f, "chunk2") == 0 ? 2 : std::strcmp(f, "block") == 0 ? 1 : 4;
    }
    const unsigned ge = grid_for(z * 16, 256);
    if (entry && A.br == 4 && A.bc == 4 && B.bc == 4)
        k_spgemm_num_e<4, 4, 4><<<ge, 256, 0, s>>>(z, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p, B.val.p, crow, C.ci.p,
                                                  C.val.p);
    else if (entry && A.br == 3 && A.bc == 3 && B.bc == 3)
        k_spgemm_num_e<3, 3, 3><<<ge, 256, 0, s>>>(z, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p, B.val.p, crow, C.ci.p,
                                                  C.val.p);
    else if (A.br == 4 && A.bc == 4 && B.bc == 4)
        num_chunked<4, 4, 4>(chunk, g, z, A, B, C, crow, s);
    else if (A.br == 3 && A.bc == 3 && B.bc == 3)
        num_chunked<3, 3, 3>(chunk, g, z, A, B, C, crow, s);
    else
        k_spgemm_num_any<<<g, 128, 0, s>>>(z, A.br, A.bc, B.bc, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p, B.val.p,
                                           crow, C.ci.p, C.val.p);
    MB_LAUNCH_CHECK();
}

// The pattern of C = A B (rows of C list their columns in increasing order),
// found or taken from `like`; C.val is allocated.  Returns false when a row
// was too long for the symbolic kernels and the one-thread-per-row product
// has filled the values as well.
static bool spgemm_pattern(const SetupBsr& A, const SetupBsr& B, SetupBsr& C, hipStream_t s, const SetupBsr* like) {
    MB_CHECK(A.bc == B.br && A.br * B.bc <= 16, MBAMG_E_INVALID, "block product shapes");
    const int n = A.n_rows;
    C = SetupBsr();
    C.n_rows = n;
    C.n_cols = B.n_cols;
    C.br = A.br;
    C.bc = B.bc;
    C.rp.alloc(n + 1);
    if (A.nnzb == 0 || B.nnzb == 0) {
        MB_HIP(hipMemsetAsync(C.rp.p, 0, sizeof(int32_t) * (n + 1), s));
        C.ci.alloc(1);
        C.val.alloc(1);
        return false;
    }
    if (like) {
        // the caller guarantees that A and B have the patterns that produced `like`
        MB_CHECK(like->n_rows == n && like->n_cols == B.n_cols, MBAMG_E_STATE, "internal: reused pattern shape");
        C.nnzb = like->nnzb;
        C.ci.alloc(std::max<int64_t>(C.nnzb, 1));
        MB_HIP(hipMemcpyAsync(C.rp.p, like->rp.p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
        if (C.nnzb)
            MB_HIP(hipMemcpyAsync(C.ci.p, like->ci.p, sizeof(int32_t) * C.nnzb, hipMemcpyDeviceToDevice, s));
    } else {
        DevBuf<int32_t> cnt(std::max(n, 1)), ovf(1);
        MB_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int32_t), s));
        // short rows of A: one thread per row while the distinct columns fit in registers
        bool per_thread = A.nnzb <= (int64_t)16 * n;
        if (const char* f = form_override("MBAMG_SYM_FORM")) per_thread = std::strcmp(f, "thread") == 0;
        if (per_thread) {
            k_spgemm_sym_t<<<grid_for(n, 128), 128, 0, s>>>(n, A.rp.p, A.ci.p, B.rp.p, B.ci.p, 0, cnt.p, nullptr,
                                                          nullptr, ovf.p);
            MB_LAUNCH_CHECK();
            if (ovf.download(s, 1)[0] != 0) {
                per_thread = false;
                MB_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int32_t), s));
            }
        }
        if (!per_thread) {
            k_spgemm_sym<<<n, WAVE, 0, s>>>(A.rp.p, A.ci.p, B.rp.p, B.ci.p, 0, cnt.p, nullptr, nullptr, ovf.p);
            MB_LAUNCH_CHECK();
        }
        if (!per_thread && ovf.download(s, 1)[0] != 0) {
            // a row has too many distinct columns for the LDS set: thread-per-row product
            k_spgemm<<<grid_for(n, 64), 64, 0, s>>>(n, A.br, A.bc, B.bc, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p,
                                                   B.val.p, 0, cnt.p, nullptr, nullptr, nullptr);
            MB_LAUNCH_CHECK();
            C.nnzb = scan_exclusive(cnt.p, n, C.rp.p, s);
            C.ci.alloc(std::max<int64_t>(C.nnzb, 1));
            C.val.alloc(std::max<int64_t>(C.nnzb * C.br * C.bc, 1));
            k_spgemm<<<grid_for(n, 64), 64, 0, s>>>(n, A.br, A.bc, B.bc, A.rp.p, A.ci.p, A.val.p, B.rp.p, B.ci.p,
                                                   B.val.p, 1, nullptr, C.rp.p, C.ci.p, C.val.p);
            MB_LAUNCH_CHECK();
            MB_HIP(hipStreamSynchronize(s));
            return false;
        }
        C.nnzb = scan_exclusive(cnt.p, n, C.rp.p, s);
        C.ci.alloc(std::max<int64_t>(C.nnzb, 1));
        if (per_thread)
            k_spgemm_sym_t<<<grid_for(n, 128), 128, 0, s>>>(n, A.rp.p, A.ci.p, B.rp.p, B.ci.p, 1, nullptr, C.rp.p,
                                                          C.ci.p, ovf.p);
        else
            k_spgemm_sym<<<n, WAVE, 0, s>>>(A.rp.p, A.ci.p, B.rp.p, B.ci.p, 1, nullptr, C.rp.p, C.ci.p, ovf.p);
        MB_LAUNCH_CHECK();
        MB_HIP(hipStreamSynchronize(s));   // cnt and ovf are released on leaving this block
    }
    C.val.alloc(std::max<int64_t>(C.nnzb * C.br * C.bc, 1));
    return true;
}

SetupBsr spgemm(const SetupBsr& A, const SetupBsr& B, hipStream_t s, const SetupBsr* like) {
    SetupBsr C;
    if (!spgemm_pattern(A, B, C, s, like)) return C;
    DevBuf<int32_t> crow(std::max<int64_t>(C.nnzb, 1));
    k_row_of<<<grid_for(C.n_rows), 256, 0, s>>>(C.n_rows, C.rp.p, crow.p);
    MB_LAUNCH_CHECK();
    spgemm_values(A, B, C, crow.p, s);
    MB_HIP(hipStreamSynchronize(s));   // crow is released on return
    return C;
}

template <int BR, int BM, int BC, int K>
static void launch_num_k(const SetupBsr* const* A, const SetupBsr* const* B, SetupBsr* const* C,
                         const int32_t* crow, hipStream_t s) {
    SpgemmVals<K> v;
    for (int k = 0; k < K; ++k) {
        v.a[k] = A[k]->val.p;
        v.b[k] = B[k]->val.p;
        v.c[k] = C[k]->val.p;
    }
    const SetupBsr& A0 = *A[0];
    const SetupBsr& B0 = *B[0];
    const int64_t z = C[0]->nnzb;
    if (z < SPGEMM_ENTRY_MAX)
        k_spgemm_num_ek<BR, BM, BC, K><<<grid_for(z * 16, 256), 256, 0, s>>>(z, A0.rp.p, A0.ci.p, B0.rp.p, B0.ci.p,
                                                                            crow, C[0]->ci.p, v);
    else
        // one lookup at a time here: the K accumulators leave no room for more (measured
        // slower with two)
        k_spgemm_num_k<BR, BM, BC, K, 1><<<grid_for(z, 128), 128, 0, s>>>(z, A0.rp.p, A0.ci.p, B0.rp.p, B0.ci.p,
                                                                         crow, C[0]->ci.p, v);
    MB_LAUNCH_CHECK();
}

void spgemm_multi(const SetupBsr* const* A, const SetupBsr* const* B, int K, SetupBsr* const* C, hipStream_t s,
                  const SetupBsr* like) {
    MB_CHECK(K >= 1 && K <= 4, MBAMG_E_INVALID, "internal: 1..4 products at once");
    for (int k = 1; k < K; ++k)
        MB_CHECK(A[k]->n_rows == A[0]->n_rows && A[k]->nnzb == A[0]->nnzb && B[k]->nnzb == B[0]->nnzb &&
                     A[k]->br == A[0]->br && A[k]->bc == A[0]->bc && B[k]->bc == B[0]->bc,
                 MBAMG_E_STATE, "internal: products grouped with different shapes");
    if (!spgemm_pattern(*A[0], *B[0], *C[0], s, like)) {
        for (int k = 1; k < K; ++k) *C[k] = spgemm(*A[k], *B[k], s, C[0]);
        return;
    }
    for (int k = 1; k < K; ++k) {
        SetupBsr& Ck = *C[k];
        Ck = SetupBsr();
        Ck.n_rows = C[0]->n_rows;
        Ck.n_cols = C[0]->n_cols;
        Ck.br = C[0]->br;
        Ck.bc = C[0]->bc;
        Ck.nnzb = C[0]->nnzb;
        Ck.rp.alloc(Ck.n_rows + 1);
        Ck.ci.alloc(std::max<int64_t>(Ck.nnzb, 1));
        Ck.val.alloc(std::max<int64_t>(Ck.nnzb * Ck.br * Ck.bc, 1));
        MB_HIP(hipMemcpyAsync(Ck.rp.p, C[0]->rp.p, sizeof(int32_t) * (Ck.n_rows + 1), hipMemcpyDeviceToDevice, s));
        if (Ck.nnzb)
            MB_HIP(hipMemcpyAsync(Ck.ci.p, C[0]->ci.p, sizeof(int32_t) * Ck.nnzb, hipMemcpyDeviceToDevice, s));
    }
    const int64_t z = C[0]->nnzb;
    if (z == 0) return;
    DevBuf<int32_t> crow(std::max<int64_t>(z, 1));
    k_row_of<<<grid_for(C[0]->n_rows), 256, 0, s>>>(C[0]->n_rows, C[0]->rp.p, crow.p);
    MB_LAUNCH_CHECK();
    const SetupBsr& A0 = *A[0];
    const SetupBsr& B0 = *B[0];
    const bool shape4 = A0.br == 4 && A0.bc == 4 && B0.bc == 4, shape3 = A0.br == 3 && A0.bc == 3 && B0.bc == 3;
    // one launch for the group, one lookup per output block and row entry (measured: pays
    // for groups of three or four, where the lookups dominate, and for tiny outputs; larger
    // pairs are faster apart); the forced single-product forms take one launch per product
    const char* fo = form_override("MBAMG_SPGEMM_FORM");
    const bool fuse = (shape4 || shape3) && (fo ? std::strcmp(fo, "fused") == 0 && K >= 2
                                                : K >= 3 || (K >= 2 && z < SPGEMM_ENTRY_MAX));
    if (!fuse) {
        for (int k = 0; k < K; ++k) spgemm_values(*A[k], *B[k], *C[k], crow.p, s);
    } else if (shape4) {
        if (K == 2) launch_num_k<4, 4, 4, 2>(A, B, C, crow.p, s);
        else if (K == 3) launch_num_k<4, 4, 4, 3>(A, B, C, crow.p, s);
        else launch_num_k<4, 4, 4, 4>(A, B, C, crow.p, s);
    } else {
        if (K == 2) launch_num_k<3, 3, 3, 2>(A, B, C, crow.p, s);
        else if (K == 3) launch_num_k<3, 3, 3, 3>(A, B, C, crow.p, s);
        else launch_num_k<3, 3, 3, 4>(A, B, C, crow.p, s);
    }
    MB_HIP(hipStreamSynchronize(s));   // crow is released on return
}

void part_layout(int n, int ns, int kind, const int32_t* perm, const int32_t* rp, const int32_t* ci,
                 const int32_t* row0, const int32_t* nrow, DevBuf<int32_t>& width, DevBuf<int32_t>& coff32,
                 int64_t& n_slots, hipStream_t s) {
    DevBuf<int32_t> rowlen(std::max(n, 1));
    k_part_rowlen<<<grid_for(n), 256, 0, s>>>(n, kind, perm, rp, ci, rowlen.p);
    width.alloc(std::max(ns, 1));
    k_part_width<<<grid_for(ns), 256, 0, s>>>(ns, kind, row0, nrow, rowlen.p, width.p);
    MB_LAUNCH_CHECK();
    coff32.alloc(ns + 1);
    n_slots = scan_exclusive(width.p, ns, coff32.p, s);
}

void part_fill_index(int ns, int kind, const int32_t* row0, const int32_t* nrow, const int32_t* width,
                     const int32_t* coff32, const int32_t* perm, const int32_t* rp, const int32_t* ci,
                     const int32_t* col_iperm, int64_t n_slots, int32_t* col, int64_t* src, int32_t* slot_blocks,
                     hipStream_t s) {
    MB_HIP(hipMemsetAsync(slot_blocks, 0, sizeof(int32_t) * std::max<int64_t>(n_slots, 1), s));
    k_part_fill_index<<<grid_for((int64_t)ns * WAVE), 256, 0, s>>>(ns, kind, row0, nrow, width, coff32, perm, rp, ci,
                                                                   col_iperm, col, src, slot_blocks);
    MB_LAUNCH_CHECK();
}

int64_t slot_offsets(int64_t n_slots, const uint32_t* mask, DevBuf<int64_t>& voff, hipStream_t s) {
    DevBuf<int32_t> cnt(std::max<int64_t>(n_slots, 1)), off32(n_slots + 1);
    k_popcount<<<grid_for(n_slots), 256, 0, s>>>(n_slots, mask, cnt.p);
    MB_LAUNCH_CHECK();
    int64_t groups = scan_exclusive(cnt.p, n_slots, off32.p, s);
    voff.alloc(std::max<int64_t>(n_slots, 1));
    k_i32_to_i64<<<grid_for(n_slots), 256, 0, s>>>(n_slots, off32.p, voff.p);
    MB_LAUNCH_CHECK();
    MB_HIP(hipStreamSynchronize(s));
    return groups;
}

void i32_to_i64(int64_t n, const int32_t* a, int64_t* b, hipStream_t s) {
    if (n <= 0) return;
    k_i32_to_i64<<<grid_for(n), 256, 0, s>>>(n, a, b);
    MB_LAUNCH_CHECK();
}

void transfer_maps(int n, int nc, const int32_t* perm, const int32_t* iperm, const int32_t* agg,
                   const int32_t* cperm, const int32_t* ciperm, const int32_t* mptr, const int32_t* midx,
                   DevBuf<int32_t>& aggp, DevBuf<int32_t>& optr, DevBuf<int32_t>& oidx, hipStream_t s) {
    aggp.alloc(std::max(n, 1));
    k_map_agg<<<grid_for(n), 256, 0, s>>>(n, perm, agg, ciperm, aggp.p);
    DevBuf<int32_t> cnt(std::max(nc, 1));
    k_map_count<<<grid_for(nc), 256, 0, s>>>(nc, cperm, mptr, cnt.p);
    MB_LAUNCH_CHECK();
    optr.alloc(nc + 1);
    scan_exclusive(cnt.p, nc, optr.p, s);
    oidx.alloc(std::max(n, 1));
    k_map_members<<<grid_for(nc), 256, 0, s>>>(nc, cperm, mptr, midx, iperm, optr.p, oidx.p);
    MB_LAUNCH_CHECK();
}

template <int T, int R, int B>
static void gj_run(CoarseWork& w, int n, hipStream_t s, double** result, const int32_t** order) {
    double* cur = w.M.p;
    double* nxt = w.M.p + (size_t)n * n;
    const int32_t* ord_in = nullptr;
    int which = 0;
    for (int k0 = 0; k0 < n; k0 += B) {
        const int b = std::min(B, n - k0);
        k_gj_panel<T, R, B><<<1, T, 0, s>>>(cur, n, k0, b, w.rowsrc.p, w.sing.p);
        if (b == n) {   // one panel: nothing outside it
            ord_in = w.rowsrc.p;
            break;
        }
        int32_t* ord_out = w.ord.p + (size_t)which * n;
        const dim3 grid((n + GJ_TILE - 1) / GJ_TILE, (n + GJ_TILE - 1) / GJ_TILE);
        k_gj_update<B><<<grid, 256, 0, s>>>(cur, nxt, n, k0, b, w.rowsrc.p, ord_in, ord_out);
        ord_in = ord_out;
        which ^= 1;
        std::swap(cur, nxt);
    }
    MB_LAUNCH_CHECK();
    *result = cur;
    *order = ord_in;
}

void coarse_inverse_launch_blocks(const SetupBsr* const* A, int nb, const int* d, DevBuf<double>& inv, CoarseWork& w,
                                  hipStream_t s) {
    // block f's dofs start after the blocks before it (node-major within each block)
    std::vector<int64_t> off(nb + 1, 0);
    for (int f = 0; f < nb; ++f) off[f + 1] = off[f] + (int64_t)A[f * nb + f]->n_rows * d[f];
    const int n = (int)off[nb];
    MB_CHECK(off[nb] <= 16384, MBAMG_E_INVALID, "coarsest level too large for the dense solve (raise max_levels)");
    w.n = n;
    w.M.alloc((size_t)2 * n * n);
    w.sing.alloc(1);
    w.rowsrc.alloc(std::max(n, 1));
    w.ord.alloc((size_t)2 * std::max(n, 1));
    inv.alloc((size_t)n * n);
    MB_HIP(hipMemsetAsync(w.sing.p, 0, sizeof(int32_t), s));
    if (n == 0) return;
    MB_HIP(hipMemsetAsync(w.M.p, 0, sizeof(double) * (size_t)n * n, s));
    for (int f = 0; f < nb; ++f)
        for (int g = 0; g < nb; ++g) {
            const SetupBsr& B = *A[f * nb + g];
            if (B.nnzb == 0) continue;
            k_dense_scatter<<<grid_for(B.n_rows, 64), 64, 0, s>>>(B.n_rows, B.br, B.bc, B.rp.p, B.ci.p, B.val.p,
                                                                 off[f], off[g], (int64_t)n, w.M.p);
            MB_LAUNCH_CHECK();
        }
    // threads T and rows per thread R set the panel width B: R * B doubles stay in registers
    double* X = nullptr;
    const int32_t* ord = nullptr;
    if (n <= 512) gj_run<512, 1, 16>(w, n, s, &X, &ord);
    else if (n <= 1024) gj_run<512, 2, 16>(w, n, s, &X, &ord);
    else if (n <= 2048) gj_run<512, 4, 16>(w, n, s, &X, &ord);
    else if (n <= 3072) gj_run<512, 6, 16>(w, n, s, &X, &ord);
    else if (n <= 4096) gj_run<512, 8, 8>(w, n, s, &X, &ord);
    else if (n <= 8192) gj_run<512, 16, 4>(w, n, s, &X, &ord);
    else gj_run<512, 32, 2>(w, n, s, &X, &ord);
    k_gj_extract<<<grid_for((int64_t)n * n), 256, 0, s>>>(X, n, ord, inv.p);
    MB_LAUNCH_CHECK();
}

void coarse_inverse_launch(const SetupBsr (&A)[2][2], const int d[2], DevBuf<double>& inv, CoarseWork& w,
                           hipStream_t s) {
    const SetupBsr* blocks[4] = {&A[0][0], &A[0][1], &A[1][0], &A[1][1]};
    coarse_inverse_launch_blocks(blocks, 2, d, inv, w, s);
}

void coarse_inverse_finish(CoarseWork& w, hipStream_t s) {
    int32_t h = 0;
    MB_HIP(hipMemcpyAsync(&h, w.sing.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    w.M.release();
    w.rowsrc.release();
    w.ord.release();
    MB_CHECK(h == 0, MBAMG_E_SINGULAR, "the coarsest matrix is singular");
}

}  // namespace mbamg
