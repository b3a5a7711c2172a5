// Solve-phase kernels for gfx950: one 64-lane wavefront per slice of 64
// block rows, one lane per block row.  Matrix values are stored slot-major and
// lane-contiguous, so every value load of a wavefront is one contiguous
// 256 B (FP32) or 512 B (FP64) segment; only block entries that are nonzero
// somewhere in the slice are stored, which keeps the streamed bytes close to
// the structural nonzeros.  All loops over slots and mask bits are
// wave-uniform (scalar branches).
#include "solve_kernels.h"

#include <algorithm>
#include <climits>

namespace mbamg {

constexpr int WPB = 4;          // waves per 256-thread block
constexpr int CHUNK = 2;        // slots whose loads are issued together

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of slices so neighbour gathers stay in its own L2.
__device__ __forceinline__ int xcd_slice(int nslices_padded_blocks) {
    const int per = nslices_padded_blocks >> 3;
    const int bid = blockIdx.x;
    const int logical = (bid & 7) * per + (bid >> 3);
    return logical * WPB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

static inline unsigned xcd_grid(int nslices) {
    int blocks = (int)ceil_div(nslices, WPB);
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

// acc[r] -= sum_c A[r,c] * x_col(c) over all slots of one part.
// MODE 0: x from xa.  MODE 1: columns below cstart from xa (already updated),
// others from xb.  MODE 2: columns below cstart from xa, others contribute 0.
template <class T, int BR, int BC, int MODE>
__device__ __forceinline__ void sell_sub(const SellView<T>& A, int s, int lane, const T* __restrict__ xa,
                                         const T* __restrict__ xb, int cstart, T (&acc)[BR]) {
    const int w = A.width[s];
    const int64_t cb = A.coff[s];
    int64_t vg = A.voff[s];
    for (int t = 0; t < w; t += CHUNK) {
        int j[CHUNK];
        uint32_t m[CHUNK];
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) {
            const bool live = t + u < w;
            m[u] = live ? A.mask[cb + t + u] : 0u;
            j[u] = live ? A.col[(cb + t + u) * WAVE + lane] : -1;
        }
        T v[CHUNK][BR * BC];
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) {
            load_masked<T, BR * BC>(A.val + vg * WAVE + lane, m[u], v[u]);
            vg += __builtin_popcount(m[u]);
        }
        T xj[CHUNK][BC];
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) {
            const int jj = j[u];
            const T* src = nullptr;
            if (MODE == 0) src = xa;
            else if (MODE == 1) src = jj < cstart ? xa : xb;
            else src = jj < cstart ? xa : nullptr;
            if (jj >= 0 && src) load_vec<T, BC>(src + (int64_t)jj * BC, xj[u]);
            else {
#pragma unroll
                for (int c = 0; c < BC; ++c) xj[u][c] = T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < CHUNK; ++u)
#pragma unroll
            for (int r = 0; r < BR; ++r)
#pragma unroll
                for (int c = 0; c < BC; ++c) acc[r] -= v[u][r * BC + c] * xj[u][c];
    }
}

// One colour of the multicolour nodal-block Gauss-Seidel sub-solve of block f
// inside Algorithm 1: for each row i of the colour
//   t_i  = D_i^-1 (b_i - sum_{j != i} A_ff[i,j] t_j - (A_fg x_g)_i)
//   xn_i = x_i + omega (t_i - x_i)
// where t_j is the updated value for rows of earlier colours and x_j otherwise;
// t_i - x_i is the sub-solve's correction e_i for the residual b - A x.
template <class T, int D, bool ZX, bool CPL>
__global__ __launch_bounds__(256) void k_gs(GsArgs<T> a, int padded_blocks) {
    const int sidx = xcd_slice(padded_blocks);
    if (sidx >= a.s_count) return;
    const int s = a.s_begin + sidx;
    const int lane = threadIdx.x & (WAVE - 1);
    const int row0 = a.sl.row0[s], nrow = a.sl.nrow[s];
    const bool act = lane < nrow;
    const int row = row0 + (act ? lane : 0);
    T acc[D];
    load_vec<T, D>(a.b + (int64_t)row * D, acc);
    if (!a.skip_off) {
        if (ZX) sell_sub<T, D, D, 2>(a.off, s, lane, a.t, nullptr, a.cstart, acc);
        else sell_sub<T, D, D, 1>(a.off, s, lane, a.t, a.x, a.cstart, acc);
    }
    if (CPL) sell_sub<T, D, D, 0>(a.cpl, s, lane, a.xg, nullptr, 0, acc);
    T dv[D * D];
    load_masked<T, D * D>(a.dinv.val + a.dinv.voff[s] * WAVE + lane, a.dinv.mask[a.dinv.coff[s]], dv);
    T tn[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T sum = T(0);
#pragma unroll
        for (int c = 0; c < D; ++c) sum += dv[r * D + c] * acc[c];
        tn[r] = sum;
    }
    if (!act) return;
    const T w = a.w_row ? a.w_row[row] : a.omega;
    T xn[D];
    if (ZX) {
#pragma unroll
        for (int r = 0; r < D; ++r) xn[r] = w * tn[r];
    } else {
        T xo[D];
        load_vec<T, D>(a.x + (int64_t)row * D, xo);
#pragma unroll
        for (int r = 0; r < D; ++r) xn[r] = xo[r] + w * (tn[r] - xo[r]);
    }
    store_vec<T, D>(a.t + (int64_t)row * D, tn);
    store_vec<T, D>(a.xn + (int64_t)row * D, xn);
}

// r = b - A x (or w = A x when b is NULL) for both block rows in one launch.
template <class T, int D>
__global__ __launch_bounds__(256) void k_resid(ResidArgs<T> a, int padded_blocks) {
    int sidx = xcd_slice(padded_blocks);
    int f = 0;
    if (sidx >= a.s_count[0]) {
        sidx -= a.s_count[0];
        f = 1;
        if (sidx >= a.s_count[1]) return;
    }
    const int g = 1 - f;
    const int lane = threadIdx.x & (WAVE - 1);
    const int row0 = a.sl[f].row0[sidx], nrow = a.sl[f].nrow[sidx];
    const bool act = lane < nrow;
    const int row = row0 + (act ? lane : 0);
    T acc[D];
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r] = T(0);
    sell_sub<T, D, D, 0>(a.diag[f], sidx, lane, a.x[f], nullptr, 0, acc);
    sell_sub<T, D, D, 0>(a.off[f], sidx, lane, a.x[f], nullptr, 0, acc);
    sell_sub<T, D, D, 0>(a.cpl[f], sidx, lane, a.x[g], nullptr, 0, acc);
    if (!act) return;
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

// coarse b_k = sum over members i of aggregate k of q_i .* r_i (per component)
template <class T, int D>
__global__ void k_restrict(TransferArgs<T> a) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int f = 0;
    if (k >= a.n_rows[0]) {
        k -= a.n_rows[0];
        f = 1;
        if (k >= a.n_rows[1]) return;
    }
    const int32_t* mp = a.map[f];
    const int32_t* mi = a.idx[f];
    T acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = T(0);
    for (int m = mp[k]; m < mp[k + 1]; ++m) {
        const int64_t i = mi[m];
        T q[D], r[D];
        load_vec<T, D>(a.q[f] + i * D, q);
        load_vec<T, D>(a.in[f] + i * D, r);
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] += q[c] * r[c];
    }
    store_vec<T, D>(a.out[f] + (int64_t)k * D, acc);
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
template <class T, int D>
static void gs_dispatch(bool zx, bool cpl, const GsArgs<T>& a, hipStream_t s) {
    if (a.s_count <= 0) return;
    unsigned grid = xcd_grid(a.s_count);
    int pb = (int)grid;
    if (zx) {
        if (cpl) k_gs<T, D, true, true><<<grid, 256, 0, s>>>(a, pb);
        else k_gs<T, D, true, false><<<grid, 256, 0, s>>>(a, pb);
    } else {
        if (cpl) k_gs<T, D, false, true><<<grid, 256, 0, s>>>(a, pb);
        else k_gs<T, D, false, false><<<grid, 256, 0, s>>>(a, pb);
    }
    MB_LAUNCH_CHECK();
}

template <class T>
void launch_gs(int d, bool zero_x, bool has_cpl, const GsArgs<T>& a, hipStream_t s) {
    switch (d) {
        case 1: gs_dispatch<T, 1>(zero_x, has_cpl, a, s); break;
        case 2: gs_dispatch<T, 2>(zero_x, has_cpl, a, s); break;
        case 3: gs_dispatch<T, 3>(zero_x, has_cpl, a, s); break;
        case 4: gs_dispatch<T, 4>(zero_x, has_cpl, a, s); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
}

template <class T>
void launch_resid(int d, const ResidArgs<T>& a, hipStream_t s) {
    const int total = a.s_count[0] + a.s_count[1];
    if (total <= 0) return;
    unsigned grid = xcd_grid(total);
    int pb = (int)grid;
    switch (d) {
        case 1: k_resid<T, 1><<<grid, 256, 0, s>>>(a, pb); break;
        case 2: k_resid<T, 2><<<grid, 256, 0, s>>>(a, pb); break;
        case 3: k_resid<T, 3><<<grid, 256, 0, s>>>(a, pb); break;
        case 4: k_resid<T, 4><<<grid, 256, 0, s>>>(a, pb); break;
        default: throw Error(MBAMG_E_INVALID, "dofs per node must be 1..4");
    }
    MB_LAUNCH_CHECK();
}

template <class T>
void launch_restrict(int d, const TransferArgs<T>& a, hipStream_t s) {
    const int total = a.n_rows[0] + a.n_rows[1];
    if (total <= 0) return;
    unsigned grid = (unsigned)ceil_div(total, 256);
    switch (d) {
        case 1: k_restrict<T, 1><<<grid, 256, 0, s>>>(a); break;
        case 2: k_restrict<T, 2><<<grid, 256, 0, s>>>(a); break;
        case 3: k_restrict<T, 3><<<grid, 256, 0, s>>>(a); break;
        case 4: k_restrict<T, 4><<<grid, 256, 0, s>>>(a); break;
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

template void launch_gs<double>(int, bool, bool, const GsArgs<double>&, hipStream_t);
template void launch_gs<float>(int, bool, bool, const GsArgs<float>&, hipStream_t);
template void launch_resid<double>(int, const ResidArgs<double>&, hipStream_t);
template void launch_resid<float>(int, const ResidArgs<float>&, hipStream_t);
template void launch_restrict<double>(int, const TransferArgs<double>&, hipStream_t);
template void launch_restrict<float>(int, const TransferArgs<float>&, hipStream_t);
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

// partial[b*KMAXQ + q] = sum over this block's elements of V_q . w
__global__ __launch_bounds__(256) void k_multidot(int64_t n, int nq, const double* __restrict__ V, int64_t ldv,
                                                  const double* __restrict__ w, double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc[KMAXQ - 1];
#pragma unroll
    for (int q = 0; q < KMAXQ - 1; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const double we = w[e];
#pragma unroll
        for (int q = 0; q < KMAXQ - 1; ++q)
            if (q < nq) acc[q] += V[q * ldv + e] * we;
    }
#pragma unroll
    for (int q = 0; q < KMAXQ - 1; ++q) {
        if (q >= nq) break;
        double r = block_sum(acc[q], sh);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * KMAXQ + q] = r;
    }
}

// w -= sum_q h_q V_q ; optionally partial norm^2 of the new w in slot nq
__global__ __launch_bounds__(256) void k_update(int64_t n, int nq, const double* __restrict__ V, int64_t ldv,
                                                const double* __restrict__ h, double* __restrict__ w, int norm,
                                                double* __restrict__ partial) {
    __shared__ double sh[4];
    double hq[KMAXQ - 1];
#pragma unroll
    for (int q = 0; q < KMAXQ - 1; ++q) hq[q] = q < nq ? h[q] : 0.0;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double we = w[e];
#pragma unroll
        for (int q = 0; q < KMAXQ - 1; ++q)
            if (q < nq) we -= hq[q] * V[q * ldv + e];
        w[e] = we;
        acc += we * we;
    }
    if (norm) {
        double r = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * KMAXQ + nq] = r;
    }
}

// out[q - q0] = sum_b partial[b*KMAXQ + q] for q in [q0, q0+cnt), in a fixed order
__global__ void k_reduce(const double* __restrict__ partial, int nb, int q0, int cnt, double* __restrict__ out) {
    __shared__ double sh[4];
    for (int q = q0; q < q0 + cnt; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) v += partial[(int64_t)b * KMAXQ + q];
        double r = block_sum(v, sh);
        if (threadIdx.x == 0) out[q - q0] = r;
        __syncthreads();
    }
}

__global__ void k_scale(int64_t n, const double* __restrict__ w, const double* __restrict__ nrm2,
                        double* __restrict__ v) {
    const double inv = 1.0 / sqrt(*nrm2);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        v[e] = w[e] * inv;
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

int krylov_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(KBLOCKS, ceil_div(n, 256))); }

static unsigned stream_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n, 256)));
}

void launch_multidot(int64_t n, int nq, const double* V, int64_t ldv, const double* w, double* partial,
                     int nblocks, hipStream_t s) {
    MB_CHECK(nq >= 1 && nq <= KMAXQ - 1, MBAMG_E_INVALID, "too many Krylov vectors");
    k_multidot<<<nblocks, 256, 0, s>>>(n, nq, V, ldv, w, partial);
    MB_LAUNCH_CHECK();
}

void launch_update(int64_t n, int nq, const double* V, int64_t ldv, const double* h, double* w, bool norm,
                   double* partial, int nblocks, hipStream_t s) {
    MB_CHECK(nq >= 0 && nq <= KMAXQ - 1, MBAMG_E_INVALID, "too many Krylov vectors");
    k_update<<<nblocks, 256, 0, s>>>(n, nq, V, ldv, h, w, norm ? 1 : 0, partial);
    MB_LAUNCH_CHECK();
}

void launch_reduce(const double* partial, int nblocks, int q0, int cnt, double* out, hipStream_t s) {
    k_reduce<<<1, 256, 0, s>>>(partial, nblocks, q0, cnt, out);
    MB_LAUNCH_CHECK();
}

void launch_scale(int64_t n, const double* w, const double* nrm2, double* v, hipStream_t s) {
    k_scale<<<stream_grid(n), 256, 0, s>>>(n, w, nrm2, v);
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
