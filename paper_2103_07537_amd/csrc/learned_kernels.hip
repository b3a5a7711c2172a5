// Learned form: per-aggregate features and the 12 -> 64 -> 64 -> 2 network
// that predicts a prolongator-smoothing weight omega_P in (0, 5/6) and a
// smoother damping omega_S in (0.3, 1.3) per aggregate.  The three dense
// layers, their input-gradient products and their weight-gradient products
// run on the matrix cores with bfloat16 operands and FP32 accumulation: the
// products that contract over the 64 hidden units take gfx950's
// v_mfma_f32_16x16x32_bf16 (two instructions per 64), the ones that contract
// over 16 (the 12 padded inputs, the 2 padded outputs, the 16 rows of a tile
// in the weight gradients) v_mfma_f32_16x16x16_bf16; biases, activations and
// the output map stay in FP32.
//
// Parameter packing (5122 FP32): W1[64][12], b1[64], W2[64][64], b2[64],
// W3[2][64], b3[2].
#include "learned_kernels.h"
#include "dpp.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace mbamg {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int OFF_W1 = 0, OFF_B1 = 768, OFF_W2 = 832, OFF_B2 = 4928, OFF_W3 = 4992, OFF_B3 = 5120;
constexpr float OMEGA_P_MAX = 5.0f / 6.0f;
constexpr float OMEGA_S_MIN = 0.3f, OMEGA_S_SPAN = 1.0f;
constexpr int MLP_WAVES = 4;                  // 256 threads, 16 rows per wave, 64 rows per block step
constexpr int MLP_MAX_BLOCKS = 256;

// float -> bfloat16, round to nearest even
__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

// Operand fragments of the 16x16x16 instruction.  For A (16 x K-chunk) lane l
// supplies row l%16, columns 4*(l/16)..+3 of the chunk; for B (K-chunk x 16)
// lane l supplies column l%16, rows 4*(l/16)..+3.  Result lane l holds rows
// 4*(l/16)..+3 of column l%16.
// Row-major tile T with leading dimension ld: rows r0.., columns k0..
__device__ __forceinline__ v4s frag_rows(const short* T, int ld, int r0, int k0, int lane) {
    const short* p = T + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
    return v4s{p[0], p[1], p[2], p[3]};
}
// the same tile read transposed: element (a, k) of the fragment is T[k0 + k][r0 + a]
__device__ __forceinline__ v4s frag_cols(const short* T, int ld, int r0, int k0, int lane) {
    const int c = r0 + (lane & 15);
    const int k = k0 + 4 * (lane >> 4);
    return v4s{T[(k + 0) * ld + c], T[(k + 1) * ld + c], T[(k + 2) * ld + c], T[(k + 3) * ld + c]};
}

// Operand fragments of the 16x16x32 instruction: as above with 8 K entries
// per lane, 8*(l/16)..+7 of the 32-wide chunk.
__device__ __forceinline__ v8s frag_rows8(const short* T, int ld, int r0, int k0, int lane) {
    const short* p = T + (r0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4);
    return v8s{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
}
__device__ __forceinline__ v8s frag_cols8(const short* T, int ld, int r0, int k0, int lane) {
    const int c = r0 + (lane & 15);
    const short* p = T + (k0 + 8 * (lane >> 4)) * ld + c;
    return v8s{p[0], p[ld], p[2 * ld], p[3 * ld], p[4 * ld], p[5 * ld], p[6 * ld], p[7 * ld]};
}

struct MlpShared {
    short W1[64 * 16];     // [out][in], inputs 12..15 zero
    short W2[64 * 64];     // [out][in]
    short W3[16 * 64];     // [out][in], outputs 2..15 zero
    float b1[64], b2[64], b3[2];
    short X[MLP_WAVES][16 * 16];
    short H1[MLP_WAVES][16 * 64];
    short H2[MLP_WAVES][16 * 64];
    short D2[MLP_WAVES][16 * 64];   // dZ2 (bfloat16)
    short D1[MLP_WAVES][16 * 64];   // dZ1 (bfloat16)
    short DO[MLP_WAVES][16 * 16];   // dO  (bfloat16), columns 2..15 zero
};

__device__ void load_params(MlpShared& S, const float* __restrict__ th) {
    for (int t = threadIdx.x; t < 64 * 16; t += blockDim.x) {
        int o = t / 16, k = t % 16;
        S.W1[t] = k < 12 ? f2bf(th[OFF_W1 + o * 12 + k]) : (short)0;
    }
    for (int t = threadIdx.x; t < 64 * 64; t += blockDim.x) S.W2[t] = f2bf(th[OFF_W2 + t]);
    for (int t = threadIdx.x; t < 16 * 64; t += blockDim.x) {
        int o = t / 64, k = t % 64;
        S.W3[t] = o < 2 ? f2bf(th[OFF_W3 + o * 64 + k]) : (short)0;
    }
    for (int t = threadIdx.x; t < 64; t += blockDim.x) {
        S.b1[t] = th[OFF_B1 + t];
        S.b2[t] = th[OFF_B2 + t];
    }
    if (threadIdx.x < 2) S.b3[threadIdx.x] = th[OFF_B3 + threadIdx.x];
}

// forward pass of one 16-row tile held by one wave; returns the 16x16 logit
// fragment (columns 0, 1 meaningful)
__device__ v4f tile_forward(MlpShared& S, int w, int lane, const float* __restrict__ x, int64_t r0, int64_t n) {
    {   // input tile: 16 rows x 16 (12 features + zero padding), 4 values per lane
        const int i = lane >> 2, k = (lane & 3) * 4;
        const int64_t row = r0 + i;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float v = (row < n && k + t < 12) ? x[row * 12 + k + t] : 0.0f;
            S.X[w][i * 16 + k + t] = f2bf(v);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag_rows(S.X[w], 16, 0, 0, lane), frag_rows(S.W1, 16, 16 * t, 0, lane), acc);
        const int col = 16 * t + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float h = fmaxf(acc[v] + S.b1[col], 0.0f);
            S.H1[w][(4 * (lane >> 4) + v) * 64 + col] = f2bf(h);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            acc = mfma32(frag_rows8(S.H1[w], 64, 0, 32 * s, lane), frag_rows8(S.W2, 64, 16 * t, 32 * s, lane), acc);
        const int col = 16 * t + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float h = fmaxf(acc[v] + S.b2[col], 0.0f);
            S.H2[w][(4 * (lane >> 4) + v) * 64 + col] = f2bf(h);
        }
    }
    __syncthreads();
    v4f o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
        o = mfma32(frag_rows8(S.H2[w], 64, 0, 32 * s, lane), frag_rows8(S.W3, 64, 0, 32 * s, lane), o);
    const int j = lane & 15;
    if (j < 2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] += S.b3[j];
    }
    return o;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ th, const float* __restrict__ x,
                                                     int64_t n, float* __restrict__ out) {
    __shared__ MlpShared S;
    load_params(S, th);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t r0 = base + 16 * w;
        v4f o = tile_forward(S, w, lane, x, r0, n);
        const int j = lane & 15;
        if (j < 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = r0 + 4 * (lane >> 4) + v;
                if (row < n) {
                    float s = sigm(o[v]);
                    out[row * 2 + j] = j == 0 ? OMEGA_P_MAX * s : OMEGA_S_MIN + OMEGA_S_SPAN * s;
                }
            }
        }
        __syncthreads();
    }
}

// Forward and backward of the mean squared error over n rows.  Each wave
// writes its partial gradient (5122 values) and partial loss to
// partial[(block*4 + wave) * 5123 + ...]; k_mlp_grad_reduce sums them in a
// fixed order.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ th, const float* __restrict__ x,
                                                  const float* __restrict__ tgt, int64_t n,
                                                  float* __restrict__ partial) {
    __shared__ MlpShared S;
    load_params(S, th);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, g4 = 4 * (lane >> 4);
    const float inv_n = 1.0f / (float)n;
    v4f gW1[4], gW2[4][4], gW3[4];
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gb3 = 0.0f, loss = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = v4f{0.f, 0.f, 0.f, 0.f};
        gW3[a] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 4; ++t) gW2[a][t] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t r0 = base + 16 * w;
        v4f o = tile_forward(S, w, lane, x, r0, n);
        // output gradient dO[i][c] = (2/n)(out - t) * dout/do
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = g4 + v;
            const int64_t row = r0 + i;
            float g = 0.0f;
            if (j < 2 && row < n) {
                float s = sigm(o[v]);
                float outv = j == 0 ? OMEGA_P_MAX * s : OMEGA_S_MIN + OMEGA_S_SPAN * s;
                float diff = outv - tgt[row * 2 + j];
                loss += diff * diff;
                float scale = j == 0 ? OMEGA_P_MAX : OMEGA_S_SPAN;
                g = 2.0f * inv_n * diff * scale * s * (1.0f - s);
            }
            gb3 += j < 2 ? g : 0.0f;
            S.DO[w][i * 16 + j] = f2bf(g);
        }
        __syncthreads();
        // dW3[c][h] += sum_i dO[i][c] H2[i][h]
#pragma unroll
        for (int t = 0; t < 4; ++t)
            gW3[t] = mfma(frag_cols(S.DO[w], 16, 0, 0, lane), frag_cols(S.H2[w], 64, 16 * t, 0, lane), gW3[t]);
        // dH2 = dO W3 ; dZ2 = dH2 * (H2 > 0)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(frag_rows(S.DO[w], 16, 0, 0, lane), frag_cols(S.W3, 64, 16 * t, 0, lane), acc);
            const int col = 16 * t + j;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = g4 + v;
                float dz = S.H2[w][i * 64 + col] > 0 ? acc[v] : 0.0f;
                gb2[t] += dz;
                S.D2[w][i * 64 + col] = f2bf(dz);
            }
        }
        __syncthreads();
        // dW2[o][h] += sum_i dZ2[i][o] H1[i][h]
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                gW2[a][t] = mfma(frag_cols(S.D2[w], 64, 16 * a, 0, lane), frag_cols(S.H1[w], 64, 16 * t, 0, lane),
                                 gW2[a][t]);
        // dH1 = dZ2 W2 ; dZ1 = dH1 * (H1 > 0)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s)
                acc = mfma32(frag_rows8(S.D2[w], 64, 0, 32 * s, lane), frag_cols8(S.W2, 64, 16 * t, 32 * s, lane),
                             acc);
            const int col = 16 * t + j;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = g4 + v;
                float dz = S.H1[w][i * 64 + col] > 0 ? acc[v] : 0.0f;
                gb1[t] += dz;
                S.D1[w][i * 64 + col] = f2bf(dz);
            }
        }
        __syncthreads();
        // dW1[o][k] += sum_i dZ1[i][o] X[i][k]
#pragma unroll
        for (int a = 0; a < 4; ++a)
            gW1[a] = mfma(frag_cols(S.D1[w], 64, 16 * a, 0, lane), frag_cols(S.X[w], 16, 0, 0, lane), gW1[a]);
        __syncthreads();
    }
    // write this wave's partial: result lane layout is rows g4+v, column j
    float* P = partial + ((int64_t)blockIdx.x * MLP_WAVES + w) * (N_MLP_PARAMS + 1);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 16 * a + g4 + v;
            if (j < 12) P[OFF_W1 + o * 12 + j] = gW1[a][v];
#pragma unroll
            for (int t = 0; t < 4; ++t) P[OFF_W2 + o * 64 + 16 * t + j] = gW2[a][t][v];
        }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = g4 + v;
            if (c < 2) P[OFF_W3 + c * 64 + 16 * t + j] = gW3[t][v];
        }
    // bias sums: lanes j, j+16, j+32, j+48 hold the same column
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float b1v = gb1[t], b2v = gb2[t];
        b1v += __shfl_xor(b1v, 16, 64);
        b1v += __shfl_xor(b1v, 32, 64);
        b2v += __shfl_xor(b2v, 16, 64);
        b2v += __shfl_xor(b2v, 32, 64);
        if (lane < 16) {
            P[OFF_B1 + 16 * t + j] = b1v;
            P[OFF_B2 + 16 * t + j] = b2v;
        }
    }
    gb3 += __shfl_xor(gb3, 16, 64);
    gb3 += __shfl_xor(gb3, 32, 64);
    if (lane < 2) P[OFF_B3 + lane] = gb3;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (lane == 0) P[N_MLP_PARAMS] = loss * inv_n;
}

__global__ void k_mlp_grad_reduce(const float* __restrict__ partial, int nparts, float* __restrict__ grad,
                                  float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > N_MLP_PARAMS) return;
    float s = 0.0f;
    for (int k = 0; k < nparts; ++k) s += partial[(int64_t)k * (N_MLP_PARAMS + 1) + p];
    if (p < N_MLP_PARAMS) grad[p] = s;
    else if (loss) *loss = s;
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    th[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------------------------
// features (FP64 arithmetic, FP32 output)
// ----------------------------------------------------------------------------
__device__ inline int find_block(const int32_t* ci, int lo, int hi, int key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int c = ci[mid];
        if (c == key) return mid;
        if (c < key) lo = mid + 1; else hi = mid;
    }
    return -1;
}

// mean vector-diagonal entry of the diagonal block of row i
// a block of n <= 16 doubles into registers (16-byte loads for 4x4 blocks)
__device__ __forceinline__ void load_block_n(const double* __restrict__ p, int n, double (&v)[16]) {
    if (n == 16) {
#pragma unroll
        for (int x = 0; x < 16; x += 2) {
            const double2 t = *reinterpret_cast<const double2*>(p + x);
            v[x] = t.x;
            v[x + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int x = 0; x < 16; ++x) v[x] = x < n ? p[x] : 0.0;
    }
}

__device__ inline double vdiag(const BsrView& A, int i, int nv) {
    int p = find_block(A.ci, A.rp[i], A.rp[i + 1], i);
    if (p < 0) return 0.0;
    const double* b = A.val + (int64_t)p * A.d * A.d;
    double s = 0.0;
    for (int a = 0; a < nv; ++a) s += b[a * A.d + a];
    return s / nv;
}

__device__ inline double cvv(const BsrView& A, int p, int nv) {
    const double* b = A.val + (int64_t)p * A.d * A.d;
    double s = 0.0;
    for (int a = 0; a < nv; ++a) s += fabs(b[a * A.d + a]);
    return s / nv;
}

__device__ inline double row_fro2(const BsrView& A, int i) {
    double s = 0.0;
    const int bs = A.d * A.d;
    for (int p = A.rp[i]; p < A.rp[i + 1]; ++p)
        for (int e = 0; e < bs; ++e) {
            double v = A.val[(int64_t)p * bs + e];
            s += v * v;
        }
    return s;
}

__global__ void k_logdiag(int n, BsrView A00, int nv, double* ld) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ld[i] = log(vdiag(A00, i, nv));
}

__global__ void k_sum_partial(const double* a, int n, double* part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double* part, int nb, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        *out = s;
    }
}

__device__ inline double wave_sum(double v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}
__device__ inline double wave_min(double v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}

// One workgroup of W wavefronts per aggregate.  Members go to groups of G
// lanes (G = 16: four members per wavefront at once, for short rows; G = 64:
// one, for long coarse rows); within a group, 16 lanes take the entries of
// one block (lane x holds entry x), G / 16 blocks per pass.  The lane holding
// a block's entry 0 also reads that block's diagonal (just fetched, so cached).
template <int G, int W>
__global__ __launch_bounds__(W * WAVE) void k_features(int nagg, int n, const int32_t* __restrict__ agg,
                                                       const int32_t* __restrict__ mptr,
                                                       const int32_t* __restrict__ midx, BsrView A00, BsrView A01,
                                                       BsrView A10, BsrView A11, int nv0, int nv1,
                                                       const double* __restrict__ ld,
                                                       const double* __restrict__ ld_sum, float level_feature,
                                                       const float* __restrict__ mean,
                                                       const float* __restrict__ stdv, float* __restrict__ out) {
    static_assert(G == 16 || G == 64, "a group is one DPP row or the wavefront");
    constexpr int NT = W * WAVE;       // threads per aggregate
    constexpr int NG = NT / G;         // member groups per aggregate
    constexpr int BPP = G / 16;        // blocks per pass
    constexpr int U = 4;               // passes in flight
    __shared__ double red[W][12];
    const int k = blockIdx.x, tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int grp = tid / G, glane = tid % G;
    const int sub = glane / 16, x = glane % 16;
    const int b = mptr[k], e = mptr[k + 1];
    const double m = (double)(e - b);
    const double mu = *ld_sum / n;

    // pass 1: the members' log-diagonal statistics
    double sld = 0, mx = -1e300, mn = 1e300;
    for (int q = b + tid; q < e; q += NT) {
        const double v = ld[midx[q]];
        sld += v;
        mx = fmax(mx, v);
        mn = fmin(mn, v);
    }
    sld = wave_sum(sld);
    mx = wave_max(mx);
    mn = wave_min(mn);
    if (W > 1) {
        if (lane == 0) {
            red[wv][0] = sld;
            red[wv][1] = mx;
            red[wv][2] = mn;
        }
        __syncthreads();
        sld = 0;
        mx = -1e300;
        mn = 1e300;
        for (int w = 0; w < W; ++w) {
            sld += red[w][0];
            mx = fmax(mx, red[w][1]);
            mn = fmin(mn, red[w][2]);
        }
        __syncthreads();
    }
    const double mld = sld / m;

    // pass 2: members by groups, block entries by lanes
    const int d0 = A00.d, d1 = A11.d, dd0 = d0 * d0, dd1 = d1 * d1;
    const int a0 = x / d0, c0 = x % d0;
    const bool g2_entry = x < dd0 && a0 < nv0 && c0 >= nv0;
    double fro00 = 0, fro11 = 0, a01 = 0, a10 = 0, outw = 0, cmax = -1.0, cmin = 1e300;
    double var = 0, tot = 0, f9 = 0, f10 = 0, f11 = 0;   // last lane of each group
    for (int q = b + grp; q < e; q += NG) {
        const int i = midx[q];
        double off0 = 0, dv0 = 0, cpp = 0, g2 = 0, off1 = 0, dv1 = 0;
        // chunks of G blocks: the group first fetches their columns (and the
        // columns' aggregates), one block per lane, so no pass waits on a
        // dependent load; then U passes of BPP blocks at a time, lanes over
        // entries, with the U passes' loads issued before any is used
        for (int base = A00.rp[i], r1 = A00.rp[i + 1]; base < r1; base += G) {
            const int nb = min(G, r1 - base);
            int jn_l = -1, ag_l = -1;
            if (glane < nb) {
                jn_l = A00.ci[base + glane];
                ag_l = agg[jn_l];
            }
            for (int t0 = 0; t0 < nb; t0 += U * BPP) {
                double vv[U];
#pragma unroll
                for (int h = 0; h < U; ++h) {
                    const int t = t0 + h * BPP + sub;
                    vv[h] = t < nb && x < dd0 ? A00.val[(int64_t)(base + t) * dd0 + x] : 0.0;
                }
#pragma unroll
                for (int h = 0; h < U; ++h) {
                    const int t = t0 + h * BPP + sub;
                    const int src = t < nb ? t : 0;
                    const int jn = __shfl(jn_l, src, G), ag = __shfl(ag_l, src, G);
                    if (t >= nb || x >= dd0) continue;
                    const double v = vv[h];
                    fro00 += v * v;
                    if (g2_entry) g2 += v * v;
                    if (x != 0) continue;
                    const double* blk = A00.val + (int64_t)(base + t) * dd0;   // just fetched: cached
                    if (jn == i) {
                        if (d0 > nv0) cpp = fabs(blk[nv0 * d0 + nv0]);
                        double sd = 0.0;
                        for (int a = 0; a < nv0; ++a) sd += blk[a * d0 + a];
                        dv0 = sd / nv0;
                    } else {
                        double sc = 0.0;
                        for (int a = 0; a < nv0; ++a) sc += fabs(blk[a * d0 + a]);
                        const double c = sc / nv0;
                        off0 += c;
                        if (ag != k) outw += c;
                        else {
                            cmax = fmax(cmax, c);
                            cmin = fmin(cmin, c);
                        }
                    }
                }
            }
        }
        for (int base = A11.rp[i], r1 = A11.rp[i + 1]; base < r1; base += G) {
            const int nb = min(G, r1 - base);
            const int jn_l = glane < nb ? A11.ci[base + glane] : -1;
            for (int t0 = 0; t0 < nb; t0 += U * BPP) {
                double vv[U];
#pragma unroll
                for (int h = 0; h < U; ++h) {
                    const int t = t0 + h * BPP + sub;
                    vv[h] = t < nb && x < dd1 ? A11.val[(int64_t)(base + t) * dd1 + x] : 0.0;
                }
#pragma unroll
                for (int h = 0; h < U; ++h) {
                    const int t = t0 + h * BPP + sub;
                    const int jn = __shfl(jn_l, t < nb ? t : 0, G);
                    if (t >= nb || x >= dd1) continue;
                    const double v = vv[h];
                    fro11 += v * v;
                    if (x != 0) continue;
                    const double* blk = A11.val + (int64_t)(base + t) * dd1;
                    double sd = 0.0;
                    if (jn == i) {
                        for (int a = 0; a < nv1; ++a) sd += blk[a * d1 + a];
                        dv1 = sd / nv1;
                    } else {
                        for (int a = 0; a < nv1; ++a) sd += fabs(blk[a * d1 + a]);
                        off1 += sd / nv1;
                    }
                }
            }
        }
        if (A01.rp && x < A01.d * A01.d)
#pragma unroll 4
            for (int p = A01.rp[i] + sub; p < A01.rp[i + 1]; p += BPP) {
                const double v = A01.val[(int64_t)p * A01.d * A01.d + x];
                a01 += v * v;
            }
        if (A10.rp && x < A10.d * A10.d)
#pragma unroll 4
            for (int p = A10.rp[i] + sub; p < A10.rp[i + 1]; p += BPP) {
                const double v = A10.val[(int64_t)p * A10.d * A10.d + x];
                a10 += v * v;
            }
        off0 = group_sum<G>(off0);
        dv0 = group_sum<G>(dv0);
        cpp = group_sum<G>(cpp);
        g2 = group_sum<G>(g2);
        off1 = group_sum<G>(off1);
        dv1 = group_sum<G>(dv1);
        if (glane == G - 1) {
            const double li = ld[i];
            var += (li - mld) * (li - mld);
            tot += off0;
            f9 += off0 / dv0;
            f10 += off1 / dv1;
            if (d0 > nv0) f11 += g2 / fmax(dv0 * cpp, 1e-300);
        }
    }
    double S[12] = {var, tot, outw, f9, f10, f11, fro00, a01, a10, fro11, cmax, cmin};
#pragma unroll
    for (int t = 0; t < 10; ++t) S[t] = wave_sum(S[t]);
    S[10] = wave_max(S[10]);
    S[11] = wave_min(S[11]);
    if (W > 1) {
        if (lane < 12) {
            double v = S[0];
#pragma unroll
            for (int t = 1; t < 12; ++t)
                if (lane == t) v = S[t];
            red[wv][lane] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 12; ++t) {
            double v = red[0][t];
            for (int w = 1; w < W; ++w) v = t == 10 ? fmax(v, red[w][t]) : t == 11 ? fmin(v, red[w][t]) : v + red[w][t];
            S[t] = v;
        }
    }
    if (tid >= 12) return;
    var = S[0]; tot = S[1]; outw = S[2]; f9 = S[3]; f10 = S[4]; f11 = S[5];
    fro00 = S[6]; a01 = S[7]; a10 = S[8]; fro11 = S[9]; cmax = S[10]; cmin = S[11];
    double F;
    switch (tid) {
        case 0: F = mld - mu; break;
        case 1: F = sqrt(fmax(var / m, 0.0)); break;
        case 2: F = mx - mn; break;
        case 3: F = (cmax >= 0.0 && cmin > 0.0) ? log(cmax) - log(cmin) : 0.0; break;
        case 4: F = m / ((double)n / nagg); break;
        case 5: F = tot > 0 ? outw / tot : 0.0; break;
        case 6: F = sqrt(a01) / sqrt(fro00); break;
        case 7: F = sqrt(a10) / sqrt(fro11); break;
        case 8: F = f9 / m; break;
        case 9: F = f10 / m; break;
        case 10: F = f11 / m; break;
        default: F = level_feature; break;
    }
    float v = (float)F;
    if (mean) v = (v - mean[tid]) / stdv[tid];
    out[(int64_t)k * 12 + tid] = v;
}

// per-aggregate weights -> per-row smoother damping in colour order
template <class T>
__global__ void k_row_damping(int n, const int32_t* perm, const int32_t* agg, const double* ws, T* w_row) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) w_row[p] = (T)ws[agg[perm[p]]];
}

__global__ void k_split_weights(int nagg, const float* out2, double* wp, double* ws) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nagg) return;
    wp[k] = (double)out2[2 * k];
    ws[k] = (double)out2[2 * k + 1];
}

// ----------------------------------------------------------------------------
// host wrappers
// ----------------------------------------------------------------------------
static unsigned gridn(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, ceil_div(n, t)); }

void mlp_forward(const float* th, const float* x, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>(MLP_MAX_BLOCKS * 16, ceil_div(n, 64));
    k_mlp_forward<<<blocks, 256, 0, s>>>(th, x, n, out);
    MB_LAUNCH_CHECK();
}

void mlp_loss_grad(const float* th, const float* x, const float* t, int64_t n, float* grad, float* loss,
                   DevBuf<float>& partial, hipStream_t s) {
    MB_CHECK(n > 0, MBAMG_E_INVALID, "empty batch");
    int blocks = (int)std::min<int64_t>(MLP_MAX_BLOCKS, ceil_div(n, 64));
    const int64_t need = (int64_t)blocks * MLP_WAVES * (N_MLP_PARAMS + 1);
    if ((int64_t)partial.n < need) partial.alloc(need);
    k_mlp_grad<<<blocks, 256, 0, s>>>(th, x, t, n, partial.p);
    MB_LAUNCH_CHECK();
    k_mlp_grad_reduce<<<gridn(N_MLP_PARAMS + 1), 256, 0, s>>>(partial.p, blocks * MLP_WAVES, grad, loss);
    MB_LAUNCH_CHECK();
}

// Scratch of the allocation-free gradient: the per-wavefront partial sums of
// k_mlp_grad for the largest grid mlp_loss_grad launches (MLP_MAX_BLOCKS
// workgroups of MLP_WAVES wavefronts, N_MLP_PARAMS + 1 floats each:
// 5,245,952 floats = 20.0 MiB).  Each GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per
// device, and only that address is ever passed to a kernel.
constexpr int64_t NOALLOC_SCRATCH_FLOATS = (int64_t)MLP_MAX_BLOCKS * MLP_WAVES * (N_MLP_PARAMS + 1);
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];

constexpr int NOALLOC_MAX_DEVICES = 64;

// Device address of this device's scratch array (looked up on the first call
// on each device, with that device current).
static float* scratch_address() {
    static std::mutex mu;
    static float* addr[NOALLOC_MAX_DEVICES] = {};
    int dev = 0;
    MB_HIP(hipGetDevice(&dev));
    MB_CHECK(dev >= 0 && dev < NOALLOC_MAX_DEVICES, MBAMG_E_INVALID, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        MB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MB_CHECK(p != nullptr, MBAMG_E_HIP, "scratch symbol has no device address");
        addr[dev] = static_cast<float*>(p);
    }
    return addr[dev];
}

void mlp_loss_grad_noalloc(const float* th, const float* x, const float* t, int64_t n, float* grad, float* loss,
                           hipStream_t s) {
    MB_CHECK(n > 0, MBAMG_E_INVALID, "empty batch");
    // the same grid as mlp_loss_grad, so the partial sums and their reduction order are the same
    const int blocks = (int)std::min<int64_t>(MLP_MAX_BLOCKS, ceil_div(n, 64));
    const int64_t need = (int64_t)blocks * MLP_WAVES * (N_MLP_PARAMS + 1);
    MB_CHECK(need <= NOALLOC_SCRATCH_FLOATS, MBAMG_E_INVALID,
             "gradient scratch: the grid needs more than the 20 MiB static buffer holds");
    float* partial = scratch_address();
    // every wavefront of the grid writes all N_MLP_PARAMS + 1 of its entries and the
    // reduction reads only those: nothing needs clearing, stale entries are never read
    k_mlp_grad<<<blocks, 256, 0, s>>>(th, x, t, n, partial);
    MB_LAUNCH_CHECK();
    k_mlp_grad_reduce<<<gridn(N_MLP_PARAMS + 1), 256, 0, s>>>(partial, blocks * MLP_WAVES, grad, loss);
    MB_LAUNCH_CHECK();
}

void mlp_adam(float* th, const float* g, float* m, float* v, int64_t step, float lr, float b1, float b2, float eps,
              hipStream_t s) {
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    k_adam<<<gridn(N_MLP_PARAMS), 256, 0, s>>>(th, g, m, v, N_MLP_PARAMS, lr, b1, b2, eps, c1, c2);
    MB_LAUNCH_CHECK();
}

void aggregate_features(int nagg, int n, const int32_t* agg, const int32_t* mptr, const int32_t* midx,
                        const BsrView (&A)[2][2], int nv0, int nv1, int level, const float* mean, const float* stdv,
                        float* out, hipStream_t s) {
    DevBuf<double> ld(std::max(n, 1)), part(256), tot(1);
    k_logdiag<<<gridn(n), 256, 0, s>>>(n, A[0][0], nv0, ld.p);
    k_sum_partial<<<256, 256, 0, s>>>(ld.p, n, part.p);
    k_sum_final<<<1, 64, 0, s>>>(part.p, 256, tot.p);
    MB_CHECK(A[0][0].d <= 4 && A[1][1].d <= 4 && A[0][1].d <= 4 && A[1][0].d <= 4, MBAMG_E_INVALID,
             "features: blocks of at most 4 x 4");
    if (nagg > 0) {
        // long coarse rows: one wavefront per member, and more of them per aggregate when
        // the aggregates are few; short rows: four members per wavefront
        const bool long_rows = n > 0 && A[0][0].nnzb >= (int64_t)16 * n;
        const float lf = (float)level / 4.0f;
        if (!long_rows)
            k_features<16, 1><<<nagg, WAVE, 0, s>>>(nagg, n, agg, mptr, midx, A[0][0], A[0][1], A[1][0], A[1][1],
                                                     nv0, nv1, ld.p, tot.p, lf, mean, stdv, out);
        else if (nagg >= 1024)
            k_features<64, 4><<<nagg, 4 * WAVE, 0, s>>>(nagg, n, agg, mptr, midx, A[0][0], A[0][1], A[1][0],
                                                         A[1][1], nv0, nv1, ld.p, tot.p, lf, mean, stdv, out);
        else
            k_features<64, 8><<<nagg, 8 * WAVE, 0, s>>>(nagg, n, agg, mptr, midx, A[0][0], A[0][1], A[1][0],
                                                           A[1][1], nv0, nv1, ld.p, tot.p, lf, mean, stdv, out);
    }
    MB_LAUNCH_CHECK();
    MB_HIP(hipStreamSynchronize(s));
}

__global__ void k_normalize_features(int64_t n, const float* raw, const float* mean, const float* stdv, float* out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = (int)(t % N_FEATURES);
    out[t] = (raw[t] - mean[c]) / stdv[c];
}

void normalize_features(int nagg, const float* raw, const float* mean, const float* stdv, float* out, hipStream_t s) {
    const int64_t n = (int64_t)nagg * N_FEATURES;
    if (n == 0) return;
    k_normalize_features<<<gridn(n), 256, 0, s>>>(n, raw, mean, stdv, out);
    MB_LAUNCH_CHECK();
}

void split_weights(int nagg, const float* out2, double* wp, double* ws, hipStream_t s) {
    k_split_weights<<<gridn(nagg), 256, 0, s>>>(nagg, out2, wp, ws);
    MB_LAUNCH_CHECK();
}

template <class T>
void row_damping(int n, const int32_t* perm, const int32_t* agg, const double* ws, T* w_row, hipStream_t s) {
    k_row_damping<T><<<gridn(n), 256, 0, s>>>(n, perm, agg, ws, w_row);
    MB_LAUNCH_CHECK();
}
template void row_damping<double>(int, const int32_t*, const int32_t*, const double*, double*, hipStream_t);
template void row_damping<float>(int, const int32_t*, const int32_t*, const double*, float*, hipStream_t);

}  // namespace mbamg
