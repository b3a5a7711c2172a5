// Learned form: per-aggregate features and the 12 -> 64 -> 64 -> 2 network
// that predicts a prolongator-smoothing weight omega_P in (0, 5/6) and a
// smoother damping omega_S in (0.3, 1.3) per aggregate.  The three dense
// layers, their input-gradient products and their weight-gradient products
// run on the matrix cores (v_mfma_f32_16x16x16_bf16: bfloat16 operands, FP32
// accumulation); biases, activations and the output map stay in FP32.
//
// Parameter packing (5122 FP32): W1[64][12], b1[64], W2[64][64], b2[64],
// W3[2][64], b3[2].
#include "learned_kernels.h"

#include <algorithm>
#include <cmath>

namespace mbamg {

typedef short v4s __attribute__((ext_vector_type(4)));
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
        for (int s = 0; s < 4; ++s)
            acc = mfma(frag_rows(S.H1[w], 64, 0, 16 * s, lane), frag_rows(S.W2, 64, 16 * t, 16 * s, lane), acc);
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
    for (int s = 0; s < 4; ++s)
        o = mfma(frag_rows(S.H2[w], 64, 0, 16 * s, lane), frag_rows(S.W3, 64, 0, 16 * s, lane), o);
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
            for (int s = 0; s < 4; ++s)
                acc = mfma(frag_rows(S.D2[w], 64, 0, 16 * s, lane), frag_cols(S.W2, 64, 16 * t, 16 * s, lane), acc);
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

// One 64-lane wavefront per aggregate, one lane per member (strided), sums
// and extrema combined across the wave.
__global__ __launch_bounds__(WAVE) void k_features(int nagg, int n, const int32_t* __restrict__ agg,
                                                   const int32_t* __restrict__ mptr, const int32_t* __restrict__ midx,
                                                   BsrView A00, BsrView A01, BsrView A10, BsrView A11, int nv0,
                                                   int nv1, const double* __restrict__ ld,
                                                   const double* __restrict__ ld_sum, float level_feature,
                                                   const float* __restrict__ mean, const float* __restrict__ stdv,
                                                   float* __restrict__ out) {
    const int k = blockIdx.x, lane = threadIdx.x;
    const int b = mptr[k], e = mptr[k + 1];
    const double m = (double)(e - b);
    const double mu = *ld_sum / n;
    double sld = 0, mx = -1e300, mn = 1e300;
    for (int q = b + lane; q < e; q += WAVE) {
        double v = ld[midx[q]];
        sld += v;
        mx = fmax(mx, v);
        mn = fmin(mn, v);
    }
    sld = wave_sum(sld);
    mx = wave_max(mx);
    mn = wave_min(mn);
    const double mld = sld / m;
    double var = 0;
    double cmax = -1.0, cmin = 1e300;
    double tot = 0, outw = 0, f9 = 0, f10 = 0, f11 = 0;
    double a00 = 0, a01 = 0, a10 = 0, a11 = 0;
    const int d0 = A00.d;
    const int d1 = A11.d;
    for (int q = b + lane; q < e; q += WAVE) {
        const int i = midx[q];
        var += (ld[i] - mld) * (ld[i] - mld);
        // every block of the member's A00 and A11 rows is read once, into registers;
        // the sums run in the order of vdiag, cvv and row_fro2
        double dv0 = 0.0, dv1 = 0.0, fro00 = 0.0, fro11 = 0.0;
        double off0 = 0, off1 = 0, g2 = 0, cpp = 0;
        for (int p = A00.rp[i]; p < A00.rp[i + 1]; ++p) {
            const int jn = A00.ci[p];
            double blk[16];
            load_block_n(A00.val + (int64_t)p * d0 * d0, d0 * d0, blk);
#pragma unroll
            for (int x = 0; x < 16; ++x)
                if (x < d0 * d0) fro00 += blk[x] * blk[x];
            if (d0 > nv0)
                for (int a = 0; a < nv0; ++a)
                    for (int c = nv0; c < d0; ++c) g2 += blk[a * d0 + c] * blk[a * d0 + c];
            if (jn == i) {
                if (d0 > nv0) cpp = fabs(blk[nv0 * d0 + nv0]);
                double sd = 0.0;
                for (int a = 0; a < nv0; ++a) sd += blk[a * d0 + a];
                dv0 = sd / nv0;
                continue;
            }
            double sc = 0.0;
            for (int a = 0; a < nv0; ++a) sc += fabs(blk[a * d0 + a]);
            const double c = sc / nv0;
            off0 += c;
            if (agg[jn] != k) outw += c;
            else {
                cmax = fmax(cmax, c);
                cmin = fmin(cmin, c);
            }
        }
        for (int p = A11.rp[i]; p < A11.rp[i + 1]; ++p) {
            double blk[16];
            load_block_n(A11.val + (int64_t)p * d1 * d1, d1 * d1, blk);
#pragma unroll
            for (int x = 0; x < 16; ++x)
                if (x < d1 * d1) fro11 += blk[x] * blk[x];
            double sd = 0.0;
            if (A11.ci[p] == i) {
                for (int a = 0; a < nv1; ++a) sd += blk[a * d1 + a];
                dv1 = sd / nv1;
            } else {
                for (int a = 0; a < nv1; ++a) sd += fabs(blk[a * d1 + a]);
                off1 += sd / nv1;
            }
        }
        tot += off0;
        f9 += off0 / dv0;
        f10 += off1 / dv1;
        if (d0 > nv0) f11 += g2 / fmax(dv0 * cpp, 1e-300);
        a00 += fro00;
        a11 += fro11;
        if (A01.rp) a01 += row_fro2(A01, i);
        if (A10.rp) a10 += row_fro2(A10, i);
    }
    var = wave_sum(var);
    cmax = wave_max(cmax);
    cmin = wave_min(cmin);
    tot = wave_sum(tot);
    outw = wave_sum(outw);
    f9 = wave_sum(f9);
    f10 = wave_sum(f10);
    f11 = wave_sum(f11);
    a00 = wave_sum(a00);
    a01 = wave_sum(a01);
    a10 = wave_sum(a10);
    a11 = wave_sum(a11);
    if (lane >= 12) return;
    double F;
    switch (lane) {
        case 0: F = mld - mu; break;
        case 1: F = sqrt(fmax(var / m, 0.0)); break;
        case 2: F = mx - mn; break;
        case 3: F = (cmax >= 0.0 && cmin > 0.0) ? log(cmax) - log(cmin) : 0.0; break;
        case 4: F = m / ((double)n / nagg); break;
        case 5: F = tot > 0 ? outw / tot : 0.0; break;
        case 6: F = sqrt(a01) / sqrt(a00); break;
        case 7: F = sqrt(a10) / sqrt(a11); break;
        case 8: F = f9 / m; break;
        case 9: F = f10 / m; break;
        case 10: F = f11 / m; break;
        default: F = level_feature; break;
    }
    float v = (float)F;
    if (mean) v = (v - mean[lane]) / stdv[lane];
    out[(int64_t)k * 12 + lane] = v;
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
    if (nagg > 0)
        k_features<<<nagg, WAVE, 0, s>>>(nagg, n, agg, mptr, midx, A[0][0], A[0][1], A[1][0], A[1][1], nv0, nv1, ld.p,
                                         tot.p, (float)level / 4.0f, mean, stdv, out);
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
