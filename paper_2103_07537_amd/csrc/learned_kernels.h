// Learned-form kernels (device work in learned_kernels.hip).
#pragma once

#include "common.h"

namespace mbamg {

constexpr int N_MLP_PARAMS = 5122;
constexpr int N_FEATURES = 12;

// Read-only view of a natural-order BSR block with d x d blocks.
struct BsrView {
    const int32_t* rp;
    const int32_t* ci;
    const double* val;
    int d;
    int64_t nnzb;   // blocks (host-side launch choices)
};

// out[n][2] = (omega_P, omega_S) for normalised features x[n][12]
void mlp_forward(const float* th, const float* x, int64_t n, float* out, hipStream_t s);
// grad[5122] and loss[1] of the mean squared error against t[n][2]
void mlp_loss_grad(const float* th, const float* x, const float* t, int64_t n, float* grad, float* loss,
                   DevBuf<float>& partial, hipStream_t s);
// the same, with the partial sums in a static per-device buffer (no allocation)
void mlp_loss_grad_noalloc(const float* th, const float* x, const float* t, int64_t n, float* grad, float* loss,
                           hipStream_t s);
void mlp_adam(float* th, const float* g, float* m, float* v, int64_t step, float lr, float b1, float b2, float eps,
              hipStream_t s);
// 12 features per aggregate; normalised with (mean, stdv) when mean != NULL (synchronous)
void aggregate_features(int nagg, int n, const int32_t* agg, const int32_t* mptr, const int32_t* midx,
                        const BsrView (&A)[2][2], int nv0, int nv1, int level, const float* mean, const float* stdv,
                        float* out, hipStream_t s);
// out = (raw - mean) / stdv per feature column, in FP32 (the normalisation aggregate_features applies)
void normalize_features(int nagg, const float* raw, const float* mean, const float* stdv, float* out, hipStream_t s);
void split_weights(int nagg, const float* out2, double* wp, double* ws, hipStream_t s);
template <class T>
void row_damping(int n, const int32_t* perm, const int32_t* agg, const double* ws, T* w_row, hipStream_t s);

}  // namespace mbamg
