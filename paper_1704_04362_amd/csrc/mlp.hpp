// Learned leverage proposal kernels (mlp.hip).
#pragma once

#include "common.hpp"

namespace tp {

constexpr int kMlpParams = 17 * 128 + 128 + 128 * 128 + 128 + 128 + 1;

size_t mlp_features_ws(int64_t n1, int64_t n2);
// feat (n2 x 17); norms, when not null, receives the squared Frobenius norms
// of the lateral slices (float64) from the same pass over A
int mlp_features(const float* a, int64_t n1, int64_t n2, int64_t n3, const float* phi, float* feat, void* ws,
                 hipStream_t st, double* norms = nullptr);
int mlp_forward(const float* P, const float* feat, int64_t nrows, float* out, hipStream_t st);
size_t mlp_train_ws(int64_t ntensors, int64_t nslices);
int mlp_train_step(float* P, float* M, float* V, int64_t step, double lr, const float* feat, const float* target,
                   int64_t T, int64_t nsl, float* loss, float* grad_out, void* ws, hipStream_t st);
// w = (1 - alpha) softmax(logits) + alpha / n
int mlp_proposal(const float* logits, int64_t n, double alpha, double* w, hipStream_t st);

}  // namespace tp
