// Per-slice singular value thresholding and ADMM elementwise steps (svt.hip).
#pragma once

#include "common.hpp"

namespace tp {

int svt_blocks(int64_t n1);
size_t svt_ratio_count(int64_t K, int64_t n1);
int zero_f32(float* p, int64_t n, hipStream_t st);
int svt_identity(float* ure, float* uim, int64_t K, int64_t n, hipStream_t st);
// Block one-sided Jacobi on the rows of X (K x n1 x n2), accumulating the row
// rotations in Uh (K x n1 x n1); conv receives per-slice convergence flags.
int svt_jacobi(float* xre, float* xim, float* ure, float* uim, int64_t K, int64_t n1, int64_t n2, bool real_last,
               int max_sweeps, double tol, float* ratio, int* conv, hipStream_t st);
int svt_shrink(float* xre, float* xim, int64_t K, int64_t n1, int64_t n2, double tau, bool real_last,
               double* sig, int32_t* ranks, hipStream_t st);
int admm_pre(const float* x, const float* e, const float* y, float inv_mu, int64_t n, float* m, hipStream_t st);
int admm_post(const float* x, const uint8_t* mask, const float* l, float mu, float inv_mu, int64_t n, float* e,
              float* y, hipStream_t st);

}  // namespace tp
