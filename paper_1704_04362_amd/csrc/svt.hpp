// Per-slice singular value thresholding and ADMM elementwise steps (svt.hip).
#pragma once

#include <cmath>

#include "common.hpp"

namespace tp {

int svt_blocks(int64_t n1);
size_t svt_ratio_count(int64_t K, int64_t n1);
int zero_f32(float* p, int64_t n, hipStream_t st);
int svt_identity(float* ure, float* uim, int64_t K, int64_t n, hipStream_t st);
// Block one-sided Jacobi on the rows of X (K x n1 x n2), accumulating the row
// rotations in Uh (K x n1 x n1); conv receives per-slice convergence flags.
// Writes (when out is not null) the number of the K slices whose last
// svt_jacobi sweeps ended without meeting its convergence test.
int svt_count_unconverged(const int* conv, int64_t K, int32_t* out, hipStream_t st);
int svt_jacobi(float* xre, float* xim, float* ure, float* uim, int64_t K, int64_t n1, int64_t n2, bool real_last,
               int max_sweeps, double tol, float* ratio, int* conv, hipStream_t st);
int svt_shrink(float* xre, float* xim, int64_t K, int64_t n1, int64_t n2, double tau, bool real_last,
               double* sig, int32_t* ranks, hipStream_t st);
// Largest m for tsvd_pick (its eigenvalues and picks live in LDS).
constexpr int64_t kPickMax = 4096;
// After svt_jacobi (X = Q Y, K x m x ldx, rows orthogonal): the r rows of
// the source S (K x m x len: Q, or X itself) with the largest row norms mu
// of X, conjugated, as columns of out (K x len x r planes), scaled by 1
// (mode 0), 1 / sqrt(mu) (mode 1) or 1 / mu (mode 2); sv (K x r float64,
// may be null) receives sqrt(mu) (sqrt_sv) or mu, descending. A mu at or
// below floor_rel times the slice's largest counts as zero: value 0, zero
// column.
int tsvd_pick(const float* xre, const float* xim, int64_t ldx, const float* sre, const float* sim, int64_t len,
              int64_t K, int64_t m, int64_t r, bool real_last, int mode, bool sqrt_sv, double floor_rel, float* ore,
              float* oim, double* sv, hipStream_t st);
int admm_pre(const float* x, const float* e, const float* y, float inv_mu, int64_t n, float* m, hipStream_t st);
int admm_post(const float* x, const uint8_t* mask, const float* l, float mu, float inv_mu, int64_t n, float* e,
              float* y, hipStream_t st);
// out_k = conj(in_k)^T for every Fourier slice of a float32 planar spectrum
// (K x rows x cols in, K x cols x rows out).
int spec_conj_transpose(const float* re, const float* im, int64_t K, int64_t rows, int64_t cols, float* ore,
                        float* oim, hipStream_t st);
// Algorithm 7's stop quantities max |L - Lprev|, max |E - Eprev|,
// max |L + E - X| into out[0..2] (device), through admm_stop_floats(n) - 4
// floats of per-workgroup partials in part.
size_t admm_stop_floats(int64_t n);
int admm_stop(const float* x, const float* l, const float* lprev, const float* e, const float* eprev, int64_t n,
              float* part, float* out, hipStream_t st);
int admm_post_soft(const float* x, const float* l, float mu, float inv_mu, float thr, int64_t n, float* e, float* y,
                   hipStream_t st);
// t-transpose of an n1 x n2 x n3 tube-major tensor into out (n2 x n1 x n3);
// elements of 1 or 4 bytes.
int ttranspose(const void* in, int elem_bytes, int64_t n1, int64_t n2, int64_t n3, void* out, hipStream_t st);
// out[a][b][:] = in[ridx[a]][cidx[b]][:] (either index list may be null:
// identity; entries past *count of the listed index are zero); elements of
// 1 or 4 bytes.
int gather_slices(const void* in, int elem_bytes, int64_t in_cols, int64_t n3, const int32_t* ridx,
                  const int32_t* cidx, const int64_t* count, int64_t rows, int64_t cols, void* out,
                  hipStream_t st);
// The ADMM of Algorithm 7 on an n1 x n2 x n3 float32 tensor: completion
// (E zero on mask != 0) when mask is non-null, robust PCA with weight lam
// otherwise. Workspace: admm_workspace bytes.
size_t admm_workspace(int64_t n1, int64_t n2, int64_t n3);
// tol > 0 ends the loop at Algorithm 7's stop test (read back after every
// iteration) and gives TP_ENOCONV at the cap; tol <= 0 runs exactly `iters`
// iterations without synchronising. *iters_done (host, may be null): the
// iterations run.
int admm_run(const float* x, const uint8_t* mask, double lam, int64_t n1, int64_t n2, int64_t n3, int iters,
             double rho, double mu0, double mu_max, double tol, float* l, float* e, float* y, int32_t* ranks,
             int32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t st);
// The l1 weight of eq. tlow7 when the caller passes 0: 1/sqrt(max(n1, n2) n3)
// (the paper gives none; this is the value of the tensor robust PCA work the
// problem comes from).
inline double rpca_default_lambda(int64_t n1, int64_t n2, int64_t n3) {
  return 1.0 / std::sqrt(double(n1 > n2 ? n1 : n2) * double(n3));
}

}  // namespace tp
