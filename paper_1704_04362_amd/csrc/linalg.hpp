// Small per-slice linear algebra (linalg.hip).
#pragma once

#include "common.hpp"

namespace tp {

constexpr int kMaxS = 64;  // largest sketch / eigenproblem size

int randn_spectrum(void* re, void* im, int dtype, int64_t K, int64_t rows, int64_t cols, bool real_last,
                   uint64_t seed, uint64_t stream_id, hipStream_t st);
// G_k = X_k^H X_k, X_k rows x s (row stride ldx, slice stride sx), float64 out.
// Tall slices are split over row chunks whose partial Gram matrices go to
// (pre, pim), gram_part_doubles(K, rows, s) doubles each (none needed when 0),
// and are then added in a fixed order.
size_t gram_part_doubles(int64_t K, int64_t rows, int s);
int gram(const void* xre, const void* xim, int dtype, int64_t K, int64_t rows, int s, int64_t ldx, int64_t sx,
         bool real_last, double* gre, double* gim, double* pre, double* pim, hipStream_t st);
// C_k = X_k^H Y_k (a x b, row-major, in the data dtype) for tall X_k (rows x a)
// and Y_k (rows x b), a, b <= 64, row-split with partials (pre, pim) of
// xgram_part_doubles(K, rows, a, b) doubles each, added in a fixed order
size_t xgram_part_doubles(int64_t K, int64_t rows, int a, int b);
int xgram(const void* xre, const void* xim, int a, int64_t ldx, int64_t sx, const void* yre, const void* yim, int b,
          int64_t ldy, int64_t sy, int dtype, int64_t K, int64_t rows, bool real_last, void* ore, void* oim,
          double* pre, double* pim, hipStream_t st);
// eigenvalues descending (K x s) and eigenvectors as columns (K x s x s)
int herm_eig(const double* gre, const double* gim, int64_t K, int s, double* evals, double* vre, double* vim,
             hipStream_t st);
// T_k (s x s) with X_k T_k orthonormal on the kept columns, from G_k = X_k^H X_k
// by Cholesky with pivots <= rtol max diag(G_k) dropped (CholeskyQR)
int chol_inv(const double* gre, const double* gim, int64_t K, int s, double rtol, bool real_last, void* tre,
             void* tim, int out_dtype, hipStream_t st);
// mode 0: T = V diag(lambda^-1/2) (s x s); mode 1: T = V[:, :r] diag(sigma^-power) (s x r)
int eig_transform(const double* vre, const double* vim, const double* evals, int64_t K, int s, int r, int mode,
                  double rtol, double power, void* tre, void* tim, int out_dtype, hipStream_t st);
// out[j] = sum_k w_k sum_{i<r} |X_k[j, i]|^2 g_k[i]; part holds K x n doubles
int leverage(const void* xre, const void* xim, int dtype, int64_t K, int64_t n, int64_t ldx, int64_t sx, int r,
             bool real_last, const double* evals, int s, double rtol, double* part, double* out, hipStream_t st);
int singular_values(const double* evals, int64_t K, int s, int r, double* sv, hipStream_t st);
int gather_rows(const void* xre, const void* xim, int in_dtype, int64_t K, int64_t rows, int64_t cols,
                const int32_t* idx, const double* scale, const int64_t* count, int64_t out_rows, void* wre,
                void* wim, int out_dtype, hipStream_t st);
int convert(const void* a, int adt, void* b, int bdt, int64_t n, hipStream_t st);

// Fused truncated pseudo-inverse of small t-CUR cores (core.hip): per slice
// the range finder (q power iterations) on W (m x n, float64) with the given
// Gaussian Omega (n x s), the Jacobi eigen-decomposition of Bh^H Bh and the
// factors P = Bh U_B,r diag(1/lambda) (n x r) and U = Q U_B,r (m x r), keeping
// sigma_i > rtol sigma_1; float32 copies of P and U when those pointers are
// set. Needs m, n <= 64 and r <= s <= 32 (core_pinv_fits).
bool core_pinv_fits(int64_t m, int64_t n, int s, int64_t r);
int core_pinv(const double* wre, const double* wim, const double* ore, const double* oim, int64_t K, int64_t m,
              int64_t n, int s, int64_t r, bool real_last, int q, double rtol, double* p64re, double* p64im,
              double* u64re, double* u64im, float* p32re, float* p32im, float* u32re, float* u32im, hipStream_t st);

}  // namespace tp
