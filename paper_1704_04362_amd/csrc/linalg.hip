// Small per-Fourier-slice linear algebra for the randomized t-SVD
// (Theorem "t-SVD" and eq. circ1: the t-SVD is one matrix SVD per Fourier
// slice), t-project / t-CX (Algorithms 3-4) and the t-CUR core
// pseudo-inverse (Algorithm 5):
//  * Gaussian test matrices drawn per slice (Philox4x64-10 + Box-Muller);
//  * Gram matrices X^H X of tall slices, accumulated in float64;
//  * a Hermitian eigensolver for s x s Gram matrices (s <= 64): the LDS
//    Jacobi solver of jacobi.hpp in float64, one workgroup per slice;
//  * the derived small transforms (orthonormalisation V diag(lambda^-1/2),
//    truncation to the leading r directions with singular-value scaling);
//  * leverage reductions summed over the half spectrum with conjugate
//    weights (1 for the real slices, 2 for the others).
#include <cmath>

#include "common.hpp"
#include "jacobi.hpp"
#include "linalg.hpp"

namespace tp {
namespace {

__device__ __forceinline__ uint64_t philox4x64_w01(uint64_t seed, uint64_t stream, uint64_t index, uint64_t* w1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = index, x1 = 0, x2 = 0, x3 = 0;
  uint64_t k0 = seed, k1 = stream;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  *w1 = x1;
  return x0;
}

// Standard complex normal entries (real normal on the real slices).
template <typename T>
__global__ void randn_kernel(T* re, T* im, int64_t K, int64_t per_slice, int real_last, uint64_t seed,
                             uint64_t stream) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * per_slice) return;
  const int64_t k = e / per_slice;
  const bool real = k == 0 || (real_last && k == K - 1);
  uint64_t w1;
  const uint64_t w0 = philox4x64_w01(seed, stream, (uint64_t)e, &w1);
  const double u1 = ((double)(w0 >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)(w1 >> 11) * 0x1.0p-53;         // [0, 1)
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  if (real) {
    re[e] = (T)(rad * cs);
    im[e] = T(0);
  } else {
    re[e] = (T)(rad * cs * 0.7071067811865476);
    im[e] = (T)(rad * sn * 0.7071067811865476);
  }
}

// Partial cross products: workgroup (k, y) adds conj(x_i) y_j over the rows
// [y rch, (y + 1) rch) of slice k, X_k rows x a and Y_k rows x b (planar,
// a, b <= 64), and writes its a x b block to part[(k nch + y) a b] (float64).
// The Gram matrix X^H X is the case Y = X. On the float64 matrix cores
// (v_mfma_f64_16x16x4f64; A lane l = A[l % 16][l / 16], B lane l =
// B[l / 16][l % 16], D lane l register v = D[4 v + l / 16][l % 16]): the
// a x b output is cut into 16 x 16 tiles, tile t owned by wavefront t % 4
// (at most MAXT tiles each); rows are staged through LDS as float64, CH at
// a time, with row strides of 16 mod 32 doubles (16 consecutive columns of
// 4 rows per read). re = Xr^T Yr + Xi^T Yi, im = Xr^T Yi - Xi^T Yr.
typedef double xg_d4 __attribute__((ext_vector_type(4)));

template <typename T, int WA, int WB, int MAXT, bool SAME>
__global__ __launch_bounds__(256) void xgram_mfma_kernel(const T* __restrict__ xre, const T* __restrict__ xim, int a,
                                                         int64_t ldx, int64_t sx, const T* __restrict__ yre,
                                                         const T* __restrict__ yim, int b, int64_t ldy, int64_t sy,
                                                         int64_t K, int64_t rows, int real_last, int64_t rch,
                                                         double* __restrict__ pre, double* __restrict__ pim) {
  static_assert(!SAME || WA == WB, "a Gram matrix is square");
  constexpr int CH = 16, SA = WA + 16, SB = SAME ? 1 : WB + 16;
  __shared__ double xr_[CH][SA], xi_[CH][SA], yr_[CH][SB], yi_[CH][SB];
  const int64_t k = blockIdx.x;
  const int64_t nch = gridDim.y;
  const bool real = k == 0 || (real_last && k == K - 1);
  const T* xr = xre + k * sx;
  const T* xi = xim + k * sx;
  const T* yr = yre + k * sy;
  const T* yi = yim + k * sy;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int tb = (b + 15) >> 4, ntile = ((a + 15) >> 4) * tb;
  const int64_t rbeg = (int64_t)blockIdx.y * rch;
  const int64_t rend = (rbeg + rch) < rows ? (rbeg + rch) : rows;
  xg_d4 cr[MAXT], ci[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) cr[q] = ci[q] = xg_d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = rbeg; r0 < rend; r0 += CH) {
    for (int e = tid; e < CH * WA; e += 256) {
      const int rr = e / WA, c = e - rr * WA;
      const int64_t row = r0 + rr;
      const bool live = row < rend && c < a;
      xr_[rr][c] = live ? (double)xr[row * ldx + c] : 0.0;
      xi_[rr][c] = (live && !real) ? (double)xi[row * ldx + c] : 0.0;
    }
    if constexpr (!SAME) {
      for (int e = tid; e < CH * WB; e += 256) {
        const int rr = e / WB, c = e - rr * WB;
        const int64_t row = r0 + rr;
        const bool live = row < rend && c < b;
        yr_[rr][c] = live ? (double)yr[row * ldy + c] : 0.0;
        yi_[rr][c] = (live && !real) ? (double)yi[row * ldy + c] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < CH / 4; ++kk) {
      const int rr = 4 * kk + (l >> 4);
#pragma unroll
      for (int q = 0; q < MAXT; ++q) {
        const int t = w + 4 * q;
        if (t >= ntile) break;
        const int ti = t / tb, tj = t - ti * tb;
        const int ci_ = 16 * ti + (l & 15), cj = 16 * tj + (l & 15);
        const double ar = xr_[rr][ci_], ai = xi_[rr][ci_];
        const double br = SAME ? xr_[rr][cj] : yr_[rr][cj], bi = SAME ? xi_[rr][cj] : yi_[rr][cj];
        cr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cr[q], 0, 0, 0);
        cr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, cr[q], 0, 0, 0);
        ci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, ci[q], 0, 0, 0);
        ci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, ci[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int64_t base = (k * nch + blockIdx.y) * (int64_t)a * b;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = w + 4 * q;
    if (t >= ntile) break;
    const int ti = t / tb, tj = t - ti * tb;
    const int j = 16 * tj + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + 4 * v + (l >> 4);
      if (i < a && j < b) {
        pre[base + i * b + j] = cr[q][v];
        pim[base + i * b + j] = real ? 0.0 : ci[q][v];
      }
    }
  }
}

// out[k][e] = sum over chunks y (in order) of part[k][y][e], as type TO.
template <typename TO>
__global__ void xgram_reduce_kernel(const double* __restrict__ pre, const double* __restrict__ pim, int64_t K,
                                    int64_t nch, int ne, TO* __restrict__ ore, TO* __restrict__ oim) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * ne) return;
  const int64_t k = t / ne, e = t - k * ne;
  double sr = 0.0, si = 0.0;
#pragma unroll 8
  for (int64_t y = 0; y < nch; ++y) {
    sr += pre[(k * nch + y) * ne + e];
    si += pim[(k * nch + y) * ne + e];
  }
  ore[t] = (TO)sr;
  oim[t] = (TO)si;
}

// Eigen-decomposition of one s x s Hermitian matrix per workgroup with the
// LDS Jacobi solver; eigenvalues are returned in descending order (ties by
// index) with the matching eigenvector columns.
template <int MAXN, int NT>
__global__ __launch_bounds__(NT) void herm_eig_kernel(const double* __restrict__ gre,
                                                       const double* __restrict__ gim, int s, int max_sweeps,
                                                       double* __restrict__ evals, double* __restrict__ vre,
                                                       double* __restrict__ vim) {
  __shared__ JacobiShared<MAXN, NT> sh;
  __shared__ int order[MAXN];
  const int64_t k = blockIdx.x;
  const int ne = s * s;
  const int tid = threadIdx.x;
  for (int e = tid; e < ne; e += NT) {
    const int i = e / s, j = e - i * s;
    sh.Hr[i][j] = gre[k * ne + e];
    sh.Hi[i][j] = gim[k * ne + e];
  }
  __syncthreads();
  jacobi_eig_lds<MAXN, NT>(sh, s, max_sweeps, 1e-15);
  if (tid < s) {
    const double lt = sh.Hr[tid][tid];
    int rank = 0;
    for (int j = 0; j < s; ++j) {
      const double lj = sh.Hr[j][j];
      if (lj > lt || (lj == lt && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < ne; e += NT) {
    const int i = e / s, j = e - i * s;  // row i, sorted column j
    const int src = order[j];
    vre[k * ne + e] = sh.Vr[i][src];
    vim[k * ne + e] = sh.Vi[i][src];
  }
  if (tid < s) evals[k * s + tid] = sh.Hr[order[tid]][order[tid]];
}

// Orthonormalising transform from a Gram matrix G = X^H X (CholeskyQR):
// right-looking Cholesky G = R^H R in which a pivot at or below
// rtol * max_i G_ii drops its index (that row of R is zero: the column is
// taken as dependent on the earlier ones), then T = R^{-1} restricted to the
// kept indices (zero rows and columns elsewhere), so that X T has
// orthonormal columns on the kept indices and zero columns on the dropped
// ones. One workgroup per slice; T is s x s, row-major.
//
// Each of the 1024 threads keeps MAXN^2 / 1024 entries of the padded
// MAXN x MAXN upper triangle in registers. Step j publishes row j (already
// updated by steps < j) to LDS; after one barrier every thread applies
// G_lm -= conj(G_jl) G_jm / G_jj to its entries below row j. Row j is
// never written again, so a step needs no second barrier.
constexpr int kCholNT = 1024;

template <int MAXN, typename T>
__global__ __launch_bounds__(kCholNT) void chol_inv_kernel(const double* __restrict__ gre,
                                                           const double* __restrict__ gim, int64_t K, int s,
                                                           double rtol, int real_last, T* __restrict__ tre,
                                                           T* __restrict__ tim) {
  constexpr int NT = kCholNT, PER = MAXN * MAXN / NT;
  static_assert(PER >= 1 && PER * NT == MAXN * MAXN, "one or more whole entries per thread");
  __shared__ double Gr[MAXN][MAXN + 1], Gi[MAXN][MAXN + 1];
  __shared__ double Tr[MAXN][MAXN + 1], Ti[MAXN][MAXN + 1];
  __shared__ double rd[MAXN];
  __shared__ double dmax;
  const int64_t k = blockIdx.x;
  const bool real = k == 0 || (real_last && k == K - 1);
  const int tid = threadIdx.x;
  const int ne = s * s;
  int ri[PER], ci[PER];
  double gr[PER], gi[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + NT * u;
    ri[u] = e / MAXN;
    ci[u] = e % MAXN;
    const bool in = ri[u] < s && ci[u] < s && ci[u] >= ri[u];
    gr[u] = in ? gre[k * ne + ri[u] * s + ci[u]] : 0.0;
    gi[u] = (in && !real && ci[u] > ri[u]) ? gim[k * ne + ri[u] * s + ci[u]] : 0.0;
  }
  if (tid < 64) {
    double m = tid < s ? gre[k * ne + tid * s + tid] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (tid == 0) dmax = m;
  }
  __syncthreads();
  const double tol = rtol * dmax;
  for (int j = 0; j < s; ++j) {
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (ri[u] == j && ci[u] >= j && ci[u] < s) {
        Gr[j][ci[u]] = gr[u];
        Gi[j][ci[u]] = gi[u];
      }
    __syncthreads();
    const double d = Gr[j][j];
    if (d > tol && d > 0.0) {
      const double inv = 1.0 / d;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int l = ri[u], m = ci[u];
        if (l > j && m >= l && m < s) {
          const double ar = Gr[j][l], ai = Gi[j][l], br = Gr[j][m], bi = Gi[j][m];
          gr[u] -= (ar * br + ai * bi) * inv;
          gi[u] -= (ar * bi - ai * br) * inv;
        }
      }
    }
  }
  // pivots: the published diagonal is the value each step tested
  if (tid < MAXN) {
    const double d = tid < s ? Gr[tid][tid] : 0.0;
    rd[tid] = (tid < s && d > tol && d > 0.0) ? sqrt(d) : 0.0;
  }
  __syncthreads();
  // R (strict upper triangle, zero on dropped rows and past s) and T = diag(1 / R_ii)
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = ri[u], j = ci[u];
    if (j > i) {
      const bool live = i < s && j < s && rd[i] > 0.0;
      Gr[i][j] = live ? gr[u] / rd[i] : 0.0;
      Gi[i][j] = live ? gi[u] / rd[i] : 0.0;
    }
    Tr[i][j] = (i == j && rd[i] > 0.0) ? 1.0 / rd[i] : 0.0;
    Ti[i][j] = 0.0;
  }
  __syncthreads();
  // T = R^{-1} on the kept indices by recursive doubling over diagonal
  // blocks of the padded MAXN x MAXN factor: with T11, T22 the inverses of
  // two adjacent b x b diagonal blocks, the block above T22 is
  // T12 = -T11 (R12 T22). W = R12 T22 is kept in the (unused) lower triangle
  // of G at the transposed position. A dropped index has R_ii = 0 and a zero
  // row, and gets a zero row and column of T.
  for (int b = 1; b < MAXN; b *= 2) {
    const int nw = (MAXN / (2 * b)) * b * b;
    // W = R12 T22 (b x b per pair), stored at G[a1 + y][a0 + x]
    for (int e = tid; e < nw; e += NT) {
      const int p = e / (b * b), rem = e - p * b * b;
      const int x = rem / b, y = rem - x * b;  // W row x (block row a0 + x), column y (a1 + y)
      const int a0 = 2 * p * b, a1 = a0 + b;
      double wr = 0.0, wi = 0.0;
      for (int t = 0; t < b; ++t) {
        const double rr = Gr[a0 + x][a1 + t], rim = Gi[a0 + x][a1 + t];
        const double tr = Tr[a1 + t][a1 + y], ti = Ti[a1 + t][a1 + y];
        wr += rr * tr - rim * ti;
        wi += rr * ti + rim * tr;
      }
      Gr[a1 + y][a0 + x] = wr;
      Gi[a1 + y][a0 + x] = wi;
    }
    __syncthreads();
    // T12 = -T11 W
    for (int e = tid; e < nw; e += NT) {
      const int p = e / (b * b), rem = e - p * b * b;
      const int x = rem / b, y = rem - x * b;
      const int a0 = 2 * p * b, a1 = a0 + b;
      double vr = 0.0, vi = 0.0;
      for (int t = 0; t < b; ++t) {
        const double tr = Tr[a0 + x][a0 + t], ti = Ti[a0 + x][a0 + t];
        const double wr = Gr[a1 + y][a0 + t], wi = Gi[a1 + y][a0 + t];
        vr += tr * wr - ti * wi;
        vi += tr * wi + ti * wr;
      }
      Tr[a0 + x][a1 + y] = -vr;
      Ti[a0 + x][a1 + y] = -vi;
    }
    __syncthreads();
  }
  for (int e = tid; e < ne; e += NT) {
    const int i = e / s, j = e - i * s;
    tre[k * ne + e] = (T)Tr[i][j];
    tim[k * ne + e] = (T)(real ? 0.0 : Ti[i][j]);
  }
}

// Small transforms from an eigen-decomposition G = V diag(lambda) V^H.
// mode 0 (orthonormalise): T = V diag(w), w_i = lambda_i^{-1/2} when
//   lambda_i > rtol * lambda_0 (and > 0), else 0; T is s x s.
// mode 1 (truncate): T = V[:, :r] diag(w), w_i = lambda_i^{-p/2} for the
//   kept i < r with sigma_i = sqrt(lambda_i) > rtol * sigma_0, else 0; T is
//   s x r. p is `power`.
// Output planar in float (Tf) or double (Td).
template <typename T>
__global__ void transform_kernel(const double* __restrict__ vre, const double* __restrict__ vim,
                                 const double* __restrict__ evals, int64_t K, int s, int r, int mode, double rtol,
                                 double power, T* __restrict__ tre, T* __restrict__ tim) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int cols = mode == 0 ? s : r;
  if (e >= K * s * cols) return;
  const int64_t k = e / ((int64_t)s * cols);
  const int rem = (int)(e - k * s * cols);
  const int i = rem / cols, j = rem - i * cols;
  const double l0 = evals[k * s];
  const double lj = evals[k * s + j];
  double w = 0.0;
  if (mode == 0) {
    if (lj > 0.0 && lj > rtol * l0) w = 1.0 / sqrt(lj);
  } else {
    const double s0 = l0 > 0.0 ? sqrt(l0) : 0.0;
    const double sj = lj > 0.0 ? sqrt(lj) : 0.0;
    if (sj > 0.0 && sj > rtol * s0) w = pow(sj, -power);
  }
  const int64_t src = k * (int64_t)s * s + (int64_t)i * s + j;
  tre[e] = (T)(vre[src] * w);
  tim[e] = (T)(vim[src] * w);
}

// part[k][j] = w_k sum_{i<r} |X_k[j, i]|^2 g_k[i], with g_k[i] = 1/lambda_k[i]
// when scaled (so that X_k diag(1/sigma) is normalised), else 1; w_k the
// conjugate weights of the half spectrum (1 for the real slices, 2 for the
// others). One thread per (row j, slice k = blockIdx.x): slices on the grid
// dimension that holds more than 65,535 values.
template <typename T>
__global__ void leverage_kernel(const T* __restrict__ xre, const T* __restrict__ xim, int64_t K, int64_t n,
                                int64_t ldx, int64_t sx, int r, int real_last, const double* __restrict__ evals,
                                int s, double rtol, double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t k = blockIdx.x;
  if (j >= n) return;
  const double wk = (k == 0 || (real_last && k == K - 1)) ? 1.0 : 2.0;
  const double l0 = evals ? evals[k * s] : 0.0;
  const double s0 = l0 > 0 ? sqrt(l0) : 0.0;
  double sk = 0.0;
  for (int i = 0; i < r; ++i) {
    double g = 1.0;
    if (evals) {
      const double li = evals[k * s + i];
      const double si = li > 0 ? sqrt(li) : 0.0;
      g = (si > 0 && si > rtol * s0) ? 1.0 / li : 0.0;
    }
    const double a = (double)xre[k * sx + j * ldx + i], b = (double)xim[k * sx + j * ldx + i];
    sk += (a * a + b * b) * g;
  }
  part[k * n + j] = wk * sk;
}

// out[j] = sum over k (in order) of part[k][j].
__global__ void sum_slices_kernel(const double* __restrict__ part, int64_t K, int64_t n, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  // unrolled so that the loads of 16 slices are in flight together; the
  // additions keep their order
#pragma unroll 16
  for (int64_t k = 0; k < K; ++k) acc += part[k * n + j];
  out[j] = acc;
}

// Long spectra: thread (j, c) sums slices [c kc, (c + 1) kc) of column j in
// order and leaves the sum in the chunk's first row (read by no other
// thread); the chunk sums are then added in chunk order.
__global__ void sum_chunks_kernel(double* __restrict__ part, int64_t K, int64_t n, int64_t kc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.y * kc;
  if (j >= n) return;
  const int64_t k1 = k0 + kc < K ? k0 + kc : K;
  double acc = 0.0;
#pragma unroll 16
  for (int64_t k = k0; k < k1; ++k) acc += part[k * n + j];
  part[k0 * n + j] = acc;
}

__global__ void sum_chunk_heads_kernel(const double* __restrict__ part, int64_t K, int64_t n, int64_t kc,
                                       double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < K; k0 += kc) acc += part[k0 * n + j];
  out[j] = acc;
}

__global__ void sqrt_evals_kernel(const double* __restrict__ evals, int64_t K, int s, int r,
                                  double* __restrict__ sv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * r) return;
  const int64_t k = e / r;
  const int i = (int)(e - k * r);
  const double l = evals[k * s + i];
  sv[e] = l > 0 ? sqrt(l) : 0.0;
}

// W[k][t][c] = scale[t] * X[k][idx[t]][c] (row gather of a spectrum, with
// rows at or beyond *count set to zero); converts between float types.
template <typename Ti, typename To>
__global__ void gather_rows_kernel(const Ti* __restrict__ xre, const Ti* __restrict__ xim, int64_t K, int64_t rows,
                                   int64_t cols, const int32_t* __restrict__ idx, const double* __restrict__ scale,
                                   const int64_t* count, int64_t out_rows, To* __restrict__ wre,
                                   To* __restrict__ wim) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * out_rows * cols) return;
  const int64_t k = e / (out_rows * cols);
  const int64_t rem = e - k * out_rows * cols;
  const int64_t t = rem / cols, c = rem - t * cols;
  const int64_t lim = count ? *count : out_rows;
  if (t >= lim) {
    wre[e] = To(0);
    wim[e] = To(0);
    return;
  }
  const double sc = scale ? scale[t] : 1.0;
  const int64_t src = k * rows * cols + (int64_t)idx[t] * cols + c;
  wre[e] = (To)((double)xre[src] * sc);
  wim[e] = (To)((double)xim[src] * sc);
}

template <typename Ti, typename To>
__global__ void convert_kernel(const Ti* __restrict__ a, To* __restrict__ b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (To)a[e];
}

unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int randn_spectrum(void* re, void* im, int dtype, int64_t K, int64_t rows, int64_t cols, bool real_last,
                   uint64_t seed, uint64_t stream_id, hipStream_t st) {
  const int64_t n = K * rows * cols;
  if (n == 0) return TP_OK;
  if (dtype == TP_F64)
    hipLaunchKernelGGL(randn_kernel<double>, dim3(blocks_for(n)), dim3(256), 0, st, (double*)re, (double*)im, K,
                       rows * cols, real_last ? 1 : 0, seed, stream_id);
  else
    hipLaunchKernelGGL(randn_kernel<float>, dim3(blocks_for(n)), dim3(256), 0, st, (float*)re, (float*)im, K,
                       rows * cols, real_last ? 1 : 0, seed, stream_id);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int64_t gram_chunks(int64_t rows) {
  const int64_t c = (rows + 63) / 64;
  return c < 1 ? 1 : (c > 16 ? 16 : c);
}

size_t gram_part_doubles(int64_t K, int64_t rows, int s) { return (size_t)(K * gram_chunks(rows) * s * s); }

// launches the cross product on the matrix cores with the narrowest staging
// that covers a and b (at most 16 tiles of 16 x 16, four per wavefront)
template <typename T, bool SAME>
void launch_xgram(dim3 grid, hipStream_t st, const T* xre, const T* xim, int a, int64_t ldx, int64_t sx,
                  const T* yre, const T* yim, int b, int64_t ldy, int64_t sy, int64_t K, int64_t rows, int rl,
                  int64_t rch, double* pre, double* pim) {
  if constexpr (SAME) {
    if (a <= 32)
      hipLaunchKernelGGL((xgram_mfma_kernel<T, 32, 32, 1, true>), grid, dim3(256), 0, st, xre, xim, a, ldx, sx, yre,
                         yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
    else
      hipLaunchKernelGGL((xgram_mfma_kernel<T, 64, 64, 4, true>), grid, dim3(256), 0, st, xre, xim, a, ldx, sx, yre,
                         yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
    return;
  }
  if (a <= 32 && b <= 32)
    hipLaunchKernelGGL((xgram_mfma_kernel<T, 32, 32, 1, false>), grid, dim3(256), 0, st, xre, xim, a, ldx, sx, yre,
                       yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
  else if (b <= 32)
    hipLaunchKernelGGL((xgram_mfma_kernel<T, 64, 32, 2, false>), grid, dim3(256), 0, st, xre, xim, a, ldx, sx, yre,
                       yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
  else if (a <= 32)
    hipLaunchKernelGGL((xgram_mfma_kernel<T, 32, 64, 2, false>), grid, dim3(256), 0, st, xre, xim, a, ldx, sx, yre,
                       yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
  else
    hipLaunchKernelGGL((xgram_mfma_kernel<T, 64, 64, 4, false>), grid, dim3(256), 0, st, xre, xim, a, ldx, sx, yre,
                       yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
}

size_t xgram_part_doubles(int64_t K, int64_t rows, int a, int b) {
  return (size_t)(K * gram_chunks(rows) * a * b);
}

int xgram(const void* xre, const void* xim, int a, int64_t ldx, int64_t sx, const void* yre, const void* yim, int b,
          int64_t ldy, int64_t sy, int dtype, int64_t K, int64_t rows, bool real_last, void* ore, void* oim,
          double* pre, double* pim, hipStream_t st) {
  if (a < 1 || a > kMaxS || b < 1 || b > kMaxS) return fail(TP_EUNSUPPORTED, "cross product size outside 1..64");
  if (K == 0) return TP_OK;
  if (K > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many Fourier slices");  // slices on grid x
  if (!pre || !pim) return fail(TP_EWORKSPACE, "cross product partial buffer missing");
  const int64_t nch = gram_chunks(rows);
  const int64_t rch = (rows + nch - 1) / nch;
  const dim3 grid((unsigned)K, (unsigned)nch);
  const int rl = real_last ? 1 : 0;
  if (dtype == TP_F64)
    launch_xgram<double, false>(grid, st, (const double*)xre, (const double*)xim, a, ldx, sx, (const double*)yre,
                                (const double*)yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
  else
    launch_xgram<float, false>(grid, st, (const float*)xre, (const float*)xim, a, ldx, sx, (const float*)yre,
                               (const float*)yim, b, ldy, sy, K, rows, rl, rch, pre, pim);
  TP_LAUNCH_CHECK();
  const int ne = a * b;
  if (dtype == TP_F64)
    hipLaunchKernelGGL(xgram_reduce_kernel<double>, dim3(blocks_for(K * ne)), dim3(256), 0, st, pre, pim, K, nch, ne,
                       (double*)ore, (double*)oim);
  else
    hipLaunchKernelGGL(xgram_reduce_kernel<float>, dim3(blocks_for(K * ne)), dim3(256), 0, st, pre, pim, K, nch, ne,
                       (float*)ore, (float*)oim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int gram(const void* xre, const void* xim, int dtype, int64_t K, int64_t rows, int s, int64_t ldx, int64_t sx,
         bool real_last, double* gre, double* gim, double* pre, double* pim, hipStream_t st) {
  if (s < 1 || s > kMaxS) return fail(TP_EUNSUPPORTED, "Gram size outside 1..64");
  if (K == 0) return TP_OK;
  if (K > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many Fourier slices");  // slices on grid x
  if (!pre || !pim) return fail(TP_EWORKSPACE, "Gram partial buffer missing");
  const int64_t nch = gram_chunks(rows);
  const int64_t rch = (rows + nch - 1) / nch;
  const dim3 grid((unsigned)K, (unsigned)nch);
  const int rl = real_last ? 1 : 0;
  if (dtype == TP_F64)
    launch_xgram<double, true>(grid, st, (const double*)xre, (const double*)xim, s, ldx, sx, (const double*)xre,
                               (const double*)xim, s, ldx, sx, K, rows, rl, rch, pre, pim);
  else
    launch_xgram<float, true>(grid, st, (const float*)xre, (const float*)xim, s, ldx, sx, (const float*)xre,
                              (const float*)xim, s, ldx, sx, K, rows, rl, rch, pre, pim);
  TP_LAUNCH_CHECK();
  const int ne = s * s;
  hipLaunchKernelGGL(xgram_reduce_kernel<double>, dim3(blocks_for(K * ne)), dim3(256), 0, st, pre, pim, K, nch, ne,
                     gre, gim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int herm_eig(const double* gre, const double* gim, int64_t K, int s, double* evals, double* vre, double* vim,
             hipStream_t st) {
  if (s < 1 || s > kMaxS) return fail(TP_EUNSUPPORTED, "eigenproblem size outside 1..64");
  if (K == 0) return TP_OK;
  if (s <= 32)
    hipLaunchKernelGGL((herm_eig_kernel<32, 1024>), dim3((unsigned)K), dim3(1024), 0, st, gre, gim, s, 40, evals,
                       vre, vim);
  else
    hipLaunchKernelGGL((herm_eig_kernel<kMaxS, 1024>), dim3((unsigned)K), dim3(1024), 0, st, gre, gim, s, 40, evals,
                       vre, vim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int chol_inv(const double* gre, const double* gim, int64_t K, int s, double rtol, bool real_last, void* tre,
             void* tim, int out_dtype, hipStream_t st) {
  if (s < 1 || s > kMaxS) return fail(TP_EUNSUPPORTED, "Cholesky size outside 1..64");
  if (K == 0) return TP_OK;
  const int rl = real_last ? 1 : 0;
  const dim3 g((unsigned)K), b(kCholNT);
  if (out_dtype == TP_F64) {
    if (s <= 32)
      hipLaunchKernelGGL((chol_inv_kernel<32, double>), g, b, 0, st, gre, gim, K, s, rtol, rl, (double*)tre,
                         (double*)tim);
    else
      hipLaunchKernelGGL((chol_inv_kernel<kMaxS, double>), g, b, 0, st, gre, gim, K, s, rtol, rl, (double*)tre,
                         (double*)tim);
  } else {
    if (s <= 32)
      hipLaunchKernelGGL((chol_inv_kernel<32, float>), g, b, 0, st, gre, gim, K, s, rtol, rl, (float*)tre,
                         (float*)tim);
    else
      hipLaunchKernelGGL((chol_inv_kernel<kMaxS, float>), g, b, 0, st, gre, gim, K, s, rtol, rl, (float*)tre,
                         (float*)tim);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int eig_transform(const double* vre, const double* vim, const double* evals, int64_t K, int s, int r, int mode,
                  double rtol, double power, void* tre, void* tim, int out_dtype, hipStream_t st) {
  const int64_t n = K * s * (mode == 0 ? s : r);
  if (n == 0) return TP_OK;
  if (out_dtype == TP_F64)
    hipLaunchKernelGGL(transform_kernel<double>, dim3(blocks_for(n)), dim3(256), 0, st, vre, vim, evals, K, s, r,
                       mode, rtol, power, (double*)tre, (double*)tim);
  else
    hipLaunchKernelGGL(transform_kernel<float>, dim3(blocks_for(n)), dim3(256), 0, st, vre, vim, evals, K, s, r,
                       mode, rtol, power, (float*)tre, (float*)tim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int leverage(const void* xre, const void* xim, int dtype, int64_t K, int64_t n, int64_t ldx, int64_t sx, int r,
             bool real_last, const double* evals, int s, double rtol, double* part, double* out, hipStream_t st) {
  if (n == 0) return TP_OK;
  if (K > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many Fourier slices");
  if (blocks_for(n) > 65535) return fail(TP_EUNSUPPORTED, "too many slices to score");
  const dim3 grid((unsigned)K, blocks_for(n));
  if (dtype == TP_F64)
    hipLaunchKernelGGL(leverage_kernel<double>, grid, dim3(256), 0, st, (const double*)xre, (const double*)xim, K,
                       n, ldx, sx, r, real_last ? 1 : 0, evals, s, rtol, part);
  else
    hipLaunchKernelGGL(leverage_kernel<float>, grid, dim3(256), 0, st, (const float*)xre, (const float*)xim, K, n,
                       ldx, sx, r, real_last ? 1 : 0, evals, s, rtol, part);
  TP_LAUNCH_CHECK();
  if (K > 4096) {
    // many slices and few rows: chunks of 256 slices summed in parallel
    constexpr int64_t kc = 256;
    const int64_t nch = (K + kc - 1) / kc;
    if (nch > 65535) return fail(TP_EUNSUPPORTED, "too many Fourier slices");
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(blocks_for(n), (unsigned)nch), dim3(256), 0, st, part, K, n, kc);
    TP_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_chunk_heads_kernel, dim3(blocks_for(n)), dim3(256), 0, st, part, K, n, kc, out);
  } else {
    hipLaunchKernelGGL(sum_slices_kernel, dim3(blocks_for(n)), dim3(256), 0, st, part, K, n, out);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int singular_values(const double* evals, int64_t K, int s, int r, double* sv, hipStream_t st) {
  if (K * r == 0) return TP_OK;
  hipLaunchKernelGGL(sqrt_evals_kernel, dim3(blocks_for(K * r)), dim3(256), 0, st, evals, K, s, r, sv);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int gather_rows(const void* xre, const void* xim, int in_dtype, int64_t K, int64_t rows, int64_t cols,
                const int32_t* idx, const double* scale, const int64_t* count, int64_t out_rows, void* wre,
                void* wim, int out_dtype, hipStream_t st) {
  const int64_t n = K * out_rows * cols;
  if (n == 0) return TP_OK;
  if (in_dtype == TP_F32 && out_dtype == TP_F64)
    hipLaunchKernelGGL((gather_rows_kernel<float, double>), dim3(blocks_for(n)), dim3(256), 0, st,
                       (const float*)xre, (const float*)xim, K, rows, cols, idx, scale, count, out_rows,
                       (double*)wre, (double*)wim);
  else if (in_dtype == TP_F32 && out_dtype == TP_F32)
    hipLaunchKernelGGL((gather_rows_kernel<float, float>), dim3(blocks_for(n)), dim3(256), 0, st,
                       (const float*)xre, (const float*)xim, K, rows, cols, idx, scale, count, out_rows,
                       (float*)wre, (float*)wim);
  else if (in_dtype == TP_F64 && out_dtype == TP_F64)
    hipLaunchKernelGGL((gather_rows_kernel<double, double>), dim3(blocks_for(n)), dim3(256), 0, st,
                       (const double*)xre, (const double*)xim, K, rows, cols, idx, scale, count, out_rows,
                       (double*)wre, (double*)wim);
  else
    return fail(TP_EDTYPE, "gather_rows: unsupported conversion");
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int convert(const void* a, int adt, void* b, int bdt, int64_t n, hipStream_t st) {
  if (n == 0) return TP_OK;
  if (adt == TP_F64 && bdt == TP_F32)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(blocks_for(n)), dim3(256), 0, st, (const double*)a,
                       (float*)b, n);
  else if (adt == TP_F32 && bdt == TP_F64)
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(blocks_for(n)), dim3(256), 0, st, (const float*)a,
                       (double*)b, n);
  else
    return fail(TP_EDTYPE, "convert: unsupported conversion");
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
