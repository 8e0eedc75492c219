// Singular value thresholding of every Fourier slice (the closed-form
// L-update of Algorithm 7 with the tensor nuclear norm of eq. tnuc), the
// elementwise updates of the ADMM loops (completion, eq. tlow6, and robust
// PCA, eq. tlow7) and the slice gathers that feed CUR t-NN (Algorithm 6).
//
// SVD by block one-sided Jacobi on rows: every slice M (n1 x n2) is kept as
// X = U^H M together with Uh = U^H (both row-major, float32 planar). A step
// takes a pair of 16-row blocks (32 rows), forms their Gram matrix
// G = X_p X_p^H in float64, diagonalises it with the LDS Jacobi solver
// (G = V diag V^H) and rotates both X_p and Uh_p by V^H, which makes the 32
// rows mutually orthogonal. A round-robin tournament over the blocks visits
// all block pairs in a sweep; the disjoint pairs of a round are independent
// workgroups. A slice is converged when every pair in a sweep had
// max |G_st| / max(G_ss, G_tt) below the tolerance (measured against the
// larger row: rows stored in float32 keep a rounding floor of about
// eps_32 times the larger row); later launches for it return at once, so a
// fixed launch sequence needs no host synchronisation.
// At the end the rows of X are U^H M = Sigma V^H: sigma_i = ||x_i||, and
//   L = U diag(max(1 - tau / sigma_i, 0)) X = Uh^H (D X).
#include <cmath>

#include "common.hpp"
#include "jacobi.hpp"
#include "svt.hpp"

namespace tp {
namespace {

constexpr int RB = 16;       // rows per block
constexpr int PR = 2 * RB;   // rows per pair
constexpr int CHC = 64;      // columns staged per chunk
constexpr int NT = 256;
// Cyclic Jacobi sweeps on the 32 x 32 Gram matrix of a pair step. The outer
// sweeps revisit every pair until all of them are orthogonal, so a pair step
// need not diagonalise its Gram matrix exactly: one inner sweep costs about
// one more outer sweep in total against a full inner solve, at a fraction of
// the price per step (the inner solve dominates a step).
constexpr int kInnerSweeps = 1;

struct PairArgs {
  int64_t K, n1, n2;
  int64_t k0;        // first slice of this launch (blockIdx.y counts from it)
  float *xre, *xim;  // K x n1 x n2
  float *ure, *uim;  // K x n1 x n1
  int nb;            // number of blocks (even; the last may be partial or empty)
  int real_last;
  float* ratio;      // (nb-1) x K x (nb/2) ratios of this sweep, per round
  const int* conv;   // K flags
  double tol;
  int inner_sweeps;
};

__device__ __forceinline__ int tournament(int pos, int round, int nb) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (nb - 1));
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Staged rows of a pair step live in LDS as float64 with a row stride chosen
// per access pattern (in doubles): the Gram products read 16 rows x 4
// consecutive columns per instruction (stride = 4 mod 32 keeps that 2-way,
// the minimum for 64 eight-byte lanes), the rotations 4 rows x 16 columns
// (stride = 16 mod 32).
constexpr int kGramStride = CHC + 4;
constexpr int kRotStride = CHC + 16;
constexpr int kStage = PR * kRotStride;

// A chunk of the staged rows (columns [c0, c0 + nc) of rows[0..PR), float32
// planar) as held by one thread between its global loads and its LDS
// stores: element e = tid + NT q is row e / CHC, column e % CHC; missing rows
// and columns past nc read as zero. Loading the next chunk into registers
// before the current one is consumed keeps the global loads in flight
// during the products.
constexpr int kChunkPer = PR * CHC / NT;
constexpr int kGramDepth = 2, kRotDepth = 1;
struct ChunkRegs {
  float r[kChunkPer], i[kChunkPer];
};

__device__ __forceinline__ void load_chunk(ChunkRegs& g, const float* re, const float* im, int64_t ncols, int64_t c0,
                                           int nc, const int* rows, bool real) {
#pragma unroll
  for (int q = 0; q < kChunkPer; ++q) {
    const int e = threadIdx.x + NT * q;
    const int r = e / CHC, j = e - r * CHC;
    float vr = 0.f, vi = 0.f;
    if (j < nc && rows[r] >= 0) {
      const int64_t off = (int64_t)rows[r] * ncols + c0 + j;
      vr = re[off];
      vi = real ? 0.f : im[off];
    }
    g.r[q] = vr;
    g.i[q] = vi;
  }
}

// Stores a chunk into the float64 staging arrays with row stride S.
template <int S>
__device__ __forceinline__ void store_chunk(const ChunkRegs& g, double* sr, double* si) {
#pragma unroll
  for (int q = 0; q < kChunkPer; ++q) {
    const int e = threadIdx.x + NT * q;
    const int r = e / CHC, j = e - r * CHC;
    sr[r * S + j] = (double)g.r[q];
    si[r * S + j] = (double)g.i[q];
  }
}

// Runs body(c0, nc) over the column chunks [c0, c0 + nc) of the staged rows,
// each chunk stored to the LDS staging arrays (row stride S) before its
// body. DEPTH (1 or 2) chunks are kept in flight in registers: chunk
// c + DEPTH is loaded while chunk c is multiplied. Every thread must call
// it; body must only read the staging arrays.
template <int S, int DEPTH, class Body>
__device__ __forceinline__ void staged_chunks(const float* re, const float* im, int64_t ncols, const int* rows,
                                              bool real, double* sr, double* si, Body&& body) {
  static_assert(DEPTH == 1 || DEPTH == 2, "one or two chunks in flight");
  auto width = [ncols](int64_t c) { return (int)((ncols - c) < CHC ? (ncols - c) : CHC); };
  ChunkRegs g[DEPTH];
  load_chunk(g[0], re, im, ncols, 0, width(0), rows, real);
  if (DEPTH == 2 && CHC < ncols) load_chunk(g[DEPTH - 1], re, im, ncols, CHC, width(CHC), rows, real);
  for (int64_t c0 = 0; c0 < ncols; c0 += DEPTH * CHC) {
#pragma unroll
    for (int b = 0; b < DEPTH; ++b) {
      const int64_t c = c0 + b * CHC;
      if (c >= ncols) break;
      store_chunk<S>(g[b], sr, si);
      __syncthreads();
      if (c + DEPTH * CHC < ncols) load_chunk(g[b], re, im, ncols, c + DEPTH * CHC, width(c + DEPTH * CHC), rows, real);
      body(c, width(c));
      __syncthreads();
    }
  }
}

// Rotates rows rows[0..PR) of a row-major K x nrows x ncols planar matrix by
// V^H: out_s = sum_t conj(V_ts) in_t, on the float64 matrix cores
// (v_mfma_f64_16x16x4f64: A lane l = A[l % 16][l / 16], B lane l =
// B[l / 16][l % 16], D lane l register v = D[4 v + l / 16][l % 16], as
// measured on gfx950).
// Wavefront w owns output columns [16 w, 16 w + 16) of each staged chunk and
// both 16-row halves; the V^H fragments (A[s][t] = conj(V[t][s])) are passed
// in registers: vfr/vfi[h][kk] for row half h and contraction step kk.
__device__ void rotate_rows(const double (&vfr)[2][8], const double (&vfi)[2][8], double* sr, double* si,
                            float* re, float* im, int64_t ncols, const int* rows, bool real) {
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int j0 = 16 * w;
  staged_chunks<kRotStride, kRotDepth>(re, im, ncols, rows, real, sr, si, [&](int64_t c0, int nc) {
    d4 orr[2], oi[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      orr[h] = d4{0.0, 0.0, 0.0, 0.0};
      oi[h] = d4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int kk = 0; kk < PR / 4; ++kk) {
      const int t = 4 * kk + (l >> 4), j = j0 + (l & 15);
      const double br = sr[t * kRotStride + j], bi = si[t * kRotStride + j];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // conj(V)^T x: re = Vr xr + Vi xi, im = Vr xi - Vi xr
        orr[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(vfr[h][kk], br, orr[h], 0, 0, 0);
        orr[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(vfi[h][kk], bi, orr[h], 0, 0, 0);
        oi[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(vfr[h][kk], bi, oi[h], 0, 0, 0);
        oi[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(-vfi[h][kk], br, oi[h], 0, 0, 0);
      }
    }
    // the chunks still in flight cover later columns than the ones written
    const int j = j0 + (l & 15);
    if (j < nc) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int sidx = 16 * h + 4 * v + (l >> 4);
          if (rows[sidx] < 0) continue;
          const int64_t off = (int64_t)rows[sidx] * ncols + c0 + j;
          re[off] = (float)orr[h][v];
          if (!real) im[off] = (float)oi[h][v];
        }
    }
  });
}

__global__ __launch_bounds__(NT) void svt_pair_kernel(PairArgs a, int round) {
  __shared__ JacobiShared<PR, NT> sh;
  __shared__ double stage_r[kStage], stage_i[kStage];
  __shared__ int rows[PR];
  __shared__ double ratio_red[NT];
  __shared__ int skip;
  const int64_t k = a.k0 + blockIdx.y;
  const int pair = blockIdx.x;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  if (a.conv[k]) return;
  const bool real = k == 0 || (a.real_last && k == a.K - 1);
  const int ba = tournament(pair, round, a.nb), bb = tournament(a.nb - 1 - pair, round, a.nb);
  if (tid < PR) {
    const int blk = tid < RB ? ba : bb;
    const int64_t r = (int64_t)blk * RB + (tid % RB);
    rows[tid] = r < a.n1 ? (int)r : -1;
  }
  float* xre = a.xre + k * a.n1 * a.n2;
  float* xim = a.xim + k * a.n1 * a.n2;
  float* ure = a.ure + k * a.n1 * a.n1;
  float* uim = a.uim + k * a.n1 * a.n1;
  // Gram G_st = sum_j x_s[j] conj(x_t[j]) on the matrix cores: wavefront w
  // owns the 16 x 16 block (s0, t0); re = Xr Xr^T + Xi Xi^T,
  // im = Xi Xr^T - Xr Xi^T (A = rows s0.., B = rows t0.. transposed)
  const int s0 = 16 * (w >> 1), t0 = 16 * (w & 1);
  d4 gre = {0.0, 0.0, 0.0, 0.0}, gim = {0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  staged_chunks<kGramStride, kGramDepth>(xre, xim, a.n2, rows, real, stage_r, stage_i, [&](int64_t, int) {
#pragma unroll 4
    for (int kk = 0; kk < CHC / 4; ++kk) {
      const int j = 4 * kk + (l >> 4);
      const double ar = stage_r[(s0 + (l & 15)) * kGramStride + j], ai = stage_i[(s0 + (l & 15)) * kGramStride + j];
      const double br = stage_r[(t0 + (l & 15)) * kGramStride + j], bi = stage_i[(t0 + (l & 15)) * kGramStride + j];
      gre = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, gre, 0, 0, 0);
      gre = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, gre, 0, 0, 0);
      gim = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, gim, 0, 0, 0);
      gim = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar, bi, gim, 0, 0, 0);
    }
  });
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    sh.Hr[s0 + 4 * v + (l >> 4)][t0 + (l & 15)] = gre[v];
    sh.Hi[s0 + 4 * v + (l >> 4)][t0 + (l & 15)] = gim[v];
  }
  __syncthreads();
  // largest off-diagonal entry relative to the larger squared norm of its
  // two rows, |G_st| / max(G_ss, G_tt). Rows are stored in float32, so a
  // rotation leaves rounding of size eps_32 |x_big| in the smaller row and
  // |G_st| cannot fall below ~eps_32 max(G_ss, G_tt): the usual
  // |G_st| / sqrt(G_ss G_tt) would never reach the tolerance for pairs whose
  // norms differ by more than tol / eps_32 and every call would run its
  // full sweep budget. Scaled by the larger row, the residual rotation
  // angle is below tol relative to the pair's spectral gap, which bounds
  // the error of the thresholded result by ~tol ||M||.
  double mr = 0.0;
  for (int e = tid; e < PR * PR; e += NT) {
    const int s = e / PR, t = e - s * PR;
    if (s != t) {
      const double d = fmax(sh.Hr[s][s], sh.Hr[t][t]);
      const double gr = sh.Hr[s][t], gi = sh.Hi[s][t];
      if (d > 0.0) mr = fmax(mr, sqrt(gr * gr + gi * gi) / d);
    }
  }
  ratio_red[tid] = mr;
  __syncthreads();
  for (int ww = NT / 2; ww > 0; ww >>= 1) {
    if (tid < ww) ratio_red[tid] = fmax(ratio_red[tid], ratio_red[tid + ww]);
    __syncthreads();
  }
  if (tid == 0) {
    a.ratio[((int64_t)round * a.K + k) * (a.nb / 2) + pair] = (float)ratio_red[0];
    skip = ratio_red[0] < a.tol;
  }
  __syncthreads();
  if (skip) return;
  jacobi_eig_lds<PR, NT>(sh, PR, a.inner_sweeps, 1e-14);
  // V^H fragments for the rotations: A[s][t] = conj(V[t][s]) with
  // s = 16 h + (l % 16), t = 4 kk + (l / 16); the minus sign of the
  // imaginary part is applied in the products
  double vfr[2][8], vfi[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int kk = 0; kk < PR / 4; ++kk) {
      vfr[h][kk] = sh.Vr[4 * kk + (l >> 4)][16 * h + (l & 15)];
      vfi[h][kk] = sh.Vi[4 * kk + (l >> 4)][16 * h + (l & 15)];
    }
  rotate_rows(vfr, vfi, stage_r, stage_i, xre, xim, a.n2, rows, real);
  rotate_rows(vfr, vfi, stage_r, stage_i, ure, uim, a.n1, rows, real);
}

__global__ void svt_conv_kernel(const float* __restrict__ ratio, int64_t K, int64_t k0, int64_t k1, int nrounds,
                                int npairs, double tol, int* conv) {
  const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k1) return;
  if (conv[k]) return;
  float m = 0.f;
  for (int r = 0; r < nrounds; ++r)
#pragma unroll 8
    for (int p = 0; p < npairs; ++p) m = fmaxf(m, ratio[((int64_t)r * K + k) * npairs + p]);
  if (m < tol) conv[k] = 1;
}

// Number of slices whose sweeps ended without meeting the convergence test
// (conv[k] == 0), one workgroup, integer sums in a fixed order.
__global__ __launch_bounds__(256) void count_unconverged_kernel(const int* __restrict__ conv, int64_t K,
                                                                int32_t* __restrict__ out) {
  __shared__ int64_t red[256];
  int64_t c = 0;
  for (int64_t k = threadIdx.x; k < K; k += 256) c += conv[k] ? 0 : 1;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (int32_t)(red[0] < 0x7fffffff ? red[0] : 0x7fffffff);
}

__global__ void identity_kernel(float* re, float* im, int64_t K, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * n * n) return;
  const int64_t r = e % (n * n);
  re[e] = (r / n == r % n) ? 1.f : 0.f;
  im[e] = 0.f;
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.f;
}

__global__ void zero_int_kernel(int* p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0;
}

// Row norms of X, shrink factors d_i = max(1 - tau / sigma_i, 0), X <- D X,
// and the number of sigma_i > tau per slice. Row norms at or below
// max(n1, n2) eps_32 sigma_max are rounding residue of rows that the
// rotations have emptied (a slice has at most min(n1, n2) nonzero singular
// values) and count as zero. Three passes over all slices at once: a
// wavefront per row sums it with consecutive lanes on consecutive columns;
// one workgroup per slice turns the norms into factors (sig, K x n1, holds
// the norms and then the factors); the scaling runs over every element.
__global__ __launch_bounds__(NT) void svt_rownorm_kernel(const float* __restrict__ xre, const float* __restrict__ xim,
                                                         int64_t K, int64_t n1, int64_t n2, int real_last,
                                                         double* __restrict__ sig) {
  const int64_t row = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= K * n1) return;
  const int64_t k = row / n1;
  const bool real = k == 0 || (real_last && k == K - 1);
  const float* re = xre + row * n2;
  const float* im = xim + row * n2;
  double s2 = 0.0;
  for (int64_t j = lane; j < n2; j += 64) {
    const double a = re[j], b = real ? 0.0 : im[j];
    s2 += a * a + b * b;
  }
  s2 = wave_sum(s2);
  if (lane == 0) sig[row] = sqrt(s2);
}

__global__ __launch_bounds__(NT) void svt_factor_kernel(int64_t n1, int64_t n2, double tau, double* sig,
                                                        int32_t* ranks) {
  __shared__ double red[NT];
  __shared__ int cnt[NT];
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x;
  double* sg = sig + k * n1;
  double mx = 0.0;
  for (int64_t i = tid; i < n1; i += NT) mx = fmax(mx, sg[i]);
  red[tid] = mx;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double floor_ = (double)(n1 > n2 ? n1 : n2) * 1.1920928955078125e-07 * red[0];
  int mine = 0;
  for (int64_t i = tid; i < n1; i += NT) {
    const double sgi = sg[i];
    const bool kept = sgi > tau && sgi > floor_;
    if (kept) ++mine;
    sg[i] = kept ? 1.0 - tau / sgi : 0.0;
  }
  cnt[tid] = mine;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) cnt[tid] += cnt[tid + w];
    __syncthreads();
  }
  if (tid == 0 && ranks) ranks[k] = cnt[0];
}

__global__ void svt_scale_kernel(float* __restrict__ xre, float* __restrict__ xim, int64_t K, int64_t n1, int64_t n2,
                                 int real_last, const double* __restrict__ sig) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * n1 * n2) return;
  const int64_t row = e / n2, k = row / n1;
  const bool real = k == 0 || (real_last && k == K - 1);
  const double d = sig[row];
  xre[e] = (float)(d * xre[e]);
  if (!real) xim[e] = (float)(d * xim[e]);
}

// Leading singular (or eigen) vectors after the block Jacobi has made the m
// rows of X (row length ldx) orthogonal, X = Q Y with Q unitary. Row i of X
// is mu_i times a unit row and so mu_i = ||X_i||. Two uses:
//  * Y = G, a Hermitian positive semidefinite Gram matrix: q_i (row i of Q)
//    is a conjugated eigenvector and mu_i its eigenvalue, sigma = sqrt(mu);
//  * Y = a Fourier slice itself (m <= its row length): mu_i = sigma_i, rows
//    of Q are the conjugated left singular vectors and rows of X are sigma_i
//    times the conjugated right ones.
// For the r largest mu (descending, ties by index) column t of out (len x r
// planes per slice) is conj(row sel(t) of the source S (row length len))
// times 1, 1 / sqrt(mu) (mode 1) or 1 / mu (mode 2), and sv[k][t] =
// sqrt(mu) (sqrt_sv) or mu. One workgroup per slice. A mu at or below
// floor_rel times the slice's largest mu is rounding residue of a row the
// rotations have emptied (or of an eigenvalue that is zero): it is reported
// as 0 and its column is zero in every mode, so a rank-deficient slice gives
// the same zero columns whichever route produced X.
__global__ __launch_bounds__(NT) void tsvd_pick_kernel(const float* __restrict__ xre, const float* __restrict__ xim,
                                                       int64_t ldx, const float* __restrict__ sre,
                                                       const float* __restrict__ sim, int64_t len, int64_t K, int m,
                                                       int r, int real_last, int mode, int sqrt_sv, double floor_rel,
                                                       float* __restrict__ ore, float* __restrict__ oim,
                                                       double* __restrict__ sv) {
  __shared__ double red[NT];
  extern __shared__ double lam[];  // m row norms, then r selected rows (int)
  int* sel = reinterpret_cast<int*>(lam + m);
  const int64_t k = blockIdx.x;
  const bool real = k == 0 || (real_last && k == K - 1);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float* xr = xre + k * m * ldx;
  const float* xi = xim + k * m * ldx;
  for (int i = wv; i < m; i += NT / 64) {
    double s2 = 0.0;
    for (int64_t j = lane; j < ldx; j += 64) {
      const double a = xr[(int64_t)i * ldx + j], b = real ? 0.0 : xi[(int64_t)i * ldx + j];
      s2 += a * a + b * b;
    }
    s2 = wave_sum(s2);
    if (lane == 0) lam[i] = sqrt(s2);
  }
  // every rank below r is taken exactly once for finite norms; the default
  // keeps a non-finite input in bounds
  for (int t = tid; t < r; t += NT) sel[t] = 0;
  __syncthreads();
  for (int i = tid; i < m; i += NT) {
    const double li = lam[i];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = lam[j];
      rank += (lj > li || (lj == li && j < i)) ? 1 : 0;
    }
    if (rank < r) sel[rank] = i;
  }
  double mx = 0.0;
  for (int i = tid; i < m; i += NT) mx = fmax(mx, lam[i]);
  red[tid] = mx;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double floor_ = floor_rel * red[0];
  const float* s_r = sre + k * m * len;
  const float* s_i = sim + k * m * len;
  float* o_r = ore + k * len * r;
  float* o_i = oim + k * len * r;
  for (int64_t e = tid; e < len * r; e += NT) {
    const int64_t j = e / r;
    const int t = (int)(e - j * r);
    const int row = sel[t];
    const double l = lam[row];
    const double sc = !(l > floor_) ? 0.0 : (mode == 0 ? 1.0 : (mode == 1 ? 1.0 / sqrt(l) : 1.0 / l));
    o_r[e] = (float)(sc * s_r[(int64_t)row * len + j]);
    o_i[e] = real ? 0.f : (float)(-sc * s_i[(int64_t)row * len + j]);
  }
  if (sv)
    for (int t = tid; t < r; t += NT) {
      const double l = lam[sel[t]];
      sv[k * r + t] = !(l > floor_) ? 0.0 : (sqrt_sv ? sqrt(l) : l);
    }
}

// t-transpose (Section 2.1): out (n2 x n1 x n3) with out[j][i][t] =
// in[i][j][(n3 - t) mod n3], i.e. every frontal slice transposed and slices
// 2..n3 in reverse order; its Fourier slices are the conjugate transposes
// of those of in.
template <typename T>
__global__ void ttranspose_kernel(const T* __restrict__ in, int64_t n1, int64_t n2, int64_t n3, T* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n1 * n2 * n3) return;
  const int64_t tube = e / n3, t = e - tube * n3;
  const int64_t j = tube / n1, i = tube - j * n1;
  const int64_t ts = t == 0 ? 0 : n3 - t;
  out[e] = in[(i * n2 + j) * n3 + ts];
}

// M = X - E - Y / mu (tube-major, elementwise)
__global__ void admm_pre_kernel(const float* __restrict__ x, const float* __restrict__ e,
                                const float* __restrict__ y, float inv_mu, int64_t n, float* __restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) m[i] = x[i] - e[i] - y[i] * inv_mu;
}

// E = P_unobserved(X - L - Y/mu); Y = Y + mu (L + E - X)
__global__ void admm_post_kernel(const float* __restrict__ x, const uint8_t* __restrict__ mask,
                                 const float* __restrict__ l, float mu, float inv_mu, int64_t n,
                                 float* __restrict__ e, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float xv = x[i], lv = l[i], yv = y[i];
  const float ev = mask[i] ? 0.f : (xv - lv - yv * inv_mu);
  e[i] = ev;
  y[i] = yv + mu * (lv + ev - xv);
}

// E = shrink(X - L - Y/mu, lam/mu), the prox of (lam/mu) ||.||_1 (robust
// PCA, eq. tlow7); Y = Y + mu (L + E - X)
__global__ void admm_post_soft_kernel(const float* __restrict__ x, const float* __restrict__ l, float mu,
                                      float inv_mu, float thr, int64_t n, float* __restrict__ e,
                                      float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float xv = x[i], lv = l[i], yv = y[i];
  const float v = xv - lv - yv * inv_mu;
  const float ev = v > thr ? v - thr : (v < -thr ? v + thr : 0.f);
  e[i] = ev;
  y[i] = yv + mu * (lv + ev - xv);
}

// out[k][j][i] = conj(in[k][i][j]): the conjugate transpose of every
// Fourier slice (K x rows x cols planar in, K x cols x rows out). Reads are
// coalesced along j; the writes are strided.
__global__ void spec_conj_transpose_kernel(const float* __restrict__ re, const float* __restrict__ im, int64_t K,
                                           int64_t rows, int64_t cols, float* __restrict__ ore,
                                           float* __restrict__ oim) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = rows * cols;
  if (e >= K * per) return;
  const int64_t k = e / per, r = e - k * per, i = r / cols, j = r - i * cols;
  const int64_t o = k * per + j * rows + i;
  ore[o] = re[e];
  oim[o] = -im[e];
}

// The three quantities of Algorithm 7's convergence check for one
// iteration, reduced per workgroup: max |L - Lprev|, max |E - Eprev| and
// max |L + E - X| over the workgroup's elements (E the new iterate, read
// after the E-update; eprev a copy taken before it). One value triple per
// workgroup in part[3 * block + q]; the maxima are order independent.
__global__ __launch_bounds__(256) void admm_stop_partial_kernel(const float* __restrict__ x,
                                                                const float* __restrict__ l,
                                                                const float* __restrict__ lprev,
                                                                const float* __restrict__ e,
                                                                const float* __restrict__ eprev, int64_t n,
                                                                float* __restrict__ part) {
  __shared__ float red[3][256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float dl = 0.f, de = 0.f, rs = 0.f;
  if (i < n) {
    const float lv = l[i], ev = e[i];
    dl = fabsf(lv - lprev[i]);
    de = fabsf(ev - eprev[i]);
    rs = fabsf(lv + ev - x[i]);
  }
  red[0][threadIdx.x] = dl;
  red[1][threadIdx.x] = de;
  red[2][threadIdx.x] = rs;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmaxf(red[q][threadIdx.x], red[q][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) part[3 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// out[q] = max over the nb partial triples (one workgroup)
__global__ __launch_bounds__(256) void admm_stop_reduce_kernel(const float* __restrict__ part, int64_t nb,
                                                               float* __restrict__ out) {
  __shared__ float red[3][256];
  float m[3] = {0.f, 0.f, 0.f};
  for (int64_t b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int q = 0; q < 3; ++q) m[q] = fmaxf(m[q], part[3 * b + q]);
#pragma unroll
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = m[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmaxf(red[q][threadIdx.x], red[q][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

// out[a][b][t] = in[ra][cb][t] with ra = ridx ? ridx[a] : a and
// cb = cidx ? cidx[b] : b: picked lateral or horizontal slices of a
// tube-major tensor with in_cols lateral slices. Entries past the live pick
// count (*count, for the listed index) are written as zeros; a negative
// count (rejected weights) leaves every entry zero.
template <typename T>
__global__ void gather_slices_kernel(const T* __restrict__ in, int64_t in_cols, int64_t n3,
                                     const int32_t* __restrict__ ridx, const int32_t* __restrict__ cidx,
                                     const int64_t* __restrict__ count, int64_t rows, int64_t cols,
                                     T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols * n3) return;
  const int64_t tube = i / n3, t = i - tube * n3;
  const int64_t a = tube / cols, b = tube - a * cols;
  const int64_t lim = count ? *count : INT64_MAX;
  if ((ridx && a >= lim) || (cidx && b >= lim)) {
    out[i] = T(0);
    return;
  }
  const int64_t ra = ridx ? (int64_t)ridx[a] : a;
  const int64_t cb = cidx ? (int64_t)cidx[b] : b;
  out[i] = in[(ra * in_cols + cb) * n3 + t];
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// The Jacobi sweeps use at most two streams: the caller's and the side
// stream (three or four streams measured slower than two).
constexpr int kSvtStreams = 2;

}  // namespace

size_t svt_ratio_count(int64_t K, int64_t n1) {
  const int nb = svt_blocks(n1);
  return size_t(nb - 1) * K * (nb / 2);
}

int svt_blocks(int64_t n1) {
  int nb = (int)((n1 + RB - 1) / RB);
  if (nb < 2) nb = 2;
  if (nb % 2) ++nb;
  return nb;
}

int zero_f32(float* p, int64_t n, hipStream_t st) {
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(zero_f32_kernel, dim3(nblk(n)), dim3(256), 0, st, p, n);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int svt_identity(float* ure, float* uim, int64_t K, int64_t n, hipStream_t st) {
  if (K * n * n == 0) return TP_OK;
  hipLaunchKernelGGL(identity_kernel, dim3(nblk(K * n * n)), dim3(256), 0, st, ure, uim, K, n);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int svt_count_unconverged(const int* conv, int64_t K, int32_t* out, hipStream_t st) {
  if (!out) return TP_OK;
  hipLaunchKernelGGL(count_unconverged_kernel, dim3(1), dim3(256), 0, st, conv, K, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int svt_jacobi(float* xre, float* xim, float* ure, float* uim, int64_t K, int64_t n1, int64_t n2, bool real_last,
               int max_sweeps, double tol, float* ratio, int* conv, hipStream_t st) {
  const int nb = svt_blocks(n1);
  hipLaunchKernelGGL(zero_int_kernel, dim3(nblk(K)), dim3(256), 0, st, conv, K);
  TP_LAUNCH_CHECK();
  PairArgs a{K, n1, n2, 0, xre, xim, ure, uim, nb, real_last ? 1 : 0, ratio, conv, tol, kInnerSweeps};
  // slices [k0, k1) on stream s
  auto sweeps = [&](int64_t k0, int64_t k1, hipStream_t s) -> int {
    PairArgs g = a;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      for (int round = 0; round < nb - 1; ++round) {
        // the slices sit on a grid dimension of at most 65,535 values: longer
        // spectra take several launches per round
        for (int64_t c0 = k0; c0 < k1; c0 += 65535) {
          g.k0 = c0;
          const int64_t kc = k1 - c0 < 65535 ? k1 - c0 : 65535;
          hipLaunchKernelGGL(svt_pair_kernel, dim3(nb / 2, (unsigned)kc), dim3(NT), 0, s, g, round);
          TP_LAUNCH_CHECK();
        }
      }
      hipLaunchKernelGGL(svt_conv_kernel, dim3(nblk(k1 - k0)), dim3(256), 0, s, ratio, K, k0, k1, nb - 1, nb / 2,
                         tol, conv);
      TP_LAUNCH_CHECK();
    }
    return TP_OK;
  };
  // The slices are independent: when one launch would leave compute units
  // with a free pair-step slot (two fit per compute unit by LDS) but has more
  // workgroups than compute units, the second half of the slices runs on
  // the side stream, so that one half's pair steps fill the units that the
  // other half's launch leaves idle. Measured on 51 slices of 256 x 256 (408
  // pair steps per launch on 256 units): 7% faster than one stream; on 85
  // slices of 192 x 1140 (510 pair steps, every slot taken): 7% slower.
  int dev = 0, cus = 0;
  TP_HIP_CHECK(hipGetDevice(&dev));
  TP_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t w = K * (nb / 2);
  if (K < kSvtStreams || w <= cus || 8 * w > 7 * 2 * (int64_t)cus) return sweeps(0, K, st);
  SideStream* ss = nullptr;
  if (int rc = side_stream(&ss)) return rc;
  std::lock_guard<std::mutex> lk(ss->mu);
  const int64_t kh = K / 2;
  TP_HIP_CHECK(hipEventRecord(ss->fork, st));
  TP_HIP_CHECK(hipStreamWaitEvent(ss->s, ss->fork, 0));
  if (int rc = sweeps(kh, K, ss->s)) return rc;
  TP_HIP_CHECK(hipEventRecord(ss->join, ss->s));
  if (int rc = sweeps(0, kh, st)) return rc;
  TP_HIP_CHECK(hipStreamWaitEvent(st, ss->join, 0));
  return TP_OK;
}

int svt_shrink(float* xre, float* xim, int64_t K, int64_t n1, int64_t n2, double tau, bool real_last,
               double* sig, int32_t* ranks, hipStream_t st) {
  if (K * n1 == 0) return TP_OK;
  const int rl = real_last ? 1 : 0;
  const int64_t rows = K * n1;
  hipLaunchKernelGGL(svt_rownorm_kernel, dim3((unsigned)((rows + NT / 64 - 1) / (NT / 64))), dim3(NT), 0, st, xre,
                     xim, K, n1, n2, rl, sig);
  hipLaunchKernelGGL(svt_factor_kernel, dim3((unsigned)K), dim3(NT), 0, st, n1, n2, tau, sig, ranks);
  hipLaunchKernelGGL(svt_scale_kernel, dim3(nblk(K * n1 * n2)), dim3(256), 0, st, xre, xim, K, n1, n2, rl, sig);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int tsvd_pick(const float* xre, const float* xim, int64_t ldx, const float* sre, const float* sim, int64_t len,
              int64_t K, int64_t m, int64_t r, bool real_last, int mode, bool sqrt_sv, double floor_rel, float* ore,
              float* oim, double* sv, hipStream_t st) {
  if (K == 0 || r == 0) return TP_OK;
  if (m > kPickMax || r > m) return fail(TP_EUNSUPPORTED, "vector selection needs r <= m <= 4096");
  const size_t lds = size_t(m) * sizeof(double) + size_t(r) * sizeof(int);
  hipLaunchKernelGGL(tsvd_pick_kernel, dim3((unsigned)K), dim3(NT), lds, st, xre, xim, ldx, sre, sim, len, K, (int)m,
                     (int)r, real_last ? 1 : 0, mode, sqrt_sv ? 1 : 0, floor_rel, ore, oim, sv);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int admm_pre(const float* x, const float* e, const float* y, float inv_mu, int64_t n, float* m, hipStream_t st) {
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(admm_pre_kernel, dim3(nblk(n)), dim3(256), 0, st, x, e, y, inv_mu, n, m);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int admm_post(const float* x, const uint8_t* mask, const float* l, float mu, float inv_mu, int64_t n, float* e,
              float* y, hipStream_t st) {
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(admm_post_kernel, dim3(nblk(n)), dim3(256), 0, st, x, mask, l, mu, inv_mu, n, e, y);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int spec_conj_transpose(const float* re, const float* im, int64_t K, int64_t rows, int64_t cols, float* ore,
                        float* oim, hipStream_t st) {
  const int64_t n = K * rows * cols;
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(spec_conj_transpose_kernel, dim3(nblk(n)), dim3(256), 0, st, re, im, K, rows, cols, ore, oim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

size_t admm_stop_floats(int64_t n) { return 3 * size_t(nblk(n)) + 4; }

int admm_stop(const float* x, const float* l, const float* lprev, const float* e, const float* eprev, int64_t n,
              float* part, float* out, hipStream_t st) {
  if (n == 0) return TP_OK;
  const unsigned nb = nblk(n);
  hipLaunchKernelGGL(admm_stop_partial_kernel, dim3(nb), dim3(256), 0, st, x, l, lprev, e, eprev, n, part);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(admm_stop_reduce_kernel, dim3(1), dim3(256), 0, st, part, (int64_t)nb, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int admm_post_soft(const float* x, const float* l, float mu, float inv_mu, float thr, int64_t n, float* e, float* y,
                   hipStream_t st) {
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(admm_post_soft_kernel, dim3(nblk(n)), dim3(256), 0, st, x, l, mu, inv_mu, thr, n, e, y);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int ttranspose(const void* in, int elem_bytes, int64_t n1, int64_t n2, int64_t n3, void* out, hipStream_t st) {
  const int64_t n = n1 * n2 * n3;
  if (n == 0) return TP_OK;
  if (elem_bytes == 4)
    hipLaunchKernelGGL(ttranspose_kernel<float>, dim3(nblk(n)), dim3(256), 0, st, (const float*)in, n1, n2, n3,
                       (float*)out);
  else if (elem_bytes == 1)
    hipLaunchKernelGGL(ttranspose_kernel<uint8_t>, dim3(nblk(n)), dim3(256), 0, st, (const uint8_t*)in, n1, n2, n3,
                       (uint8_t*)out);
  else
    return fail(TP_EUNSUPPORTED, "t-transpose supports 1- and 4-byte elements");
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int gather_slices(const void* in, int elem_bytes, int64_t in_cols, int64_t n3, const int32_t* ridx,
                  const int32_t* cidx, const int64_t* count, int64_t rows, int64_t cols, void* out, hipStream_t st) {
  const int64_t n = rows * cols * n3;
  if (n == 0) return TP_OK;
  if (elem_bytes == 4)
    hipLaunchKernelGGL(gather_slices_kernel<float>, dim3(nblk(n)), dim3(256), 0, st, (const float*)in, in_cols, n3,
                       ridx, cidx, count, rows, cols, (float*)out);
  else if (elem_bytes == 1)
    hipLaunchKernelGGL(gather_slices_kernel<uint8_t>, dim3(nblk(n)), dim3(256), 0, st, (const uint8_t*)in, in_cols,
                       n3, ridx, cidx, count, rows, cols, (uint8_t*)out);
  else
    return fail(TP_EUNSUPPORTED, "slice gather supports 1- and 4-byte elements");
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
