// Per-Fourier-slice complex matrix products (the slice loops of Algorithms
// 1 and 2, and the Fourier-domain products of Algorithms 3-5).
//
// Spectra are planar (separate re / im arrays, slice-major). Every slice k
// is an independent product C_k = op(A_k) op(B_k); slices 0 and, for even
// tube length, the Nyquist slice are real and skip the imaginary work.
//
// This file holds the general kernel (any op, any size, float or double,
// LDS-tiled on the vector ALUs) and the dispatch. The matrix-core kernels
// live in gemm_f32.hip (float32 arithmetic), gemm_mfma.hip (split bf16),
// gemm_short.hip (short contractions) and gemm_tall.hip (narrow results).
#include <algorithm>

#include "common.hpp"

namespace tp {
int cgemm_mfma(const CGemm& p, int prec, hipStream_t st, bool* handled);
int cgemm_short(const CGemm& p, int split, hipStream_t st, bool* handled);
int cgemm_tall(const CGemm& p, int split, hipStream_t st, bool* handled);
int cgemm_f32mfma(const CGemm& p, hipStream_t st, bool* handled);

namespace {

constexpr int BK = 16, NT = 256;

struct GemmArgs {
  int64_t M, N, Kd;
  const void *are, *aim, *bre, *bim;
  void *cre, *cim;
  int64_t lda, ldb, ldc, sa, sb, sc;
  int op_a, op_b;
  int64_t K;
  int real_last;
  const int64_t* kdim_dev;
};

// BM x BN tile per workgroup, 4 x 4 outputs per thread (rows ty + TY i,
// columns tx + TX j with TY = BM / 4, TX = BN / 4): 64 x 64 in general,
// 128 x 32 for products with at most 32 columns (the range-finder sketches)
// so that no thread computes columns past the end.
template <typename T, int BM, int BN>
__global__ __launch_bounds__(NT) void cgemm_simt_kernel(GemmArgs g) {
  constexpr int TY = BM / 4, TX = BN / 4;
  static_assert(TY * TX == NT, "4 x 4 outputs per thread");
  __shared__ T As_re[BK][BM + 1], As_im[BK][BM + 1];
  __shared__ T Bs_re[BK][BN + 1], Bs_im[BK][BN + 1];
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int64_t k = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const bool real = (k == 0) || (g.real_last && k == g.K - 1);
  int64_t Kd = g.Kd;
  if (g.kdim_dev) {
    const int64_t lim = *g.kdim_dev;
    Kd = lim < Kd ? (lim < 0 ? 0 : lim) : Kd;
  }
  const T* are = (const T*)g.are + k * g.sa;
  const T* aim = (const T*)g.aim + k * g.sa;
  const T* bre = (const T*)g.bre + k * g.sb;
  const T* bim = (const T*)g.bim + k * g.sb;

  T cr[4][4], ci[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) cr[i][j] = ci[i][j] = T(0);

  // the next k step's tile values are loaded into registers while the
  // current one is consumed from LDS
  constexpr int RA = (BM * BK) / NT, RB = (BN * BK) / NT;
  T ra_r[RA], ra_i[RA], rb_r[RB], rb_i[RB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int mm, kk;
      if (g.op_a == 0) {
        kk = tid % BK;
        mm = tid / BK + r * (NT / BK);
      } else {
        mm = tid % BM;
        kk = tid / BM + r * (NT / BM);
      }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      T vr = T(0), vi = T(0);
      if (gm < g.M && gk < Kd) {
        const int64_t off = g.op_a == 0 ? gm * g.lda + gk : gk * g.lda + gm;
        vr = are[off];
        if (!real) vi = g.op_a == 0 ? aim[off] : -aim[off];
      }
      ra_r[r] = vr;
      ra_i[r] = vi;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int nn, kk;
      if (g.op_b == 0) {
        nn = tid % BN;
        kk = tid / BN + r * (NT / BN);
      } else {
        kk = tid % BK;
        nn = tid / BK + r * (NT / BK);
      }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      T vr = T(0), vi = T(0);
      if (gn < g.N && gk < Kd) {
        const int64_t off = g.op_b == 0 ? gk * g.ldb + gn : gn * g.ldb + gk;
        vr = bre[off];
        if (!real) vi = g.op_b == 0 ? bim[off] : -bim[off];
      }
      rb_r[r] = vr;
      rb_i[r] = vi;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int mm, kk;
      if (g.op_a == 0) {
        kk = tid % BK;
        mm = tid / BK + r * (NT / BK);
      } else {
        mm = tid % BM;
        kk = tid / BM + r * (NT / BM);
      }
      As_re[kk][mm] = ra_r[r];
      As_im[kk][mm] = ra_i[r];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int nn, kk;
      if (g.op_b == 0) {
        nn = tid % BN;
        kk = tid / BN + r * (NT / BN);
      } else {
        kk = tid % BK;
        nn = tid / BK + r * (NT / BK);
      }
      Bs_re[kk][nn] = rb_r[r];
      Bs_im[kk][nn] = rb_i[r];
    }
  };

  if (Kd > 0) load(0);
  for (int64_t k0 = 0; k0 < Kd; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < Kd) load(k0 + BK);
    if (real) {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        T a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As_re[kk][ty + TY * i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs_re[kk][tx + TX * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) cr[i][j] += a[i] * b[j];
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        T ar[4], ai[4], br[4], bi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ar[i] = As_re[kk][ty + TY * i];
          ai[i] = As_im[kk][ty + TY * i];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          br[j] = Bs_re[kk][tx + TX * j];
          bi[j] = Bs_im[kk][tx + TX * j];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cr[i][j] += ar[i] * br[j] - ai[i] * bi[j];
            ci[i][j] += ar[i] * bi[j] + ai[i] * br[j];
          }
      }
    }
    __syncthreads();
  }
  T* cre = (T*)g.cre + k * g.sc;
  T* cim = (T*)g.cim + k * g.sc;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gm = m0 + ty + TY * i;
    if (gm >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gn = n0 + tx + TX * j;
      if (gn >= g.N) continue;
      cre[gm * g.ldc + gn] = cr[i][j];
      cim[gm * g.ldc + gn] = real ? T(0) : ci[i][j];
    }
  }
}

}  // namespace

// Most launches put the Fourier slices on a grid dimension that holds at
// most 65,535 values. Longer spectra (tubes above 131,070) are taken in
// chunks of that many slices. Every kernel treats slice 0 of its launch as
// the real DC slice, so a chunk after the first starts one slice early: that
// slice comes out wrong (imaginary part dropped) and is then recomputed by
// the preceding chunk, which runs later because the chunks are enqueued
// last first.
constexpr int64_t kLaunchSlices = 65535;

int cgemm(const CGemm& p, int dtype, int prec, hipStream_t st) {
  if (p.K == 0 || p.M == 0 || p.N == 0) return TP_OK;
  if (p.K > kLaunchSlices) {
    const size_t es = dtype == TP_F64 ? 8 : 4;
    const int64_t step = kLaunchSlices - 1;
    const int64_t nlater = (p.K - kLaunchSlices + step - 1) / step;
    for (int64_t c = nlater; c >= 0; --c) {
      const int64_t lo = c == 0 ? 0 : kLaunchSlices + (c - 1) * step - 1;
      const int64_t hi = c == 0 ? kLaunchSlices : std::min(p.K, kLaunchSlices + c * step);
      CGemm q = p;
      q.K = hi - lo;
      q.are = (const char*)p.are + lo * p.sa * es;
      q.aim = (const char*)p.aim + lo * p.sa * es;
      q.bre = (const char*)p.bre + lo * p.sb * es;
      q.bim = (const char*)p.bim + lo * p.sb * es;
      q.cre = (char*)p.cre + lo * p.sc * es;
      q.cim = (char*)p.cim + lo * p.sc * es;
      q.real_last = p.real_last && hi == p.K;
      if (int rc = cgemm(q, dtype, prec, st)) return rc;
    }
    return TP_OK;
  }
  if (dtype == TP_F32 && (prec == TP_PREC_F32 || prec == TP_PREC_BF16X3)) {
    const int split = prec == TP_PREC_BF16X3 ? 1 : 0;
    bool handled = false;
    // narrow results with a long contraction (range-finder products)
    if (int rc = cgemm_tall(p, split, st, &handled)) return rc;
    if (handled) return TP_OK;
    // short contractions: output-bound kernel on the matrix cores
    if (int rc = cgemm_short(p, split, st, &handled)) return rc;
    if (handled) return TP_OK;
  }
  if (dtype == TP_F32 && prec == TP_PREC_F32) {
    // large float32 products on the float32 matrix cores
    bool handled = false;
    if (int rc = cgemm_f32mfma(p, st, &handled)) return rc;
    if (handled) return TP_OK;
  }
  if (dtype == TP_F32 && prec != TP_PREC_F64) {
    bool handled = false;
    if (int rc = cgemm_mfma(p, prec, st, &handled)) return rc;
    if (handled) return TP_OK;
  }
  GemmArgs g{p.M, p.N, p.Kd, p.are, p.aim, p.bre, p.bim, p.cre, p.cim, p.lda, p.ldb, p.ldc,
             p.sa, p.sb, p.sc, p.op_a, p.op_b, p.K, p.real_last ? 1 : 0, p.kdim_dev};
  if (p.K > 65535) return fail(TP_EUNSUPPORTED, "more than 65535 Fourier slices");
  const bool narrow = p.N <= 32;
  const int64_t bm = narrow ? 128 : 64, bn = narrow ? 32 : 64;
  dim3 grid((unsigned)((p.N + bn - 1) / bn), (unsigned)((p.M + bm - 1) / bm), (unsigned)p.K);
  if (dtype == TP_F64) {
    if (narrow)
      hipLaunchKernelGGL((cgemm_simt_kernel<double, 128, 32>), grid, dim3(NT), 0, st, g);
    else
      hipLaunchKernelGGL((cgemm_simt_kernel<double, 64, 64>), grid, dim3(NT), 0, st, g);
  } else {
    if (narrow)
      hipLaunchKernelGGL((cgemm_simt_kernel<float, 128, 32>), grid, dim3(NT), 0, st, g);
    else
      hipLaunchKernelGGL((cgemm_simt_kernel<float, 64, 64>), grid, dim3(NT), 0, st, g);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
