// Per-slice complex products with a short contraction (at most 64): the
// reconstruction of the t-CUR approximation (Algorithm 5),
// Zhat_k = (Chat_k P_k)(U_k^H Rhat_k) with an r-deep contraction, and any
// other float32 slice product of that shape. Such a product writes
// 8 M N bytes per slice and reads a few percent of that, so it is bound
// by the output stream. The arithmetic runs on the float32 matrix cores
// (v_mfma_f32_16x16x4f32) for float32 products and on the bf16 matrix cores
// with split operands (three bf16 products per real product) for the
// split precision.
//
// Tiling: a 256-thread workgroup owns a 256 x 128 output block of one
// Fourier slice, walked as four 64-row tiles; wavefront w owns columns
// 32 w .. 32 w + 31 (2 matrix-core tiles of 16 across, 4 down per row tile).
// Each wavefront reads its own B columns once, straight from global memory
// into registers. The A tiles (64 rows x KP, KP = contraction rounded up to
// 8, or to 32 for split operands) are shared by the four wavefronts through
// two LDS buffers: the next one is loaded into registers while the current
// one is consumed. The tiles compute
// C^T = B^T A^T so that a lane ends with four consecutive columns of one
// row of C and stores them with one 16-byte store; a row tile is stored as
// soon as it is complete, so its stores drain while the next one is on the
// matrix cores.
#include "common.hpp"

namespace tp {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int QM = 64, QN = 128, QT = 256;
constexpr int QMT = 4;  // row tiles of 64 per workgroup

struct QArgs {
  int64_t M, N, Kd;
  const float *are, *aim, *bre, *bim;
  float *cre, *cim;
  int64_t lda, ldb, ldc, sa, sb, sc;
  int64_t K;
  int real_last;
  int vec;  // 16-byte stores allowed (ldc, sc multiples of 4, aligned planes)
  const int64_t* kdim_dev;
};

// Stores the 16 x 32 strip of row tile mt held by a lane as C^T fragments:
// lane (gq, c) has C[m0 + 16 mt + c][n0 + 16 nt + 4 gq + v], v = 0..3.
__device__ __forceinline__ void store_strip(const QArgs& g, float* cre, float* cim, int64_t m, int64_t n0, int gq,
                                            const f32x4 (&vr)[2], const f32x4 (&vi)[2], bool real) {
  if (m >= g.M) return;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int64_t n = n0 + 16 * nt + 4 * gq;
    const f32x4 xr = vr[nt];
    const f32x4 xi = real ? f32x4{0.f, 0.f, 0.f, 0.f} : vi[nt];
    if (g.vec && n + 3 < g.N) {
      *reinterpret_cast<f32x4*>(cre + m * g.ldc + n) = xr;
      *reinterpret_cast<f32x4*>(cim + m * g.ldc + n) = xi;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (n + v < g.N) {
          cre[m * g.ldc + n + v] = xr[v];
          cim[m * g.ldc + n + v] = xi[v];
        }
    }
  }
}

__device__ __forceinline__ int64_t eff_kd(const QArgs& g) {
  int64_t kd = g.Kd;
  if (g.kdim_dev) {
    const int64_t lim = *g.kdim_dev;
    kd = lim < kd ? (lim < 0 ? 0 : lim) : kd;
  }
  return kd;
}

// float32 matrix cores (TP_PREC_F32 and any product that asks for float32)
template <int KP>
__global__ __launch_bounds__(QT) void cgemm_short_kernel(QArgs g) {
  static_assert(KP % 8 == 0 && KP <= 64, "contraction padded to a multiple of 8");
  constexpr int LDM = QM + 16;        // padded row of the transposed A tile
  constexpr int NS = KP / 4;           // matrix-core k steps
  constexpr int RA = QM * KP / QT;     // A values per thread and plane
  __shared__ float atr[2][KP][LDM], ati[2][KP][LDM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gq = lane >> 4, c = lane & 15;
  const int64_t k = blockIdx.z;
  const int64_t mbase = (int64_t)blockIdx.y * (QM * QMT), n0 = (int64_t)blockIdx.x * QN + 32 * wave;
  const bool real = (k == 0) || (g.real_last && k == g.K - 1);
  const int64_t kd = eff_kd(g);
  const float* are = g.are + k * g.sa;
  const float* aim = g.aim + k * g.sa;
  const float* bre = g.bre + k * g.sb;
  const float* bim = g.bim + k * g.sb;
  // B fragments, loaded once for all row tiles: lane (gq, c) of tile nt at
  // step s holds B[4 s + gq][n0 + 16 nt + c]
  float br[NS][2], bi[NS][2];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int64_t kk = 4 * s + gq, n = n0 + 16 * nt + c;
      const bool in = kk < kd && n < g.N;
      br[s][nt] = in ? bre[kk * g.ldb + n] : 0.f;
      bi[s][nt] = (in && !real) ? bim[kk * g.ldb + n] : 0.f;
    }
  // A tiles: thread value u is entry e = tid + QT u of the 64 x KP tile
  float pr[RA], pi[RA];
  auto load_a = [&](int64_t m0) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int e = tid + QT * u, m = e / KP, kk = e - m * KP;
      const bool in = kk < kd && m0 + m < g.M;
      pr[u] = in ? are[(m0 + m) * g.lda + kk] : 0.f;
      pi[u] = (in && !real) ? aim[(m0 + m) * g.lda + kk] : 0.f;
    }
  };
  // transposed and swizzled: at[kk][m ^ sw(kk)] = A[m0 + m][kk]
  auto put_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int e = tid + QT * u, m = e / KP, kk = e - m * KP;
      const int ms = m ^ ((kk >> 1) & 15);
      atr[buf][kk][ms] = pr[u];
      ati[buf][kk][ms] = pi[u];
    }
  };
  const int nmt = (int)((g.M - mbase + QM - 1) / QM) < QMT ? (int)((g.M - mbase + QM - 1) / QM) : QMT;
  load_a(mbase);
  put_a(0);
  __syncthreads();
  float* cre = g.cre + k * g.sc;
  float* cim = g.cim + k * g.sc;
  for (int t = 0; t < nmt; ++t) {
    const int buf = t & 1;
    const int64_t m0 = mbase + (int64_t)t * QM;
    if (t + 1 < nmt) load_a(m0 + QM);
    // one 16-row strip at a time, stored as soon as it is complete so that
    // its stores drain while the next strip is on the matrix cores
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 cr[2], ci[2];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) cr[nt] = ci[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int kk = 4 * s + gq, cs = c ^ ((kk >> 1) & 15);
        const float ar = atr[buf][kk][16 * mt + cs], ai = ati[buf][kk][16 * mt + cs];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          // C^T tile += B^T A^T: Re = Br Ar - Bi Ai, Im = Br Ai + Bi Ar
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[s][nt], ar, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-bi[s][nt], ai, cr[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[s][nt], ai, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bi[s][nt], ar, ci[nt], 0, 0, 0);
        }
      }
      store_strip(g, cre, cim, m0 + 16 * mt + c, n0, gq, cr, ci, real);
    }
    if (t + 1 < nmt) put_a(buf ^ 1);
    __syncthreads();
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 bneg(bf16x8 x) {
  u32x4 u = __builtin_bit_cast(u32x4, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

// Split bf16 matrix cores (TP_PREC_BF16X3): every float32 value x is
// hi + lo with hi = bf16(x) and lo = bf16(x - hi); a real product keeps
// hi*hi + hi*lo + lo*hi (v_mfma_f32_16x16x32_bf16, float32 accumulation).
// An A tile is staged split in LDS, [plane][m][k] with planes hi re,
// lo re, hi im, lo im; lane (gq, c) of a 32-deep step reads the 8
// consecutive k values 8 gq .. 8 gq + 7 of row 16 mt + c.
template <int KP>
__global__ __launch_bounds__(QT) void cgemm_short_split_kernel(QArgs g) {
  static_assert(KP % 32 == 0 && KP <= 64, "contraction padded to a multiple of 32");
  constexpr int LDK = KP + 16;  // row bytes 2 LDK = 32 mod 64: conflict-free 16-byte fragment reads
  constexpr int NS = KP / 32;
  constexpr int RA = QM * KP / QT;
  __shared__ __align__(16) __bf16 as[2][4][QM][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gq = lane >> 4, c = lane & 15;
  const int64_t k = blockIdx.z;
  const int64_t mbase = (int64_t)blockIdx.y * (QM * QMT), n0 = (int64_t)blockIdx.x * QN + 32 * wave;
  const bool real = (k == 0) || (g.real_last && k == g.K - 1);
  const int64_t kd = eff_kd(g);
  const float* are = g.are + k * g.sa;
  const float* aim = g.aim + k * g.sa;
  const float* bre = g.bre + k * g.sb;
  const float* bim = g.bim + k * g.sb;
  // B^T fragments, split once for all row tiles: lane (gq, c) of tile nt at
  // step s holds B[32 s + 8 gq + j][n0 + 16 nt + c], j = 0..7
  bf16x8 brh[NS][2], brl[NS][2], bih[NS][2], bil[NS][2];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int64_t n = n0 + 16 * nt + c;
      float xr[8], xi[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t kk = 32 * s + 8 * gq + j;
        const bool in = kk < kd && n < g.N;
        xr[j] = in ? bre[kk * g.ldb + n] : 0.f;
        xi[j] = (in && !real) ? bim[kk * g.ldb + n] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const __bf16 h = (__bf16)xr[j], h2 = (__bf16)xi[j];
        brh[s][nt][j] = h;
        brl[s][nt][j] = (__bf16)(xr[j] - (float)h);
        bih[s][nt][j] = h2;
        bil[s][nt][j] = (__bf16)(xi[j] - (float)h2);
      }
    }
  float pr[RA], pi[RA];
  auto load_a = [&](int64_t m0) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int e = tid + QT * u, m = e / KP, kk = e - m * KP;
      const bool in = kk < kd && m0 + m < g.M;
      pr[u] = in ? are[(m0 + m) * g.lda + kk] : 0.f;
      pi[u] = (in && !real) ? aim[(m0 + m) * g.lda + kk] : 0.f;
    }
  };
  auto put_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int e = tid + QT * u, m = e / KP, kk = e - m * KP;
      const __bf16 hr = (__bf16)pr[u], hi = (__bf16)pi[u];
      as[buf][0][m][kk] = hr;
      as[buf][1][m][kk] = (__bf16)(pr[u] - (float)hr);
      as[buf][2][m][kk] = hi;
      as[buf][3][m][kk] = (__bf16)(pi[u] - (float)hi);
    }
  };
  const int nmt = (int)((g.M - mbase + QM - 1) / QM) < QMT ? (int)((g.M - mbase + QM - 1) / QM) : QMT;
  load_a(mbase);
  put_a(0);
  __syncthreads();
  float* cre = g.cre + k * g.sc;
  float* cim = g.cim + k * g.sc;
  for (int t = 0; t < nmt; ++t) {
    const int buf = t & 1;
    const int64_t m0 = mbase + (int64_t)t * QM;
    if (t + 1 < nmt) load_a(m0 + QM);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 cr[2], ci[2];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) cr[nt] = ci[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int row = 16 * mt + c, col = 32 * s + 8 * gq;
        const bf16x8 arh = *reinterpret_cast<const bf16x8*>(&as[buf][0][row][col]);
        const bf16x8 arl = *reinterpret_cast<const bf16x8*>(&as[buf][1][row][col]);
        const bf16x8 aih = *reinterpret_cast<const bf16x8*>(&as[buf][2][row][col]);
        const bf16x8 ail = *reinterpret_cast<const bf16x8*>(&as[buf][3][row][col]);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const bf16x8 nih = bneg(bih[s][nt]), nil = bneg(bil[s][nt]);
          // Re^T = Br^T Ar^T - Bi^T Ai^T, Im^T = Br^T Ai^T + Bi^T Ar^T
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(brh[s][nt], arh, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(brh[s][nt], arl, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(brl[s][nt], arh, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, aih, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, ail, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, aih, cr[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(brh[s][nt], aih, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(brh[s][nt], ail, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(brl[s][nt], aih, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bih[s][nt], arh, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bih[s][nt], arl, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bil[s][nt], arh, ci[nt], 0, 0, 0);
        }
      }
      store_strip(g, cre, cim, m0 + 16 * mt + c, n0, gq, cr, ci, real);
    }
    if (t + 1 < nmt) put_a(buf ^ 1);
    __syncthreads();
  }
}

}  // namespace

// Takes float32 products C_k = A_k B_k (no transposes) with a contraction of
// at most 64 and at least 64 x 64 outputs per slice, in float32 (split = 0)
// or split bf16 (split = 1); *handled says whether it did.
int cgemm_short(const CGemm& p, int split, hipStream_t st, bool* handled) {
  *handled = false;
  if (p.op_a != 0 || p.op_b != 0) return TP_OK;
  if (p.Kd < 1 || p.Kd > 64 || p.M < 64 || p.N < 64) return TP_OK;
  if (p.K > 65535 || (p.M + QM - 1) / QM > 65535) return TP_OK;
  const uintptr_t al = reinterpret_cast<uintptr_t>(p.cre) | reinterpret_cast<uintptr_t>(p.cim);
  QArgs g{p.M, p.N, p.Kd, (const float*)p.are, (const float*)p.aim, (const float*)p.bre, (const float*)p.bim,
          (float*)p.cre, (float*)p.cim, p.lda, p.ldb, p.ldc, p.sa, p.sb, p.sc, p.K, p.real_last ? 1 : 0,
          (al % 16 == 0 && p.ldc % 4 == 0 && p.sc % 4 == 0) ? 1 : 0, p.kdim_dev};
  const dim3 grid((unsigned)((p.N + QN - 1) / QN), (unsigned)((p.M + QM * QMT - 1) / (QM * QMT)), (unsigned)p.K);
  if (split) {
    if (p.Kd <= 32)
      hipLaunchKernelGGL(cgemm_short_split_kernel<32>, grid, dim3(QT), 0, st, g);
    else
      hipLaunchKernelGGL(cgemm_short_split_kernel<64>, grid, dim3(QT), 0, st, g);
  } else {
    switch ((p.Kd + 7) / 8) {
      case 1: hipLaunchKernelGGL(cgemm_short_kernel<8>, grid, dim3(QT), 0, st, g); break;
      case 2: hipLaunchKernelGGL(cgemm_short_kernel<16>, grid, dim3(QT), 0, st, g); break;
      case 3: hipLaunchKernelGGL(cgemm_short_kernel<24>, grid, dim3(QT), 0, st, g); break;
      case 4: hipLaunchKernelGGL(cgemm_short_kernel<32>, grid, dim3(QT), 0, st, g); break;
      case 5: hipLaunchKernelGGL(cgemm_short_kernel<40>, grid, dim3(QT), 0, st, g); break;
      case 6: hipLaunchKernelGGL(cgemm_short_kernel<48>, grid, dim3(QT), 0, st, g); break;
      case 7: hipLaunchKernelGGL(cgemm_short_kernel<56>, grid, dim3(QT), 0, st, g); break;
      default: hipLaunchKernelGGL(cgemm_short_kernel<64>, grid, dim3(QT), 0, st, g); break;
    }
  }
  TP_LAUNCH_CHECK();
  *handled = true;
  return TP_OK;
}

}  // namespace tp
