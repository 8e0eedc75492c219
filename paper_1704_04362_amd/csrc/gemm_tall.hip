// Per-slice complex products with a narrow result: C_k = op(A_k) B_k with
// at most 64 columns and a long contraction, op = identity or conjugate
// transpose. These are the range-finder products of the randomized t-SVD
// and of the leverage estimates in t-CUR (Algorithms 4 and 5): Y = X Omega,
// Z = X^H Q and the projections, with X a full Fourier slice and Omega / Q
// a few dozen columns wide. Float32 products run on the float32 matrix cores
// (v_mfma_f32_16x16x4f32); split-precision products keep
// hi*hi + hi*lo + lo*hi of bf16 parts (v_mfma_f32_16x16x32_bf16), float32
// accumulation in both.
//
// Tiling: a 256-thread workgroup owns 64 rows x NB (32 or 64) columns of
// one Fourier slice and walks the contraction in 32-deep steps; wavefront w
// owns rows 16 w .. 16 w + 15 and all NB columns. A step's A and B tiles are
// staged in LDS (two buffers) and the next step's values are loaded into
// registers while the current step is on the matrix cores.
#include "common.hpp"

namespace tp {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, KB = 32, TT = 256;

struct TArgs {
  int64_t M, N, Kd;
  const float *are, *aim, *bre, *bim;
  float *cre, *cim;
  int64_t lda, ldb, ldc, sa, sb, sc;
  int64_t K;
  int real_last;
  const int64_t* kdim_dev;
};

__device__ __forceinline__ bf16x8 bneg(bf16x8 x) {
  u32x4 u = __builtin_bit_cast(u32x4, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

// Loader of one 32-deep step into registers. A values: entry u of the
// thread is (m, kk) with, for op = N, m = e / KB, kk = e % KB (rows of A
// read along k) and, for op = C, kk = e / TM, m = e % TM (rows of A^stored
// read along m), e = tid + TT u. B values: (kk, n) = (e / NB, e % NB).
template <int OPA, int NB>
struct StepLoad {
  static constexpr int RA = TM * KB / TT, RB = KB * NB / TT;
  float ar[RA], ai[RA], br[RB], bi[RB];

  __device__ __forceinline__ static void a_index(int e, int& m, int& kk) {
    if (OPA == 0) {
      m = e / KB;
      kk = e % KB;
    } else {
      kk = e / TM;
      m = e % TM;
    }
  }

  __device__ __forceinline__ void load(const TArgs& g, const float* are, const float* aim, const float* bre,
                                       const float* bim, int64_t m0, int64_t k0, int64_t kd, bool real, int tid) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      int m, kk;
      a_index(tid + TT * u, m, kk);
      const int64_t gm = m0 + m, gk = k0 + kk;
      const bool in = gm < g.M && gk < kd;
      const int64_t off = OPA == 0 ? gm * g.lda + gk : gk * g.lda + gm;
      ar[u] = in ? are[off] : 0.f;
      const float v = (in && !real) ? aim[off] : 0.f;
      ai[u] = OPA == 0 ? v : -v;  // conjugate for op = C
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int e = tid + TT * u, kk = e / NB, n = e % NB;
      const int64_t gk = k0 + kk;
      const bool in = n < g.N && gk < kd;
      br[u] = in ? bre[gk * g.ldb + n] : 0.f;
      bi[u] = (in && !real) ? bim[gk * g.ldb + n] : 0.f;
    }
  }
};

__device__ __forceinline__ int64_t tall_kd(const TArgs& g) {
  int64_t kd = g.Kd;
  if (g.kdim_dev) {
    const int64_t lim = *g.kdim_dev;
    kd = lim < kd ? (lim < 0 ? 0 : lim) : kd;
  }
  return kd;
}

// lane (gq, c) holds C[m0 + 16 w + 4 gq + v][16 nt + c], v = 0..3
template <int NB>
__device__ __forceinline__ void tall_store(const TArgs& g, int64_t k, int64_t m0, int wave, int gq, int c,
                                           const f32x4 (&cr)[NB / 16], const f32x4 (&ci)[NB / 16], bool real) {
  float* cre = g.cre + k * g.sc;
  float* cim = g.cim + k * g.sc;
#pragma unroll
  for (int nt = 0; nt < NB / 16; ++nt) {
    const int64_t n = 16 * nt + c;
    if (n >= g.N) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t m = m0 + 16 * wave + 4 * gq + v;
      if (m < g.M) {
        cre[m * g.ldc + n] = cr[nt][v];
        cim[m * g.ldc + n] = real ? 0.f : ci[nt][v];
      }
    }
  }
}

// float32 matrix cores. LDS holds A^T (k rows, m contiguous; column m of
// row kk at m ^ ((kk >> 2) & 15)) and B (k rows, n contiguous).
template <int OPA, int NB>
__global__ __launch_bounds__(TT) void cgemm_tall_kernel(TArgs g) {
  constexpr int LDA = TM + 16, LDB = NB + 16, NTL = NB / 16;
  __shared__ float as[2][2][KB][LDA];
  __shared__ float bs[2][2][KB][LDB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gq = lane >> 4, c = lane & 15;
  const int64_t k = blockIdx.z, m0 = (int64_t)blockIdx.y * TM;
  const bool real = (k == 0) || (g.real_last && k == g.K - 1);
  const int64_t kd = tall_kd(g);
  const float* are = g.are + k * g.sa;
  const float* aim = g.aim + k * g.sa;
  const float* bre = g.bre + k * g.sb;
  const float* bim = g.bim + k * g.sb;
  using L = StepLoad<OPA, NB>;
  L ld;
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < L::RA; ++u) {
      int m, kk;
      L::a_index(tid + TT * u, m, kk);
      const int ms = m ^ ((kk >> 2) & 15);
      as[b][0][kk][ms] = ld.ar[u];
      as[b][1][kk][ms] = ld.ai[u];
    }
#pragma unroll
    for (int u = 0; u < L::RB; ++u) {
      const int e = tid + TT * u, kk = e / NB, n = e % NB;
      bs[b][0][kk][n] = ld.br[u];
      bs[b][1][kk][n] = ld.bi[u];
    }
  };
  f32x4 cr[NTL], ci[NTL];
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt) cr[nt] = ci[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nsteps = (kd + KB - 1) / KB;
  if (nsteps > 0) {
    ld.load(g, are, aim, bre, bim, m0, 0, kd, real, tid);
    put(0);
    __syncthreads();
  }
  for (int64_t st = 0; st < nsteps; ++st) {
    const int b = (int)(st & 1);
    if (st + 1 < nsteps) ld.load(g, are, aim, bre, bim, m0, (st + 1) * KB, kd, real, tid);
#pragma unroll
    for (int s = 0; s < KB / 4; ++s) {
      const int kk = 4 * s + gq;
      const int ms = (16 * wave + c) ^ ((kk >> 2) & 15);
      const float xr = as[b][0][kk][ms], xi = as[b][1][kk][ms];
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        const float yr = bs[b][0][kk][16 * nt + c], yi = bs[b][1][kk][16 * nt + c];
        // Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br
        cr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, yr, cr[nt], 0, 0, 0);
        cr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-xi, yi, cr[nt], 0, 0, 0);
        ci[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, yi, ci[nt], 0, 0, 0);
        ci[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yr, ci[nt], 0, 0, 0);
      }
    }
    if (st + 1 < nsteps) put(b ^ 1);
    __syncthreads();
  }
  tall_store<NB>(g, k, m0, wave, gq, c, cr, ci, real);
}

// Split bf16 matrix cores. LDS holds the four planes (hi re, lo re, hi im,
// lo im) of A as [m][k] and of B^T as [n][k], k contiguous, so that a lane
// reads its 8 consecutive k values of a 32-deep step with one 16-byte read.
template <int OPA, int NB>
__global__ __launch_bounds__(TT) void cgemm_tall_split_kernel(TArgs g) {
  // 96-byte rows (32 mod 64): the 16-byte fragment reads are free of bank conflicts
  constexpr int LK = KB + 16, NTL = NB / 16;
  __shared__ __align__(16) __bf16 as[2][4][TM][LK];
  __shared__ __align__(16) __bf16 bs[2][4][NB][LK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gq = lane >> 4, c = lane & 15;
  const int64_t k = blockIdx.z, m0 = (int64_t)blockIdx.y * TM;
  const bool real = (k == 0) || (g.real_last && k == g.K - 1);
  const int64_t kd = tall_kd(g);
  const float* are = g.are + k * g.sa;
  const float* aim = g.aim + k * g.sa;
  const float* bre = g.bre + k * g.sb;
  const float* bim = g.bim + k * g.sb;
  using L = StepLoad<OPA, NB>;
  L ld;
  auto split_put = [](__bf16* hi, __bf16* lo, float x) {
    const __bf16 h = (__bf16)x;
    *hi = h;
    *lo = (__bf16)(x - (float)h);
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < L::RA; ++u) {
      int m, kk;
      L::a_index(tid + TT * u, m, kk);
      split_put(&as[b][0][m][kk], &as[b][1][m][kk], ld.ar[u]);
      split_put(&as[b][2][m][kk], &as[b][3][m][kk], ld.ai[u]);
    }
#pragma unroll
    for (int u = 0; u < L::RB; ++u) {
      const int e = tid + TT * u, kk = e / NB, n = e % NB;
      split_put(&bs[b][0][n][kk], &bs[b][1][n][kk], ld.br[u]);
      split_put(&bs[b][2][n][kk], &bs[b][3][n][kk], ld.bi[u]);
    }
  };
  f32x4 cr[NTL], ci[NTL];
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt) cr[nt] = ci[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nsteps = (kd + KB - 1) / KB;
  if (nsteps > 0) {
    ld.load(g, are, aim, bre, bim, m0, 0, kd, real, tid);
    put(0);
    __syncthreads();
  }
  for (int64_t st = 0; st < nsteps; ++st) {
    const int b = (int)(st & 1);
    if (st + 1 < nsteps) ld.load(g, are, aim, bre, bim, m0, (st + 1) * KB, kd, real, tid);
    const int row = 16 * wave + c, col = 8 * gq;
    const bf16x8 arh = *reinterpret_cast<const bf16x8*>(&as[b][0][row][col]);
    const bf16x8 arl = *reinterpret_cast<const bf16x8*>(&as[b][1][row][col]);
    const bf16x8 aih = *reinterpret_cast<const bf16x8*>(&as[b][2][row][col]);
    const bf16x8 ail = *reinterpret_cast<const bf16x8*>(&as[b][3][row][col]);
    const bf16x8 nih = bneg(aih), nil = bneg(ail);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      const int n = 16 * nt + c;
      const bf16x8 brh = *reinterpret_cast<const bf16x8*>(&bs[b][0][n][col]);
      const bf16x8 brl = *reinterpret_cast<const bf16x8*>(&bs[b][1][n][col]);
      const bf16x8 bih = *reinterpret_cast<const bf16x8*>(&bs[b][2][n][col]);
      const bf16x8 bil = *reinterpret_cast<const bf16x8*>(&bs[b][3][n][col]);
      // Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br (three split terms each)
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brh, cr[nt], 0, 0, 0);
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brl, cr[nt], 0, 0, 0);
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, brh, cr[nt], 0, 0, 0);
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, bih, cr[nt], 0, 0, 0);
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, bil, cr[nt], 0, 0, 0);
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, bih, cr[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bih, ci[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bil, ci[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bih, ci[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brh, ci[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brl, ci[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, brh, ci[nt], 0, 0, 0);
    }
    if (st + 1 < nsteps) put(b ^ 1);
    __syncthreads();
  }
  tall_store<NB>(g, k, m0, wave, gq, c, cr, ci, real);
}

template <int OPA, int NB>
void launch_tall(const TArgs& g, int split, dim3 grid, hipStream_t st) {
  if (split)
    hipLaunchKernelGGL((cgemm_tall_split_kernel<OPA, NB>), grid, dim3(TT), 0, st, g);
  else
    hipLaunchKernelGGL((cgemm_tall_kernel<OPA, NB>), grid, dim3(TT), 0, st, g);
}

}  // namespace

// Takes float32 products C_k = op(A_k) B_k (op_b = N) with at most 64
// result columns (any contraction length), in float32 (split = 0)
// or split bf16 (split = 1); *handled says whether it did.
int cgemm_tall(const CGemm& p, int split, hipStream_t st, bool* handled) {
  *handled = false;
  if (p.op_b != 0 || p.N < 1 || p.N > 64 || p.Kd < 1 || p.M < 32) return TP_OK;
  if (p.K > 65535 || (p.M + TM - 1) / TM > 65535) return TP_OK;
  TArgs g{p.M, p.N, p.Kd, (const float*)p.are, (const float*)p.aim, (const float*)p.bre, (const float*)p.bim,
          (float*)p.cre, (float*)p.cim, p.lda, p.ldb, p.ldc, p.sa, p.sb, p.sc, p.K, p.real_last ? 1 : 0,
          p.kdim_dev};
  const dim3 grid(1u, (unsigned)((p.M + TM - 1) / TM), (unsigned)p.K);
  if (p.op_a == 0) {
    if (p.N <= 32)
      launch_tall<0, 32>(g, split, grid, st);
    else
      launch_tall<0, 64>(g, split, grid, st);
  } else {
    if (p.N <= 32)
      launch_tall<1, 32>(g, split, grid, st);
    else
      launch_tall<1, 64>(g, split, grid, st);
  }
  TP_LAUNCH_CHECK();
  *handled = true;
  return TP_OK;
}

}  // namespace tp
