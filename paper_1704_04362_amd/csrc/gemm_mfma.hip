// Matrix-core kernels for the large per-slice complex products of
// Algorithms 1 and 2 (the Fourier-slice loop) on float32 spectra.
//
// Complex products use three real products (3M):
//   P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
//   Re C = P1 - P2, Im C = P3 - P1 - P2,
// and the two real slices (DC, Nyquist) use P1 alone.
//
// TP_PREC_BF16X3 splits every float32 operand value into bf16 hi + lo (round
// to nearest even; x - hi is exact in float32) and accumulates
// hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x32_bf16 in float32; the dropped
// lo*lo term is below 2^-16 of each product. TP_PREC_BF16 keeps hi*hi only.
//
// Tiling: a 256-thread workgroup owns a 128 x 128 tile of one Fourier slice;
// each of its four wavefronts owns 64 x 64 (4 x 4 MFMA tiles of 16 x 16,
// three accumulators each). Per 32-deep k step the workgroup reads the
// float32 planes of A (128 x 32) and B (32 x 128) with coalesced loads into
// registers (prefetched one step ahead), forms Ar+Ai / Br+Bi, splits, and
// stores bf16 planes k-contiguous in LDS (rows padded to 40 elements, which
// makes the 16-byte fragment reads conflict free). Every wavefront then reads
// its fragments with 16-byte LDS reads and issues 4 x 4 x 9 MFMAs.
#include <type_traits>

#include "common.hpp"

namespace tp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32, NT = 256;
constexpr int LDK = BK + 8;  // padded k-extent of an LDS row (bf16 elements)

struct MArgs {
  int64_t M, N, Kd;
  const float *are, *aim, *bre, *bim;
  float *cre, *cim;
  int64_t lda, ldb, ldc, sa, sb, sc;
  int64_t K;
  int real_last;
  const int64_t* kdim_dev;
};

template <int SPLIT>
struct Frag {
  bf16x8 v[SPLIT];
};

// Split 4 float32 values into bf16 hi (and lo) quads.
template <int SPLIT>
__device__ __forceinline__ void split4(const float (&x)[4], bf16x4& hi, bf16x4& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    if constexpr (SPLIT == 2) lo[e] = (__bf16)(x[e] - (float)h);
  }
}

template <int SPLIT, bool REAL>
__device__ __forceinline__ void cgemm_bf16_body(const MArgs& g, int64_t k, __bf16* sA, __bf16* sB) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  constexpr bool real = REAL;
  int64_t Kd = g.Kd;
  if (g.kdim_dev) {
    const int64_t lim = *g.kdim_dev;
    Kd = lim < Kd ? (lim < 0 ? 0 : lim) : Kd;
  }
  const float* are = g.are + k * g.sa;
  const float* aim = g.aim + k * g.sa;
  const float* bre = g.bre + k * g.sb;
  const float* bim = g.bim + k * g.sb;

  f32x4 acc[3][4][4];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[v][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // register staging of the next k step: A as 4 float4 per plane, B as
  // 4 k-quads of one column per plane
  float ra[2][4][4], rb[2][4][4];

  // offsets inside one slice are 32-bit (checked on the host), so the loads
  // use a scalar base with a 32-bit vector offset
  const uint32_t M = (uint32_t)g.M, N = (uint32_t)g.N, KdU = (uint32_t)Kd;
  const uint32_t lda = (uint32_t)g.lda, ldb = (uint32_t)g.ldb;
  // Loads are never predicated off: an address outside the live tile is
  // replaced by the slice origin (always valid) and its value is cleared at
  // LDS-store time with a bit mask, so no load sits under a branch or feeds
  // an instruction before the MFMA phase, and a step's loads stay in flight
  // together. A float4 at a column gk < Kd stays inside its row because rows
  // are padded to lda >= Kd with lda and gk multiples of 4.
  uint32_t amask = 0, bmask = 0;  // bit 4*j+e: element kept
  auto load_tile = [&](uint32_t k0) {
    amask = 0;
    bmask = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t f = tid + NT * j;
      const uint32_t gm = (uint32_t)m0 + (f >> 3), gk = k0 + 4 * (f & 7);
      const bool ok = gm < M && gk < KdU;
      const uint32_t off = ok ? gm * lda + gk : 0u;
      const float4 x = *reinterpret_cast<const float4*>(are + off);
      ra[0][j][0] = x.x; ra[0][j][1] = x.y; ra[0][j][2] = x.z; ra[0][j][3] = x.w;
      if constexpr (!REAL) {
        const float4 y = *reinterpret_cast<const float4*>(aim + off);
        ra[1][j][0] = y.x; ra[1][j][1] = y.y; ra[1][j][2] = y.z; ra[1][j][3] = y.w;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) amask |= (ok && gk + e < KdU) ? (1u << (4 * j + e)) : 0u;
    }
    const uint32_t gn = (uint32_t)n0 + (tid & 127);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t gk = k0 + 4 * ((tid >> 7) + 2 * j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool ok = gn < N && gk + e < KdU;
        const uint32_t off = ok ? (gk + e) * ldb + gn : 0u;
        rb[0][j][e] = bre[off];
        if constexpr (!REAL) rb[1][j][e] = bim[off];
        bmask |= ok ? (1u << (4 * j + e)) : 0u;
      }
    }
  };

  auto keep = [](float v, uint32_t mask, int bit) {
    return __uint_as_float(__float_as_uint(v) & (0u - ((mask >> bit) & 1u)));
  };
  auto put = [&](__bf16* base, int plane_rows, int v, int row, int kq, float x0, float x1, float x2, float x3) {
    const float x[4] = {x0, x1, x2, x3};
    bf16x4 hi, lo;
    split4<SPLIT>(x, hi, lo);
    *reinterpret_cast<bf16x4*>(&base[((v * SPLIT + 0) * plane_rows + row) * LDK + 4 * kq]) = hi;
    if constexpr (SPLIT == 2) *reinterpret_cast<bf16x4*>(&base[((v * SPLIT + 1) * plane_rows + row) * LDK + 4 * kq]) = lo;
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = tid + NT * j;
      const int row = f >> 3, kq = f & 7;
      float r[4], i[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        r[e] = keep(ra[0][j][e], amask, 4 * j + e);
        i[e] = REAL ? 0.f : keep(ra[1][j][e], amask, 4 * j + e);
      }
      put(sA, BM, 0, row, kq, r[0], r[1], r[2], r[3]);
      if constexpr (!REAL) {
        put(sA, BM, 1, row, kq, i[0], i[1], i[2], i[3]);
        put(sA, BM, 2, row, kq, r[0] + i[0], r[1] + i[1], r[2] + i[2], r[3] + i[3]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = tid & 127, kq = (tid >> 7) + 2 * j;
      float r[4], i[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        r[e] = keep(rb[0][j][e], bmask, 4 * j + e);
        i[e] = REAL ? 0.f : keep(rb[1][j][e], bmask, 4 * j + e);
      }
      put(sB, BN, 0, n, kq, r[0], r[1], r[2], r[3]);
      if constexpr (!REAL) {
        put(sB, BN, 1, n, kq, i[0], i[1], i[2], i[3]);
        put(sB, BN, 2, n, kq, r[0] + i[0], r[1] + i[1], r[2] + i[2], r[3] + i[3]);
      }
    }
  };

  const int64_t nsteps = (Kd + BK - 1) / BK;
  if (nsteps > 0) load_tile(0u);
  for (int64_t ks = 0; ks < nsteps; ++ks) {
    __syncthreads();
    store_tile();
    __syncthreads();
    if (ks + 1 < nsteps) load_tile((uint32_t)((ks + 1) * BK));
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    // one pass per carried value (r, i, s) with a compile-time index, so the
    // accumulators stay in registers
    auto pass = [&](auto vtag) {
      constexpr int v = decltype(vtag)::value;
      Frag<SPLIT> b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int sp = 0; sp < SPLIT; ++sp)
          b[j].v[sp] = *reinterpret_cast<const bf16x8*>(&sB[((v * SPLIT + sp) * BN + wc * 64 + j * 16 + fr) * LDK + fk]);
      Frag<SPLIT> a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int sp = 0; sp < SPLIT; ++sp)
          a[i].v[sp] = *reinterpret_cast<const bf16x8*>(&sA[((v * SPLIT + sp) * BM + wr * 64 + i * 16 + fr) * LDK + fk]);
      // one split term over all 16 tiles before the next, so consecutive
      // MFMAs never wait on each other's accumulator
#pragma unroll
      for (int term = 0; term < (SPLIT == 2 ? 3 : 1); ++term) {
        const int sa = term == 2 ? 1 : 0, sb = term == 1 ? 1 : 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[v][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i].v[sa], b[j].v[sb], acc[v][i][j], 0, 0, 0);
      }
    };
    pass(std::integral_constant<int, 0>{});
    if constexpr (!REAL) {
      pass(std::integral_constant<int, 1>{});
      pass(std::integral_constant<int, 2>{});
    }
  }

  // epilogue: lane holds rows 4*(lane/16)+e, column lane%16 of each 16x16 tile
  float* cre = g.cre + k * g.sc;
  float* cim = g.cim + k * g.sc;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gm = m0 + wr * 64 + i * 16 + 4 * (lane >> 4) + e;
        const int64_t gn = n0 + wc * 64 + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          const float p1 = acc[0][i][j][e];
          if (real) {
            cre[gm * g.ldc + gn] = p1;
            cim[gm * g.ldc + gn] = 0.f;
          } else {
            const float p2 = acc[1][i][j][e], p3 = acc[2][i][j][e];
            cre[gm * g.ldc + gn] = p1 - p2;
            cim[gm * g.ldc + gn] = p3 - p1 - p2;
          }
        }
      }
}

// One launch covers every Fourier slice; each workgroup runs the real or the
// complex body for its slice (the branch is uniform and taken once).
template <int SPLIT>
__global__ __launch_bounds__(NT, 1) void cgemm_bf16_kernel(MArgs g) {
  // LDS: [value r/i/s][split][row][LDK]
  __shared__ __attribute__((aligned(16))) __bf16 sA[3 * SPLIT * BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 sB[3 * SPLIT * BN * LDK];
  // complex slices first in launch order, the two cheaper real slices last
  const int64_t z = blockIdx.z;
  const int64_t nreal = (g.real_last && g.K > 1) ? 2 : 1;
  const int64_t ncomplex = g.K - nreal;
  if (z < ncomplex) {
    cgemm_bf16_body<SPLIT, false>(g, z + 1, sA, sB);
  } else {
    cgemm_bf16_body<SPLIT, true>(g, z == ncomplex ? 0 : g.K - 1, sA, sB);
  }
}

}  // namespace

// Takes the product when it is an as-stored (NN) product of float32 spectra
// with 16-byte aligned rows; reports handled = false otherwise.
int cgemm_mfma(const CGemm& p, int prec, hipStream_t st, bool* handled) {
  *handled = false;
  if (prec != TP_PREC_BF16X3 && prec != TP_PREC_BF16) return TP_OK;
  if (p.op_a != 0 || p.op_b != 0) return TP_OK;
  if (p.lda % 4 != 0 || p.sa % 4 != 0) return TP_OK;
  const uintptr_t al = reinterpret_cast<uintptr_t>(p.are) | reinterpret_cast<uintptr_t>(p.aim);
  if (al % 16 != 0) return TP_OK;
  if (p.K > 65535) return TP_OK;
  // per-slice offsets must fit in 32 bits
  const int64_t lim = int64_t(1) << 31;
  if (p.M * p.lda >= lim || p.Kd * p.ldb >= lim || p.M * p.ldc >= lim) return TP_OK;
  MArgs g{p.M, p.N, p.Kd, (const float*)p.are, (const float*)p.aim, (const float*)p.bre, (const float*)p.bim,
          (float*)p.cre, (float*)p.cim, p.lda, p.ldb, p.ldc, p.sa, p.sb, p.sc, p.K, p.real_last ? 1 : 0,
          p.kdim_dev};
  const unsigned gx = (unsigned)((p.N + BN - 1) / BN), gy = (unsigned)((p.M + BM - 1) / BM);
  if (prec == TP_PREC_BF16X3)
    hipLaunchKernelGGL(cgemm_bf16_kernel<2>, dim3(gx, gy, (unsigned)p.K), dim3(NT), 0, st, g);
  else
    hipLaunchKernelGGL(cgemm_bf16_kernel<1>, dim3(gx, gy, (unsigned)p.K), dim3(NT), 0, st, g);
  TP_LAUNCH_CHECK();
  *handled = true;
  return TP_OK;
}

}  // namespace tp
