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
  // split contraction: part p of ksplit takes [p kchunk, (p + 1) kchunk)
  // and writes its planes to pre / pim [p][k][M][N]
  int ksplit;
  int64_t kchunk;
  float *pre, *pim;
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
__device__ __forceinline__ void cgemm_bf16_body(const MArgs& g, int64_t k, int part, __bf16* sA, __bf16* sB) {
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

  // contraction range of this part (kchunk is a multiple of BK)
  const int64_t kbeg = (int64_t)part * g.kchunk;
  const int64_t kend = kbeg + g.kchunk < Kd ? kbeg + g.kchunk : Kd;
  const int64_t nsteps = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nsteps > 0) load_tile((uint32_t)kbeg);
  for (int64_t ks = 0; ks < nsteps; ++ks) {
    __syncthreads();
    store_tile();
    __syncthreads();
    if (ks + 1 < nsteps) load_tile((uint32_t)(kbeg + (ks + 1) * BK));
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

  // epilogue: lane holds rows 4*(lane/16)+e, column lane%16 of each 16x16
  // tile; a part of a split contraction writes its own planes (row stride N)
  const bool parted = g.ksplit > 1;
  float* cre = parted ? g.pre + ((int64_t)part * g.K + k) * g.M * g.N : g.cre + k * g.sc;
  float* cim = parted ? g.pim + ((int64_t)part * g.K + k) * g.M * g.N : g.cim + k * g.sc;
  const int64_t ldc = parted ? g.N : g.ldc;
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
            cre[gm * ldc + gn] = p1;
            cim[gm * ldc + gn] = 0.f;
          } else {
            const float p2 = acc[1][i][j][e], p3 = acc[2][i][j][e];
            cre[gm * ldc + gn] = p1 - p2;
            cim[gm * ldc + gn] = p3 - p1 - p2;
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
  // complex slices first in launch order, the two cheaper real slices last;
  // the parts of a split contraction are the fastest-varying index
  const int part = (int)(blockIdx.z % (unsigned)g.ksplit);
  const int64_t z = blockIdx.z / (unsigned)g.ksplit;
  const int64_t nreal = (g.real_last && g.K > 1) ? 2 : 1;
  const int64_t ncomplex = g.K - nreal;
  if (z < ncomplex) {
    cgemm_bf16_body<SPLIT, false>(g, z + 1, part, sA, sB);
  } else {
    cgemm_bf16_body<SPLIT, true>(g, z == ncomplex ? 0 : g.K - 1, part, sA, sB);
  }
}


// ---------------------------------------------------------------------------
// Products of pre-split operands (the t-product path).
//
// The forward transforms write each operand as four bf16 planes
// hi(re), lo(re), hi(im), lo(im) [p][k][major][ld] with the contraction index
// contiguous (A as rows x ld, B transposed as columns x ld; ld a multiple of
// 32, zero beyond the live contraction length), so the products stream
// ready-made matrix-core fragments: no conversion in the main loop. Complex
// slices use four real products (4M: Re C = Ar Br - Ai Bi, Im C = Ar Bi +
// Ai Br, the minus sign applied by negating the Ai fragments), each as
// hi*hi + hi*lo + lo*hi for TERMS = 3 (bf16x3) or hi*hi for TERMS = 1;
// the real slices (DC, Nyquist) take Ar Br only.
//
// Tiling: 512 threads (8 wavefronts, two per SIMD so that one wavefront's
// waits are covered by the other's products) own a 128 x 128 tile; the
// wavefronts form a 2 x 4 grid, each owning 64 x 32 (4 x 2 tiles of
// v_mfma_f32_16x16x32_bf16). A 32-deep k step of both operands (4 planes x
// 128 rows x 64 bytes each, 64 KB) is staged through registers into one of
// two LDS buffers while the other is consumed, so each step ends with a
// single barrier. LDS rows are 64 bytes with the four 16-byte chunks
// XOR-swizzled by (row >> 1) & 3; with that swizzle the fragment reads
// (16 consecutive rows x 4 chunks per wavefront) and the staging writes
// (16 rows x 4 chunks) measure free of bank conflicts on gfx950
// (SQ_LDS_BANK_CONFLICT), which other row swizzles are not.
// ---------------------------------------------------------------------------
constexpr int SBM = 128, SBN = 128, SBK = 32, SNT = 512;
constexpr int WTI = 4, WTJ = 2;  // 16 x 16 tiles per wavefront (rows, columns)

struct SArgs {
  const __bf16* a;  // planes of A: [4][K][M][lda]
  const __bf16* b;  // planes of B^T: [4][K][N][ldb]
  float *cre, *cim;
  int64_t M, N, Kd;  // Kd: padded contraction length (multiple of 32)
  int64_t lda, ldb, ldc;
  int64_t pa, pb;  // plane strides (elements)
  int64_t sa, sb, sc;
  int64_t K;
  int real_last;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int swz(int row, int q) { return row * 4 + (q ^ ((row >> 1) & 3)); }

template <int TERMS, bool REAL>
__device__ __forceinline__ void split_body(const SArgs& g, int64_t k, int64_t tm, int64_t tn, u32x4* lds) {
  constexpr int NPL = REAL ? 2 : 4;  // planes read
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int64_t m0 = tm * SBM, n0 = tn * SBN;
  // per-slice bases; the row offsets below fit in 32 bits (checked on the host)
  const __bf16* abase = g.a + k * g.sa;
  const __bf16* bbase = g.b + k * g.sb;
  // staging chunk p of this thread: plane p, tile row tid >> 2, 16-byte chunk
  // tid & 3 of the 64-byte k step; rows beyond M (N) read the last row (their
  // results are never stored). Offsets are in 16-byte units inside one plane
  // of one slice.
  const int srow = tid >> 2, sq = tid & 3;
  uint32_t aoff, boff;
  {
    const int64_t ga = m0 + srow < g.M ? m0 + srow : g.M - 1;
    const int64_t gb = n0 + srow < g.N ? n0 + srow : g.N - 1;
    aoff = (uint32_t)(ga * (g.lda / 8)) + (uint32_t)sq;
    boff = (uint32_t)(gb * (g.ldb / 8)) + (uint32_t)sq;
  }
  const u32x4* ap[NPL];
  const u32x4* bp[NPL];
#pragma unroll
  for (int p = 0; p < NPL; ++p) {
    ap[p] = reinterpret_cast<const u32x4*>(abase + p * g.pa);
    bp[p] = reinterpret_cast<const u32x4*>(bbase + p * g.pb);
  }
  // two register sets of staged operands: a step is loaded two steps
  // before it is consumed, so a load has a whole step of products to land
  u32x4 ra0[NPL], rb0[NPL], ra1[NPL], rb1[NPL];
  auto load = [&](u32x4 (&ra)[NPL], u32x4 (&rb)[NPL], int64_t ks) {
    const uint32_t kq = (uint32_t)(ks * (SBK / 8));
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
      ra[p] = ap[p][aoff + kq];
      rb[p] = bp[p][boff + kq];
    }
  };
  // LDS: buffer b holds [A planes][B planes], each plane SBM rows x 4 chunks
  auto store = [&](const u32x4 (&ra)[NPL], const u32x4 (&rb)[NPL], int buf) {
    u32x4* sa = lds + buf * (2 * 4 * SBM * 4);
    u32x4* sb = sa + 4 * SBM * 4;
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
      sa[p * SBM * 4 + swz(srow, sq)] = ra[p];
      sb[p * SBM * 4 + swz(srow, sq)] = rb[p];
    }
  };

  f32x4 cr[WTI][WTJ], ci[WTI][WTJ];
#pragma unroll
  for (int i = 0; i < WTI; ++i)
#pragma unroll
    for (int j = 0; j < WTJ; ++j) {
      cr[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      ci[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  const int64_t nsteps = g.Kd / SBK;
  const int64_t last = nsteps - 1;
  const int fr = lane & 15, fq = lane >> 4;
  auto compute = [&](int buf) {
    const u32x4* sa = lds + buf * (2 * 4 * SBM * 4);
    const u32x4* sb = sa + 4 * SBM * 4;
    bf16x8 b[WTJ][NPL];
#pragma unroll
    for (int j = 0; j < WTJ; ++j)
#pragma unroll
      for (int p = 0; p < NPL; ++p) {
        const int row = wc * (16 * WTJ) + j * 16 + fr;
        b[j][p] = __builtin_bit_cast(bf16x8, sb[p * SBM * 4 + swz(row, fq)]);
      }
#pragma unroll
    for (int i = 0; i < WTI; ++i) {
      bf16x8 a[NPL], an[2];
      const int row = wr * (16 * WTI) + i * 16 + fr;
#pragma unroll
      for (int p = 0; p < NPL; ++p) a[p] = __builtin_bit_cast(bf16x8, sa[p * SBM * 4 + swz(row, fq)]);
      if constexpr (!REAL) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          u32x4 v = __builtin_bit_cast(u32x4, a[2 + h]);
          v ^= u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
          an[h] = __builtin_bit_cast(bf16x8, v);
        }
      }
      // term-outer order: consecutive products update different accumulators
#pragma unroll
      for (int term = 0; term < TERMS; ++term) {
        const int ha = term == 2 ? 1 : 0, hb = term == 1 ? 1 : 0;
#pragma unroll
        for (int j = 0; j < WTJ; ++j)
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ha], b[j][hb], cr[i][j], 0, 0, 0);
        if constexpr (!REAL) {
#pragma unroll
          for (int j = 0; j < WTJ; ++j)
            ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ha], b[j][2 + hb], ci[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < WTJ; ++j)
            cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(an[ha], b[j][2 + hb], cr[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < WTJ; ++j)
            ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2 + ha], b[j][hb], ci[i][j], 0, 0, 0);
        }
      }
    }
  };

  if (nsteps > 0) {
    // step 0 into buffer 0, step 1 in flight in set 1 (steps past the last
    // re-read the last one: valid memory, never consumed)
    load(ra0, rb0, 0);
    store(ra0, rb0, 0);
    load(ra1, rb1, 1 <= last ? 1 : last);
  }
  __syncthreads();
  // step ks computes from buffer ks & 1 while set (ks + 1) & 1 (step ks + 1,
  // loaded a step earlier) goes to the other buffer and set ks & 1 takes
  // step ks + 2; unrolled by two so that the sets swap statically. The loads
  // stay ahead of the products (scheduling barrier).
  for (int64_t ks = 0; ks < nsteps; ks += 2) {
    load(ra0, rb0, ks + 2 <= last ? ks + 2 : last);
    __builtin_amdgcn_sched_barrier(0);
    compute(0);
    store(ra1, rb1, 1);
    __syncthreads();
    if (ks + 1 >= nsteps) break;
    load(ra1, rb1, ks + 3 <= last ? ks + 3 : last);
    __builtin_amdgcn_sched_barrier(0);
    compute(1);
    store(ra0, rb0, 0);
    __syncthreads();
  }

  // epilogue: lane holds rows 4 (lane / 16) + e, column lane % 16 of a tile
  float* cre = g.cre + k * g.sc;
  float* cim = g.cim + k * g.sc;
#pragma unroll
  for (int i = 0; i < WTI; ++i)
#pragma unroll
    for (int j = 0; j < WTJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gm = m0 + wr * (16 * WTI) + i * 16 + 4 * (lane >> 4) + e;
        const int64_t gn = n0 + wc * (16 * WTJ) + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          cre[gm * g.ldc + gn] = cr[i][j][e];
          cim[gm * g.ldc + gn] = REAL ? 0.f : ci[i][j][e];
        }
      }
}

// C[k] = sum over the parts of a split contraction, in part order.
__global__ void ksplit_reduce_kernel(const float* __restrict__ pre, const float* __restrict__ pim, int ksplit,
                                     int64_t K, int64_t M, int64_t N, float* __restrict__ cre, float* __restrict__ cim,
                                     int64_t ldc, int64_t sc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = M * N;
  if (e >= K * per) return;
  const int64_t k = e / per, r = e - k * per, m = r / N, n = r - m * N;
  float sr = 0.f, si = 0.f;
  for (int p = 0; p < ksplit; ++p) {
    sr += pre[(int64_t)p * K * per + e];
    si += pim[(int64_t)p * K * per + e];
  }
  cre[k * sc + m * ldc + n] = sr;
  cim[k * sc + m * ldc + n] = si;
}

// Workgroups are dispatched to the eight XCDs round robin (workgroup L on
// XCD L mod 8, position L / 8 there), each XCD with its own L2. The tile map
// gives every XCD a contiguous run of complex-slice tiles (so the tiles of
// one Fourier slice, which share its A row blocks and B column blocks, read
// them through one L2) followed by a contiguous run of the cheaper
// real-slice tiles, both dealt as evenly as the round robin allows: XCD x
// takes one extra complex tile when x < (complex tiles mod 8) and one extra
// real tile when (x - that remainder) mod 8 < (real tiles mod 8), which
// reproduces the dispatcher's per-XCD counts.
constexpr int kXcds = 8;

template <int TERMS>
__global__ __launch_bounds__(SNT, 1) void cgemm_split_kernel(SArgs g, int64_t gm, int64_t gn) {
  __shared__ u32x4 lds[2 * 2 * 4 * SBM * 4];  // 2 buffers x (A, B) x 4 planes x 128 rows x 4 chunks: 128 KB
  const int64_t per = gm * gn;
  const int64_t nreal = (g.real_last && g.K > 1) ? 2 : 1;
  const int64_t ncomplex = g.K - nreal;
  const int64_t Tc = ncomplex * per, Tr = nreal * per;
  const int64_t cq = Tc / kXcds, crem = Tc % kXcds, rq = Tr / kXcds, rrem = Tr % kXcds;
  const int64_t L = blockIdx.x;
  const int x = (int)(L % kXcds);
  const int64_t pos = L / kXcds;
  const int64_t cc = cq + (x < crem ? 1 : 0);
  int64_t id;
  if (pos < cc) {
    id = x * cq + (x < crem ? x : crem) + pos;
  } else {
    int64_t rs = x * rq;
    for (int y = 0; y < x; ++y) rs += ((y - crem + kXcds) % kXcds) < rrem ? 1 : 0;
    id = Tc + rs + (pos - cc);
  }
  const int64_t zi = id / per, t = id - zi * per;
  const int64_t tm = t / gn, tn = t - tm * gn;
  if (zi < ncomplex)
    split_body<TERMS, false>(g, zi + 1, tm, tn, lds);
  else
    split_body<TERMS, true>(g, zi == ncomplex ? 0 : g.K - 1, tm, tn, lds);
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
  // a long contraction with few output tiles is split into parts that
  // write float32 partial planes, summed in part order afterwards, when the
  // caller provides the scratch
  int ksplit = cgemm_ksplit(p.K, p.M, p.N, p.Kd);
  if (ksplit > 1 && (!p.part_re || !p.part_im || p.part_cap < int64_t(ksplit) * p.K * p.M * p.N)) ksplit = 1;
  const int64_t kchunk = ksplit > 1 ? ((p.Kd + ksplit - 1) / ksplit + BK - 1) / BK * BK : p.Kd;
  MArgs g{p.M, p.N, p.Kd, (const float*)p.are, (const float*)p.aim, (const float*)p.bre, (const float*)p.bim,
          (float*)p.cre, (float*)p.cim, p.lda, p.ldb, p.ldc, p.sa, p.sb, p.sc, p.K, p.real_last ? 1 : 0,
          p.kdim_dev, ksplit, kchunk, p.part_re, p.part_im};
  const unsigned gx = (unsigned)((p.N + BN - 1) / BN), gy = (unsigned)((p.M + BM - 1) / BM);
  const unsigned gz = (unsigned)(p.K * ksplit);
  if (prec == TP_PREC_BF16X3)
    hipLaunchKernelGGL(cgemm_bf16_kernel<2>, dim3(gx, gy, gz), dim3(NT), 0, st, g);
  else
    hipLaunchKernelGGL(cgemm_bf16_kernel<1>, dim3(gx, gy, gz), dim3(NT), 0, st, g);
  TP_LAUNCH_CHECK();
  if (ksplit > 1) {
    const int64_t n = p.K * p.M * p.N;
    hipLaunchKernelGGL(ksplit_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p.part_re,
                       p.part_im, ksplit, p.K, p.M, p.N, (float*)p.cre, (float*)p.cim, p.ldc, p.sc);
    TP_LAUNCH_CHECK();
  }
  *handled = true;
  return TP_OK;
}

// Parts of a split contraction: enough workgroups to cover the compute
// units about twice, each part at least 32 steps of the contraction, at
// most 64 parts.
int cgemm_ksplit(int64_t K, int64_t M, int64_t N, int64_t Kd) {
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN) * K;
  if (tiles >= 256 || Kd < 64 * BK) return 1;
  int64_t s = (512 + tiles - 1) / tiles;
  s = s < Kd / (32 * BK) ? s : Kd / (32 * BK);
  s = s < 64 ? s : 64;
  return s > 1 ? (int)s : 1;
}

int cgemm_split(const SplitGemm& p, hipStream_t st) {
  if (p.K == 0 || p.M == 0 || p.N == 0) return TP_OK;
  if (p.Kd % SBK || p.lda % SBK || p.ldb % SBK || p.lda < p.Kd || p.ldb < p.Kd)
    return fail(TP_EINVAL, "split operands need a contraction stride that is a multiple of 32");
  if ((reinterpret_cast<uintptr_t>(p.a) | reinterpret_cast<uintptr_t>(p.b)) % 16)
    return fail(TP_EINVAL, "split operands must be 16-byte aligned");
  if (p.K > 65535) return fail(TP_EUNSUPPORTED, "more than 65535 Fourier slices");
  // row offsets inside one plane of one slice are 32-bit in 16-byte units
  if ((p.M * p.lda) / 8 >= (int64_t(1) << 32) || (p.N * p.ldb) / 8 >= (int64_t(1) << 32))
    return fail(TP_EUNSUPPORTED, "slice too large for the split product");
  SArgs g{(const __bf16*)p.a, (const __bf16*)p.b, p.cre, p.cim, p.M, p.N, p.Kd, p.lda, p.ldb, p.ldc, p.pa, p.pb, p.sa, p.sb, p.sc, p.K,
          p.real_last ? 1 : 0};
  const int64_t gm = (p.M + SBM - 1) / SBM, gn = (p.N + SBN - 1) / SBN;
  const int64_t tiles = gm * gn * p.K;
  if (tiles > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many product tiles");
  if (p.terms == 3)
    hipLaunchKernelGGL(cgemm_split_kernel<3>, dim3((unsigned)tiles), dim3(SNT), 0, st, g, gm, gn);
  else
    hipLaunchKernelGGL(cgemm_split_kernel<1>, dim3((unsigned)tiles), dim3(SNT), 0, st, g, gm, gn);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
