// Per-slice complex products in float32 on the float32 matrix cores
// (v_mfma_f32_16x16x4f32): the slice loop of Algorithm 1 and the large
// Fourier-domain products of the dense t-SVD (Gram matrices A^H A, A A^H
// and U = A V) when the arithmetic is plain float32 (TP_PREC_F32).
//
// Complex slices use three real products (3M):
//   P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
//   Re C = P1 - P2, Im C = P3 - P1 - P2,
// with the sums Ar + Ai and Br + Bi formed once per staged element, so the
// matrix cores do three quarters of the four-product work (this kernel is
// bound by them); the real slices (DC, Nyquist) take P1 alone. Conjugate
// transposes (op = 1) are applied while staging: the operand is read
// transposed and its imaginary part negated before the sum is formed.
//
// Tiling: a 256-thread workgroup owns a 128 x 128 tile of one Fourier
// slice; each of its four wavefronts owns 64 x 64 (4 x 4 matrix-core tiles
// of 16 x 16, three accumulators each). A 16-deep step of both operands is
// staged through registers (loaded one step ahead, never predicated off)
// into one of two LDS buffers as three planes (re, im, re + im), stored per
// row with the contraction index permuted so that a lane's four values for
// the four 4-deep sub-steps are one 16-byte chunk: position 4 (k mod 4) +
// k / 4 of the row, chunk c of row r stored at chunk c ^ (r mod 4). A
// fragment read (16 rows x 4 chunks per wavefront) then covers 1 KB of LDS
// once.
//
// Products with few output tiles and a long contraction split the
// contraction into parts that write float32 partial planes, summed in part
// order afterwards (deterministic).
#include "common.hpp"

namespace tp {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int FM = 128, FN = 128, FK = 16, FT = 256;

struct FArgs {
  int64_t M, N, Kd;
  const float *are, *aim, *bre, *bim;
  float *cre, *cim;
  int64_t lda, ldb, ldc, sa, sb, sc;
  int op_a, op_b;
  int64_t K;
  int real_last;
  const int64_t* kdim_dev;
  int ksplit;
  int64_t kchunk;
  float *pre, *pim;  // partial planes [part][K][M][N] when ksplit > 1
};

// LDS float offset of element (row, k) of a staged 16-deep operand block
__device__ __forceinline__ int lds_pos(int row, int k) {
  const int c = k & 3, w = k >> 2;
  return row * 16 + 4 * (c ^ (row & 3)) + w;
}

// Stages one 16-deep step of an operand (rows of op(X): 128 x 16) from
// global memory into registers. along_k: the stored operand is contiguous
// along the contraction index (op_a = 0 for A, op_b = 1 for B); otherwise
// along the rows. Thread t covers 8 elements. Loads are never predicated
// off: an element outside the operand reads the slice origin instead (always
// valid) and is cleared when it is stored to LDS, so all eight loads stay in
// flight together behind the products of the current step.
struct Stage {
  float re[8], im[8];
  uint32_t keep;  // bit p: element p lies inside the operand
};

__device__ __forceinline__ void stage_coords(bool along_k, int p, int& row, int& kk) {
  const int t = threadIdx.x;
  if (along_k) {
    row = (t >> 4) + 16 * p;
    kk = t & 15;
  } else {
    row = (t & 127);
    kk = (t >> 7) + 2 * p;
  }
}

template <bool REAL>
__device__ __forceinline__ void load_stage(Stage& s, const float* xr, const float* xi, int64_t ld, bool along_k,
                                           int64_t r0, int64_t rows, int64_t k0, int64_t kend) {
  s.keep = 0;
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    int row, kk;
    stage_coords(along_k, p, row, kk);
    const int64_t gr = r0 + row, gk = k0 + kk;
    const bool ok = gr < rows && gk < kend;
    const int64_t off = ok ? (along_k ? gr * ld + gk : gk * ld + gr) : 0;
    s.re[p] = xr[off];
    if (!REAL) s.im[p] = xi[off];
    s.keep |= ok ? (1u << p) : 0u;
  }
}

template <bool REAL>
__device__ __forceinline__ void store_stage(const Stage& s, bool along_k, bool conj, float* lre, float* lim,
                                            float* lsum) {
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    int row, kk;
    stage_coords(along_k, p, row, kk);
    const bool ok = (s.keep >> p) & 1u;
    const int o = lds_pos(row, kk);
    const float vr = ok ? s.re[p] : 0.f;
    lre[o] = vr;
    if (!REAL) {
      const float vi = ok ? (conj ? -s.im[p] : s.im[p]) : 0.f;
      lim[o] = vi;
      lsum[o] = vr + vi;
    }
  }
}

template <bool REAL>
__device__ __forceinline__ void f32_body(const FArgs& g, int64_t k, int part, float* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * FM, n0 = (int64_t)blockIdx.x * FN;
  int64_t Kd = g.Kd;
  if (g.kdim_dev) {
    const int64_t lim = *g.kdim_dev;
    Kd = lim < Kd ? (lim < 0 ? 0 : lim) : Kd;
  }
  const int64_t kbeg = (int64_t)part * g.kchunk;
  const int64_t kend = kbeg + g.kchunk < Kd ? kbeg + g.kchunk : Kd;
  const float* are = g.are + k * g.sa;
  const float* aim = g.aim + k * g.sa;
  const float* bre = g.bre + k * g.sb;
  const float* bim = g.bim + k * g.sb;
  const bool a_along_k = g.op_a == 0, b_along_k = g.op_b != 0;
  const bool a_conj = g.op_a != 0, b_conj = g.op_b != 0;

  // LDS: 2 buffers x [A re, A im, A sum, B re, B im, B sum] x 128 rows x 16
  constexpr int PL = FM * FK;
  auto buf = [&](int b, int which) { return lds + (b * 6 + which) * PL; };

  // p1 = Ar Br, p2 = Ai Bi, p3 = (Ar + Ai)(Br + Bi)
  f32x4 p1[4][4], p2[4][4], p3[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      p1[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      p2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      p3[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  Stage sa, sb;
  const int64_t nsteps = kend > kbeg ? (kend - kbeg + FK - 1) / FK : 0;
  if (nsteps > 0) {
    load_stage<REAL>(sa, are, aim, g.lda, a_along_k, m0, g.M, kbeg, kend);
    load_stage<REAL>(sb, bre, bim, g.ldb, b_along_k, n0, g.N, kbeg, kend);
  }
  const int fr = lane & 15, fq = lane >> 4;
  for (int64_t st = 0; st < nsteps; ++st) {
    const int b = (int)(st & 1);
    store_stage<REAL>(sa, a_along_k, a_conj, buf(b, 0), buf(b, 1), buf(b, 2));
    store_stage<REAL>(sb, b_along_k, b_conj, buf(b, 3), buf(b, 4), buf(b, 5));
    __syncthreads();
    if (st + 1 < nsteps) {
      const int64_t k0 = kbeg + (st + 1) * FK;
      load_stage<REAL>(sa, are, aim, g.lda, a_along_k, m0, g.M, k0, kend);
      load_stage<REAL>(sb, bre, bim, g.ldb, b_along_k, n0, g.N, k0, kend);
    }
    // fragments: lane (fq, fr) reads row fr of a 16-row tile, chunk fq:
    // the values for k = fq + 4 s, s = 0..3 (sub-step s of the 16-deep step)
    f32x4 br_[4], bi_[4], bs_[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = wc * 64 + j * 16 + fr;
      const int o = row * 16 + 4 * (fq ^ (row & 3));
      br_[j] = *reinterpret_cast<const f32x4*>(buf(b, 3) + o);
      if (!REAL) {
        bi_[j] = *reinterpret_cast<const f32x4*>(buf(b, 4) + o);
        bs_[j] = *reinterpret_cast<const f32x4*>(buf(b, 5) + o);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wr * 64 + i * 16 + fr;
      const int o = row * 16 + 4 * (fq ^ (row & 3));
      const f32x4 ar = *reinterpret_cast<const f32x4*>(buf(b, 0) + o);
      f32x4 ai = f32x4{0.f, 0.f, 0.f, 0.f}, as = f32x4{0.f, 0.f, 0.f, 0.f};
      if (!REAL) {
        ai = *reinterpret_cast<const f32x4*>(buf(b, 1) + o);
        as = *reinterpret_cast<const f32x4*>(buf(b, 2) + o);
      }
      // product-outer order: consecutive matrix-core operations update
      // different accumulators, so none waits for the one before it
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s], br_[j][s], p1[i][j], 0, 0, 0);
        if (!REAL) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s], bi_[j][s], p2[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[s], bs_[j][s], p3[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // lane holds rows 4 (lane / 16) + v, column lane % 16 of each 16 x 16 tile
  float *cre, *cim;
  int64_t ldc;
  if (g.ksplit > 1) {
    const int64_t per = g.M * g.N;
    cre = g.pre + ((int64_t)part * g.K + k) * per;
    cim = g.pim + ((int64_t)part * g.K + k) * per;
    ldc = g.N;
  } else {
    cre = g.cre + k * g.sc;
    cim = g.cim + k * g.sc;
    ldc = g.ldc;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wr * 64 + i * 16 + 4 * fq + v;
        const int64_t gn = n0 + wc * 64 + j * 16 + fr;
        if (gm < g.M && gn < g.N) {
          const float a = p1[i][j][v], c = p2[i][j][v];
          cre[gm * ldc + gn] = REAL ? a : a - c;
          cim[gm * ldc + gn] = REAL ? 0.f : p3[i][j][v] - a - c;
        }
      }
}

__global__ __launch_bounds__(FT, 1) void cgemm_f32_kernel(FArgs g) {
  __shared__ __attribute__((aligned(16))) float lds[2 * 6 * FM * FK];  // 96 KB
  const int part = (int)(blockIdx.z % (unsigned)g.ksplit);
  const int64_t k = blockIdx.z / (unsigned)g.ksplit;
  const bool real = k == 0 || (g.real_last && k == g.K - 1);
  if (real)
    f32_body<true>(g, k, part, lds);
  else
    f32_body<false>(g, k, part, lds);
}

// C[k] = sum over the parts, in part order
__global__ void f32_ksplit_reduce_kernel(const float* __restrict__ pre, const float* __restrict__ pim, int ksplit,
                                         int64_t K, int64_t M, int64_t N, float* __restrict__ cre,
                                         float* __restrict__ cim, int64_t ldc, int64_t sc) {
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

}  // namespace

// Parts of a split contraction for the float32 matrix-core product: enough
// workgroups to cover the compute units about twice, each part at least
// 64 steps of 16, at most 64 parts.
int cgemm_f32_ksplit(int64_t K, int64_t M, int64_t N, int64_t Kd) {
  const int64_t tiles = ((M + FM - 1) / FM) * ((N + FN - 1) / FN) * K;
  if (tiles >= 256 || Kd < 128 * FK) return 1;
  int64_t s = (512 + tiles - 1) / tiles;
  s = s < Kd / (64 * FK) ? s : Kd / (64 * FK);
  s = s < 64 ? s : 64;
  return s > 1 ? (int)s : 1;
}

// Takes float32 products with at least 16 rows and columns and a contraction
// of at least 64; reports handled = false for the others.
int cgemm_f32mfma(const CGemm& p, hipStream_t st, bool* handled) {
  *handled = false;
  if (p.M < 16 || p.N < 16 || p.Kd < 64) return TP_OK;
  if (p.K > 65535) return TP_OK;
  int ksplit = cgemm_f32_ksplit(p.K, p.M, p.N, p.Kd);
  if (ksplit > 1 && (!p.part_re || !p.part_im || p.part_cap < int64_t(ksplit) * p.K * p.M * p.N)) ksplit = 1;
  if (p.K * ksplit > 65535) ksplit = 1;
  const int64_t kchunk = ksplit > 1 ? ((p.Kd + ksplit - 1) / ksplit + FK - 1) / FK * FK : p.Kd;
  FArgs g{p.M, p.N, p.Kd, (const float*)p.are, (const float*)p.aim, (const float*)p.bre, (const float*)p.bim,
          (float*)p.cre, (float*)p.cim, p.lda, p.ldb, p.ldc, p.sa, p.sb, p.sc, p.op_a, p.op_b, p.K,
          p.real_last ? 1 : 0, p.kdim_dev, ksplit, kchunk, p.part_re, p.part_im};
  const int64_t gx = (p.N + FN - 1) / FN, gy = (p.M + FM - 1) / FM;
  if (gx > 0x7fffffff || gy > 65535) return TP_OK;
  hipLaunchKernelGGL(cgemm_f32_kernel, dim3((unsigned)gx, (unsigned)gy, (unsigned)(p.K * ksplit)), dim3(FT), 0, st,
                     g);
  TP_LAUNCH_CHECK();
  if (ksplit > 1) {
    const int64_t n = p.K * p.M * p.N;
    hipLaunchKernelGGL(f32_ksplit_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p.part_re,
                       p.part_im, ksplit, p.K, p.M, p.N, (float*)p.cre, (float*)p.cim, p.ldc, p.sc);
    TP_LAUNCH_CHECK();
  }
  *handled = true;
  return TP_OK;
}

}  // namespace tp
