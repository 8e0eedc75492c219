// Learned lateral-leverage proposal: cheap per-slice features, a small MLP
// (17 -> 128 -> 128 -> 1, ReLU) on the fp16 matrix cores with float32
// accumulation, per-tensor softmax with a KL loss against the exact
// leverage distribution, backward pass and Adam. Not part of the paper,
// which estimates leverage with a randomized routine it cites without
// describing; the exact scores (eq. cur-col-prob) stay the fallback.
//
// Features of lateral slice j of an n1 x n2 x n3 tensor A: the sketch
// s_j = Phi^T vec(A_{:j:}) with a caller-supplied (n1 n3) x 16 matrix Phi,
// whitened as z_j = G^{-1/2} s_j sqrt(n2), G = sum_j s_j s_j^T, and
// f_j = log(n2 a_j / sum a), a_j = ||A_{:j:}||_F^2.
//
// Parameters are one float32 array (the master copy) laid out as
//   W1 (17 x 128) | b1 (128) | W2 (128 x 128) | b2 (128) | w3 (128) | b3 (1)
// (h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), o = h2 w3 + b3); the
// forward and backward passes use fp16 copies of W1 and W2 and fp16
// activations as matrix-core operands.
#include <cmath>

#include "common.hpp"
#include "jacobi.hpp"
#include "mlp.hpp"

namespace tp {
namespace {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DS = 16, DIN = 17, KIN = 32, HID = 128;
constexpr int OFF_W1 = 0, OFF_B1 = DIN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
constexpr int NPARAM = OFF_B3 + 1;
static_assert(NPARAM == kMlpParams, "parameter layout");

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
// The sketch is the contraction S = X Phi with X (n2 x n1 n3), row j =
// vec(A_{:j:}). In the tube-major layout horizontal slice i of A is an
// n2 x n3 row-major block, so S = sum_i A_{i::} Phi_i with Phi_i the rows
// i n3 .. i n3 + n3 - 1 of Phi: per horizontal slice a (64 slices x n3) by
// (n3 x 16) product on the fp32 matrix cores (v_mfma_f32_16x16x4f32), one
// 16-slice tile per wavefront. Lane l of a wavefront owns row l % 16 of the
// tile and tube entries 4 (l / 16) .. 4 (l / 16) + 3 of every 16-entry tube
// block (one float4 load); its four values feed four matrix-core steps,
// with Phi_i read at the same tube positions from a transposed LDS copy.
constexpr int SJ = 64;   // lateral slices per workgroup (4 tiles of 16)
constexpr int SIR = 16;  // horizontal slices per workgroup
constexpr int SNT = 256;

// Tubes are taken in chunks of at most kSketchChunk entries (a multiple of
// 16), so that two chunks of Phi_i fit in 64 KB of LDS at any tube length.
constexpr int kSketchChunk = 496;
__device__ __host__ __forceinline__ int sketch_chunk(int64_t n3) {
  const int64_t r = (n3 + 15) / 16 * 16;
  return (int)(r < kSketchChunk ? r : kSketchChunk);
}
__device__ __host__ __forceinline__ int sketch_ldk(int64_t n3) { return sketch_chunk(n3) + 4; }

// partial[(y n2 + j) (DS + 1) + d]: the chunk-y sums (float32) of the
// sketch (d < DS) and of the squared norm (d = DS) of lateral slice j.
__global__ __launch_bounds__(SNT) void sketch_mfma_kernel(const float* __restrict__ a, const float* __restrict__ phi,
                                                           int64_t n1, int64_t n2, int64_t n3,
                                                           float* __restrict__ partial) {
  extern __shared__ float phs[];  // [2][DS][ldk]: a tube chunk of Phi_i transposed, double buffered
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kc = sketch_chunk(n3), ldk = kc + 4;
  const int64_t j0 = (int64_t)blockIdx.x * SJ;
  const int64_t i0 = (int64_t)blockIdx.y * SIR;
  const int64_t rows = (n1 - i0) < SIR ? (n1 - i0) : SIR;
  const int g = lane >> 4, r = lane & 15;
  const int64_t j = j0 + wave * 16 + r;
  const bool jok = j < n2;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float nrm = 0.f;
  // steps over (horizontal slice, tube chunk); the buffer written in a step
  // was last read two steps earlier, before the previous step's barrier
  int step = 0;
  for (int64_t ii = 0; ii < rows; ++ii) {
    const int64_t i = i0 + ii;
    const float* src = phi + i * n3 * DS;
    const float* arow = a + (i * n2 + j) * n3;
    for (int64_t k0 = 0; k0 < n3; k0 += kc, ++step) {
      float* buf = phs + (step & 1) * DS * ldk;
      // this chunk of Phi_i, zero beyond the tube's end
      for (int e = tid; e < kc * DS; e += SNT) {
        const int kk = e / DS, d = e - kk * DS;
        buf[d * ldk + kk] = k0 + kk < n3 ? src[(k0 + kk) * DS + d] : 0.f;
      }
      __syncthreads();
      const int nkb = (int)((n3 - k0 < kc ? n3 - k0 : kc) + 15) / 16;
      for (int kb = 0; kb < nkb; ++kb) {
        const int kk = kb * 16 + 4 * g;
        const int64_t k = k0 + kk;
        float4 x = {0.f, 0.f, 0.f, 0.f};
        if (jok && k < n3) x = *reinterpret_cast<const float4*>(arow + k);
        const float4 p = *reinterpret_cast<const float4*>(buf + r * ldk + kk);
        nrm += x.x * x.x + x.y * x.y + x.z * x.z + x.w * x.w;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, p.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, p.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, p.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, p.w, acc, 0, 0, 0);
      }
    }
  }
  // lane l holds S[row 4 g + v][d = l % 16] of the wavefront's tile
  float* out = partial + ((int64_t)blockIdx.y * n2) * (DS + 1);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t jj = j0 + wave * 16 + 4 * g + v;
    if (jj < n2) out[jj * (DS + 1) + r] = acc[v];
  }
  nrm += __shfl_xor(nrm, 16);
  nrm += __shfl_xor(nrm, 32);
  if (g == 0 && jok) out[j * (DS + 1) + DS] = nrm;
}

// The same contraction for tubes of at most 16 NKB entries with every load
// of a horizontal slice issued at once: lane (g, r) holds the NKB float4
// pieces 4 g + 16 b (b < NKB) of its tube, and the next slice's pieces and
// its share of the next Phi_i are fetched into registers before the
// current slice's matrix-core steps, so that HBM latency overlaps the
// arithmetic. Phi_i is staged transposed in two LDS buffers (one barrier
// per slice).
template <int NKB>
__global__ __launch_bounds__(SNT) void sketch_mfma_pipe_kernel(const float* __restrict__ a,
                                                                const float* __restrict__ phi, int64_t n1,
                                                                int64_t n2, int64_t n3, float* __restrict__ partial) {
  constexpr int LDK = 16 * NKB + 4;
  constexpr int PH = 16 * NKB * DS / SNT;  // Phi_i entries per thread (padded tube)
  static_assert(PH * SNT == 16 * NKB * DS, "whole Phi_i per workgroup");
  __shared__ __align__(16) float phs[2][DS][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * SJ;
  const int64_t i0 = (int64_t)blockIdx.y * SIR;
  const int64_t rows = (n1 - i0) < SIR ? (n1 - i0) : SIR;
  const int g = lane >> 4, r = lane & 15;
  const int64_t j = j0 + wave * 16 + r;
  const bool jok = j < n2;
  auto load_a = [&](int64_t i, float4 (&x)[NKB]) {
    const float* arow = a + (i * n2 + (jok ? j : 0)) * n3;
#pragma unroll
    for (int b = 0; b < NKB; ++b) {
      const int64_t k = 16 * b + 4 * g;
      x[b] = (jok && k < n3) ? *reinterpret_cast<const float4*>(arow + k) : float4{0.f, 0.f, 0.f, 0.f};
    }
  };
  // thread's Phi entries: e = tid + SNT u of the padded (16 NKB) x DS block
  auto load_phi = [&](int64_t i, float (&v)[PH]) {
    const float* src = phi + i * n3 * DS;
#pragma unroll
    for (int u = 0; u < PH; ++u) {
      const int e = tid + SNT * u;
      v[u] = (e / DS) < n3 ? src[e] : 0.f;
    }
  };
  float4 xc[NKB], xn[NKB];
  float pv[PH];
  load_a(i0, xc);
  load_phi(i0, pv);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float nrm = 0.f;
  for (int64_t ii = 0; ii < rows; ++ii) {
    float(*buf)[LDK] = phs[ii & 1];
#pragma unroll
    for (int u = 0; u < PH; ++u) {
      const int e = tid + SNT * u;
      buf[e % DS][e / DS] = pv[u];
    }
    if (ii + 1 < rows) {
      load_a(i0 + ii + 1, xn);
      load_phi(i0 + ii + 1, pv);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NKB; ++b) {
      const float4 x = xc[b];
      const float4 p = *reinterpret_cast<const float4*>(&buf[r][16 * b + 4 * g]);
      nrm += x.x * x.x + x.y * x.y + x.z * x.z + x.w * x.w;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, p.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, p.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, p.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, p.w, acc, 0, 0, 0);
    }
#pragma unroll
    for (int b = 0; b < NKB; ++b) xc[b] = xn[b];
  }
  float* out = partial + ((int64_t)blockIdx.y * n2) * (DS + 1);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t jj = j0 + wave * 16 + 4 * g + v;
    if (jj < n2) out[jj * (DS + 1) + r] = acc[v];
  }
  nrm += __shfl_xor(nrm, 16);
  nrm += __shfl_xor(nrm, 32);
  if (g == 0 && jok) out[j * (DS + 1) + DS] = nrm;
}

// Per block of SJS lateral slices: the float64 sums over the row chunks
// (sk[j][0..DS] = sketch and squared norm), and the block's share of the
// Gram matrix G = sum_j s_j s_j^T and of sum_j a_j (gpart[blk][0..DS*DS]).
constexpr int SJS = 16;
__global__ __launch_bounds__(256) void sketch_sum_kernel(const float* __restrict__ partial, int64_t nch, int64_t n2,
                                                          double* __restrict__ sk, double* __restrict__ gpart) {
  __shared__ double s[SJS][DS + 1];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * SJS;
  const int64_t nj = (n2 - j0) < SJS ? (n2 - j0) : SJS;
  // entries e of the block's (nj x (DS + 1)) run are contiguous in every chunk
  for (int e = tid; e < SJS * (DS + 1); e += 256) {
    const int t = e / (DS + 1);
    double v = 0.0;
    if (t < nj) {
      const float* src = partial + j0 * (DS + 1) + e;
      const int64_t stride = n2 * (DS + 1);
      int64_t y = 0;
      for (; y + 8 <= nch; y += 8) {
        float f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) f[u] = src[(y + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += (double)f[u];
      }
      for (; y < nch; ++y) v += (double)src[y * stride];
      sk[j0 * (DS + 1) + e] = v;
    }
    s[t][e - t * (DS + 1)] = v;
  }
  __syncthreads();
  {
    const int p = tid / DS, q = tid % DS;
    double gsum = 0.0;
    for (int t = 0; t < SJS; ++t) gsum += s[t][p] * s[t][q];
    gpart[blockIdx.x * (DS * DS + 1) + tid] = gsum;
  }
  if (tid == 0) {
    double at = 0.0;
    for (int t = 0; t < SJS; ++t) at += s[t][DS];
    gpart[blockIdx.x * (DS * DS + 1) + DS * DS] = at;
  }
}

// G and sum a from the block shares (fixed order), then the whitening
// W = G^{-1/2} sqrt(n2) (the symmetric inverse square root, unique for a
// positive definite G). With A = G / tr(G) (eigenvalues in (0, 1)), the
// coupled Newton-Schulz iteration T = (3 I - Z Y) / 2, Y <- Y T, Z <- T Z
// from Y = A, Z = I takes Z to A^{-1/2} (Higham, Functions of Matrices,
// sec. 6.3); it stops once max |T - I| <= 1e-12 (the T applied last is then
// I to second order). If it has not converged after kNsIters steps (G
// singular or nearly so) the float64 Jacobi solver diagonalises G instead
// and W = V diag(lambda^{-1/2}) V^T over the positive eigenvalues.
// wt[0..DS*DS) = W (row-major), wt[DS*DS] = sum a.
constexpr int kNsIters = 64;

__global__ __launch_bounds__(256) void sketch_whiten_kernel(const double* __restrict__ gpart, int64_t nblk,
                                                             int64_t n2, double* __restrict__ wt) {
  static_assert(DS * DS == 256, "one Gram entry per thread");
  __shared__ JacobiShared<DS, 256> sh;
  __shared__ double Y[DS][DS + 1], Z[DS][DS + 1], T[DS][DS + 1];
  __shared__ double dev[4];
  const int tid = threadIdx.x;
  const int p = tid / DS, q = tid % DS;
  double g = 0.0;
  for (int64_t b = 0; b < nblk; ++b) g += gpart[b * (DS * DS + 1) + tid];
  sh.Hr[p][q] = g;
  sh.Hi[p][q] = 0.0;
  if (tid == 0) {
    double at = 0.0;
    for (int64_t b = 0; b < nblk; ++b) at += gpart[b * (DS * DS + 1) + DS * DS];
    wt[DS * DS] = at;
  }
  __syncthreads();
  double tr = 0.0;
  for (int c = 0; c < DS; ++c) tr += sh.Hr[c][c];
  bool done = false;
  if (tr > 0.0 && tr < INFINITY) {
    const double inv = 1.0 / tr;
    Y[p][q] = 0.5 * (sh.Hr[p][q] + sh.Hr[q][p]) * inv;
    Z[p][q] = p == q ? 1.0 : 0.0;
    __syncthreads();
    for (int it = 0; it < kNsIters; ++it) {
      double zy = 0.0;
#pragma unroll
      for (int c = 0; c < DS; ++c) zy += Z[p][c] * Y[c][q];
      const double t = (p == q ? 1.5 : 0.0) - 0.5 * zy;
      double d = fabs(t - (p == q ? 1.0 : 0.0));
      d = d == d ? d : INFINITY;  // a NaN never converges
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o));
      T[p][q] = t;
      if ((tid & 63) == 0) dev[tid >> 6] = d;
      __syncthreads();
      double yn = 0.0, zn = 0.0;
#pragma unroll
      for (int c = 0; c < DS; ++c) {
        yn += Y[p][c] * T[c][q];
        zn += T[p][c] * Z[c][q];
      }
      const double m = fmax(fmax(dev[0], dev[1]), fmax(dev[2], dev[3]));
      __syncthreads();
      Y[p][q] = yn;
      Z[p][q] = zn;
      __syncthreads();
      if (m <= 1e-12) {
        done = true;
        break;
      }
    }
  }
  if (done) {
    wt[tid] = Z[p][q] * sqrt((double)n2 / tr);
    return;
  }
  jacobi_eig_lds<DS, 256>(sh, DS, 30, 1e-15);
  double t = 0.0;
  for (int c = 0; c < DS; ++c) {
    const double l = sh.Hr[c][c];
    if (l > 0.0) t += sh.Vr[p][c] * sh.Vr[q][c] / sqrt(l);
  }
  wt[tid] = t * sqrt((double)n2);
}

// feat[j] = [s_j^T W, log(n2 a_j / sum a)]; optionally a_j itself.
__global__ void sketch_apply_kernel(const double* __restrict__ sk, const double* __restrict__ wt, int64_t n2,
                                    float* __restrict__ feat, double* __restrict__ norms) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 * DIN) return;
  const int64_t j = e / DIN;
  const int d = (int)(e - j * DIN);
  double v;
  if (d < DS) {
    v = 0.0;
    for (int q = 0; q < DS; ++q) v += sk[j * (DS + 1) + q] * wt[q * DS + d];
  } else {
    const double aj = sk[j * (DS + 1) + DS];
    v = log((double)n2 * aj / wt[DS * DS]);
    if (norms) norms[j] = aj;
  }
  feat[e] = (float)v;
}

// ---------------------------------------------------------------------------
// MLP on the matrix cores
// ---------------------------------------------------------------------------
constexpr int TR = 64;  // rows per tile
constexpr int NT = 256;
constexpr int LX = KIN + 8, LH = HID + 8;

// acc += A[16 rows][K] * B[K][16 cols] with element strides:
// A(i, k) = A[i * asi + k * ask], B(k, j) = B[k * bsk + j * bsj].
__device__ __forceinline__ f32x4 mfma_tile(const _Float16* A, int asi, int ask, const _Float16* B, int bsk, int bsj,
                                           int K, f32x4 acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kq = 4 * (lane >> 4);
  for (int k0 = 0; k0 < K; k0 += 16) {
    half4 a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a[e] = A[r * asi + (k0 + kq + e) * ask];
      b[e] = B[(k0 + kq + e) * bsk + r * bsj];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

struct MlpShared {
  _Float16 X[TR][LX];    // input tile, features padded to KIN
  _Float16 W1[KIN][LH];  // W1 padded (rows 17..31 zero)
  _Float16 W2[HID][LH];
  _Float16 H1[TR][LH];
  _Float16 H2[TR][LH];
  _Float16 D[TR][LH];    // dH2, then dH1
  float b1[HID], b2[HID], w3[HID];
  float z[TR][HID + 4];  // staging for row sums
  float dout[TR];
};

// Forward pass of one tile; leaves H1, H2 (post-ReLU, fp16) in LDS and the
// logits in out (when set). Pre-activations are positive exactly where the
// stored post-activations are, which the backward pass uses as the masks.
__device__ void mlp_tile_forward(MlpShared& s, const float* __restrict__ P, const float* __restrict__ feat,
                                 int64_t nrows, int64_t r0, float* out) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < TR * KIN; e += NT) {
    const int r = e / KIN, c = e % KIN;
    const int64_t row = r0 + r;
    s.X[r][c] = (_Float16)((c < DIN && row < nrows) ? feat[row * DIN + c] : 0.f);
  }
  for (int e = tid; e < KIN * HID; e += NT) {
    const int r = e / HID, c = e % HID;
    s.W1[r][c] = (_Float16)(r < DIN ? P[OFF_W1 + r * HID + c] : 0.f);
  }
  for (int e = tid; e < HID * HID; e += NT) s.W2[e / HID][e % HID] = (_Float16)P[OFF_W2 + e];
  for (int e = tid; e < HID; e += NT) {
    s.b1[e] = P[OFF_B1 + e];
    s.b2[e] = P[OFF_B2 + e];
    s.w3[e] = P[OFF_W3 + e];
  }
  __syncthreads();
  // layer 1: wave w owns rows 16w..16w+15, all 8 column tiles
  for (int nt = 0; nt < HID / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_tile(&s.X[16 * wave][0], LX, 1, &s.W1[0][16 * nt], LH, 1, KIN, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * wave + 4 * (lane >> 4) + e, col = 16 * nt + (lane & 15);
      s.H1[row][col] = (_Float16)fmaxf(acc[e] + s.b1[col], 0.f);
    }
  }
  __syncthreads();
  for (int nt = 0; nt < HID / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_tile(&s.H1[16 * wave][0], LH, 1, &s.W2[0][16 * nt], LH, 1, HID, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * wave + 4 * (lane >> 4) + e, col = 16 * nt + (lane & 15);
      const float h = fmaxf(acc[e] + s.b2[col], 0.f);
      s.H2[row][col] = (_Float16)h;
      s.z[row][col] = h * s.w3[col];
    }
  }
  __syncthreads();
  if (out && tid < TR) {
    float o = P[OFF_B3];
    for (int c = 0; c < HID; ++c) o += s.z[tid][c];
    if (r0 + tid < nrows) out[r0 + tid] = o;
  }
  __syncthreads();
}

__global__ __launch_bounds__(NT) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                         int64_t nrows, float* __restrict__ out) {
  __shared__ MlpShared s;
  mlp_tile_forward(s, P, feat, nrows, (int64_t)blockIdx.x * TR, out);
}

// Per tensor: p = softmax(o), loss = KL(p* || p), dO = (p - p*) / T.
__global__ __launch_bounds__(256) void softmax_grad_kernel(const float* __restrict__ o,
                                                           const float* __restrict__ target, int64_t nsl, int64_t T,
                                                           float* __restrict__ dout, float* __restrict__ loss_part) {
  __shared__ double red[256];
  const int64_t t = blockIdx.x;
  const int tid = threadIdx.x;
  const float* ot = o + t * nsl;
  const float* pt = target + t * nsl;
  double m = -INFINITY;
  for (int64_t j = tid; j < nsl; j += 256) m = fmax(m, (double)ot[j]);
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double mx = red[0];
  __syncthreads();
  double se = 0.0;
  for (int64_t j = tid; j < nsl; j += 256) se += exp((double)ot[j] - mx);
  red[tid] = se;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double lse = mx + log(red[0]);
  __syncthreads();
  // the target row is normalised here (any positive scale is accepted)
  double qs = 0.0;
  for (int64_t j = tid; j < nsl; j += 256) qs += (double)pt[j];
  red[tid] = qs;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double qinv = red[0] > 0.0 ? 1.0 / red[0] : 0.0;
  __syncthreads();
  double kl = 0.0;
  for (int64_t j = tid; j < nsl; j += 256) {
    const double lp = (double)ot[j] - lse;
    const double q = (double)pt[j] * qinv;
    if (q > 0) kl += q * (log(q) - lp);
    dout[t * nsl + j] = (float)((exp(lp) - q) / (double)T);
  }
  red[tid] = kl;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) loss_part[t] = (float)(red[0] / (double)T);
}

// Backward of one tile: recomputes the forward pass, then writes this
// tile's gradient contribution (parameter layout) to partial[tile].
__global__ __launch_bounds__(NT) void mlp_backward_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                          const float* __restrict__ dout, int64_t nrows,
                                                          float* __restrict__ partial) {
  __shared__ MlpShared s;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t r0 = (int64_t)blockIdx.x * TR;
  mlp_tile_forward(s, P, feat, nrows, r0, nullptr);
  float* g = partial + (int64_t)blockIdx.x * NPARAM;
  if (tid < TR) s.dout[tid] = (r0 + tid < nrows) ? dout[r0 + tid] : 0.f;
  __syncthreads();
  // w3, b3 and dH2 = dO w3 (.) [h2 > 0]
  for (int c = tid; c < HID; c += NT) {
    float gw = 0.f;
    for (int r = 0; r < TR; ++r) gw += (float)s.H2[r][c] * s.dout[r];
    g[OFF_W3 + c] = gw;
  }
  if (tid == 0) {
    float gb = 0.f;
    for (int r = 0; r < TR; ++r) gb += s.dout[r];
    g[OFF_B3] = gb;
  }
  for (int e = tid; e < TR * HID; e += NT) {
    const int r = e / HID, c = e % HID;
    s.D[r][c] = (_Float16)((float)s.H2[r][c] > 0.f ? s.dout[r] * s.w3[c] : 0.f);
  }
  __syncthreads();
  // b2 = column sums of dH2; W2 = H1^T dH2
  for (int c = tid; c < HID; c += NT) {
    float gb = 0.f;
    for (int r = 0; r < TR; ++r) gb += (float)s.D[r][c];
    g[OFF_B2 + c] = gb;
  }
  for (int t = wave; t < (HID / 16) * (HID / 16); t += NT / 64) {
    const int it = t / (HID / 16), jt = t % (HID / 16);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_tile(&s.H1[0][16 * it], 1, LH, &s.D[0][16 * jt], LH, 1, TR, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * it + 4 * (lane >> 4) + e, col = 16 * jt + (lane & 15);
      g[OFF_W2 + row * HID + col] = acc[e];
    }
  }
  // dH1 = (dH2 W2^T) (.) [h1 > 0], staged in z as float
  for (int nt = 0; nt < HID / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_tile(&s.D[16 * wave][0], LH, 1, &s.W2[16 * nt][0], 1, LH, HID, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * wave + 4 * (lane >> 4) + e, col = 16 * nt + (lane & 15);
      s.z[row][col] = (float)s.H1[row][col] > 0.f ? acc[e] : 0.f;
    }
  }
  __syncthreads();
  for (int e = tid; e < TR * HID; e += NT) s.D[e / HID][e % HID] = (_Float16)s.z[e / HID][e % HID];
  __syncthreads();
  // b1 = column sums of dH1 (float); W1 = X^T dH1
  for (int c = tid; c < HID; c += NT) {
    float gb = 0.f;
    for (int r = 0; r < TR; ++r) gb += s.z[r][c];
    g[OFF_B1 + c] = gb;
  }
  for (int t = wave; t < (KIN / 16) * (HID / 16); t += NT / 64) {
    const int it = t / (HID / 16), jt = t % (HID / 16);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_tile(&s.X[0][16 * it], 1, LX, &s.D[0][16 * jt], LH, 1, TR, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * it + 4 * (lane >> 4) + e, col = 16 * jt + (lane & 15);
      if (row < DIN) g[OFF_W1 + row * HID + col] = acc[e];
    }
  }
}

__global__ void grad_reduce_kernel(const float* __restrict__ partial, int64_t ntiles, float* __restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float s = 0.f;
  for (int64_t t = 0; t < ntiles; ++t) s += partial[t * NPARAM + p];
  grad[p] = s;
}

__global__ void loss_reduce_kernel(const float* __restrict__ part, int64_t T, float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int64_t t = 0; t < T; ++t) s += part[t];
    *loss = s;
  }
}

__global__ void adam_kernel(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
                            const float* __restrict__ G, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.f - b1) * g;
  const float v = b2 * V[p] + (1.f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// w = (1 - alpha) softmax(o) + alpha / n (a defensive mixture with the
// uniform distribution), float64, one workgroup. A network output that is
// not finite (diverged or corrupted parameters) gives the uniform
// distribution, the mixture's defensive part, so the picks stay valid.
__global__ __launch_bounds__(256) void proposal_kernel(const float* __restrict__ o, int64_t n, double alpha,
                                                       double* __restrict__ w) {
  __shared__ double red[256];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  double m = -INFINITY;
  int nonfinite = 0;
  for (int64_t j = tid; j < n; j += 256) {
    const float v = o[j];
    nonfinite |= !isfinite(v);
    m = fmax(m, (double)v);
  }
  if (nonfinite) bad = 1;  // benign race: every writer stores 1
  red[tid] = m;
  __syncthreads();
  if (bad) {
    for (int64_t j = tid; j < n; j += 256) w[j] = 1.0 / (double)n;
    return;
  }
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double mx = red[0];
  __syncthreads();
  double se = 0.0;
  for (int64_t j = tid; j < n; j += 256) se += exp((double)o[j] - mx);
  red[tid] = se;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double z = red[0];
  for (int64_t j = tid; j < n; j += 256) w[j] = (1.0 - alpha) * exp((double)o[j] - mx) / z + alpha / (double)n;
}

unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t mlp_features_ws(int64_t n1, int64_t n2) {
  const int64_t nch = (n1 + SIR - 1) / SIR, nbs = (n2 + SJS - 1) / SJS;
  return align_up(size_t(nch) * n2 * (DS + 1) * 4) + align_up(size_t(n2) * (DS + 1) * 8) +
         align_up(size_t(nbs) * (DS * DS + 1) * 8) + align_up(size_t(DS * DS + 1) * 8) + 1024;
}

int mlp_features(const float* a, int64_t n1, int64_t n2, int64_t n3, const float* phi, float* feat, void* ws,
                 hipStream_t st, double* norms) {
  if (n3 % 4) return fail(TP_EUNSUPPORTED, "feature extraction needs n3 divisible by 4");
  const size_t lds = size_t(2) * DS * sketch_ldk(n3) * 4;
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(phi)) % 16)
    return fail(TP_EINVAL, "A and phi must be 16-byte aligned");
  const int64_t nch = (n1 + SIR - 1) / SIR, nb = (n2 + SJ - 1) / SJ, nbs = (n2 + SJS - 1) / SJS;
  if (nch > 65535) return fail(TP_EUNSUPPORTED, "too many horizontal slices");
  Arena ar(ws, mlp_features_ws(n1, n2));
  float* part = ar.take<float>(nch * n2 * (DS + 1));
  double* sk = ar.take<double>(n2 * (DS + 1));
  double* gpart = ar.take<double>(nbs * (DS * DS + 1));
  double* wt = ar.take<double>(DS * DS + 1);
  if (!ar.ok()) return fail(TP_EWORKSPACE, "feature workspace too small");
  const dim3 grid((unsigned)nb, (unsigned)nch);
  if (n3 <= 32)
    hipLaunchKernelGGL(sketch_mfma_pipe_kernel<2>, grid, dim3(SNT), 0, st, a, phi, n1, n2, n3, part);
  else if (n3 <= 64)
    hipLaunchKernelGGL(sketch_mfma_pipe_kernel<4>, grid, dim3(SNT), 0, st, a, phi, n1, n2, n3, part);
  else if (n3 <= 128)
    hipLaunchKernelGGL(sketch_mfma_pipe_kernel<8>, grid, dim3(SNT), 0, st, a, phi, n1, n2, n3, part);
  else
    hipLaunchKernelGGL(sketch_mfma_kernel, grid, dim3(SNT), lds, st, a, phi, n1, n2, n3, part);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(sketch_sum_kernel, dim3((unsigned)nbs), dim3(256), 0, st, part, nch, n2, sk, gpart);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(sketch_whiten_kernel, dim3(1), dim3(256), 0, st, gpart, nbs, n2, wt);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(sketch_apply_kernel, dim3(nblk(n2 * DIN)), dim3(256), 0, st, sk, wt, n2, feat, norms);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int mlp_forward(const float* P, const float* feat, int64_t nrows, float* out, hipStream_t st) {
  if (nrows == 0) return TP_OK;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((nrows + TR - 1) / TR)), dim3(NT), 0, st, P, feat, nrows,
                     out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

size_t mlp_train_ws(int64_t ntensors, int64_t nslices) {
  const int64_t rows = ntensors * nslices, ntiles = (rows + TR - 1) / TR;
  return 3 * align_up(size_t(rows) * 4) + align_up(size_t(ntiles) * NPARAM * 4) + align_up(size_t(NPARAM) * 4) +
         align_up(size_t(ntensors) * 4) + 2048;
}

int mlp_train_step(float* P, float* M, float* V, int64_t step, double lr, const float* feat, const float* target,
                   int64_t T, int64_t nsl, float* loss, float* grad_out, void* ws, hipStream_t st) {
  const int64_t rows = T * nsl, ntiles = (rows + TR - 1) / TR;
  Arena ar(ws, mlp_train_ws(T, nsl));
  float* o = ar.take<float>(rows);
  float* dout = ar.take<float>(rows);
  float* part = ar.take<float>(ntiles * NPARAM);
  float* grad = ar.take<float>(NPARAM);
  float* lpart = ar.take<float>(T);
  if (!ar.ok()) return fail(TP_EWORKSPACE, "training workspace too small");
  if (int rc = mlp_forward(P, feat, rows, o, st)) return rc;
  hipLaunchKernelGGL(softmax_grad_kernel, dim3((unsigned)T), dim3(256), 0, st, o, target, nsl, T, dout, lpart);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(mlp_backward_kernel, dim3((unsigned)ntiles), dim3(NT), 0, st, P, feat, dout, rows, part);
  TP_LAUNCH_CHECK();
  float* g = grad_out ? grad_out : grad;
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(nblk(NPARAM)), dim3(256), 0, st, part, ntiles, g);
  TP_LAUNCH_CHECK();
  if (loss) {
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(64), 0, st, lpart, T, loss);
    TP_LAUNCH_CHECK();
  }
  if (step > 0) {
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(NPARAM)), dim3(256), 0, st, P, M, V, g, (float)lr, (float)b1,
                       (float)b2, 1e-8f, (float)c1, (float)c2);
    TP_LAUNCH_CHECK();
  }
  return TP_OK;
}

int mlp_proposal(const float* logits, int64_t n, double alpha, double* w, hipStream_t st) {
  hipLaunchKernelGGL(proposal_kernel, dim3(1), dim3(256), 0, st, logits, n, alpha, w);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
