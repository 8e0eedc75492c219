// Slice picks of Algorithm 2 (lines "pick i with probability min{1, c p_i}",
// the rescaling D_tt = 1/min{1, sqrt(c p_i)}) and the same loops in
// Algorithms 4 and 5, plus the with-replacement and uniform
// without-replacement schemes used by the paper's corollaries.
//
// The paper fixes neither the generator nor the arithmetic of the coin
// flips. Every decision here is an exact integer comparison, so any
// implementation that follows the same steps picks the same slices:
//  * weights w_i >= 0 are quantised to q_i = floor(w_i 2^(B-e)) where
//    w_max = m 2^e, m in [0.5, 1), and B = 62 - ceil(log2 n); the scaling is
//    by a power of two, so it is exact, and S = sum q_i < 2^62;
//  * u_i is word 0 of Philox4x64-10 (Salmon et al., SC'11) with key
//    (seed, stream_id) and counter (i, 0, 0, 0);
//  * Bernoulli: keep i iff c q_i >= S or floor(u_i S / 2^64) < c q_i;
//  * IID: draw t takes T = floor(u_t S / 2^64) and the first i whose
//    inclusive prefix sum of q exceeds T;
//  * uniform: the c smallest u_i (ties to the smaller i).
// Scales are float64 1/sqrt(min(1, c q_i / S)) (IID: 1/sqrt(c q_j / S),
// uniform: sqrt(n / c)).
#include "common.hpp"

namespace tp {
namespace {

constexpr int SB = 1024;  // threads of the single-workgroup kernels

struct Meta {
  unsigned long long S;
  int ok;
};

__device__ __forceinline__ uint64_t philox_word0(uint64_t seed, uint64_t stream, uint64_t index) {
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
  return x0;
}

// Exclusive block scan over SB threads; also returns the block total.
template <typename T>
__device__ T block_exclusive_scan(T v, T* wave_tot, T* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wave_tot[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < SB / 64; ++w) {
      const T t = wave_tot[w];
      wave_tot[w] = acc;
      acc += t;
    }
    wave_tot[SB / 64] = acc;
  }
  __syncthreads();
  const T r = wave_tot[wid] + x - v;
  *total = wave_tot[SB / 64];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int ceil_log2(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

// Validates and quantises the weights; for IID also forms inclusive
// prefix sums. Leaves meta->ok = 0 and *count = -1 on bad weights.
__global__ __launch_bounds__(SB) void prepare_kernel(const double* __restrict__ w, int64_t n, int want_prefix,
                                                     unsigned long long* __restrict__ q,
                                                     unsigned long long* __restrict__ P, Meta* meta,
                                                     int64_t* count) {
  __shared__ double smax[SB];
  __shared__ int sbad[SB];
  __shared__ unsigned long long wave_tot[SB / 64 + 1];
  double m = 0.0;
  int bad = 0;
  for (int64_t i = threadIdx.x; i < n; i += SB) {
    const double v = w[i];
    if (!(v >= 0.0) || isinf(v)) bad = 1;
    else m = fmax(m, v);
  }
  smax[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = SB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  const double wmax = smax[0];
  if (sbad[0] || !(wmax > 0.0)) {
    if (threadIdx.x == 0) {
      meta->ok = 0;
      meta->S = 0;
      *count = -1;
    }
    return;
  }
  int e = 0;
  (void)frexp(wmax, &e);
  const int shift = 62 - ceil_log2(n) - e;
  unsigned long long carry = 0;
  for (int64_t base = 0; base < n; base += SB) {
    const int64_t i = base + threadIdx.x;
    unsigned long long qi = 0;
    if (i < n) {
      qi = (unsigned long long)floor(ldexp(w[i], shift));
      q[i] = qi;
    }
    unsigned long long tot;
    const unsigned long long ex = block_exclusive_scan<unsigned long long>(qi, wave_tot, &tot);
    if (want_prefix && i < n) P[i] = carry + ex + qi;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    meta->S = carry;
    meta->ok = 1;
  }
}

__global__ __launch_bounds__(SB) void bernoulli_kernel(const unsigned long long* __restrict__ q, int64_t n,
                                                       int64_t c, uint64_t seed, uint64_t stream,
                                                       const Meta* meta, int32_t* __restrict__ idx,
                                                       double* __restrict__ scale, int64_t* count) {
  __shared__ unsigned long long wave_tot[SB / 64 + 1];
  if (!meta->ok) return;
  const unsigned long long S = meta->S;
  unsigned long long written = 0;
  for (int64_t base = 0; base < n; base += SB) {
    const int64_t i = base + threadIdx.x;
    unsigned long long keep = 0;
    unsigned long long t = 0;
    if (i < n) {
      t = (unsigned long long)c * q[i];
      if (t >= S) {
        keep = 1;
      } else {
        const uint64_t u = philox_word0(seed, stream, (uint64_t)i);
        keep = (__umul64hi(u, S) < t) ? 1 : 0;
      }
    }
    unsigned long long tot;
    const unsigned long long pos = block_exclusive_scan<unsigned long long>(keep, wave_tot, &tot);
    if (keep) {
      const double p = fmin(1.0, (double)t / (double)S);
      idx[written + pos] = (int32_t)i;
      scale[written + pos] = 1.0 / sqrt(p);
    }
    written += tot;
  }
  if (threadIdx.x == 0) *count = (int64_t)written;
}

__global__ void iid_kernel(const unsigned long long* __restrict__ q, const unsigned long long* __restrict__ P,
                           int64_t n, int64_t c, uint64_t seed, uint64_t stream, const Meta* meta,
                           int32_t* __restrict__ idx, double* __restrict__ scale, int64_t* count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!meta->ok) return;
  if (t == 0) *count = c;
  if (t >= c) return;
  const unsigned long long S = meta->S;
  const uint64_t u = philox_word0(seed, stream, (uint64_t)t);
  const unsigned long long T = __umul64hi(u, S);
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (P[mid] > T) hi = mid;
    else lo = mid + 1;
  }
  idx[t] = (int32_t)lo;
  scale[t] = 1.0 / sqrt((double)((unsigned long long)c * q[lo]) / (double)S);
}

__global__ __launch_bounds__(SB) void uniform_kernel(int64_t n, int64_t c, uint64_t seed, uint64_t stream,
                                                     unsigned long long* __restrict__ keys,
                                                     int32_t* __restrict__ idx, double* __restrict__ scale,
                                                     int64_t* count) {
  __shared__ unsigned int hist[256];
  __shared__ unsigned long long sprefix, smask;
  __shared__ long long srank;
  __shared__ unsigned long long wave_tot[SB / 64 + 1];
  for (int64_t i = threadIdx.x; i < n; i += SB) keys[i] = philox_word0(seed, stream, (uint64_t)i);
  if (threadIdx.x == 0) {
    sprefix = 0;
    smask = 0;
    srank = c - 1;
  }
  __syncthreads();
  // radix select of the element of rank c-1 (0-based), most significant
  // byte first
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int b = threadIdx.x; b < 256; b += SB) hist[b] = 0;
    __syncthreads();
    const unsigned long long prefix = sprefix, mask = smask;
    for (int64_t i = threadIdx.x; i < n; i += SB) {
      const unsigned long long k = keys[i];
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      long long r = srank;
      int d = 0;
      for (; d < 256; ++d) {
        if (r < (long long)hist[d]) break;
        r -= hist[d];
      }
      srank = r;
      sprefix = prefix | ((unsigned long long)d << shift);
      smask = mask | (255ull << shift);
    }
    __syncthreads();
  }
  const unsigned long long v = sprefix;
  const long long take_eq = srank + 1;  // how many keys equal to v are kept
  unsigned long long written = 0, eq_seen = 0;
  const double sc = sqrt((double)n / (double)c);
  for (int64_t base = 0; base < n; base += SB) {
    const int64_t i = base + threadIdx.x;
    const unsigned long long k = i < n ? keys[i] : ~0ull;
    const unsigned long long is_eq = (i < n && k == v) ? 1 : 0;
    unsigned long long eq_tot;
    const unsigned long long eq_rank = eq_seen + block_exclusive_scan<unsigned long long>(is_eq, wave_tot, &eq_tot);
    eq_seen += eq_tot;
    const unsigned long long keep = (i < n && (k < v || (is_eq && (long long)eq_rank < take_eq))) ? 1 : 0;
    unsigned long long tot;
    const unsigned long long pos = block_exclusive_scan<unsigned long long>(keep, wave_tot, &tot);
    if (keep) {
      idx[written + pos] = (int32_t)i;
      scale[written + pos] = sc;
    }
    written += tot;
  }
  if (threadIdx.x == 0) *count = (int64_t)written;
}

}  // namespace

size_t sampler_ws(int64_t n) { return 3 * align_up(size_t(n) * 8) + 256; }

namespace {
// out = sum of n pick counts, or -1 if any of them is -1 (rejected weights)
__global__ void join_counts_kernel(const int64_t* __restrict__ counts, int n, int64_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t t = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t c = counts[i];
    if (c < 0) {
      t = -1;
      break;
    }
    t += c;
  }
  *out = t;
}
}  // namespace

int join_counts(const int64_t* counts, int n, int64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(join_counts_kernel, dim3(1), dim3(64), 0, st, counts, n, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int sample_slices(const double* w, int64_t n, int64_t c, int mode, uint64_t seed, uint64_t stream_id, int32_t* idx,
                  double* scale, int64_t* count, void* ws, hipStream_t st) {
  Arena ar(ws, sampler_ws(n));
  auto* q = ar.take<unsigned long long>(n);
  auto* P = ar.take<unsigned long long>(n);
  auto* keys = ar.take<unsigned long long>(n);
  auto* meta = ar.take<Meta>(1);
  if (!ar.ok()) return fail(TP_EWORKSPACE, "sampler workspace too small");
  if (mode == TP_S_UNIFORM) {
    hipLaunchKernelGGL(uniform_kernel, dim3(1), dim3(SB), 0, st, n, c, seed, stream_id, keys, idx, scale, count);
    TP_LAUNCH_CHECK();
    return TP_OK;
  }
  hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(SB), 0, st, w, n, mode == TP_S_IID ? 1 : 0, q, P, meta, count);
  TP_LAUNCH_CHECK();
  if (mode == TP_S_BERNOULLI) {
    hipLaunchKernelGGL(bernoulli_kernel, dim3(1), dim3(SB), 0, st, q, n, c, seed, stream_id, meta, idx, scale, count);
  } else {
    const int64_t blocks = (c + 255) / 256;
    hipLaunchKernelGGL(iid_kernel, dim3((unsigned)blocks), dim3(256), 0, st, q, P, n, c, seed, stream_id, meta, idx,
                       scale, count);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
