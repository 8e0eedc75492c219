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
//
// Up to 8192 slices a single workgroup quantises, scans and picks; above
// that every pass runs one thread per slice over many workgroups, with the
// per-workgroup integer sums scanned by one workgroup in between (integer
// sums are exact, so both routes give the same bits).
#include <algorithm>

#include "common.hpp"

namespace tp {
namespace {

constexpr int SB = 1024;    // threads of the single-workgroup kernels
constexpr int64_t kSmallN = 8192;  // up to this many slices one workgroup picks

struct Meta {
  unsigned long long S;
  int ok;
  int shift;  // the quantisation scale: q_i = floor(w_i 2^shift)
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

// Bernoulli (Algorithm 2's coin flips): slice i is kept iff c q_i >= S or
// floor(u_i S / 2^64) < c q_i.
__device__ __forceinline__ unsigned long long bern_keep(unsigned long long qi, int64_t i, int64_t c, uint64_t seed,
                                                        uint64_t stream, unsigned long long S) {
  const unsigned long long t = (unsigned long long)c * qi;
  if (t >= S) return 1;
  const uint64_t u = philox_word0(seed, stream, (uint64_t)i);
  return __umul64hi(u, S) < t ? 1 : 0;
}

// Up to kSmallN slices one workgroup does the whole pick (fewer launches):
// it validates and quantises the weights and, for IID, forms the inclusive
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
      keep = bern_keep(q[i], i, c, seed, stream, S);
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

// The multi-workgroup passes below give each thread one candidate slice;
// PB threads per workgroup.
constexpr int PB = 256;

// Inclusive scan over a PB-thread workgroup; also returns the total.
__device__ unsigned long long block_inclusive_scan(unsigned long long v, unsigned long long* wave_tot,
                                                   unsigned long long* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wave_tot[wid] = x;
  __syncthreads();
  unsigned long long off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < PB / 64; ++w) {
    const unsigned long long t = wave_tot[w];
    off += w < wid ? t : 0ull;
    tot += t;
  }
  *total = tot;
  __syncthreads();
  return off + x;
}

// Pass 1 of the weight check: per-workgroup maximum and a flag for any
// negative, infinite or NaN weight.
__global__ __launch_bounds__(PB) void weight_stats_kernel(const double* __restrict__ w, int64_t n,
                                                          double* __restrict__ part_max, int* __restrict__ part_bad) {
  __shared__ double smax[PB];
  __shared__ int sbad[PB];
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  double m = 0.0;
  int bad = 0;
  if (i < n) {
    const double v = w[i];
    if (!(v >= 0.0) || isinf(v)) bad = 1;
    else m = v;
  }
  smax[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int k = PB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + k]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_max[blockIdx.x] = smax[0];
    part_bad[blockIdx.x] = sbad[0];
  }
}

// Pass 2 (one workgroup): the maximum weight, the quantisation scale and the
// verdict; rejected weights leave meta->ok = 0 and *count = -1.
__global__ __launch_bounds__(PB) void weight_meta_kernel(const double* __restrict__ part_max,
                                                         const int* __restrict__ part_bad, int64_t nb, int64_t n,
                                                         Meta* meta, int64_t* count) {
  __shared__ double smax[PB];
  __shared__ int sbad[PB];
  double m = 0.0;
  int bad = 0;
  for (int64_t b = threadIdx.x; b < nb; b += PB) {
    m = fmax(m, part_max[b]);
    bad |= part_bad[b];
  }
  smax[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int k = PB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + k]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double wmax = smax[0];
  if (sbad[0] || !(wmax > 0.0)) {
    meta->ok = 0;
    meta->S = 0;
    meta->shift = 0;
    *count = -1;
    return;
  }
  int e = 0;
  (void)frexp(wmax, &e);
  meta->ok = 1;
  meta->shift = 62 - ceil_log2(n) - e;
}

// Pass 3: q_i = floor(w_i 2^shift) (a power-of-two scaling: exact), and the
// per-workgroup sums of q.
__global__ __launch_bounds__(PB) void quantize_kernel(const double* __restrict__ w, int64_t n, const Meta* meta,
                                                      unsigned long long* __restrict__ q,
                                                      unsigned long long* __restrict__ part) {
  __shared__ unsigned long long wave_tot[PB / 64];
  if (!meta->ok) return;
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  unsigned long long qi = 0;
  if (i < n) {
    qi = (unsigned long long)floor(ldexp(w[i], meta->shift));
    q[i] = qi;
  }
  unsigned long long tot;
  (void)block_inclusive_scan(qi, wave_tot, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One workgroup: exclusive prefix sums of nb per-workgroup totals in place
// (exact integers), the grand total into *total; does nothing when meta
// marks rejected weights.
__global__ __launch_bounds__(PB) void scan_parts_kernel(unsigned long long* __restrict__ part, int64_t nb,
                                                        const Meta* meta, unsigned long long* __restrict__ total) {
  __shared__ unsigned long long wave_tot[PB / 64];
  if (meta && !meta->ok) return;
  unsigned long long carry = 0;
  for (int64_t base = 0; base < nb; base += PB) {
    const int64_t b = base + threadIdx.x;
    const unsigned long long v = b < nb ? part[b] : 0ull;
    unsigned long long tot;
    const unsigned long long inc = block_inclusive_scan(v, wave_tot, &tot);
    if (b < nb) part[b] = carry + inc - v;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// IID: inclusive prefix sums P_i of q from the workgroup offsets.
__global__ __launch_bounds__(PB) void prefix_kernel(const unsigned long long* __restrict__ q, int64_t n,
                                                    const Meta* meta, const unsigned long long* __restrict__ part,
                                                    unsigned long long* __restrict__ P) {
  __shared__ unsigned long long wave_tot[PB / 64];
  if (!meta->ok) return;
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  const unsigned long long qi = i < n ? q[i] : 0ull;
  unsigned long long tot;
  const unsigned long long inc = block_inclusive_scan(qi, wave_tot, &tot);
  if (i < n) P[i] = part[blockIdx.x] + inc;
}

// Bernoulli, multi-workgroup pass 1: keep decisions and their
// per-workgroup counts.
__global__ __launch_bounds__(PB) void bernoulli_count_kernel(const unsigned long long* __restrict__ q, int64_t n,
                                                             int64_t c, uint64_t seed, uint64_t stream,
                                                             const Meta* meta, unsigned long long* __restrict__ part) {
  __shared__ unsigned long long wave_tot[PB / 64];
  if (!meta->ok) return;
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  const unsigned long long keep = i < n ? bern_keep(q[i], i, c, seed, stream, meta->S) : 0ull;
  unsigned long long tot;
  (void)block_inclusive_scan(keep, wave_tot, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Pass 2: every kept slice writes its index and scale
// 1/sqrt(min(1, c q_i / S)) at its rank among the kept ones (ascending slice
// order, as Algorithm 2 fills S and D); workgroup 0 writes the count.
__global__ __launch_bounds__(PB) void bernoulli_write_kernel(const unsigned long long* __restrict__ q, int64_t n,
                                                             int64_t c, uint64_t seed, uint64_t stream,
                                                             const Meta* meta,
                                                             const unsigned long long* __restrict__ part,
                                                             const unsigned long long* __restrict__ kept,
                                                             int32_t* __restrict__ idx, double* __restrict__ scale,
                                                             int64_t* count) {
  __shared__ unsigned long long wave_tot[PB / 64];
  if (!meta->ok) return;
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  const unsigned long long S = meta->S;
  unsigned long long keep = 0, t = 0;
  if (i < n) {
    t = (unsigned long long)c * q[i];
    keep = bern_keep(q[i], i, c, seed, stream, S);
  }
  unsigned long long tot;
  const unsigned long long pos = part[blockIdx.x] + block_inclusive_scan(keep, wave_tot, &tot) - keep;
  if (keep) {
    const double p = fmin(1.0, (double)t / (double)S);
    idx[pos] = (int32_t)i;
    scale[pos] = 1.0 / sqrt(p);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = (int64_t)*kept;
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

// Uniform picks without replacement: the c smallest pairs (u_i, i) in
// lexicographic order, which is the c smallest u_i with ties to the smaller
// i. The pair of rank c-1 is found by a radix select: one pass over all keys
// histograms their top byte, the keys in the byte that holds rank c-1 are
// gathered (about n/256 of them), and one workgroup finishes the select on
// that short list, first on the remaining key bits, then on the index among
// equal keys.
constexpr int UG = 128;  // workgroups of the key pass (histogram rows)

struct UMeta {
  unsigned long long v;     // key of the pair of rank c-1
  long long iv;             // its index
  long long rank;           // rank of that pair among the gathered keys
  unsigned long long ncand; // number of gathered keys
  int digit;                // top byte of v
};

__global__ __launch_bounds__(PB) void uniform_keys_kernel(int64_t n, uint64_t seed, uint64_t stream,
                                                          unsigned long long* __restrict__ keys,
                                                          unsigned int* __restrict__ rows) {
  __shared__ unsigned int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x; i < n; i += (int64_t)gridDim.x * PB) {
    const unsigned long long k = philox_word0(seed, stream, (uint64_t)i);
    keys[i] = k;
    atomicAdd(&hist[k >> 56], 1u);
  }
  __syncthreads();
  rows[(size_t)blockIdx.x * 256 + threadIdx.x] = hist[threadIdx.x];
}

// One workgroup of 1024 threads: the top byte that holds rank c-1 and the
// rank within it. Thread t sums bin t mod 256 over every fourth row.
__global__ __launch_bounds__(SB) void uniform_bin_kernel(const unsigned int* __restrict__ rows, int nrows, int64_t c,
                                                         UMeta* um) {
  __shared__ unsigned int part[SB];
  __shared__ unsigned long long wave_tot[PB / 64];
  const int bin = threadIdx.x & 255, q4 = threadIdx.x >> 8;
  unsigned int h = 0;
#pragma unroll 8
  for (int r = q4; r < nrows; r += 4) h += rows[(size_t)r * 256 + bin];
  part[threadIdx.x] = h;
  __syncthreads();
  // inclusive scan of the 256 bin totals by the first four waves
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long hb = 0, inc = 0;
  if (threadIdx.x < 256) {
    hb = (unsigned long long)part[bin] + part[bin + 256] + part[bin + 512] + part[bin + 768];
    inc = hb;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned long long y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    if (lane == 63) wave_tot[wid] = inc;
  }
  __syncthreads();
  if (threadIdx.x >= 256) return;
  for (int w = 0; w < wid; ++w) inc += wave_tot[w];
  const unsigned long long below = inc - hb, want = (unsigned long long)(c - 1);
  if (below <= want && want < inc) {
    um->digit = bin;
    um->rank = (long long)(want - below);
    um->ncand = 0;
  }
}

__global__ __launch_bounds__(PB) void uniform_gather_kernel(const unsigned long long* __restrict__ keys, int64_t n,
                                                            UMeta* um, unsigned long long* __restrict__ ckey,
                                                            unsigned long long* __restrict__ cidx) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  const unsigned long long k = i < n ? keys[i] : 0ull;
  const bool hit = i < n && (int)(k >> 56) == um->digit;
  // one counter update per wave
  const unsigned long long ball = __ballot(hit);
  if (!ball) return;
  const int leader = __ffsll((long long)ball) - 1;
  unsigned long long base = 0;
  if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(&um->ncand, (unsigned long long)__popcll(ball));
  base = __shfl(base, leader, 64);
  if (!hit) return;
  const unsigned int below =
      __builtin_amdgcn_mbcnt_hi((unsigned int)(ball >> 32), __builtin_amdgcn_mbcnt_lo((unsigned int)ball, 0u));
  ckey[base + below] = k;
  cidx[base + below] = (unsigned long long)i;
}

// One workgroup: the pair of rank um->rank among the m gathered ones,
// 8 bits at a time (key bits 55..0, then index bits 31..0 among the keys
// equal to the selected one). A pass whose chosen digit holds a single
// candidate ends the select: that candidate is the pair.
__global__ __launch_bounds__(SB) void uniform_pick_kernel(const unsigned long long* __restrict__ ckey,
                                                          const unsigned long long* __restrict__ cidx, UMeta* um) {
  __shared__ unsigned int hist[256];
  __shared__ unsigned long long sprefix, smask, sv, siv;
  __shared__ long long srank;
  __shared__ int sone;
  const int64_t m = (int64_t)um->ncand;
  if (threadIdx.x == 0) {
    sprefix = (unsigned long long)um->digit << 56;
    smask = 255ull << 56;
    srank = um->rank;
    sv = 0;
  }
  for (int pass = 0; pass < 11; ++pass) {
    const bool on_key = pass < 7;
    const int shift = on_key ? 48 - 8 * pass : 24 - 8 * (pass - 7);
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    __syncthreads();
    const unsigned long long prefix = sprefix, mask = smask, v = sv;
    for (int64_t j = threadIdx.x; j < m; j += SB) {
      const unsigned long long k = ckey[j];
      if (on_key) {
        if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255ull], 1u);
      } else if (k == v) {
        const unsigned long long x = cidx[j];
        if ((x & mask) == prefix) atomicAdd(&hist[(x >> shift) & 255ull], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // the digit holding rank srank: lane l owns digits 4l..4l+3
      const int l = threadIdx.x;
      const unsigned int h0 = hist[4 * l], h1 = hist[4 * l + 1], h2 = hist[4 * l + 2], h3 = hist[4 * l + 3];
      const unsigned long long own = (unsigned long long)h0 + h1 + h2 + h3;
      unsigned long long inc = own;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(inc, d, 64);
        if (l >= d) inc += y;
      }
      const long long r = srank, below = (long long)(inc - own);
      if (below <= r && r < (long long)inc) {
        long long rr = r - below;
        int d = 4 * l;
        unsigned int h = h0;
        if (rr >= (long long)h) { rr -= h; ++d; h = h1;
          if (rr >= (long long)h) { rr -= h; ++d; h = h2;
            if (rr >= (long long)h) { rr -= h; ++d; h = h3; } } }
        srank = rr;
        sprefix = prefix | ((unsigned long long)d << shift);
        smask = mask | (255ull << shift);
        sone = h == 1;
      }
    }
    __syncthreads();
    if (sone) {
      const unsigned long long pf = sprefix, mk = smask;
      for (int64_t j = threadIdx.x; j < m; j += SB) {
        const unsigned long long k = ckey[j];
        if (on_key) {
          if ((k & mk) == pf) {
            sv = k;
            siv = cidx[j];
          }
        } else if (k == v && (cidx[j] & mk) == pf) {
          siv = cidx[j];
        }
      }
      __syncthreads();
      break;
    }
    if (threadIdx.x == 0) {
      if (pass == 6) {
        sv = sprefix;  // the key is fixed; select the index among equals
        sprefix = 0;
        smask = 0;
      } else if (pass == 10) {
        siv = sprefix;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    um->v = sv;
    um->iv = (long long)siv;
  }
}

__device__ __forceinline__ unsigned long long uniform_keep(const unsigned long long* keys, int64_t i, int64_t n,
                                                           const UMeta* um) {
  if (i >= n) return 0;
  const unsigned long long k = keys[i], v = um->v;
  return (k < v || (k == v && i <= um->iv)) ? 1ull : 0ull;
}

__global__ __launch_bounds__(PB) void uniform_count_kernel(const unsigned long long* __restrict__ keys, int64_t n,
                                                           const UMeta* um, unsigned long long* __restrict__ part) {
  __shared__ unsigned long long wave_tot[PB / 64];
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  unsigned long long tot;
  (void)block_inclusive_scan(uniform_keep(keys, i, n, um), wave_tot, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(PB) void uniform_write_kernel(const unsigned long long* __restrict__ keys, int64_t n,
                                                           int64_t c, const UMeta* um,
                                                           const unsigned long long* __restrict__ part,
                                                           int32_t* __restrict__ idx, double* __restrict__ scale,
                                                           int64_t* count) {
  __shared__ unsigned long long wave_tot[PB / 64];
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  const unsigned long long keep = uniform_keep(keys, i, n, um);
  unsigned long long tot;
  const unsigned long long pos = part[blockIdx.x] + block_inclusive_scan(keep, wave_tot, &tot) - keep;
  if (keep) {
    idx[pos] = (int32_t)i;
    scale[pos] = sqrt((double)n / (double)c);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = c;
}

int64_t sampler_blocks(int64_t n) { return (n + PB - 1) / PB; }

int uniform_rows(int64_t n) { return (int)std::min<int64_t>(UG, sampler_blocks(n)); }

}  // namespace

size_t sampler_ws(int64_t n) {
  const size_t nb = size_t(sampler_blocks(n));
  return 3 * align_up(size_t(n) * 8) + 3 * align_up(nb * 8) + align_up(nb * 4) +
         align_up(size_t(uniform_rows(n)) * 256 * 4) + 4 * 256;
}

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
  const int64_t nb = sampler_blocks(n);
  Arena ar(ws, sampler_ws(n));
  auto* q = ar.take<unsigned long long>(n);
  auto* P = ar.take<unsigned long long>(n);
  auto* keys = ar.take<unsigned long long>(n);
  auto* part = ar.take<unsigned long long>(nb);
  auto* part_max = ar.take<double>(nb);
  auto* bpart = ar.take<unsigned long long>(nb);
  auto* part_bad = ar.take<int>(nb);
  auto* rows = ar.take<unsigned int>(size_t(uniform_rows(n)) * 256);
  auto* meta = ar.take<Meta>(1);
  auto* kept = ar.take<unsigned long long>(1);
  auto* um = ar.take<UMeta>(1);
  if (!ar.ok()) return fail(TP_EWORKSPACE, "sampler workspace too small");
  const dim3 grid((unsigned)nb), blk(PB);
  if (mode != TP_S_UNIFORM && n <= kSmallN) {
    hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(SB), 0, st, w, n, mode == TP_S_IID ? 1 : 0, q, P, meta, count);
    if (mode == TP_S_BERNOULLI) {
      hipLaunchKernelGGL(bernoulli_kernel, dim3(1), dim3(SB), 0, st, q, n, c, seed, stream_id, meta, idx, scale,
                         count);
    } else {
      hipLaunchKernelGGL(iid_kernel, dim3((unsigned)((c + 255) / 256)), dim3(256), 0, st, q, P, n, c, seed,
                         stream_id, meta, idx, scale, count);
    }
    TP_LAUNCH_CHECK();
    return TP_OK;
  }
  if (mode == TP_S_UNIFORM) {
    // the c smallest (key, index) pairs; q and P hold the gathered keys
    const int nrows = uniform_rows(n);
    hipLaunchKernelGGL(uniform_keys_kernel, dim3(nrows), blk, 0, st, n, seed, stream_id, keys, rows);
    hipLaunchKernelGGL(uniform_bin_kernel, dim3(1), dim3(SB), 0, st, rows, nrows, c, um);
    hipLaunchKernelGGL(uniform_gather_kernel, grid, blk, 0, st, keys, n, um, P, q);
    hipLaunchKernelGGL(uniform_pick_kernel, dim3(1), dim3(SB), 0, st, P, q, um);
    hipLaunchKernelGGL(uniform_count_kernel, grid, blk, 0, st, keys, n, um, bpart);
    hipLaunchKernelGGL(scan_parts_kernel, dim3(1), blk, 0, st, bpart, nb, nullptr, kept);
    hipLaunchKernelGGL(uniform_write_kernel, grid, blk, 0, st, keys, n, c, um, bpart, idx, scale, count);
    TP_LAUNCH_CHECK();
    return TP_OK;
  }
  // weights: check and maximum, scale, quantised values and their sum S
  hipLaunchKernelGGL(weight_stats_kernel, grid, blk, 0, st, w, n, part_max, part_bad);
  hipLaunchKernelGGL(weight_meta_kernel, dim3(1), blk, 0, st, part_max, part_bad, nb, n, meta, count);
  hipLaunchKernelGGL(quantize_kernel, grid, blk, 0, st, w, n, meta, q, part);
  hipLaunchKernelGGL(scan_parts_kernel, dim3(1), blk, 0, st, part, nb, meta, &meta->S);
  TP_LAUNCH_CHECK();
  if (mode == TP_S_BERNOULLI) {
    hipLaunchKernelGGL(bernoulli_count_kernel, grid, blk, 0, st, q, n, c, seed, stream_id, meta, bpart);
    hipLaunchKernelGGL(scan_parts_kernel, dim3(1), blk, 0, st, bpart, nb, meta, kept);
    hipLaunchKernelGGL(bernoulli_write_kernel, grid, blk, 0, st, q, n, c, seed, stream_id, meta, bpart, kept, idx,
                       scale, count);
  } else {
    hipLaunchKernelGGL(prefix_kernel, grid, blk, 0, st, q, n, meta, part, P);
    const int64_t blocks = (c + 255) / 256;
    hipLaunchKernelGGL(iid_kernel, dim3((unsigned)blocks), dim3(256), 0, st, q, P, n, c, seed, stream_id, meta, idx,
                       scale, count);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
