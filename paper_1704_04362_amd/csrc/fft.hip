// Tube transforms along the third mode (Section 2.1 "Operators": fft/ifft
// along mode 3, MATLAB convention; the transforms that open and close
// Algorithm 1).
//
// Layout: the tensor is tube-major (each tube X_{ij:} is n3 contiguous
// values); the spectrum is slice-major planar, re[k][tube] / im[k][tube],
// holding the K = n3/2 + 1 non-redundant slices.
//
// Forward kernel (one wavefront = 64 tubes):
//   1. the 64 tubes are read with 16-byte loads, consecutive lanes reading
//      consecutive pieces of a tube, and staged in LDS with a row stride of
//      n3 + 1 words so that the transposed read below is conflict free;
//      gathers of picked slices and their scales are applied here;
//   2. every lane packs its real tube as z[m] = x[2m] + i x[2m+1] and runs a
//      length-n3/2 complex FFT in registers (radix 4/2/5/3 Cooley-Tukey and
//      a direct DFT for other prime factors, fully unrolled, twiddles from a
//      per-device constant table);
//   3. the half spectrum of the real tube is separated from Z by conjugate
//      symmetry, X[k] = (Z[k] + conj Z[M-k])/2 + W_n3^k (Z[k] - conj Z[M-k])/2i,
//      and each slice k is written with one coalesced store per wavefront.
// The inverse kernel runs these steps backwards. Long tubes (n3 above 256
// without a specialised kernel, prime factors up to 13) use a
// workgroup-per-tube mixed-radix transform in LDS; even ones beyond its LDS
// budget (up to 2^19) a four-step transform through HBM; lengths from 257
// with a larger prime factor, up to 2048 (float32) / 1024 (float64),
// Bluestein's chirp-z transform in LDS; the rest a direct O(n3^2) transform.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace tp {
namespace {

// --------------------------------------------------------------------------
// Twiddle tables: W_L^e = exp(-2 pi i e / L) for the lengths below, stored
// back to back (re, im interleaved), computed on the host in long double.
// --------------------------------------------------------------------------
constexpr int kTwLens[] = {1, 2, 4, 8, 16, 32, 64, 128, 256, 5, 10, 20, 25, 50, 100, 200, 7, 21, 84, 168};
constexpr int kTwCount = sizeof(kTwLens) / sizeof(int);

constexpr int tw_offset(int L) {
  int off = 0;
  for (int i = 0; i < kTwCount; ++i) {
    if (kTwLens[i] == L) return off;
    off += kTwLens[i];
  }
  return -1;
}
constexpr int kTwTotal = tw_offset(168) + 168;

__constant__ double g_tw64[2 * kTwTotal];
__constant__ float g_tw32[2 * kTwTotal];

template <typename T>
__device__ __forceinline__ T tw_re(int L, int e);
template <typename T>
__device__ __forceinline__ T tw_im(int L, int e);
template <>
__device__ __forceinline__ double tw_re<double>(int L, int e) { return g_tw64[2 * (tw_offset(L) + e)]; }
template <>
__device__ __forceinline__ double tw_im<double>(int L, int e) { return g_tw64[2 * (tw_offset(L) + e) + 1]; }
template <>
__device__ __forceinline__ float tw_re<float>(int L, int e) { return g_tw32[2 * (tw_offset(L) + e)]; }
template <>
__device__ __forceinline__ float tw_im<float>(int L, int e) { return g_tw32[2 * (tw_offset(L) + e) + 1]; }

std::mutex g_tw_mutex;
std::vector<int> g_tw_ready;  // per device

int ensure_twiddles() {
  int dev = 0;
  TP_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tw_mutex);
  if (dev < (int)g_tw_ready.size() && g_tw_ready[dev]) return TP_OK;
  std::vector<double> t64(2 * kTwTotal);
  std::vector<float> t32(2 * kTwTotal);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int i = 0; i < kTwCount; ++i) {
    int L = kTwLens[i], off = tw_offset(L);
    for (int e = 0; e < L; ++e) {
      long double ang = two_pi * (long double)e / (long double)L;
      long double c = cosl(ang), s = -sinl(ang);
      // exact values where the angle is a multiple of pi/2
      if ((4 * e) % L == 0) {
        int q = (4 * e) / L;
        c = (q == 0) ? 1.0L : (q == 2 ? -1.0L : 0.0L);
        s = (q == 1) ? -1.0L : (q == 3 ? 1.0L : 0.0L);
      }
      t64[2 * (off + e)] = (double)c;
      t64[2 * (off + e) + 1] = (double)s;
      t32[2 * (off + e)] = (float)c;
      t32[2 * (off + e) + 1] = (float)s;
    }
  }
  TP_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_tw64), t64.data(), t64.size() * sizeof(double)));
  TP_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_tw32), t32.data(), t32.size() * sizeof(float)));
  if (dev >= (int)g_tw_ready.size()) g_tw_ready.resize(dev + 1, 0);
  g_tw_ready[dev] = 1;
  return TP_OK;
}

// --------------------------------------------------------------------------
// In-register complex FFT of length M (decimation in time).
// --------------------------------------------------------------------------
constexpr int radix_of(int M) {
  return (M % 4 == 0) ? 4 : (M % 2 == 0) ? 2 : (M % 5 == 0) ? 5 : (M % 3 == 0) ? 3 : M;
}

template <typename T, int M>
__device__ __forceinline__ void cfft(T (&re)[M], T (&im)[M]) {
  if constexpr (M > 1) {
    static_assert(tw_offset(M) >= 0, "no twiddle table for this transform length");
    constexpr int p = radix_of(M);
    constexpr int Q = M / p;
    T sr[p][Q], si[p][Q];
#pragma unroll
    for (int r = 0; r < p; ++r)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        sr[r][q] = re[q * p + r];
        si[r][q] = im[q * p + r];
      }
#pragma unroll
    for (int r = 0; r < p; ++r) cfft<T, Q>(sr[r], si[r]);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      T tr[p], ti[p];
#pragma unroll
      for (int r = 0; r < p; ++r) {
        const int e = (r * k) % M;
        if (e == 0) {
          tr[r] = sr[r][k];
          ti[r] = si[r][k];
        } else {
          const T wr = tw_re<T>(M, e), wi = tw_im<T>(M, e);
          tr[r] = sr[r][k] * wr - si[r][k] * wi;
          ti[r] = sr[r][k] * wi + si[r][k] * wr;
        }
      }
      if constexpr (p == 2) {
        re[k] = tr[0] + tr[1];
        im[k] = ti[0] + ti[1];
        re[k + Q] = tr[0] - tr[1];
        im[k + Q] = ti[0] - ti[1];
      } else if constexpr (p == 4) {
        const T ar = tr[0] + tr[2], ai = ti[0] + ti[2];
        const T br = tr[0] - tr[2], bi = ti[0] - ti[2];
        const T cr = tr[1] + tr[3], ci = ti[1] + ti[3];
        // (t1 - t3) * (-i)
        const T dr = ti[1] - ti[3], di = tr[3] - tr[1];
        re[k] = ar + cr;
        im[k] = ai + ci;
        re[k + 2 * Q] = ar - cr;
        im[k + 2 * Q] = ai - ci;
        re[k + Q] = br + dr;
        im[k + Q] = bi + di;
        re[k + 3 * Q] = br - dr;
        im[k + 3 * Q] = bi - di;
      } else {
        // generic p-point DFT with W_p^{rs} = W_M^{r s Q}
#pragma unroll
        for (int s = 0; s < p; ++s) {
          T accr = tr[0], acci = ti[0];
#pragma unroll
          for (int r = 1; r < p; ++r) {
            const int e = (r * s * Q) % M;
            if (e == 0) {
              accr += tr[r];
              acci += ti[r];
            } else {
              const T wr = tw_re<T>(M, e), wi = tw_im<T>(M, e);
              accr += tr[r] * wr - ti[r] * wi;
              acci += tr[r] * wi + ti[r] * wr;
            }
          }
          re[k + s * Q] = accr;
          im[k + s * Q] = acci;
        }
      }
    }
  }
}

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};

struct FwdArgs {
  int64_t rows, cols, in_cols;
  int64_t ntubes;  // output slots: major x ld
  const int32_t* row_idx;
  const int32_t* col_idx;
  const double* row_scale;
  const double* col_scale;
  const int64_t* count;
  int64_t ld;    // slots per major index (>= cols, or >= rows when colmajor)
  int colmajor;  // slot t = col * ld + row instead of row * ld + col
  // > 0 (column-major spectra with ld a multiple of the tile): workgroup b
  // takes the tile (b / nmaj) of major index b mod nmaj, so workgroups that
  // run together read neighbouring tubes of the tube-major input instead of
  // tubes a whole input row apart
  int64_t nmaj;
};

// Input tube offset and scale of output slot t; returns false for a slot
// that is to be written as zeros (padding, or beyond the live sample count).
__device__ __forceinline__ bool tube_source(const FwdArgs& a, int64_t t, int64_t& src, double& s) {
  const int64_t maj = t / a.ld, mn = t - maj * a.ld;
  const int64_t ra = a.colmajor ? mn : maj, cb = a.colmajor ? maj : mn;
  if (ra >= a.rows || cb >= a.cols) return false;
  int64_t lim = a.count ? *a.count : INT64_MAX;
  if (a.row_idx && ra >= lim) return false;
  if (a.col_idx && cb >= lim) return false;
  const int64_t ir = a.row_idx ? a.row_idx[ra] : ra;
  const int64_t ic = a.col_idx ? a.col_idx[cb] : cb;
  src = ir * a.in_cols + ic;
  s = (a.row_scale ? a.row_scale[ra] : 1.0) * (a.col_scale ? a.col_scale[cb] : 1.0);
  return true;
}

constexpr int kTile = 64;  // tubes per workgroup (one wavefront)

// Output of one spectrum value: planar float (re, im planes [k][slot]) or,
// with SPLIT, four bf16 planes [p][k][slot] = hi(re), lo(re), hi(im), lo(im)
// (hi = round-to-nearest-even bf16 of x, lo = bf16 of x - hi), the operand
// format of the matrix-core products.
template <typename T, bool SPLIT>
__device__ __forceinline__ void emit(T* ore, T* oim, int64_t K, int64_t ks, int64_t k, int64_t t, T vr, T vi) {
  if constexpr (SPLIT) {
    __bf16* b = reinterpret_cast<__bf16*>(ore);
    const __bf16 hr = (__bf16)vr, hi = (__bf16)vi;
    const int64_t ps = K * ks, o = k * ks + t;
    b[o] = hr;
    b[ps + o] = (__bf16)(vr - (float)hr);
    b[2 * ps + o] = hi;
    b[3 * ps + o] = (__bf16)(vi - (float)hi);
  } else {
    ore[k * ks + t] = vr;
    oim[k * ks + t] = vi;
  }
}

// Long tubes are staged through LDS in two halves (HALF): half the LDS per
// workgroup, so twice as many wavefronts fit on a compute unit to hide the
// memory latency of this HBM-bound kernel; each lane picks its half tube out
// of LDS between the two stagings.
template <typename T, int N, bool SPLIT = false>
__global__ __launch_bounds__(kTile) void rfft_kernel(const T* __restrict__ x, FwdArgs a, T* __restrict__ ore,
                                                     T* __restrict__ oim) {
  constexpr int M = N / 2;
  static_assert(N <= 2 || tw_offset(N) >= 0, "no twiddle table for this tube length");
  constexpr int VN = Vec16<T>::n;
  constexpr bool HALF = N >= 32 && N % (2 * VN) == 0;
  constexpr int SPAN = HALF ? N / 2 : N;  // tube entries staged at once
  constexpr int PAD = SPAN + 1;
  using V = typename Vec16<T>::type;
  __shared__ T lds[kTile * PAD];
  __shared__ int64_t s_src[kTile];
  __shared__ double s_scl[kTile];
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t tile0 = a.nmaj > 0 ? (b % a.nmaj) * a.ld + (b / a.nmaj) * kTile : b * kTile;
  {
    const int64_t t = tile0 + lane;
    int64_t src = -1;
    double s = 0.0;
    if (!(t < a.ntubes && tube_source(a, t, src, s))) src = -1;
    s_src[lane] = src;
    s_scl[lane] = s;
  }
  __syncthreads();

  // stage tube entries [h SPAN, (h + 1) SPAN) of the 64 tubes
  auto stage = [&](int h) {
    if constexpr (N % VN == 0) {
      constexpr int CH = SPAN / VN;
#pragma unroll
      for (int it = 0; it < CH; ++it) {
        const int f = it * kTile + lane;
        const int tl = f / CH, part = f - tl * CH;
        const int64_t src = s_src[tl];
        const double s = s_scl[tl];
        T v[VN];
#pragma unroll
        for (int e = 0; e < VN; ++e) v[e] = T(0);
        if (src >= 0) {
          const V w = *reinterpret_cast<const V*>(x + src * N + h * SPAN + part * VN);
          const T* wp = reinterpret_cast<const T*>(&w);
#pragma unroll
          for (int e = 0; e < VN; ++e) v[e] = (s == 1.0) ? wp[e] : (T)((double)wp[e] * s);
        }
#pragma unroll
        for (int e = 0; e < VN; ++e) lds[tl * PAD + part * VN + e] = v[e];
      }
    } else {
      for (int it = 0; it < N; ++it) {
        const int f = it * kTile + lane;
        const int tl = f / N, e = f - tl * N;
        const int64_t src = s_src[tl];
        const double s = s_scl[tl];
        T v = T(0);
        if (src >= 0) v = (s == 1.0) ? x[src * N + e] : (T)((double)x[src * N + e] * s);
        lds[tl * PAD + e] = v;
      }
    }
  };

  const int64_t t = tile0 + lane;
  const int64_t ks = a.ntubes;
  constexpr int64_t K = N / 2 + 1;
  if constexpr (N == 1) {
    stage(0);
    __syncthreads();
    if (t >= a.ntubes) return;
    emit<T, SPLIT>(ore, oim, K, ks, 0, t, lds[lane * PAD], T(0));
  } else {
    // z[m] = x[2m] + i x[2m+1]; a half holds z[h SPAN/2 .. (h+1) SPAN/2)
    T zr[M], zi[M];
#pragma unroll
    for (int h = 0; h < N / SPAN; ++h) {
      if (h > 0) __syncthreads();
      stage(h);
      __syncthreads();
#pragma unroll
      for (int m = 0; m < SPAN / 2; ++m) {
        zr[h * (SPAN / 2) + m] = lds[lane * PAD + 2 * m];
        zi[h * (SPAN / 2) + m] = lds[lane * PAD + 2 * m + 1];
      }
    }
    if (t >= a.ntubes) return;
    cfft<T, M>(zr, zi);
    emit<T, SPLIT>(ore, oim, K, ks, 0, t, zr[0] + zi[0], T(0));
    emit<T, SPLIT>(ore, oim, K, ks, M, t, zr[0] - zi[0], T(0));
#pragma unroll
    for (int k = 1; k < M; ++k) {
      const int j = M - k;
      const T er = (zr[k] + zr[j]) * T(0.5), ei = (zi[k] - zi[j]) * T(0.5);
      const T orr = (zi[k] + zi[j]) * T(0.5), oi = (zr[j] - zr[k]) * T(0.5);
      const T wr = tw_re<T>(N, k), wi = tw_im<T>(N, k);
      emit<T, SPLIT>(ore, oim, K, ks, k, t, er + (orr * wr - oi * wi), ei + (orr * wi + oi * wr));
    }
  }
}

// Output staging of the inverse transform: the 64 tubes of a workgroup are
// transposed through LDS in NH pieces of N / NH entries (two for the longer
// tubes, which halves the LDS a workgroup holds and doubles the workgroups
// that fit on a CU).
template <int N>
struct InvStage {
  static constexpr int VN = 4;
  static constexpr int NH = (N >= 64 && N % (2 * VN) == 0) ? 2 : 1;
  static constexpr int SPAN = N / NH;
  static constexpr int PAD = SPAN + 1;
};

template <typename T, int N>
__global__ __launch_bounds__(kTile) void irfft_kernel(const T* __restrict__ xre, const T* __restrict__ xim,
                                                      int64_t ntubes, T* __restrict__ y) {
  constexpr int M = N / 2;
  static_assert(N <= 2 || tw_offset(N) >= 0, "no twiddle table for this tube length");
  using ST = InvStage<N>;
  constexpr int NH = ST::NH, SPAN = ST::SPAN, PAD = ST::PAD;
  constexpr int VN = Vec16<T>::n;
  using V = typename Vec16<T>::type;
  __shared__ T lds[kTile * PAD];
  const int lane = threadIdx.x;
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  const int64_t t = tile0 + lane;
  const int64_t ks = ntubes;
  // the time-domain tube of this lane: y[2 m] = zr[m], y[2 m + 1] = zi[m]
  // once the transform is done (y[0] = zr[0] for N = 1)
  constexpr int MZ = M > 0 ? M : 1;
  T zr[MZ], zi[MZ];
  if (t < ntubes) {
    if constexpr (N == 1) {
      zr[0] = xre[t];
    } else {
      // the half spectrum is read into zr / zi and turned into conj(Z),
      // Z[k] = E[k] + i O[k], in place: slot k takes X[k] for k < M and
      // X[M] is held apart; the pair (k, M - k) is rewritten together
#pragma unroll
      for (int k = 0; k < M; ++k) {
        zr[k] = xre[(int64_t)k * ks + t];
        zi[k] = k == 0 ? T(0) : xim[(int64_t)k * ks + t];
      }
      const T xmr = xre[(int64_t)M * ks + t];
      auto zpart = [&](int k, T xkr, T xki, T xjr, T xji, T& outr, T& outi) {
        const T er = (xkr + xjr) * T(0.5), ei = (xki - xji) * T(0.5);
        const T dr = (xkr - xjr) * T(0.5), di = (xki + xji) * T(0.5);
        // O = d * conj(W_N^k); Z = E + i O; store conj(Z)
        const T wr = tw_re<T>(N, k), wi = -tw_im<T>(N, k);
        const T orr = dr * wr - di * wi, oi = dr * wi + di * wr;
        outr = er - oi;
        outi = -(ei + orr);
      };
      {
        // k = 0 pairs with X[M] (imaginary parts of both are dropped)
        T o0r, o0i;
        zpart(0, zr[0], T(0), xmr, T(0), o0r, o0i);
        zr[0] = o0r;
        zi[0] = o0i;
      }
#pragma unroll
      for (int k = 1; k <= M / 2; ++k) {
        const int j = M - k;
        const T xkr = zr[k], xki = zi[k], xjr = zr[j], xji = zi[j];
        T okr, oki, ojr, oji;
        zpart(k, xkr, xki, xjr, xji, okr, oki);
        zpart(j, xjr, xji, xkr, xki, ojr, oji);
        zr[k] = okr;
        zi[k] = oki;
        zr[j] = ojr;
        zi[j] = oji;
      }
      cfft<T, M>(zr, zi);
      const T inv = T(1) / T(M);
#pragma unroll
      for (int m = 0; m < M; ++m) {
        zr[m] = zr[m] * inv;
        zi[m] = -zi[m] * inv;
      }
    }
  }
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    if (h > 0) __syncthreads();
    if (t < ntubes) {
#pragma unroll
      for (int e = 0; e < SPAN; ++e) {
        const int g = h * SPAN + e;  // entry of the tube
        lds[lane * PAD + e] = (g & 1) ? zi[g >> 1] : zr[g >> 1];
      }
    }
    __syncthreads();
    if constexpr (SPAN % VN == 0) {
      constexpr int CH = SPAN / VN;
#pragma unroll
      for (int it = 0; it < CH; ++it) {
        const int f = it * kTile + lane;
        const int tl = f / CH, part = f - tl * CH;
        const int64_t tt = tile0 + tl;
        if (tt < ntubes) {
          V w;
          T* wp = reinterpret_cast<T*>(&w);
#pragma unroll
          for (int e = 0; e < VN; ++e) wp[e] = lds[tl * PAD + part * VN + e];
          *reinterpret_cast<V*>(y + tt * N + h * SPAN + part * VN) = w;
        }
      }
    } else {
      for (int it = 0; it < SPAN; ++it) {
        const int f = it * kTile + lane;
        const int tl = f / SPAN, e = f - tl * SPAN;
        const int64_t tt = tile0 + tl;
        if (tt < ntubes) y[tt * N + h * SPAN + e] = lds[tl * PAD + e];
      }
    }
  }
}

// Direct transforms for lengths without a specialised kernel. Every term
// uses a root exp(-2 pi i m / N) with m = k n mod N; up to kDirectTable
// points the N roots are evaluated once per workgroup into LDS (the same
// sincospi values the direct formula takes), beyond that per term.
constexpr int kDirectTable = 2048;

template <bool TABLE>
__device__ __forceinline__ void direct_root(const double* tw, int m, int N, double& sn, double& cs) {
  if (TABLE) {
    cs = tw[m];
    sn = tw[N + m];
  } else {
    sincospi(2.0 * (double)m / (double)N, &sn, &cs);
  }
}

__device__ __forceinline__ void direct_table(double* tw, int N) {
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)N, &sn, &cs);
    tw[m] = cs;
    tw[N + m] = sn;
  }
  __syncthreads();
}

template <typename T, bool TABLE>
__global__ void rdft_direct_kernel(const T* __restrict__ x, int N, FwdArgs a, T* __restrict__ ore,
                                   T* __restrict__ oim) {
  extern __shared__ double tw[];  // TABLE: cos, then sin, of 2 pi m / N
  if (TABLE) direct_table(tw, N);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ntubes) return;
  const int K = N / 2 + 1;
  int64_t src;
  double s;
  const bool live = tube_source(a, t, src, s);
  for (int k = 0; k < K; ++k) {
    double accr = 0, acci = 0;
    if (live) {
      int m = 0;  // k n mod N
      for (int n = 0; n < N; ++n) {
        double sn, cs;
        direct_root<TABLE>(tw, m, N, sn, cs);
        const double v = (double)(T)((double)x[src * N + n] * s);
        accr += v * cs;
        acci -= v * sn;
        m += k;
        m = m >= N ? m - N : m;
      }
    }
    ore[(int64_t)k * a.ntubes + t] = (T)accr;
    oim[(int64_t)k * a.ntubes + t] = (k == 0 || 2 * k == N) ? T(0) : (T)acci;
  }
}

template <typename T, bool TABLE>
__global__ void irdft_direct_kernel(const T* __restrict__ xre, const T* __restrict__ xim, int N, int64_t ntubes,
                                    T* __restrict__ y) {
  extern __shared__ double tw[];
  if (TABLE) direct_table(tw, N);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntubes) return;
  const int K = N / 2 + 1;
  for (int n = 0; n < N; ++n) {
    double acc = 0;
    int m = 0;  // k n mod N
    for (int k = 0; k < K; ++k) {
      const double wk = (k == 0 || 2 * k == N) ? 1.0 : 2.0;
      double sn, cs;
      direct_root<TABLE>(tw, m, N, sn, cs);
      const double xr = (double)xre[(int64_t)k * ntubes + t];
      const double xi = (k == 0 || 2 * k == N) ? 0.0 : (double)xim[(int64_t)k * ntubes + t];
      acc += wk * (xr * cs - xi * sn);
      m += n;
      m = m >= N ? m - N : m;
    }
    y[t * N + n] = (T)(acc / N);
  }
}

// --------------------------------------------------------------------------
// Long tubes (n3 above 256 without a specialised kernel): one workgroup per
// tube, the whole tube as n3 complex values in LDS, an in-place mixed-radix
// decimation-in-time FFT. The input is loaded in digit-reversed order for
// the radix sequence r_0, r_1, ... (4s first, then 2, 3, 5, then primes up
// to kLongMaxRadix); stage q combines r_q sub-transforms of span m (the
// product of the earlier radices) into transforms of span m r_q: for the
// butterfly (group g, offset j < m) the inputs a[g + j + s m] take the
// twiddle W_{m r_q}^{j s} and go through an r_q-point DFT, written back to
// the same positions. Twiddles and the small DFTs' roots are evaluated with
// sincospi in float64.
// --------------------------------------------------------------------------
constexpr int kLongMaxStages = 24;
constexpr int kLongMaxRadix = 13;
constexpr int kLongNT = 256;
constexpr int64_t kLongMin = 257;

struct LongPlan {
  int n, nst;
  int rad[kLongMaxStages];
};

// source index of the element that the digit-reversed load puts at pos
__device__ __forceinline__ int long_src(const LongPlan& pl, int pos) {
  int out = 0, m = pl.n;
  for (int q = 0; q < pl.nst; ++q) {
    const int p = pl.rad[q];
    m /= p;
    out += (pos % p) * m;
    pos /= p;
  }
  return out;
}

template <typename T>
__device__ void long_stages(const LongPlan& pl, T* ar, T* ai) {
  const int n = pl.n;
  int m = 1;
  for (int q = 0; q < pl.nst; ++q) {
    const int p = pl.rad[q], span = m * p;
    // roots of the p-point DFT
    double cw[kLongMaxRadix], sw[kLongMaxRadix];
    for (int e = 0; e < p; ++e) sincospi(-2.0 * e / p, &sw[e], &cw[e]);
    for (int b = threadIdx.x; b < n / p; b += kLongNT) {
      const int j = b % m, g = (b / m) * span;
      double vr[kLongMaxRadix], vi[kLongMaxRadix];
      for (int t = 0; t < p; ++t) {
        const double xr = (double)ar[g + j + t * m], xi = (double)ai[g + j + t * m];
        const int e = (j * t) % span;
        double sn, cs;
        sincospi(-2.0 * e / span, &sn, &cs);
        vr[t] = xr * cs - xi * sn;
        vi[t] = xr * sn + xi * cs;
      }
      for (int t = 0; t < p; ++t) {
        double accr = 0.0, acci = 0.0;
        for (int u = 0; u < p; ++u) {
          const int e = (u * t) % p;
          accr += vr[u] * cw[e] - vi[u] * sw[e];
          acci += vr[u] * sw[e] + vi[u] * cw[e];
        }
        ar[g + j + t * m] = (T)accr;
        ai[g + j + t * m] = (T)acci;
      }
    }
    __syncthreads();
    m = span;
  }
}

template <typename T>
__global__ __launch_bounds__(kLongNT) void rfft_long_kernel(const T* __restrict__ x, FwdArgs a, LongPlan pl,
                                                            T* __restrict__ ore, T* __restrict__ oim) {
  extern __shared__ unsigned char long_lds[];
  T* ar = reinterpret_cast<T*>(long_lds);
  T* ai = ar + pl.n;
  const int64_t t = blockIdx.x;
  const int n = pl.n, K = n / 2 + 1;
  const int64_t ks = a.ntubes;
  int64_t src = -1;
  double s = 0.0;
  const bool live = tube_source(a, t, src, s);
  for (int pos = threadIdx.x; pos < n; pos += kLongNT) {
    T v = T(0);
    if (live) {
      const T xv = x[src * n + long_src(pl, pos)];
      v = (s == 1.0) ? xv : (T)((double)xv * s);
    }
    ar[pos] = v;
    ai[pos] = T(0);
  }
  __syncthreads();
  long_stages<T>(pl, ar, ai);
  for (int k = threadIdx.x; k < K; k += kLongNT) {
    ore[(int64_t)k * ks + t] = ar[k];
    oim[(int64_t)k * ks + t] = (k == 0 || 2 * k == n) ? T(0) : ai[k];
  }
}

// inverse: the Hermitian extension of the half spectrum, conjugated, goes
// through the forward stages; y = Re(result) / n
template <typename T>
__global__ __launch_bounds__(kLongNT) void irfft_long_kernel(const T* __restrict__ xre, const T* __restrict__ xim,
                                                             int64_t ntubes, LongPlan pl, T* __restrict__ y) {
  extern __shared__ unsigned char long_lds[];
  T* ar = reinterpret_cast<T*>(long_lds);
  T* ai = ar + pl.n;
  const int64_t t = blockIdx.x;
  const int n = pl.n, K = n / 2 + 1;
  for (int pos = threadIdx.x; pos < n; pos += kLongNT) {
    const int k = long_src(pl, pos);
    T vr, vi;
    if (k < K) {
      vr = xre[(int64_t)k * ntubes + t];
      vi = (k == 0 || 2 * k == n) ? T(0) : xim[(int64_t)k * ntubes + t];
    } else {
      // X[k] = conj(X[n - k])
      vr = xre[(int64_t)(n - k) * ntubes + t];
      vi = -xim[(int64_t)(n - k) * ntubes + t];
    }
    ar[pos] = vr;
    ai[pos] = -vi;
  }
  __syncthreads();
  long_stages<T>(pl, ar, ai);
  const T inv = T(1) / T(n);
  for (int e = threadIdx.x; e < n; e += kLongNT) y[t * n + e] = ar[e] * inv;
}

// Radix plan of a long tube; false when n has a prime factor above
// kLongMaxRadix, too many stages, or does not fit the LDS budget.
bool long_plan(int64_t n, int elem_bytes, LongPlan& pl) {
  if (n < kLongMin || 2 * n * elem_bytes > 64 * 1024) return false;
  pl.n = (int)n;
  pl.nst = 0;
  int64_t r = n;
  for (int p : {4, 2, 3, 5, 7, 11, 13}) {
    while (r % p == 0) {
      if (pl.nst == kLongMaxStages) return false;
      pl.rad[pl.nst++] = p;
      r /= p;
    }
  }
  return r == 1;
}

// --------------------------------------------------------------------------
// Tubes beyond the LDS budget: a four-step transform through HBM, with the
// caller's output as the only intermediate storage. The real tube x of even
// length n is packed as z[m] = x[2m] + i x[2m+1], m < N = n/2, and with
// N = N1 N2, m = j1 + N1 j2, k = k2 + N2 k1 its DFT factors as
//   Z[k2 + N2 k1] = sum_j1 W_N1^{j1 k1} W_N^{j1 k2} sum_j2 z[j1 + N1 j2] W_N2^{j2 k2}
// (W_L = exp(-2 pi i / L)). Forward:
//   tube pass: per tube and j1 the inner length-N2 transform over j2 and the
//     twiddle W_N^{j1 k2}, written to spectrum slice k2 + N2 j1 of that
//     tube's slot;
//   slice pass: per slot block and pair {k2, N2 - k2} the outer length-N1
//     transforms over j1 (the partner Z[N - k] of every Z[k] of the pair is
//     in the pair), then X[k] = E[k] + W_n^k O[k] for k <= N, with
//     E[k] = (Z[k] + conj Z[N-k]) / 2, O[k] = (Z[k] - conj Z[N-k]) / 2i, written
//     to slice k: exactly the slices the pair's intermediate values occupy, so
//     each workgroup overwrites only what it has read.
// Inverse (the steps reversed, conjugated, into the output tensor):
//   slice pass: per slot block and k2, Z[k] = E[k] + i O[k] from the half
//     spectrum (E = (X[k] + conj X[N-k]) / 2, O = (X[k] - conj X[N-k]) W_n^-k / 2),
//     the inverse transform over k1 and the twiddle W_N^{-j1 k2}, written
//     into the tube at packed position j1 + N1 k2;
//   tube pass: per tube and j1 the inverse transform over k2, 1/N, and the
//     real and imaginary parts as x[2m], x[2m+1] at the positions it read.
// Both short transforms run in LDS as the mixed-radix stages above, several
// sequences per workgroup (FsGeom: slots x j1 values of length N2 <= 256 in
// the tube pass, slots x the pair of length N1 <= 1024 in the slice pass, at
// most 64 KB of LDS), so tubes up to n = 2 x 256 x 1024 with no prime factor
// above 13 take this path; longer or other lengths beyond the LDS budget
// take the direct transform.
// --------------------------------------------------------------------------
constexpr int kFsMaxN2 = 256, kFsMaxN1 = 1024, kFsNT = 512;
constexpr int kFsBatch = 8;  // elements whose loads a thread keeps in flight

template <typename T>
struct FsGeom;
template <>
struct FsGeom<float> {
  static constexpr int tubes = 8, j1s = 4, stubes = 4;  // tube pass: 8 slots x 4 j1; slice pass: 4 slots
};
template <>
struct FsGeom<double> {
  static constexpr int tubes = 4, j1s = 4, stubes = 2;
};

struct FourStep {
  int N1, N2;
  LongPlan p1, p2;  // radix plans of lengths N1 and N2
};

// Launch order. Workgroup L runs on XCD L mod 8, each XCD with its own L2;
// the logical index (L mod 8) q + L / 8 (q = ceil(total / 8)) gives every XCD
// a contiguous range of logical work, so the workgroups that share cache
// lines (neighbouring slots, neighbouring j1) run together on one XCD.
// Returns false for the padding beyond `total`.
__device__ __forceinline__ bool fs_logical(int64_t total, int64_t& G) {
  const int64_t L = blockIdx.x, q = (total + 7) / 8;
  G = (L % 8) * q + L / 8;
  return G < total;
}

// tube passes: 4 x 4 groups of (slot block, j1 block), j1 groups fastest,
// so that reads (contiguous in j1) and writes (contiguous in slots) both
// share lines within a group
__device__ __forceinline__ bool fs_tube_block(int64_t nslot_blocks, int64_t nj_blocks, int64_t& sb, int64_t& jb) {
  const int64_t ngj = (nj_blocks + 3) / 4, ngs = (nslot_blocks + 3) / 4;
  int64_t G;
  if (!fs_logical(ngj * ngs * 16, G)) return false;
  const int64_t g = G / 16, w = G % 16;
  jb = (g % ngj) * 4 + (w % 4);
  sb = (g / ngj) * 4 + (w / 4);
  return jb < nj_blocks && sb < nslot_blocks;
}

// sincospi in the arithmetic of the data (float tubes take float roots:
// their rounding is that of the data)
__device__ __forceinline__ void fs_sincospi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void fs_sincospi(double x, double* s, double* c) { sincospi(x, s, c); }

// One radix-P butterfly of a decimation-in-time stage of span m P: the P
// inputs a[base + t m] take the twiddle W_{mP}^{j t} (j t < m P) and go through
// a P-point DFT with roots (cw, sw); P is a compile-time constant, so the DFT
// is fully unrolled with its root indices folded.
template <int P, typename T>
__device__ __forceinline__ void fs_bfly(T* ar, T* ai, int base, int m, int j, int span, const T* cw, const T* sw) {
  T vr[P], vi[P];
  vr[0] = ar[base];
  vi[0] = ai[base];
#pragma unroll
  for (int t = 1; t < P; ++t) {
    const T xr = ar[base + t * m], xi = ai[base + t * m];
    T sn, cs;
    fs_sincospi(T(-2) * T(j * t) / T(span), &sn, &cs);
    vr[t] = xr * cs - xi * sn;
    vi[t] = xr * sn + xi * cs;
  }
#pragma unroll
  for (int t = 0; t < P; ++t) {
    T accr = vr[0], acci = vi[0];
#pragma unroll
    for (int u = 1; u < P; ++u) {
      const int e = (u * t) % P;
      accr += vr[u] * cw[e] - vi[u] * sw[e];
      acci += vr[u] * sw[e] + vi[u] * cw[e];
    }
    ar[base + t * m] = accr;
    ai[base + t * m] = acci;
  }
}

// mixed-radix stages of `nseq` sequences of length pl.n, sequence s at
// offset s * pl.n (loaded in digit-reversed order), in the data's precision
template <typename T>
__device__ void multi_stages(const LongPlan& pl, T* ar, T* ai, int nseq) {
  const int n = pl.n;
  int m = 1;
  for (int q = 0; q < pl.nst; ++q) {
    const int p = pl.rad[q], span = m * p, per = n / p;
    T cw[kLongMaxRadix], sw[kLongMaxRadix];
#pragma unroll
    for (int e = 0; e < kLongMaxRadix; ++e) {
      cw[e] = T(1);
      sw[e] = T(0);
      if (e < p) fs_sincospi(T(-2) * T(e) / T(p), &sw[e], &cw[e]);
    }
    for (int b = threadIdx.x; b < nseq * per; b += kFsNT) {
      const int sq = b / per, bb = b - sq * per;
      const int bm = bb / m, j = bb - bm * m;
      const int base = sq * n + bm * span + j;
      switch (p) {
        case 2: fs_bfly<2, T>(ar, ai, base, m, j, span, cw, sw); break;
        case 3: fs_bfly<3, T>(ar, ai, base, m, j, span, cw, sw); break;
        case 4: fs_bfly<4, T>(ar, ai, base, m, j, span, cw, sw); break;
        case 5: fs_bfly<5, T>(ar, ai, base, m, j, span, cw, sw); break;
        case 7: fs_bfly<7, T>(ar, ai, base, m, j, span, cw, sw); break;
        case 11: fs_bfly<11, T>(ar, ai, base, m, j, span, cw, sw); break;
        default: fs_bfly<13, T>(ar, ai, base, m, j, span, cw, sw); break;
      }
    }
    __syncthreads();
    m = span;
  }
}

// position at which the digit-reversed load puts source index src (the
// inverse of long_src)
__device__ __forceinline__ int long_dst(const LongPlan& pl, int src) {
  int pos = 0, w = 1;
  int digits[kLongMaxStages];
  for (int q = pl.nst - 1; q >= 0; --q) {
    digits[q] = src % pl.rad[q];
    src /= pl.rad[q];
  }
  for (int q = 0; q < pl.nst; ++q) {
    pos += digits[q] * w;
    w *= pl.rad[q];
  }
  return pos;
}

// exp(-2 pi i e / L) for 0 <= e < L
__device__ __forceinline__ void fs_root(int e, int L, double& c, double& s) {
  sincospi(-2.0 * (double)e / (double)L, &s, &c);
}

// forward tube pass: workgroup (slot block, j1 block)
template <typename T>
__global__ __launch_bounds__(kFsNT) void fs_fwd_tube_kernel(const T* __restrict__ x, FwdArgs a, FourStep fs,
                                                            T* __restrict__ ore, T* __restrict__ oim) {
  constexpr int TB = FsGeom<T>::tubes, JB = FsGeom<T>::j1s;
  extern __shared__ unsigned char fs_lds[];
  const int N1 = fs.N1, N2 = fs.N2, N = N1 * N2;
  T* ar = reinterpret_cast<T*>(fs_lds);
  T* ai = ar + TB * JB * N2;
  const int64_t ks = a.ntubes;
  int64_t sbk, jbk;
  if (!fs_tube_block((ks + TB - 1) / TB, (N1 + JB - 1) / JB, sbk, jbk)) return;
  const int64_t t0 = sbk * TB;
  const int j10 = (int)jbk * JB;
  // input tube and scale of each slot of the block
  __shared__ int64_t s_src[TB];
  __shared__ double s_sc[TB];
  if (threadIdx.x < TB) {
    const int64_t t = t0 + threadIdx.x;
    int64_t src = -1;
    double sc = 1.0;
    if (!(t < ks && tube_source(a, t, src, sc))) src = -1;
    s_src[threadIdx.x] = src;
    s_sc[threadIdx.x] = sc;
  }
  __syncthreads();
  // sequence (tube u, j1 offset v) at (u JB + v) N2 holds z[j1 + N1 j2] at
  // the digit-reversed position of j2; threads take consecutive j1 of one
  // (tube, j2) (contiguous input runs), kFsBatch loads in flight per thread
  // (indices first, then the batch's loads unconditionally from clamped
  // addresses so that they all stay in flight, then the LDS stores)
  const int total = TB * JB * N2;
  for (int e0 = threadIdx.x; e0 < total; e0 += kFsBatch * kFsNT) {
    int64_t off[kFsBatch];
    double sc[kFsBatch];
    int li[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int e = e0 + q * kFsNT;
      off[q] = -1;
      sc[q] = 1.0;
      li[q] = -1;
      if (e < total) {
        const int v = e % JB, r = e / JB;
        const int j2 = r % N2, u = r / N2;
        const int j1 = j10 + v;
        li[q] = (u * JB + v) * N2 + long_dst(fs.p2, j2);
        const int64_t src = s_src[u];
        if (src >= 0 && j1 < N1) {
          off[q] = src * (int64_t)(2 * N) + 2 * ((int64_t)j1 + (int64_t)N1 * j2);
          sc[q] = s_sc[u];
        }
      }
    }
    T vr[kFsBatch], vi[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int64_t o = off[q] < 0 ? 0 : off[q];
      vr[q] = x[o];
      vi[q] = x[o + 1];
    }
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      if (li[q] < 0) continue;
      const bool ok = off[q] >= 0;
      ar[li[q]] = !ok ? T(0) : (sc[q] == 1.0) ? vr[q] : (T)((double)vr[q] * sc[q]);
      ai[li[q]] = !ok ? T(0) : (sc[q] == 1.0) ? vi[q] : (T)((double)vi[q] * sc[q]);
    }
  }
  __syncthreads();
  multi_stages<T>(fs.p2, ar, ai, TB * JB);
  // twiddle W_N^{j1 k2}; value (t, j1, k2) goes to slice k2 + N2 j1 of slot t
  for (int e = threadIdx.x; e < TB * JB * N2; e += kFsNT) {
    const int k2 = e / (TB * JB), r = e - k2 * (TB * JB);
    const int v = r / TB, u = r - v * TB;  // slots fastest: neighbouring stores
    const int64_t t = t0 + u;
    const int j1 = j10 + v;
    if (t >= ks || j1 >= N1) continue;
    const int li = (u * JB + v) * N2 + k2;
    double c, sn;
    fs_root((int)((unsigned)(j1 * k2) % (unsigned)N), N, c, sn);  // j1 k2 < 2^18
    const double xr = (double)ar[li], xi = (double)ai[li];
    const int64_t o = ((int64_t)k2 + (int64_t)N2 * j1) * ks + t;
    ore[o] = (T)(xr * c - xi * sn);
    oim[o] = (T)(xr * sn + xi * c);
  }
}

// forward slice pass: workgroup (slot block, pair {k2, N2 - k2})
template <typename T>
__global__ __launch_bounds__(kFsNT) void fs_fwd_slice_kernel(FourStep fs, int64_t ks, T* __restrict__ ore,
                                                             T* __restrict__ oim) {
  constexpr int TB = FsGeom<T>::stubes;
  extern __shared__ unsigned char fs_lds[];
  const int N1 = fs.N1, N2 = fs.N2, N = N1 * N2;
  T* ar = reinterpret_cast<T*>(fs_lds);
  T* ai = ar + 2 * TB * N1;
  const int64_t nsb = (ks + TB - 1) / TB;
  int64_t G;
  if (!fs_logical(nsb * (N2 / 2 + 1), G)) return;
  const int64_t t0 = (G % nsb) * TB;  // slot blocks fastest
  const int ka = (int)(G / nsb), kb = (N2 - ka) % N2;
  const int nk = ka == kb ? 1 : 2;
  // sequence (h, u) at (h TB + u) N1 holds the values of slice k2 = (ka, kb)[h]
  // of slot t0 + u, position pos holding j1 = long_src(pos); kFsBatch loads
  // in flight per thread
  const int total = nk * TB * N1;
  for (int e0 = threadIdx.x; e0 < total; e0 += kFsBatch * kFsNT) {
    int64_t off[kFsBatch];
    int li[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int e = e0 + q * kFsNT;
      off[q] = -1;
      li[q] = -1;
      if (e < total) {
        const int pos = e / (nk * TB), r = e - pos * (nk * TB);
        const int h = r / TB, u = r - h * TB;
        const int64_t t = t0 + u;
        li[q] = (h * TB + u) * N1 + pos;
        if (t < ks) off[q] = ((int64_t)(h ? kb : ka) + (int64_t)N2 * long_src(fs.p1, pos)) * ks + t;
      }
    }
    T vr[kFsBatch], vi[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int64_t o = off[q] < 0 ? 0 : off[q];
      vr[q] = ore[o];
      vi[q] = oim[o];
    }
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      if (li[q] < 0) continue;
      ar[li[q]] = off[q] < 0 ? T(0) : vr[q];
      ai[li[q]] = off[q] < 0 ? T(0) : vi[q];
    }
  }
  __syncthreads();
  multi_stages<T>(fs.p1, ar, ai, nk * TB);
  // X[k] = E[k] + W_n^k O[k] for the k of this pair (and k = N with k2 = 0)
  const int n = 2 * N;
  const int nout = nk * N1 + (ka == 0 ? 1 : 0);
  for (int e = threadIdx.x; e < nout * TB; e += kFsNT) {
    const int q = e / TB, u = e - q * TB;
    const int64_t t = t0 + u;
    if (t >= ks) continue;
    // the q-th output of the pair: slice (ka, kb)[q / N1] + N2 (q mod N1), or N
    const int k = q < nk * N1 ? (q < N1 ? ka : kb) + N2 * (q % N1) : N;
    // Z[k mod N] and Z[(N - k) mod N], both among the pair's sequences
    const int kk = k % N, km = (N - kk) % N;
    const int ha = kk % N2 == ka ? 0 : 1, hb = km % N2 == ka ? 0 : 1;
    const int ia = (ha * TB + u) * N1 + kk / N2, ib = (hb * TB + u) * N1 + km / N2;
    const double zr = (double)ar[ia], zi = (double)ai[ia];
    const double wr = (double)ar[ib], wi = -(double)ai[ib];  // conj Z[N - k]
    const double er = 0.5 * (zr + wr), ei = 0.5 * (zi + wi);
    const double orr = 0.5 * (zi - wi), oi = -0.5 * (zr - wr);  // (Z - conj Z[N-k]) / 2i
    double c, sn;
    fs_root(k, n, c, sn);
    const double xr = er + (orr * c - oi * sn);
    const double xi = (k == 0 || k == N) ? 0.0 : ei + (orr * sn + oi * c);
    const int64_t o = (int64_t)k * ks + t;
    ore[o] = (T)xr;
    oim[o] = (T)xi;
  }
}

// inverse slice pass: workgroup (slot block, k2)
template <typename T>
__global__ __launch_bounds__(kFsNT) void fs_inv_slice_kernel(const T* __restrict__ xre, const T* __restrict__ xim,
                                                             int64_t ntubes, FourStep fs, T* __restrict__ y) {
  constexpr int TB = FsGeom<T>::stubes;
  extern __shared__ unsigned char fs_lds[];
  const int N1 = fs.N1, N2 = fs.N2, N = N1 * N2, n = 2 * N;
  T* ar = reinterpret_cast<T*>(fs_lds);
  T* ai = ar + TB * N1;
  const int64_t nsb = (ntubes + TB - 1) / TB;
  int64_t G;
  if (!fs_logical(nsb * N2, G)) return;
  const int64_t t0 = (G % nsb) * TB;  // slot blocks fastest
  const int k2 = (int)(G / nsb);
  // conj Z[k2 + N2 k1] at position pos of sequence u (k1 = long_src(pos)):
  // the forward stages of the conjugate give the conjugate of the inverse;
  // kFsBatch elements' loads in flight per thread
  const int total = TB * N1;
  for (int e0 = threadIdx.x; e0 < total; e0 += kFsBatch * kFsNT) {
    int64_t oa[kFsBatch], ob[kFsBatch];
    int kq[kFsBatch], li[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int e = e0 + q * kFsNT;
      oa[q] = ob[q] = 0;
      kq[q] = -1;
      li[q] = -1;
      if (e < total) {
        const int pos = e / TB, u = e - pos * TB;
        const int64_t t = t0 + u;
        li[q] = u * N1 + pos;
        if (t < ntubes) {
          const int k = k2 + N2 * long_src(fs.p1, pos);
          kq[q] = k;
          oa[q] = (int64_t)k * ntubes + t;
          ob[q] = (int64_t)(N - k) * ntubes + t;  // 1 <= N - k <= N
        }
      }
    }
    T ar0[kFsBatch], ai0[kFsBatch], br0[kFsBatch], bi0[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      ar0[q] = xre[oa[q]];
      ai0[q] = xim[oa[q]];
      br0[q] = xre[ob[q]];
      bi0[q] = xim[ob[q]];
    }
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      if (li[q] < 0) continue;
      T vr = T(0), vi = T(0);
      const int k = kq[q];
      if (k >= 0) {
        const double xr = (double)ar0[q], xi = k == 0 ? 0.0 : (double)ai0[q];
        const double yr = (double)br0[q], yi = (N - k) == N ? 0.0 : -(double)bi0[q];  // conj X[N-k]
        const double er = 0.5 * (xr + yr), ei = 0.5 * (xi + yi);
        const double dr = 0.5 * (xr - yr), di = 0.5 * (xi - yi);
        double c, sn;
        fs_root(k, n, c, sn);  // W_n^k; O = D conj(W_n^k)
        const double orr = dr * c + di * sn, oi = di * c - dr * sn;
        // Z = E + i O, conjugated
        vr = (T)(er - oi);
        vi = (T)(-(ei + orr));
      }
      ar[li[q]] = vr;
      ai[li[q]] = vi;
    }
  }
  __syncthreads();
  multi_stages<T>(fs.p1, ar, ai, TB);
  // u[j1] = conj(stage result) W_N^{-j1 k2}, stored at packed position
  // j1 + N1 k2 of the slot's tube
  for (int e = threadIdx.x; e < TB * N1; e += kFsNT) {
    const int u = e / N1, j1 = e - u * N1;
    const int64_t t = t0 + u;
    if (t >= ntubes) continue;
    const double vr = (double)ar[u * N1 + j1], vi = -(double)ai[u * N1 + j1];
    double c, sn;
    fs_root((int)((unsigned)(j1 * k2) % (unsigned)N), N, c, sn);  // W_N^{j1 k2}; times its conjugate
    const int64_t o = t * (int64_t)n + 2 * ((int64_t)j1 + (int64_t)N1 * k2);
    y[o] = (T)(vr * c + vi * sn);
    y[o + 1] = (T)(vi * c - vr * sn);
  }
}

// inverse tube pass: workgroup (slot block, j1 block), in place in y
template <typename T>
__global__ __launch_bounds__(kFsNT) void fs_inv_tube_kernel(int64_t ntubes, FourStep fs, T* __restrict__ y) {
  constexpr int TB = FsGeom<T>::tubes, JB = FsGeom<T>::j1s;
  extern __shared__ unsigned char fs_lds[];
  const int N1 = fs.N1, N2 = fs.N2, N = N1 * N2, n = 2 * N;
  T* ar = reinterpret_cast<T*>(fs_lds);
  T* ai = ar + TB * JB * N2;
  int64_t sbk, jbk;
  if (!fs_tube_block((ntubes + TB - 1) / TB, (N1 + JB - 1) / JB, sbk, jbk)) return;
  const int64_t t0 = sbk * TB;
  const int j10 = (int)jbk * JB;
  const int total = TB * JB * N2;
  for (int e0 = threadIdx.x; e0 < total; e0 += kFsBatch * kFsNT) {
    int64_t off[kFsBatch];
    int li[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int e = e0 + q * kFsNT;
      off[q] = -1;
      li[q] = -1;
      if (e < total) {
        const int v = e % JB, r = e / JB;
        const int k2 = r % N2, u = r / N2;
        const int64_t t = t0 + u;
        const int j1 = j10 + v;
        li[q] = (u * JB + v) * N2 + long_dst(fs.p2, k2);
        if (t < ntubes && j1 < N1) off[q] = t * (int64_t)n + 2 * ((int64_t)j1 + (int64_t)N1 * k2);
      }
    }
    T vr[kFsBatch], vi[kFsBatch];
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      const int64_t o = off[q] < 0 ? 0 : off[q];
      vr[q] = y[o];
      vi[q] = y[o + 1];
    }
#pragma unroll
    for (int q = 0; q < kFsBatch; ++q) {
      if (li[q] < 0) continue;
      ar[li[q]] = off[q] < 0 ? T(0) : vr[q];
      ai[li[q]] = off[q] < 0 ? T(0) : -vi[q];  // conjugate in, conjugate out
    }
  }
  __syncthreads();
  multi_stages<T>(fs.p2, ar, ai, TB * JB);
  const double inv = 1.0 / (double)N;
  for (int e = threadIdx.x; e < TB * JB * N2; e += kFsNT) {
    const int u = e / (JB * N2), r = e - u * (JB * N2);
    const int j2 = r / JB, v = r - j2 * JB;  // j1 fastest: neighbouring stores
    const int64_t t = t0 + u;
    const int j1 = j10 + v;
    if (t >= ntubes || j1 >= N1) continue;
    const int li = (u * JB + v) * N2 + j2;
    const int64_t o = t * (int64_t)n + 2 * ((int64_t)j1 + (int64_t)N1 * j2);
    y[o] = (T)((double)ar[li] * inv);
    y[o + 1] = (T)(-(double)ai[li] * inv);
  }
}

// radix plan of a short length (factors 4, 2, 3, 5, 7, 11, 13), no size limits
bool radix_plan(int64_t n, LongPlan& pl) {
  pl.n = (int)n;
  pl.nst = 0;
  int64_t r = n;
  for (int p : {4, 2, 3, 5, 7, 11, 13}) {
    while (r % p == 0) {
      if (pl.nst == kLongMaxStages) return false;
      pl.rad[pl.nst++] = p;
      r /= p;
    }
  }
  return r == 1;
}

// --------------------------------------------------------------------------
// Lengths with a prime factor above 13 (up to kBlueMax): Bluestein's
// chirp-z transform in LDS, one workgroup per tube. With the chirp
// w[m] = exp(-i pi m^2 / n), the DFT is X[k] = w[k] sum_m (x[m] w[m])
// conj(w[k - m]) (from 2 m k = m^2 + k^2 - (k - m)^2), a circular
// convolution of length L >= 2n - 1 (L without prime factors above 13)
// evaluated by three mixed-radix transforms of length L: a = x w and the
// filter b (conj w at m and L - m) forward, then the inverse of A B through
// the conjugate. The inverse tube transform is the forward one of the
// conjugated Hermitian extension, conjugated and scaled by 1/n.
// --------------------------------------------------------------------------
constexpr int kBlueMax = 2048;  // float32 tubes; float64 up to half of it

struct BluePlan {
  int n;
  LongPlan pl;  // length L
};

// chirp exp(-i pi m^2 / n) in double (m^2 reduced mod 2n, exact in int64)
__device__ __forceinline__ void blue_chirp(int m, int n, double& c, double& s) {
  const int64_t e = ((int64_t)m * m) % (2 * (int64_t)n);
  sincospi(-(double)e / (double)n, &s, &c);
}

// DFT of n complex values: load(m) gives input m < n, store(k, re, im)
// takes output k < nout (<= n). LDS: ar | br (2L values, br = ar + L) and
// ai | bi, so the two forward transforms run as one two-sequence pass.
constexpr int kBluePer = 2 * kBlueMax / kFsNT;  // L / threads at most

template <typename T, typename Load, typename Store>
__device__ void bluestein(const BluePlan& bp, T* ar, T* ai, Load load, int nout, Store store) {
  const int n = bp.n, L = bp.pl.n;
  T* br = ar + L;
  T* bi = ai + L;
  for (int m = threadIdx.x; m < L; m += kFsNT) {
    T a_r = T(0), a_i = T(0), b_r = T(0), b_i = T(0);
    if (m < n) {
      double c, sn, xr, xi;
      blue_chirp(m, n, c, sn);
      load(m, xr, xi);
      a_r = (T)(xr * c - xi * sn);
      a_i = (T)(xr * sn + xi * c);
      b_r = (T)c;
      b_i = (T)(-sn);
    } else if (m > L - n) {
      double c, sn;
      blue_chirp(L - m, n, c, sn);
      b_r = (T)c;
      b_i = (T)(-sn);
    }
    const int pos = long_dst(bp.pl, m);
    ar[pos] = a_r;
    ai[pos] = a_i;
    br[pos] = b_r;
    bi[pos] = b_i;
  }
  __syncthreads();
  multi_stages<T>(bp.pl, ar, ai, 2);
  // conj(A B), through registers, into ar/ai in digit-reversed order
  T pr[kBluePer], pi[kBluePer];
#pragma unroll
  for (int q = 0; q < kBluePer; ++q) {
    const int m = threadIdx.x + q * kFsNT;
    if (m < L) {
      const double xr = (double)ar[m], xi = (double)ai[m], yr = (double)br[m], yi = (double)bi[m];
      pr[q] = (T)(xr * yr - xi * yi);
      pi[q] = (T)(-(xr * yi + xi * yr));
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kBluePer; ++q) {
    const int m = threadIdx.x + q * kFsNT;
    if (m < L) {
      const int pos = long_dst(bp.pl, m);
      ar[pos] = pr[q];
      ai[pos] = pi[q];
    }
  }
  __syncthreads();
  multi_stages<T>(bp.pl, ar, ai, 1);
  const double inv = 1.0 / (double)L;
  for (int k = threadIdx.x; k < nout; k += kFsNT) {
    double c, sn;
    blue_chirp(k, n, c, sn);
    const double yr = (double)ar[k] * inv, yi = -(double)ai[k] * inv;  // the convolution at k
    store(k, yr * c - yi * sn, yr * sn + yi * c);
  }
}

template <typename T>
__global__ __launch_bounds__(kFsNT) void rdft_blue_kernel(const T* __restrict__ x, FwdArgs a, BluePlan bp,
                                                          T* __restrict__ ore, T* __restrict__ oim) {
  extern __shared__ unsigned char blue_lds[];
  const int n = bp.n, L = bp.pl.n, K = n / 2 + 1;
  T* ar = reinterpret_cast<T*>(blue_lds);
  T* ai = ar + 2 * L;
  const int64_t t = blockIdx.x;
  const int64_t ks = a.ntubes;
  int64_t src = -1;
  double sc = 1.0;
  const bool live = tube_source(a, t, src, sc);
  auto load = [&](int m, double& xr, double& xi) {
    xr = live ? (double)x[src * n + m] * sc : 0.0;
    xi = 0.0;
  };
  auto store = [&](int k, double re, double im) {
    ore[(int64_t)k * ks + t] = (T)re;
    oim[(int64_t)k * ks + t] = (k == 0 || 2 * k == n) ? T(0) : (T)im;
  };
  bluestein<T>(bp, ar, ai, load, K, store);
}

// inverse: the forward transform of the conjugated Hermitian extension,
// conjugated (only the real part is kept) and scaled by 1/n
template <typename T>
__global__ __launch_bounds__(kFsNT) void irdft_blue_kernel(const T* __restrict__ xre, const T* __restrict__ xim,
                                                           int64_t ntubes, BluePlan bp, T* __restrict__ y) {
  extern __shared__ unsigned char blue_lds[];
  const int n = bp.n, L = bp.pl.n, K = n / 2 + 1;
  T* ar = reinterpret_cast<T*>(blue_lds);
  T* ai = ar + 2 * L;
  const int64_t t = blockIdx.x;
  auto load = [&](int k, double& re, double& im) {
    if (k < K) {
      re = (double)xre[(int64_t)k * ntubes + t];
      im = (k == 0 || 2 * k == n) ? 0.0 : (double)xim[(int64_t)k * ntubes + t];
    } else {
      re = (double)xre[(int64_t)(n - k) * ntubes + t];
      im = -(double)xim[(int64_t)(n - k) * ntubes + t];
    }
    im = -im;
  };
  const double inv = 1.0 / (double)n;
  auto store = [&](int e, double re, double) { y[t * n + e] = (T)(re * inv); };
  bluestein<T>(bp, ar, ai, load, n, store);
}

// Bluestein plan: L = the smallest length >= 2n - 1 without prime factors
// above 13; the four L-long sequences must fit in 64 KB of LDS.
bool blue_plan(int64_t n, int elem_bytes, BluePlan& bp) {
  if (n < 2 || n > (elem_bytes == 4 ? kBlueMax : kBlueMax / 2)) return false;
  for (int64_t L = 2 * n - 1;; ++L) {
    if (4 * L * elem_bytes > 64 * 1024) return false;
    if (radix_plan(L, bp.pl)) {
      bp.n = (int)n;
      return true;
    }
  }
}

// Four-step plan of an even n: N = n/2 = N1 N2 with N2 the largest divisor
// <= kFsMaxN2 that leaves N1 <= kFsMaxN1, both without prime factors above 13.
bool four_step_plan(int64_t n, FourStep& fs) {
  if (n % 2 || n < 4) return false;
  const int64_t N = n / 2;
  if (N > (int64_t)kFsMaxN1 * kFsMaxN2) return false;
  for (int64_t n2 = kFsMaxN2 < N ? kFsMaxN2 : N; n2 >= 1; --n2) {
    if (N % n2) continue;
    const int64_t n1 = N / n2;
    if (n1 > kFsMaxN1) break;
    if (radix_plan(n1, fs.p1) && radix_plan(n2, fs.p2)) {
      fs.N1 = (int)n1;
      fs.N2 = (int)n2;
      return true;
    }
  }
  return false;
}

// 1D grid of a launch with `total` logical workgroups (padded to whole
// rounds over the eight XCDs)
inline int64_t fs_grid(int64_t total) { return (total + 7) / 8 * 8; }
inline int64_t fs_tube_grid(int64_t nslot_blocks, int64_t nj_blocks) {
  return fs_grid(((nj_blocks + 3) / 4) * ((nslot_blocks + 3) / 4) * 16);
}

template <typename T>
int fs_forward(const T* x, const FwdArgs& a, const FourStep& fs, T* re, T* im, hipStream_t st) {
  constexpr int TB = FsGeom<T>::tubes, JB = FsGeom<T>::j1s, SB = FsGeom<T>::stubes;
  const int64_t gt = fs_tube_grid((a.ntubes + TB - 1) / TB, (fs.N1 + JB - 1) / JB);
  const int64_t gs = fs_grid((a.ntubes + SB - 1) / SB * (fs.N2 / 2 + 1));
  if (gt > 0x7fffffffLL || gs > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
  const size_t lt = size_t(2) * TB * JB * fs.N2 * sizeof(T), ls = size_t(2) * 2 * SB * fs.N1 * sizeof(T);
  hipLaunchKernelGGL(fs_fwd_tube_kernel<T>, dim3((unsigned)gt), dim3(kFsNT), lt, st, x, a, fs, re, im);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(fs_fwd_slice_kernel<T>, dim3((unsigned)gs), dim3(kFsNT), ls, st, fs, a.ntubes, re, im);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

template <typename T>
int fs_inverse(const T* re, const T* im, int64_t ntubes, const FourStep& fs, T* y, hipStream_t st) {
  constexpr int TB = FsGeom<T>::tubes, JB = FsGeom<T>::j1s, SB = FsGeom<T>::stubes;
  const int64_t gt = fs_tube_grid((ntubes + TB - 1) / TB, (fs.N1 + JB - 1) / JB);
  const int64_t gs = fs_grid((ntubes + SB - 1) / SB * fs.N2);
  if (gt > 0x7fffffffLL || gs > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
  const size_t lt = size_t(2) * TB * JB * fs.N2 * sizeof(T), ls = size_t(2) * SB * fs.N1 * sizeof(T);
  hipLaunchKernelGGL(fs_inv_slice_kernel<T>, dim3((unsigned)gs), dim3(kFsNT), ls, st, re, im, ntubes, fs, y);
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(fs_inv_tube_kernel<T>, dim3((unsigned)gt), dim3(kFsNT), lt, st, ntubes, fs, y);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

template <typename T>
using FwdKernel = void (*)(const T*, FwdArgs, T*, T*);
template <typename T>
using InvKernel = void (*)(const T*, const T*, int64_t, T*);

template <typename T>
FwdKernel<T> pick_fwd(int64_t n) {
  switch (n) {
    case 1: return rfft_kernel<T, 1>;
    case 2: return rfft_kernel<T, 2>;
    case 4: return rfft_kernel<T, 4>;
    case 8: return rfft_kernel<T, 8>;
    case 16: return rfft_kernel<T, 16>;
    case 32: return rfft_kernel<T, 32>;
    case 64: return rfft_kernel<T, 64>;
    case 128: return rfft_kernel<T, 128>;
    case 10: return rfft_kernel<T, 10>;
    case 20: return rfft_kernel<T, 20>;
    case 50: return rfft_kernel<T, 50>;
    case 100: return rfft_kernel<T, 100>;
    case 168: return rfft_kernel<T, 168>;
    default: return nullptr;
  }
}

template <typename T>
InvKernel<T> pick_inv(int64_t n) {
  switch (n) {
    case 1: return irfft_kernel<T, 1>;
    case 2: return irfft_kernel<T, 2>;
    case 4: return irfft_kernel<T, 4>;
    case 8: return irfft_kernel<T, 8>;
    case 16: return irfft_kernel<T, 16>;
    case 32: return irfft_kernel<T, 32>;
    case 64: return irfft_kernel<T, 64>;
    case 128: return irfft_kernel<T, 128>;
    case 10: return irfft_kernel<T, 10>;
    case 20: return irfft_kernel<T, 20>;
    case 50: return irfft_kernel<T, 50>;
    case 100: return irfft_kernel<T, 100>;
    case 168: return irfft_kernel<T, 168>;
    default: return nullptr;
  }
}

template <typename T>
int fwd_impl(const T* x, int64_t n3, const TubeGather& g, T* re, T* im, hipStream_t st) {
  FwdArgs a{g.rows, g.cols, g.in_cols, g.rows * g.cols, g.row_idx, g.col_idx, g.row_scale, g.col_scale, g.count,
            g.cols, 0, 0};
  if (a.ntubes == 0) return TP_OK;
  if (auto k = pick_fwd<T>(n3)) {
    const int64_t blocks = (a.ntubes + kTile - 1) / kTile;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTile), 0, st, x, a, re, im);
  } else if (LongPlan pl; long_plan(n3, (int)sizeof(T), pl)) {
    if (a.ntubes > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
    hipLaunchKernelGGL(rfft_long_kernel<T>, dim3((unsigned)a.ntubes), dim3(kLongNT), 2 * n3 * sizeof(T), st, x, a,
                       pl, re, im);
  } else if (FourStep fs; n3 >= kLongMin && four_step_plan(n3, fs)) {
    return fs_forward<T>(x, a, fs, (T*)re, (T*)im, st);
  } else if (BluePlan bp; n3 >= kLongMin && blue_plan(n3, (int)sizeof(T), bp)) {
    if (a.ntubes > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
    hipLaunchKernelGGL(rdft_blue_kernel<T>, dim3((unsigned)a.ntubes), dim3(kFsNT), 4 * bp.pl.n * sizeof(T), st, x, a,
                       bp, re, im);
  } else {
    const int64_t blocks = (a.ntubes + 127) / 128;
    if (n3 <= kDirectTable)
      hipLaunchKernelGGL((rdft_direct_kernel<T, true>), dim3((unsigned)blocks), dim3(128), 2 * n3 * sizeof(double), st,
                         x, (int)n3, a, re, im);
    else
      hipLaunchKernelGGL((rdft_direct_kernel<T, false>), dim3((unsigned)blocks), dim3(128), 0, st, x, (int)n3, a, re,
                         im);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

template <typename T>
int inv_impl(const T* re, const T* im, int64_t n3, int64_t ntubes, T* y, hipStream_t st) {
  if (ntubes == 0) return TP_OK;
  if (auto k = pick_inv<T>(n3)) {
    const int64_t blocks = (ntubes + kTile - 1) / kTile;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTile), 0, st, re, im, ntubes, y);
  } else if (LongPlan pl; long_plan(n3, (int)sizeof(T), pl)) {
    if (ntubes > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
    hipLaunchKernelGGL(irfft_long_kernel<T>, dim3((unsigned)ntubes), dim3(kLongNT), 2 * n3 * sizeof(T), st, re, im,
                       ntubes, pl, y);
  } else if (FourStep fs; n3 >= kLongMin && four_step_plan(n3, fs)) {
    return fs_inverse<T>(re, im, ntubes, fs, y, st);
  } else if (BluePlan bp; n3 >= kLongMin && blue_plan(n3, (int)sizeof(T), bp)) {
    if (ntubes > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
    hipLaunchKernelGGL(irdft_blue_kernel<T>, dim3((unsigned)ntubes), dim3(kFsNT), 4 * bp.pl.n * sizeof(T), st, re, im,
                       ntubes, bp, y);
  } else {
    const int64_t blocks = (ntubes + 127) / 128;
    if (n3 <= kDirectTable)
      hipLaunchKernelGGL((irdft_direct_kernel<T, true>), dim3((unsigned)blocks), dim3(128), 2 * n3 * sizeof(double),
                         st, re, im, (int)n3, ntubes, y);
    else
      hipLaunchKernelGGL((irdft_direct_kernel<T, false>), dim3((unsigned)blocks), dim3(128), 0, st, re, im, (int)n3,
                         ntubes, y);
  }
  TP_LAUNCH_CHECK();
  return TP_OK;
}

template <bool SPLIT>
FwdKernel<float> pick_fwd_split(int64_t n) {
  switch (n) {
    case 1: return rfft_kernel<float, 1, true>;
    case 2: return rfft_kernel<float, 2, true>;
    case 4: return rfft_kernel<float, 4, true>;
    case 8: return rfft_kernel<float, 8, true>;
    case 16: return rfft_kernel<float, 16, true>;
    case 32: return rfft_kernel<float, 32, true>;
    case 64: return rfft_kernel<float, 64, true>;
    case 128: return rfft_kernel<float, 128, true>;
    case 10: return rfft_kernel<float, 10, true>;
    case 20: return rfft_kernel<float, 20, true>;
    case 50: return rfft_kernel<float, 50, true>;
    case 100: return rfft_kernel<float, 100, true>;
    default: return nullptr;
  }
}

}  // namespace

bool fft_supported(int64_t n3) { return pick_fwd<float>(n3) != nullptr; }

bool fft_split_supported(int64_t n3) { return pick_fwd_split<true>(n3) != nullptr; }

int fft_forward_split(const float* x, int64_t n3, const TubeGather& g, bool colmajor, int64_t ld, void* planes,
                      hipStream_t st) {
  if (int rc = ensure_twiddles()) return rc;
  auto k = pick_fwd_split<true>(n3);
  if (!k) return fail(TP_EUNSUPPORTED, "no split-output transform for this tube length");
  if (ld < (colmajor ? g.rows : g.cols)) return fail(TP_EINVAL, "split spectrum stride below its extent");
  FwdArgs a{g.rows, g.cols, g.in_cols, (colmajor ? g.cols : g.rows) * ld, g.row_idx, g.col_idx, g.row_scale,
            g.col_scale, g.count, ld, colmajor ? 1 : 0, (colmajor && ld % kTile == 0) ? g.cols : 0};
  if (a.ntubes == 0) return TP_OK;
  const int64_t blocks = (a.ntubes + kTile - 1) / kTile;
  if (blocks > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTile), 0, st, x, a, (float*)planes, (float*)nullptr);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int fft_forward(const void* x, int dtype, int64_t n3, const TubeGather& g, void* re, void* im, hipStream_t st) {
  if (int rc = ensure_twiddles()) return rc;
  if ((g.rows * g.cols + kTile - 1) / kTile > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many tubes");
  if (dtype == TP_F64)
    return fwd_impl<double>((const double*)x, n3, g, (double*)re, (double*)im, st);
  return fwd_impl<float>((const float*)x, n3, g, (float*)re, (float*)im, st);
}

int fft_inverse(const void* re, const void* im, int dtype, int64_t n3, int64_t rows, int64_t cols, void* x,
                hipStream_t st) {
  if (int rc = ensure_twiddles()) return rc;
  if (dtype == TP_F64)
    return inv_impl<double>((const double*)re, (const double*)im, n3, rows * cols, (double*)x, st);
  return inv_impl<float>((const float*)re, (const float*)im, n3, rows * cols, (float*)x, st);
}

}  // namespace tp
