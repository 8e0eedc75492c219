// Slice statistics feeding the sampling probabilities of Section 3:
// squared Frobenius norms of lateral slices ||A_{:j:}||_F^2 (eq.
// nonoptimal_probs and, with horizontal norms of B, eq. nearly_optimal_probs)
// and of horizontal slices ||A_{i::}||_F^2.
//
// Squares are formed and summed in float64 (a float32 square is exact in
// float64), always in the same order, so results are reproducible run to
// run. No floating-point atomics.
#include "common.hpp"

namespace tp {
namespace {

constexpr int LT = 32;      // tubes (lateral slices) per workgroup (64 measured 2% slower in the rt-product)
constexpr int LROWS = 16;   // horizontal slices per workgroup
constexpr int LNT = 256;    // threads per workgroup

template <typename T>
struct V16;
template <>
struct V16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct V16<double> {
  using type = double2;
  static constexpr int n = 2;
};

// Workgroup (bx, by) sums rows [by*LROWS, +LROWS) for tubes [bx*LT, +LT).
// In every row those LT tubes are one contiguous run of LT*n3 values; a
// thread always owns the same 16-byte pieces of that run, so it accumulates
// its pieces over all rows with independent coalesced loads, and the pieces
// of a tube are added in a fixed order at the end through LDS.
template <typename T>
__global__ __launch_bounds__(LNT) void lateral_partial_kernel(const T* __restrict__ a, int64_t n1, int64_t n2,
                                                               int64_t n3, double* __restrict__ partial) {
  using V = typename V16<T>::type;
  constexpr int VN = V16<T>::n;
  extern __shared__ double piece[];  // [LT][CH]
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * LT;
  const int64_t i0 = (int64_t)blockIdx.y * LROWS;
  const int64_t ntub = (n2 - j0) < LT ? (n2 - j0) : LT;
  const bool vec = (n3 % VN) == 0;
  const int64_t CH = vec ? n3 / VN : n3;
  const int64_t npieces = ntub * CH;
  const int64_t rows = (n1 - i0) < LROWS ? (n1 - i0) : LROWS;
  for (int64_t f0 = 0; f0 < LT * CH; f0 += LNT) {
    const int64_t f = f0 + tid;
    double s = 0.0;
    if (f < npieces) {
      if (vec) {
        // all LROWS loads in flight at once: rows past the end re-read the
        // last row and are masked out of the sum
        V w[LROWS];
#pragma unroll
        for (int r = 0; r < LROWS; ++r) {
          const int64_t rr = r < rows ? r : rows - 1;
          w[r] = *reinterpret_cast<const V*>(a + ((i0 + rr) * n2 + j0) * n3 + f * VN);
        }
#pragma unroll
        for (int r = 0; r < LROWS; ++r) {
          const T* wp = reinterpret_cast<const T*>(&w[r]);
          double q = 0.0;
#pragma unroll
          for (int e = 0; e < VN; ++e) q += (double)wp[e] * (double)wp[e];
          s += r < rows ? q : 0.0;
        }
      } else {
        for (int64_t r = 0; r < rows; ++r) {
          const double v = (double)a[((i0 + r) * n2 + j0) * n3 + f];
          s += v * v;
        }
      }
    }
    if (f < LT * CH) piece[f] = s;
  }
  __syncthreads();
  if (tid < ntub) {
    double t = 0.0;
    for (int64_t p = 0; p < CH; ++p) t += piece[tid * CH + p];
    partial[(int64_t)blockIdx.y * n2 + j0 + tid] = t;
  }
}

// Long tubes (the piece table of the kernel above would exceed 64 KB): one
// workgroup per (tube j, block of LROWS rows), each thread summing fixed
// 16-byte pieces of the block's tubes, then a fixed-order tree over the
// threads.
template <typename T>
__global__ __launch_bounds__(LNT) void lateral_long_kernel(const T* __restrict__ a, int64_t n1, int64_t n2,
                                                            int64_t n3, double* __restrict__ partial) {
  using V = typename V16<T>::type;
  constexpr int VN = V16<T>::n;
  __shared__ double red[LNT];
  const int64_t j = blockIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * LROWS;
  const int64_t rows = (n1 - i0) < LROWS ? (n1 - i0) : LROWS;
  double s = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    const T* tube = a + ((i0 + r) * n2 + j) * n3;
    if (n3 % VN == 0) {
      for (int64_t f = threadIdx.x; f < n3 / VN; f += LNT) {
        const V w = *reinterpret_cast<const V*>(tube + f * VN);
        const T* wp = reinterpret_cast<const T*>(&w);
#pragma unroll
        for (int e = 0; e < VN; ++e) s += (double)wp[e] * (double)wp[e];
      }
    } else {
      for (int64_t f = threadIdx.x; f < n3; f += LNT) s += (double)tube[f] * (double)tube[f];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = LNT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * n2 + j] = red[0];
}

__global__ void reduce_partials_kernel(const double* __restrict__ partial, int64_t nb, int64_t n,
                                       double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
#pragma unroll 8
  for (int64_t b = 0; b < nb; ++b) s += partial[b * n + j];
  out[j] = s;
}

// One workgroup per horizontal slice (a contiguous run of n2*n3 values).
template <typename T>
__global__ __launch_bounds__(256) void horizontal_kernel(const T* __restrict__ a, int64_t n2, int64_t n3,
                                                         double* __restrict__ out) {
  using V = typename V16<T>::type;
  constexpr int VN = V16<T>::n;
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  const int64_t len = n2 * n3;
  const T* row = a + i * len;
  double s = 0.0;
  if (len % VN == 0) {
    for (int64_t f = threadIdx.x; f < len / VN; f += 256) {
      const V w = *reinterpret_cast<const V*>(row + f * VN);
      const T* wp = reinterpret_cast<const T*>(&w);
#pragma unroll
      for (int e = 0; e < VN; ++e) s += (double)wp[e] * (double)wp[e];
    }
  } else {
    for (int64_t f = threadIdx.x; f < len; f += 256) s += (double)row[f] * (double)row[f];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

__global__ void fill_zero_kernel(double* out, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = 0.0;
}

__global__ void fill_value_kernel(double* out, int64_t n, double v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = v;
}

__global__ void normprod_kernel(const double* a, const double* b, int64_t n, double* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = sqrt(a[j] * b[j]);
}

int64_t lateral_blocks(int64_t n1) { return (n1 + LROWS - 1) / LROWS; }

}  // namespace

size_t lateral_norms_ws(int64_t n1, int64_t n2, int64_t) { return align_up(size_t(lateral_blocks(n1)) * n2 * 8); }

int lateral_norms(const void* a, int dtype, int64_t n1, int64_t n2, int64_t n3, double* out, double* ws,
                  hipStream_t st) {
  if (n2 == 0) return TP_OK;
  const int64_t nb = lateral_blocks(n1);
  const int vn = dtype == TP_F64 ? 2 : 4;
  const int64_t CH = (n3 % vn == 0) ? n3 / vn : n3;
  const size_t lds = size_t(LT) * CH * sizeof(double);
  if (n1 == 0) {
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, out, n2);
    TP_LAUNCH_CHECK();
    return TP_OK;
  }
  if (lds > 64 * 1024) {
    if (n2 > 0x7fffffffLL) return fail(TP_EUNSUPPORTED, "too many lateral slices");
    dim3 grid((unsigned)n2, (unsigned)nb);
    if (dtype == TP_F64)
      hipLaunchKernelGGL(lateral_long_kernel<double>, grid, dim3(LNT), 0, st, (const double*)a, n1, n2, n3, ws);
    else
      hipLaunchKernelGGL(lateral_long_kernel<float>, grid, dim3(LNT), 0, st, (const float*)a, n1, n2, n3, ws);
  } else {
    dim3 grid((unsigned)((n2 + LT - 1) / LT), (unsigned)nb);
    if (dtype == TP_F64)
      hipLaunchKernelGGL(lateral_partial_kernel<double>, grid, dim3(LNT), lds, st, (const double*)a, n1, n2, n3, ws);
    else
      hipLaunchKernelGGL(lateral_partial_kernel<float>, grid, dim3(LNT), lds, st, (const float*)a, n1, n2, n3, ws);
  }
  TP_LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, ws, nb, n2, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int horizontal_norms(const void* a, int dtype, int64_t n1, int64_t n2, int64_t n3, double* out, hipStream_t st) {
  if (n1 == 0) return TP_OK;
  if (dtype == TP_F64)
    hipLaunchKernelGGL(horizontal_kernel<double>, dim3((unsigned)n1), dim3(256), 0, st, (const double*)a, n2, n3, out);
  else
    hipLaunchKernelGGL(horizontal_kernel<float>, dim3((unsigned)n1), dim3(256), 0, st, (const float*)a, n2, n3, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(fill_value_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int combine_normprod(const double* a, const double* b, int64_t n, double* out, hipStream_t st) {
  if (n == 0) return TP_OK;
  hipLaunchKernelGGL(normprod_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
