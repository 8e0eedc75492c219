// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "tprod.h"

namespace tp {

// thread-local error text behind tp_last_error()
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

#define TP_HIP_CHECK(expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::tp::fail(TP_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

#define TP_LAUNCH_CHECK()                                                                       \
  do {                                                                                          \
    hipError_t e_ = hipGetLastError();                                                          \
    if (e_ != hipSuccess)                                                                       \
      return ::tp::fail(TP_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e_)); \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// A second stream per device (streams.cpp), created on first use, with the
// events that fork it from, and join it to, a caller's stream: independent
// work of one call runs on it beside the caller's stream and is joined back
// before the call's later work. mu serialises the enqueue of one fork-join
// section.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::mutex mu;
};
int side_stream(SideStream** out);

// Bump allocator over a caller workspace. With a null base it only counts
// (dry run), which is how the *_workspace queries size a call: they run the
// same sequence of takes as the call itself.
struct Arena {
  char* base;
  size_t cap;
  size_t used = 0;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t n) {
    size_t off = align_up(used);
    used = off + n * sizeof(T);
    return (used <= cap && base) ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool ok() const { return base != nullptr && used <= cap; }
  bool dry() const { return base == nullptr; }
};

// Sizes a spectrum of the given shape occupies (re and im planes).
inline size_t spectrum_bytes(int64_t K, int64_t rows, int64_t cols, int dtype) {
  size_t es = dtype == TP_F64 ? 8 : 4;
  return 2 * align_up(size_t(K) * rows * cols * es);
}

inline int64_t half_count(int64_t n3) { return n3 / 2 + 1; }

// ---------------------------------------------------------------------------
// Tube transforms (fft.hip)
// ---------------------------------------------------------------------------

// Which tubes feed the forward transform and how they are scaled.
// Output tube (a, b), a < rows, b < cols, is read from input tube
//   (row_idx ? row_idx[a] : a, col_idx ? col_idx[b] : b)
// of a tensor with in_cols tubes per row, multiplied by
//   (row_scale ? row_scale[a] : 1) * (col_scale ? col_scale[b] : 1).
// If `count` is set, output tubes whose gathered coordinate (a when row_idx
// is set, b when col_idx is set) is >= *count are written as zeros.
struct TubeGather {
  int64_t rows = 0, cols = 0, in_cols = 0;
  const int32_t* row_idx = nullptr;
  const int32_t* col_idx = nullptr;
  const double* row_scale = nullptr;
  const double* col_scale = nullptr;
  const int64_t* count = nullptr;
};

int fft_forward(const void* x, int dtype, int64_t n3, const TubeGather& g, void* re, void* im,
                hipStream_t st);
int fft_inverse(const void* re, const void* im, int dtype, int64_t n3, int64_t rows, int64_t cols, void* x,
                hipStream_t st);
bool fft_supported(int64_t n3);
// Forward transform of float32 tubes into the split operand format of the
// matrix-core products: four bf16 planes [hi re, lo re, hi im, lo im][k][slot]
// with slot = row * ld + col (colmajor: col * ld + row); slots past the live
// rows / columns are zero.
bool fft_split_supported(int64_t n3);
int fft_forward_split(const float* x, int64_t n3, const TubeGather& g, bool colmajor, int64_t ld, void* planes,
                      hipStream_t st);

// C_k = A_k B_k from split operands (gemm_mfma.hip): a holds the planes of A
// ([4][K][M][lda]), b those of B transposed ([4][K][N][ldb]); Kd, lda, ldb are
// multiples of 32 and the contraction entries past the live length are
// zero. C is float32 planar [K][M][ldc]. terms: 3 (bf16x3) or 1 (bf16).
struct SplitGemm {
  const void* a = nullptr;
  const void* b = nullptr;
  float* cre = nullptr;
  float* cim = nullptr;
  int64_t K = 0, M = 0, N = 0, Kd = 0, lda = 0, ldb = 0, ldc = 0;
  int64_t pa = 0, pb = 0, sa = 0, sb = 0, sc = 0;
  bool real_last = false;
  int terms = 3;
};
int cgemm_split(const SplitGemm& p, hipStream_t st);

// Launch tracing (trace.cpp): with tp_trace_enable(1) (2: only scopes named
// "*.gemm"), a scope records HIP events on its stream around the work
// enqueued inside it.
class TraceScope {
 public:
  TraceScope(const char* name, hipStream_t st);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t e0_ = nullptr, e1_ = nullptr;
  bool live_ = false;
};

// ---------------------------------------------------------------------------
// Per-slice complex products (gemm.hip)
// ---------------------------------------------------------------------------

// C_k = op(A_k) op(B_k) for k < K over planar complex spectra. M, N, Kd are
// the dimensions of the product (op(A_k) is M x Kd). lda/ldb/ldc are row
// strides of the stored matrices, sa/sb/sc the slice strides (elements).
// kdim_dev, when set, caps Kd at *kdim_dev (sample counts known only on the
// device). Slices 0 and (real_last) K-1 are real.
struct CGemm {
  int64_t K = 0, M = 0, N = 0, Kd = 0;
  const void *are = nullptr, *aim = nullptr, *bre = nullptr, *bim = nullptr;
  void *cre = nullptr, *cim = nullptr;
  int64_t lda = 0, ldb = 0, ldc = 0, sa = 0, sb = 0, sc = 0;
  int op_a = 0, op_b = 0;  // 0 = N, 1 = conjugate transpose
  bool real_last = false;
  const int64_t* kdim_dev = nullptr;
  // optional float32 scratch for a split contraction (products with few
  // output tiles and a long contraction): part_cap floats per plane
  float *part_re = nullptr, *part_im = nullptr;
  int64_t part_cap = 0;
};

int cgemm(const CGemm& p, int dtype, int prec, hipStream_t st);
// Number of contraction parts the matrix-core product would use for an
// M x N x Kd product over K slices (1 = no split), and the scratch floats
// per plane it needs for them.
int cgemm_ksplit(int64_t K, int64_t M, int64_t N, int64_t Kd);
// The same for the float32 matrix-core product (gemm_f32.hip).
int cgemm_f32_ksplit(int64_t K, int64_t M, int64_t N, int64_t Kd);
inline int64_t cgemm_ksplit_floats(int64_t K, int64_t M, int64_t N, int64_t Kd) {
  const int s = cgemm_ksplit(K, M, N, Kd), s2 = cgemm_f32_ksplit(K, M, N, Kd);
  const int m = s > s2 ? s : s2;
  return m > 1 ? int64_t(m) * K * M * N : 0;
}

// ---------------------------------------------------------------------------
// Slice statistics (stats.hip)
// ---------------------------------------------------------------------------
size_t lateral_norms_ws(int64_t n1, int64_t n2, int64_t n3);
int lateral_norms(const void* a, int dtype, int64_t n1, int64_t n2, int64_t n3, double* out, double* ws,
                  hipStream_t st);
int horizontal_norms(const void* a, int dtype, int64_t n1, int64_t n2, int64_t n3, double* out,
                     hipStream_t st);
int combine_normprod(const double* a, const double* b, int64_t n, double* out, hipStream_t st);
int fill_f64(double* p, int64_t n, double v, hipStream_t st);

// ---------------------------------------------------------------------------
// Sampling (sample.hip)
// ---------------------------------------------------------------------------
size_t sampler_ws(int64_t n);
// w: device float64 weights (ignored for uniform mode).
int sample_slices(const double* w, int64_t n, int64_t c, int mode, uint64_t seed, uint64_t stream_id,
                  int32_t* idx, double* scale, int64_t* count, void* ws, hipStream_t st);
// Workspace bytes tp_tsample needs for these arguments (the n-dependent
// part plus the lateral-norm partials of A for the norm-based kinds).
size_t tsample_ws_full(int kind, const tp_tensor* A, int64_t n);
// *out = sum of the n device counts, or -1 if any is -1.
int join_counts(const int64_t* counts, int n, int64_t* out, hipStream_t st);

}  // namespace tp
