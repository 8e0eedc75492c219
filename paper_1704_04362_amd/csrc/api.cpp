// C ABI: argument validation, workspace planning and the order in which the
// kernels of each call are enqueued. No device memory is allocated here.
#include <cmath>
#include <string>

#include "common.hpp"

namespace tp {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t numel(const tp_tensor* t) { return t->n1 * t->n2 * t->n3; }

int check_tensor(const tp_tensor* t, const char* name) {
  if (!t) return fail(TP_EINVAL, std::string(name) + " is null");
  if (t->dtype != TP_F32 && t->dtype != TP_F64) return fail(TP_EDTYPE, std::string(name) + ": unknown dtype");
  if (t->n1 < 0 || t->n2 < 0 || t->n3 < 1)
    return fail(TP_ESHAPE, std::string(name) + ": dimensions must satisfy n1, n2 >= 0 and n3 >= 1");
  if (numel(t) > 0 && !t->data) return fail(TP_EINVAL, std::string(name) + ": data is null");
  return TP_OK;
}

int check_spectrum(const tp_spectrum* s, const char* name) {
  if (!s) return fail(TP_EINVAL, std::string(name) + " is null");
  if (s->dtype != TP_F32 && s->dtype != TP_F64) return fail(TP_EDTYPE, std::string(name) + ": unknown dtype");
  if (s->K < 1 || s->rows < 0 || s->cols < 0) return fail(TP_ESHAPE, std::string(name) + ": bad dimensions");
  if (s->rows * s->cols > 0 && (!s->re || !s->im)) return fail(TP_EINVAL, std::string(name) + ": null plane");
  return TP_OK;
}

int check_prec(int dtype, int prec) {
  if (prec == TP_PREC_F64) {
    if (dtype != TP_F64) return fail(TP_EDTYPE, "TP_PREC_F64 needs float64 data");
    return TP_OK;
  }
  if (prec == TP_PREC_F32 || prec == TP_PREC_BF16X3 || prec == TP_PREC_BF16) {
    if (dtype != TP_F32) return fail(TP_EDTYPE, "float32-input precisions need float32 data");
    return TP_OK;
  }
  return fail(TP_EDTYPE, "unknown precision");
}

int check_sample(const tp_sample* s, int64_t n) {
  if (!s->idx || !s->scale || !s->count) return fail(TP_EINVAL, "sample: null idx/scale/count");
  if (s->cap < 1) return fail(TP_EINVAL, "sample: capacity must be >= 1");
  if (s->cap > n) return fail(TP_ESHAPE, "sample: capacity exceeds the number of slices");
  if (s->cap > 0x7fffffff) return fail(TP_EUNSUPPORTED, "sample: capacity above 2^31-1");
  return TP_OK;
}

int64_t round_up32(int64_t n) { return (n + 31) / 32 * 32; }

// the t-product takes the split-operand matrix-core path for float32 data
// at the bf16 precisions when the tube length has a specialised transform
bool use_split(int dtype, int prec, int64_t n3) {
  return dtype == TP_F32 && (prec == TP_PREC_BF16X3 || prec == TP_PREC_BF16) && fft_split_supported(n3);
}

struct Plane {
  void* re;
  void* im;
};

Plane take_spectrum(Arena& ar, int64_t K, int64_t rows, int64_t cols, int dtype) {
  const size_t n = size_t(K) * rows * cols;
  if (dtype == TP_F64) {
    double* r = ar.take<double>(n);
    double* i = ar.take<double>(n);
    return {r, i};
  }
  float* r = ar.take<float>(n);
  float* i = ar.take<float>(n);
  return {r, i};
}

}  // namespace
}  // namespace tp

using namespace tp;

extern "C" {

const char* tp_status_string(int status) {
  switch (status) {
    case TP_OK: return "ok";
    case TP_EINVAL: return "invalid argument";
    case TP_ESHAPE: return "shape mismatch";
    case TP_EDTYPE: return "unsupported dtype or precision";
    case TP_EWORKSPACE: return "workspace missing or too small";
    case TP_EHIP: return "HIP runtime error";
    case TP_ENOCONV: return "iteration limit reached";
    case TP_EUNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

const char* tp_last_error(void) { return g_last_error.c_str(); }

int tp_version(void) { return 100; }

int tp_tfft(const tp_tensor* X, tp_spectrum* Xh, void* stream) {
  if (int rc = check_tensor(X, "X")) return rc;
  if (int rc = check_spectrum(Xh, "Xh")) return rc;
  if (Xh->dtype != X->dtype) return fail(TP_EDTYPE, "X and Xh dtypes differ");
  if (Xh->K != half_count(X->n3) || Xh->rows != X->n1 || Xh->cols != X->n2)
    return fail(TP_ESHAPE, "Xh must be (n3/2+1) x n1 x n2");
  TubeGather g;
  g.rows = X->n1;
  g.cols = X->n2;
  g.in_cols = X->n2;
  return fft_forward(X->data, X->dtype, X->n3, g, Xh->re, Xh->im, S(stream));
}

int tp_tifft(const tp_spectrum* Xh, tp_tensor* X, void* stream) {
  if (int rc = check_tensor(X, "X")) return rc;
  if (int rc = check_spectrum(Xh, "Xh")) return rc;
  if (Xh->dtype != X->dtype) return fail(TP_EDTYPE, "X and Xh dtypes differ");
  if (Xh->K != half_count(X->n3) || Xh->rows != X->n1 || Xh->cols != X->n2)
    return fail(TP_ESHAPE, "Xh must be (n3/2+1) x n1 x n2");
  return fft_inverse(Xh->re, Xh->im, X->dtype, X->n3, X->n1, X->n2, X->data, S(stream));
}

int tp_spectrum_matmul(const tp_spectrum* A, int op_a, const tp_spectrum* B, int op_b, tp_spectrum* C,
                       int real_last, int prec, void* stream) {
  if (int rc = check_spectrum(A, "A")) return rc;
  if (int rc = check_spectrum(B, "B")) return rc;
  if (int rc = check_spectrum(C, "C")) return rc;
  if ((op_a != 0 && op_a != 1) || (op_b != 0 && op_b != 1)) return fail(TP_EINVAL, "op must be 0 or 1");
  if (A->dtype != B->dtype || A->dtype != C->dtype) return fail(TP_EDTYPE, "spectra dtypes differ");
  if (int rc = check_prec(A->dtype, prec)) return rc;
  if (A->K != B->K || A->K != C->K) return fail(TP_ESHAPE, "spectra have different slice counts");
  const int64_t M = op_a ? A->cols : A->rows, Ka = op_a ? A->rows : A->cols;
  const int64_t Kb = op_b ? B->cols : B->rows, N = op_b ? B->rows : B->cols;
  if (Ka != Kb || C->rows != M || C->cols != N) return fail(TP_ESHAPE, "inner or outer dimensions do not match");
  CGemm p;
  p.K = A->K;
  p.M = M;
  p.N = N;
  p.Kd = Ka;
  p.are = A->re;
  p.aim = A->im;
  p.bre = B->re;
  p.bim = B->im;
  p.cre = C->re;
  p.cim = C->im;
  p.lda = A->cols;
  p.ldb = B->cols;
  p.ldc = C->cols;
  p.sa = A->rows * A->cols;
  p.sb = B->rows * B->cols;
  p.sc = C->rows * C->cols;
  p.op_a = op_a;
  p.op_b = op_b;
  p.real_last = real_last != 0 && A->K > 1;
  return cgemm(p, A->dtype, prec, S(stream));
}

size_t tp_slice_norms_workspace(const tp_tensor* A, int mode) {
  if (!A || mode != 0) return 0;
  return lateral_norms_ws(A->n1, A->n2, A->n3);
}

int tp_slice_norms(const tp_tensor* A, int mode, double* out, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_tensor(A, "A")) return rc;
  if (mode != 0 && mode != 1) return fail(TP_EINVAL, "mode must be 0 (lateral) or 1 (horizontal)");
  const int64_t n = mode == 0 ? A->n2 : A->n1;
  if (n > 0 && !out) return fail(TP_EINVAL, "out is null");
  if (mode == 1) return horizontal_norms(A->data, A->dtype, A->n1, A->n2, A->n3, out, S(stream));
  const size_t need = lateral_norms_ws(A->n1, A->n2, A->n3);
  if (need > 0 && (!ws || ws_bytes < need)) return fail(TP_EWORKSPACE, "slice-norm workspace too small");
  return lateral_norms(A->data, A->dtype, A->n1, A->n2, A->n3, out, (double*)ws, S(stream));
}

size_t tp_tsample_workspace(int64_t n) {
  if (n < 1) return 0;
  // sampler state, two weight vectors, and the lateral-norm partials of a
  // tensor with up to n lateral slices and n1 rows are sized by the call;
  // this is the part that depends on n only.
  return sampler_ws(n) + 2 * align_up(size_t(n) * 8);
}

}  // extern "C"

size_t tp::tsample_ws_full(int kind, const tp_tensor* A, int64_t n) {
  size_t s = tp_tsample_workspace(n);
  if ((kind == TP_P_NORM2 || kind == TP_P_NORMPROD) && A) s += lateral_norms_ws(A->n1, A->n2, A->n3);
  return s;
}

extern "C" {

int tp_tsample(int kind, const tp_tensor* A, const tp_tensor* B, const double* w, int64_t n, int64_t c, int mode,
               uint64_t seed, uint64_t stream_id, tp_sample* out, void* ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(TP_EINVAL, "out is null");
  if (mode != TP_S_BERNOULLI && mode != TP_S_IID && mode != TP_S_UNIFORM) return fail(TP_EINVAL, "unknown mode");
  if (kind == TP_P_NORM2 || kind == TP_P_NORMPROD) {
    if (int rc = check_tensor(A, "A")) return rc;
    if (n != A->n2) return fail(TP_ESHAPE, "n must equal A->n2 for lateral-slice probabilities");
    if (kind == TP_P_NORMPROD) {
      if (int rc = check_tensor(B, "B")) return rc;
      if (B->n1 != A->n2 || B->n3 != A->n3) return fail(TP_ESHAPE, "B must be n2 x n4 x n3");
      if (B->dtype != A->dtype) return fail(TP_EDTYPE, "A and B dtypes differ");
    }
  } else if (kind == TP_P_USER) {
    if (!w) return fail(TP_EINVAL, "user weights are null");
  } else if (kind != TP_P_UNIFORM) {
    return fail(TP_EINVAL, "probability kind not available in tp_tsample");
  }
  if (n < 1) return fail(TP_ESHAPE, "need at least one slice");
  if (n > 0x7fffffff) return fail(TP_EUNSUPPORTED, "more than 2^31-1 slices");
  if (c < 1 || c > n) return fail(TP_EINVAL, "need 1 <= c <= n");
  if (!out->idx || !out->scale || !out->count) return fail(TP_EINVAL, "sample: null idx/scale/count");
  const int64_t need_cap = mode == TP_S_BERNOULLI ? n : c;
  if (out->cap < need_cap)
    return fail(TP_EINVAL, mode == TP_S_BERNOULLI ? "Bernoulli picks need capacity >= n" : "capacity must be >= c");
  const size_t need = tsample_ws_full(kind, A, n);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "sampling workspace too small");

  Arena ar(ws, ws_bytes);
  void* sws = ar.take<char>(sampler_ws(n));
  double* wa = ar.take<double>(n);
  double* wb = ar.take<double>(n);
  double* part = nullptr;
  if (kind == TP_P_NORM2 || kind == TP_P_NORMPROD) part = ar.take<double>(lateral_norms_ws(A->n1, A->n2, A->n3) / 8);
  if (!ar.ok()) return fail(TP_EWORKSPACE, "sampling workspace too small");
  hipStream_t st = S(stream);
  const double* weights = w;
  if (mode != TP_S_UNIFORM) {
    if (kind == TP_P_UNIFORM) {
      if (int rc = fill_f64(wa, n, 1.0, st)) return rc;
      weights = wa;
    } else if (kind == TP_P_NORM2 || kind == TP_P_NORMPROD) {
      if (int rc = lateral_norms(A->data, A->dtype, A->n1, A->n2, A->n3, wa, part, st)) return rc;
      weights = wa;
      if (kind == TP_P_NORMPROD) {
        if (int rc = horizontal_norms(B->data, B->dtype, B->n1, B->n2, B->n3, wb, st)) return rc;
        if (int rc = combine_normprod(wa, wb, n, wa, st)) return rc;
      }
    }
  }
  return sample_slices(weights, n, c, mode, seed, stream_id, out->idx, out->scale, out->count, sws, st);
}

size_t tp_tprod_workspace(const tp_tensor* A, const tp_tensor* B, const tp_sample* sample, int prec) {
  if (!A || !B) return 0;
  const int64_t K = half_count(A->n3);
  const int64_t inner = sample ? sample->cap : A->n2;
  if (use_split(A->dtype, prec, A->n3)) {
    const int64_t ldk = round_up32(inner);
    return align_up(size_t(8) * K * A->n1 * ldk) + align_up(size_t(8) * K * B->n2 * ldk) +
           spectrum_bytes(K, A->n1, B->n2, TP_F32) + 1024;
  }
  const int64_t part = A->dtype == TP_F32 ? cgemm_ksplit_floats(K, A->n1, B->n2, inner) : 0;
  return spectrum_bytes(K, A->n1, inner, A->dtype) + spectrum_bytes(K, inner, B->n2, A->dtype) +
         spectrum_bytes(K, A->n1, B->n2, A->dtype) + 2 * align_up(size_t(4) * part) + 1024;
}

int tp_tprod(const tp_tensor* A, const tp_tensor* B, const tp_sample* sample, tp_tensor* C, int prec, void* ws,
             size_t ws_bytes, void* stream) {
  if (int rc = check_tensor(A, "A")) return rc;
  if (int rc = check_tensor(B, "B")) return rc;
  if (int rc = check_tensor(C, "C")) return rc;
  if (A->dtype != B->dtype || A->dtype != C->dtype) return fail(TP_EDTYPE, "A, B, C dtypes differ");
  if (int rc = check_prec(A->dtype, prec)) return rc;
  if (A->n2 != B->n1 || A->n3 != B->n3) return fail(TP_ESHAPE, "t-product needs A n1 x n2 x n3 and B n2 x n4 x n3");
  if (C->n1 != A->n1 || C->n2 != B->n2 || C->n3 != A->n3) return fail(TP_ESHAPE, "C must be n1 x n4 x n3");
  if (sample)
    if (int rc = check_sample(sample, A->n2)) return rc;
  const size_t need = tp_tprod_workspace(A, B, sample, prec);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "t-product workspace too small");
  if (numel(C) == 0) return TP_OK;

  const int64_t n1 = A->n1, n2 = A->n2, n4 = B->n2, n3 = A->n3, K = half_count(n3);
  const int64_t inner = sample ? sample->cap : n2;
  const bool real_last = (n3 % 2 == 0) && K > 1;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  // stage names for launch tracing (exact product / rt-product)
  const char* nm_fa = sample ? "rtprod.fft_a" : "tprod.fft_a";
  const char* nm_fb = sample ? "rtprod.fft_b" : "tprod.fft_b";
  const char* nm_mm = sample ? "rtprod.gemm" : "tprod.gemm";
  const char* nm_if = sample ? "rtprod.ifft" : "tprod.ifft";

  TubeGather ga;
  ga.rows = n1;
  ga.cols = inner;
  ga.in_cols = n2;
  TubeGather gb;
  gb.rows = inner;
  gb.cols = n4;
  gb.in_cols = n4;
  if (sample) {
    // C = A*S*D: picked lateral slices of A; R = D*S^T*B: the matching
    // horizontal slices of B (Algorithm 2); both read straight from the
    // original tensors and transformed once.
    ga.col_idx = sample->idx;
    ga.col_scale = sample->scale;
    ga.count = sample->count;
    gb.row_idx = sample->idx;
    gb.row_scale = sample->scale;
    gb.count = sample->count;
  }

  if (use_split(A->dtype, prec, n3)) {
    // matrix-core path: both operands transformed straight into split bf16
    // planes with the contraction index contiguous (B transposed), padded
    // to a multiple of 32 with zeros
    const int64_t ldk = round_up32(inner);
    void* Ap = ar.take<char>(size_t(8) * K * n1 * ldk);
    void* Bp = ar.take<char>(size_t(8) * K * n4 * ldk);
    Plane Ch = take_spectrum(ar, K, n1, n4, TP_F32);
    if (!ar.ok()) return fail(TP_EWORKSPACE, "t-product workspace too small");
    {
      TraceScope ts(nm_fa, st);
      if (int rc = fft_forward_split((const float*)A->data, n3, ga, false, ldk, Ap, st)) return rc;
    }
    {
      TraceScope ts(nm_fb, st);
      if (int rc = fft_forward_split((const float*)B->data, n3, gb, true, ldk, Bp, st)) return rc;
    }
    SplitGemm g;
    g.a = Ap;
    g.b = Bp;
    g.cre = (float*)Ch.re;
    g.cim = (float*)Ch.im;
    g.K = K;
    g.M = n1;
    g.N = n4;
    g.Kd = ldk;
    g.lda = ldk;
    g.ldb = ldk;
    g.ldc = n4;
    g.pa = K * n1 * ldk;
    g.pb = K * n4 * ldk;
    g.sa = n1 * ldk;
    g.sb = n4 * ldk;
    g.sc = n1 * n4;
    g.real_last = real_last;
    g.terms = prec == TP_PREC_BF16X3 ? 3 : 1;
    {
      TraceScope ts(nm_mm, st);
      if (int rc = cgemm_split(g, st)) return rc;
    }
    TraceScope ts(nm_if, st);
    return fft_inverse(Ch.re, Ch.im, TP_F32, n3, n1, n4, C->data, st);
  }

  Plane Ah = take_spectrum(ar, K, n1, inner, A->dtype);
  Plane Bh = take_spectrum(ar, K, inner, n4, A->dtype);
  Plane Ch = take_spectrum(ar, K, n1, n4, A->dtype);
  // scratch for a split contraction of a product with few output tiles
  const int64_t part = A->dtype == TP_F32 ? cgemm_ksplit_floats(K, n1, n4, inner) : 0;
  float* part_re = part ? ar.take<float>(part) : nullptr;
  float* part_im = part ? ar.take<float>(part) : nullptr;
  if (!ar.ok()) return fail(TP_EWORKSPACE, "t-product workspace too small");
  if (inner > 0) {
    TraceScope ts(sample ? "rtprod.fft_ab" : "tprod.fft_ab", st);
    if (int rc = fft_forward(A->data, A->dtype, n3, ga, Ah.re, Ah.im, st)) return rc;
    if (int rc = fft_forward(B->data, B->dtype, n3, gb, Bh.re, Bh.im, st)) return rc;
  }
  CGemm p;
  p.K = K;
  p.M = n1;
  p.N = n4;
  p.Kd = inner;
  p.are = Ah.re;
  p.aim = Ah.im;
  p.bre = Bh.re;
  p.bim = Bh.im;
  p.cre = Ch.re;
  p.cim = Ch.im;
  p.lda = inner;
  p.ldb = n4;
  p.ldc = n4;
  p.sa = n1 * inner;
  p.sb = inner * n4;
  p.sc = n1 * n4;
  p.real_last = real_last;
  p.kdim_dev = sample ? sample->count : nullptr;
  p.part_re = part_re;
  p.part_im = part_im;
  p.part_cap = part;
  {
    TraceScope ts(nm_mm, st);
    if (int rc = cgemm(p, A->dtype, prec, st)) return rc;
  }
  TraceScope ts(nm_if, st);
  return fft_inverse(Ch.re, Ch.im, A->dtype, n3, n1, n4, C->data, st);
}

}  // extern "C"
