// C ABI of the randomized decompositions: tubal-rank-r t-SVD by a Gaussian
// range finder (the t-SVD theorem computed slice by slice in the Fourier
// domain), tubal leverage scores (eqs. cur-col-prob, colprob_rows_exact) and
// t-CUR (Algorithm 5). Validation, workspace planning and kernel order only.
#include <algorithm>
#include <cmath>
#include <string>

#include "common.hpp"
#include "linalg.hpp"
#include "svt.hpp"

namespace tp {
namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct Spec {
  void* re = nullptr;
  void* im = nullptr;
};

Spec take(Arena& ar, int64_t n, int dtype) {
  Spec s;
  if (dtype == TP_F64) {
    s.re = ar.take<double>(n);
    s.im = ar.take<double>(n);
  } else {
    s.re = ar.take<float>(n);
    s.im = ar.take<float>(n);
  }
  return s;
}

// Batched product C_k = op(A_k) op(B_k) over row-major slices.
int mm(const Spec& A, int op_a, int64_t a_rows, int64_t a_cols, const Spec& B, int op_b, int64_t b_rows,
       int64_t b_cols, const Spec& C, int64_t K, bool real_last, int dtype, int prec, hipStream_t st,
       const int64_t* kdim_dev = nullptr) {
  CGemm p;
  p.K = K;
  p.M = op_a ? a_cols : a_rows;
  p.Kd = op_a ? a_rows : a_cols;
  p.N = op_b ? b_rows : b_cols;
  p.are = A.re;
  p.aim = A.im;
  p.bre = B.re;
  p.bim = B.im;
  p.cre = C.re;
  p.cim = C.im;
  p.lda = a_cols;
  p.ldb = b_cols;
  p.ldc = p.N;
  p.sa = a_rows * a_cols;
  p.sb = b_rows * b_cols;
  p.sc = p.M * p.N;
  p.op_a = op_a;
  p.op_b = op_b;
  p.real_last = real_last;
  p.kdim_dev = kdim_dev;
  return cgemm(p, dtype, prec, st);
}

// Range finder for a batch of m x n slices X_k: an orthonormal basis Q_k
// (m x s) of the range of X_k Omega_k after q power iterations, the
// projected matrix Bh_k = X_k^H Q_k (n x s), and the eigen-decomposition of
// Bh_k^H Bh_k = Q_k^H X_k X_k^H Q_k = U_B diag(lambda) U_B^H, so that the
// singular values of Q^H X are sqrt(lambda) with left vectors U_B and right
// vectors Bh U_B diag(lambda)^-1/2 (Halko, Martinsson, Tropp 2011).
struct RangeFinder {
  int64_t K, m, n;
  int s;
  int dtype;  // of X, Q, Bh
  bool real_last;
  Spec omega, Y, Q, Bh, Z, T;
  double *gre, *gim, *evals, *ure, *uim;
  double *pre = nullptr, *pim = nullptr;  // partial Gram matrices of tall slices

  bool carve(Arena& ar) {
    omega = take(ar, K * n * s, dtype);
    Y = take(ar, K * m * s, dtype);
    Q = take(ar, K * m * s, dtype);
    Bh = take(ar, K * n * s, dtype);
    Z = take(ar, K * n * s, dtype);
    T = take(ar, K * s * s, dtype);
    gre = ar.take<double>(K * s * s);
    gim = ar.take<double>(K * s * s);
    ure = ar.take<double>(K * s * s);
    uim = ar.take<double>(K * s * s);
    evals = ar.take<double>(K * s);
    size_t np = gram_part_doubles(K, std::max(m, n), s);
    if (n <= kMaxS) np = std::max(np, xgram_part_doubles(K, m, (int)n, s));
    if (np) {
      pre = ar.take<double>(np);
      pim = ar.take<double>(np);
    }
    return ar.dry() || ar.ok();
  }

  // out = orthonormal basis of the columns of X (rows x s) by CholeskyQR:
  // X^H X = R^H R, out = X R^{-1}, with pivots at or below rtol times the
  // largest diagonal entry dropped (zero columns).
  int orth(const Spec& X, int64_t rows, const Spec& out, int prec, hipStream_t st, double rtol_pivot = 0.0) const {
    const double rtol = rtol_pivot > 0.0 ? rtol_pivot : (dtype == TP_F64 ? 1e-24 : 1e-11);
    if (int rc = gram(X.re, X.im, dtype, K, rows, s, s, rows * s, real_last, gre, gim, pre, pim, st)) return rc;
    if (int rc = chol_inv(gre, gim, K, s, rtol, real_last, T.re, T.im, dtype, st)) return rc;
    return mm(X, 0, rows, s, T, 0, s, s, out, K, real_last, dtype, prec, st);
  }

  // Bh = X^H Q (n x s): a row-split cross product when X is narrow (the
  // range finder of C and of the t-CUR core), the general product otherwise
  int project(const Spec& X, int prec, hipStream_t st) const {
    if (n <= kMaxS)
      return xgram(X.re, X.im, (int)n, n, m * n, Q.re, Q.im, s, s, m * s, dtype, K, m, real_last, Bh.re, Bh.im, pre,
                   pim, st);
    return mm(X, 1, m, n, Q, 0, m, s, Bh, K, real_last, dtype, prec, st);
  }

  int run(const Spec& X, int q, uint64_t seed, uint64_t stream_id, int prec, hipStream_t st,
          const int64_t* ncols_dev = nullptr) {
    if (int rc = randn_spectrum(omega.re, omega.im, dtype, K, n, s, real_last, seed, stream_id, st)) return rc;
    // Y = X Omega
    if (int rc = mm(X, 0, m, n, omega, 0, n, s, Y, K, real_last, dtype, prec, st, ncols_dev)) return rc;
    return finish(X, q, prec, st, ncols_dev);
  }

  // The rest of the range finder from a sketch already in Y (m x s): the
  // Gaussian one of run(), or picked columns of X (the t-CX basis).
  int finish(const Spec& X, int q, int prec, hipStream_t st, const int64_t* ncols_dev = nullptr) {
    // Q = orth(orth(Y))
    if (int rc = orth(Y, m, Q, prec, st)) return rc;
    if (int rc = orth(Q, m, Y, prec, st)) return rc;
    std::swap(Q, Y);
    for (int it = 0; it < q; ++it) {
      // Z = orth(X^H Q), Q = orth(orth(X Z))
      if (int rc = project(X, prec, st)) return rc;
      if (int rc = orth(Bh, n, Z, prec, st)) return rc;
      if (int rc = mm(X, 0, m, n, Z, 0, n, s, Y, K, real_last, dtype, prec, st, ncols_dev)) return rc;
      if (int rc = orth(Y, m, Q, prec, st)) return rc;
      if (int rc = orth(Q, m, Y, prec, st)) return rc;
      std::swap(Q, Y);
    }
    if (int rc = project(X, prec, st)) return rc;
    if (int rc = gram(Bh.re, Bh.im, dtype, K, n, s, s, n * s, real_last, gre, gim, pre, pim, st)) return rc;
    return herm_eig(gre, gim, K, s, evals, ure, uim, st);
  }
};

int check_tensor(const tp_tensor* t, const char* name) {
  if (!t) return fail(TP_EINVAL, std::string(name) + " is null");
  if (t->dtype != TP_F32 && t->dtype != TP_F64) return fail(TP_EDTYPE, std::string(name) + ": unknown dtype");
  if (t->n1 < 1 || t->n2 < 1 || t->n3 < 1) return fail(TP_ESHAPE, std::string(name) + ": empty tensor");
  if (!t->data) return fail(TP_EINVAL, std::string(name) + ": data is null");
  return TP_OK;
}

int check_prec(int dtype, int prec) {
  if (prec == TP_PREC_F64) return dtype == TP_F64 ? TP_OK : fail(TP_EDTYPE, "TP_PREC_F64 needs float64 data");
  if (prec == TP_PREC_F32 || prec == TP_PREC_BF16X3)
    return dtype == TP_F32 ? TP_OK : fail(TP_EDTYPE, "float32 precisions need float32 data");
  return fail(TP_EDTYPE, "precision not available for decompositions");
}

constexpr int kOversample = 10;
constexpr int kPowerIters = 1;
constexpr int kCorePowerIters = 2;
// stream ids of the generator draws inside one call
constexpr uint64_t kStreamColPick = 0, kStreamRowPick = 1, kStreamOmegaA = 2, kStreamOmegaC = 3, kStreamOmegaW = 4;

// r + p columns, rounded up to a multiple of 4 (row strides the matrix-core
// products accept) when that still fits the slices and the small solvers.
int sketch_size(int64_t r, int64_t p, int64_t m, int64_t n) {
  int64_t s = r + p;
  const int64_t s4 = (s + 3) / 4 * 4;
  if (s4 <= std::min<int64_t>(m, n) && s4 <= kMaxS) s = s4;
  s = std::min<int64_t>(s, std::min<int64_t>(m, n));
  s = std::max<int64_t>(s, r);
  return (int)s;
}

// A probability kind and a pick mode that go together. Uniform picks
// without replacement use no weights, so they take TP_P_UNIFORM only
// (another kind would be computed and then ignored); the learned proposal
// exists for lateral slices (columns) only.
int check_pick_rule(int kind, int mode, bool columns) {
  if (mode != TP_S_BERNOULLI && mode != TP_S_IID && mode != TP_S_UNIFORM) return fail(TP_EINVAL, "unknown mode");
  const bool known = kind == TP_P_USER || kind == TP_P_UNIFORM || kind == TP_P_NORM2 || kind == TP_P_LEV ||
                     (columns && kind == TP_P_LEARNED);
  if (!known) return fail(TP_EINVAL, "unsupported probability kind");
  if (mode == TP_S_UNIFORM && kind != TP_P_UNIFORM)
    return fail(TP_EINVAL, "TP_S_UNIFORM picks use no weights: pass TP_P_UNIFORM");
  return TP_OK;
}

// Every buffer of one tp_tsvd_rand call, carved in a fixed order so that the
// workspace query (dry run) and the call agree.
struct TsvdLayout {
  Spec Ah, Ub, Vs, Us, Ubs, Vsc;
  RangeFinder rf;
  double* lpart = nullptr;
  bool carve(Arena& ar, int64_t K, int64_t n1, int64_t n2, int s, int64_t r, int dt, bool real_last) {
    Ah = take(ar, K * n1 * n2, dt);  // the spectrum of A, later that of A_r
    lpart = ar.take<double>(K * std::max(n1, n2));
    rf = RangeFinder{K, n1, n2, s, dt, real_last};
    rf.carve(ar);
    Ub = take(ar, K * s * r, dt);
    Vs = take(ar, K * n2 * r, dt);
    Us = take(ar, K * n1 * r, dt);
    Ubs = take(ar, K * s * r, dt);
    Vsc = take(ar, K * n2 * r, dt);
    return ar.dry() || ar.ok();
  }
};

// Sketch width of tp_tsvd_rand: r + p (rounded as sketch_size does), or the
// capacity of the picked slices when the basis comes from them.
int tsvd_sketch(const tp_tensor* A, int64_t r, int64_t p, const tp_sample* slices) {
  if (slices) return (int)std::min<int64_t>(slices->cap, int64_t(1) << 30);
  return sketch_size(r, p, A->n1, A->n2);
}

struct TcurLayout {
  double *wbuf = nullptr, *wbuf2 = nullptr, *part = nullptr, *lpart = nullptr;
  void* sws = nullptr;
  void* mlpws = nullptr;  // learned column proposal (TP_P_LEARNED)
  size_t mlp_bytes = 0;
  Spec Ah, UbA, Vs;          // column leverage
  RangeFinder rfA, rfC, cf;  // range finders on A, C and the core
  Spec Ch, UbC, Us;          // C and its row leverage
  Spec Rh, W, Tr, Tp, P64, U64, P, Ur, F, G, Zh;
  int sA = 0, sC = 0, sw = 0;
  bool carve(Arena& ar, int64_t K, int64_t n1, int64_t n2, int64_t n3, int64_t capc, int64_t capl, int64_t r,
             int col_kind, int row_kind, bool want_z, int dt, bool real_last) {
    const int64_t nmax = std::max(n1, n2);
    wbuf = ar.take<double>(nmax);
    wbuf2 = ar.take<double>(nmax);
    sws = ar.take<char>(sampler_ws(nmax));
    part = ar.take<double>(lateral_norms_ws(n1, n2, n3) / 8 + 1);
    lpart = ar.take<double>(K * nmax);
    if (col_kind == TP_P_LEARNED) {
      tp_tensor a{nullptr, dt, n1, n2, n3};
      mlp_bytes = tp_mlp_proposal_workspace(&a);
      mlpws = ar.take<char>(mlp_bytes);
    }
    if (col_kind == TP_P_LEV) {
      sA = sketch_size(r, kOversample, n1, n2);
      Ah = take(ar, K * n1 * n2, dt);
      rfA = RangeFinder{K, n1, n2, sA, dt, real_last};
      rfA.carve(ar);
      UbA = take(ar, K * sA * r, dt);
      Vs = take(ar, K * n2 * r, dt);
    }
    Ch = take(ar, K * n1 * capc, dt);
    if (row_kind == TP_P_LEV) {
      sC = sketch_size(r, kOversample, n1, capc);
      rfC = RangeFinder{K, n1, capc, sC, dt, real_last};
      rfC.carve(ar);
      UbC = take(ar, K * sC * r, dt);
      Us = take(ar, K * n1 * r, dt);
    }
    if (want_z) {
      Rh = take(ar, K * capl * n2, dt);
      W = take(ar, K * capl * capc, TP_F64);
      sw = sketch_size(r, kOversample, capl, capc);
      cf = RangeFinder{K, capl, capc, sw, TP_F64, real_last};
      cf.carve(ar);
      Tr = take(ar, K * sw * r, TP_F64);
      Tp = take(ar, K * sw * r, TP_F64);
      P64 = take(ar, K * capc * r, TP_F64);
      U64 = take(ar, K * capl * r, TP_F64);
      P = take(ar, K * capc * r, dt);
      Ur = take(ar, K * capl * r, dt);
      F = take(ar, K * n1 * r, dt);
      G = take(ar, K * r * n2, dt);
      Zh = take(ar, K * n1 * n2, dt);
    }
    return ar.dry() || ar.ok();
  }
};

// Lateral leverage of A (eq. cur-col-prob) from the rank-r randomized t-SVD
// (p = 10, q = 1): lay.wbuf gets n2 unnormalised scores.
int col_leverage(TcurLayout& lay, const void* A, int dt, int64_t n1, int64_t n2, int64_t n3, int64_t K, int64_t r,
                 uint64_t seed, int prec, bool real_last, double rtol, hipStream_t st) {
  TubeGather g;
  g.rows = n1;
  g.cols = n2;
  g.in_cols = n2;
  const int s = lay.sA;
  if (int rc = fft_forward(A, dt, n3, g, lay.Ah.re, lay.Ah.im, st)) return rc;
  if (int rc = lay.rfA.run(lay.Ah, kPowerIters, seed, kStreamOmegaA, prec, st)) return rc;
  if (int rc = eig_transform(lay.rfA.ure, lay.rfA.uim, lay.rfA.evals, K, s, (int)r, 1, rtol, 0.0, lay.UbA.re,
                             lay.UbA.im, dt, st))
    return rc;
  if (int rc = mm(lay.rfA.Bh, 0, n2, s, lay.UbA, 0, s, r, lay.Vs, K, real_last, dt, prec, st)) return rc;
  return leverage(lay.Vs.re, lay.Vs.im, dt, K, n2, r, n2 * r, (int)r, real_last, lay.rfA.evals, s, rtol, lay.lpart,
                  lay.wbuf, st);
}

// Horizontal leverage of C (eq. colprob_rows_exact) from the top-r left
// singular slices of the spectrum in lay.Ch: lay.wbuf2 gets n1 scores.
int row_leverage(TcurLayout& lay, int dt, int64_t n1, int64_t K, int64_t r, uint64_t seed, int prec, bool real_last,
                 double rtol, const int64_t* ccount, hipStream_t st) {
  const int s = lay.sC;
  if (int rc = lay.rfC.run(lay.Ch, kPowerIters, seed, kStreamOmegaC, prec, st, ccount)) return rc;
  if (int rc = eig_transform(lay.rfC.ure, lay.rfC.uim, lay.rfC.evals, K, s, (int)r, 1, rtol, 0.0, lay.UbC.re,
                             lay.UbC.im, dt, st))
    return rc;
  if (int rc = mm(lay.rfC.Q, 0, n1, s, lay.UbC, 0, s, r, lay.Us, K, real_last, dt, prec, st)) return rc;
  return leverage(lay.Us.re, lay.Us.im, dt, K, n1, r, n1 * r, (int)r, real_last, nullptr, s, rtol, lay.lpart,
                  lay.wbuf2, st);
}

// The core and the reconstruction shared by t-CUR and CUR t-NN, from the
// spectra lay.Ch (n1 x capc) and lay.Rh (capl x n2): W_k = D S^T Chat_k (the
// rows ridx of Chat_k, times rscale when given), Uhat_k = pinv_r(W_k) in
// float64 through a range finder on W_k (pinv_r(W) = V_r diag(1/sigma)
// U_r^H with U_r = Q U_B,r and V_r = Bh U_B,r diag(1/sigma)), then
// Zhat_k = (Chat_k P_k)(U_r,k^H Rhat_k) and Z = ifft(Zhat).
int cur_core(TcurLayout& lay, int64_t n1, int64_t n2, int64_t n3, int64_t K, int64_t capc, int64_t capl, int64_t r,
             const int32_t* ridx, const double* rscale, const int64_t* rcount, uint64_t seed, int dt, int prec,
             bool real_last, void* Z, const tp_spectrum* core, hipStream_t st) {
  const int sw = lay.sw;
  if (int rc = gather_rows(lay.Ch.re, lay.Ch.im, dt, K, n1, capc, ridx, rscale, rcount, capl, lay.W.re, lay.W.im,
                           TP_F64, st))
    return rc;
  // keep sigma_i > max(l, c) eps sigma_1 among the leading r
  const double core_rtol = double(std::max(capl, capc)) * 2.220446049250313e-16;
  Spec Pw = lay.P64, Uw = lay.U64;
  if (core_pinv_fits(capl, capc, sw, r)) {
    // small cores: the whole range finder, eigen-decomposition and factors
    // in one workgroup per Fourier slice
    if (int rc = randn_spectrum(lay.cf.omega.re, lay.cf.omega.im, TP_F64, K, capc, sw, real_last, seed,
                                kStreamOmegaW, st))
      return rc;
    const bool f32 = dt == TP_F32;
    if (int rc = core_pinv((const double*)lay.W.re, (const double*)lay.W.im, (const double*)lay.cf.omega.re,
                           (const double*)lay.cf.omega.im, K, capl, capc, sw, r, real_last, kCorePowerIters,
                           core_rtol, (double*)lay.P64.re, (double*)lay.P64.im, (double*)lay.U64.re,
                           (double*)lay.U64.im, f32 ? (float*)lay.P.re : nullptr, f32 ? (float*)lay.P.im : nullptr,
                           f32 ? (float*)lay.Ur.re : nullptr, f32 ? (float*)lay.Ur.im : nullptr, st))
      return rc;
    if (f32) {
      Pw = lay.P;
      Uw = lay.Ur;
    }
  } else {
    if (int rc = lay.cf.run(lay.W, kCorePowerIters, seed, kStreamOmegaW, TP_PREC_F64, st)) return rc;
    if (int rc = eig_transform(lay.cf.ure, lay.cf.uim, lay.cf.evals, K, sw, (int)r, 1, core_rtol, 2.0, lay.Tp.re,
                               lay.Tp.im, TP_F64, st))
      return rc;
    if (int rc = eig_transform(lay.cf.ure, lay.cf.uim, lay.cf.evals, K, sw, (int)r, 1, core_rtol, 0.0, lay.Tr.re,
                               lay.Tr.im, TP_F64, st))
      return rc;
    // P = Bh U_B,r diag(sigma^-2) = V_r diag(1/sigma) (c x r); U_r = Q U_B,r (l x r)
    if (int rc = mm(lay.cf.Bh, 0, capc, sw, lay.Tp, 0, sw, r, lay.P64, K, real_last, TP_F64, TP_PREC_F64, st))
      return rc;
    if (int rc = mm(lay.cf.Q, 0, capl, sw, lay.Tr, 0, sw, r, lay.U64, K, real_last, TP_F64, TP_PREC_F64, st))
      return rc;
    if (dt == TP_F32) {
      if (int rc = convert(lay.P64.re, TP_F64, lay.P.re, TP_F32, K * capc * r, st)) return rc;
      if (int rc = convert(lay.P64.im, TP_F64, lay.P.im, TP_F32, K * capc * r, st)) return rc;
      if (int rc = convert(lay.U64.re, TP_F64, lay.Ur.re, TP_F32, K * capl * r, st)) return rc;
      if (int rc = convert(lay.U64.im, TP_F64, lay.Ur.im, TP_F32, K * capl * r, st)) return rc;
      Pw = lay.P;
      Uw = lay.Ur;
    }
  }
  if (core) {
    // Uhat_k = pinv_r(W_k) = P_k U_r,k^H (c x l, float64)
    Spec out;
    out.re = core->re;
    out.im = core->im;
    if (int rc = mm(lay.P64, 0, capc, r, lay.U64, 1, capl, r, out, K, real_last, TP_F64, TP_PREC_F64, st)) return rc;
  }
  if (!Z) return TP_OK;
  // Zhat_k = Chat_k Uhat_k Rhat_k = (Chat_k P_k) (U_r,k^H Rhat_k), then ifft
  if (int rc = mm(lay.Ch, 0, n1, capc, Pw, 0, capc, r, lay.F, K, real_last, dt, prec, st)) return rc;
  if (dt == TP_F32) {
    // U_r^H Rhat as the conjugate transpose of Rhat^H U_r, a narrow product
    // (r columns) that the streaming kernel takes; staged in Zhat's buffer,
    // which the next product overwrites
    if (int rc = mm(lay.Rh, 1, capl, n2, Uw, 0, capl, r, lay.Zh, K, real_last, dt, prec, st)) return rc;
    if (int rc = spec_conj_transpose((const float*)lay.Zh.re, (const float*)lay.Zh.im, K, n2, r, (float*)lay.G.re,
                                     (float*)lay.G.im, st))
      return rc;
  } else if (int rc = mm(Uw, 1, capl, r, lay.Rh, 0, capl, n2, lay.G, K, real_last, dt, prec, st)) {
    return rc;
  }
  if (int rc = mm(lay.F, 0, n1, r, lay.G, 0, r, n2, lay.Zh, K, real_last, dt, prec, st)) return rc;
  return fft_inverse(lay.Zh.re, lay.Zh.im, dt, n3, n1, n2, Z, st);
}

// Time-domain parts of CUR t-NN: the picked slices C (n1 x c) and R (l x n2)
// with their masks, and the ADMM iterates of each.
struct CurNNLayout {
  float *cx = nullptr, *cl = nullptr, *ce = nullptr, *cy = nullptr;
  float *rx = nullptr, *rl = nullptr, *re = nullptr, *ry = nullptr;
  uint8_t *cm = nullptr, *rm = nullptr;
  void* admm = nullptr;
  size_t admm_bytes = 0;
  bool carve(Arena& ar, int64_t n1, int64_t n2, int64_t n3, int64_t c, int64_t l, bool masked) {
    const int64_t nc = n1 * c * n3, nr = l * n2 * n3;
    cx = ar.take<float>(nc);
    cl = ar.take<float>(nc);
    ce = ar.take<float>(nc);
    cy = ar.take<float>(nc);
    rx = ar.take<float>(nr);
    rl = ar.take<float>(nr);
    re = ar.take<float>(nr);
    ry = ar.take<float>(nr);
    if (masked) {
      cm = ar.take<uint8_t>(nc);
      rm = ar.take<uint8_t>(nr);
    }
    admm_bytes = std::max(admm_workspace(n1, c, n3), admm_workspace(l, n2, n3));
    admm = ar.take<char>(admm_bytes);
    return ar.dry() || ar.ok();
  }
};

// Orthogonal projection of every Fourier slice of X onto the range of the
// matching slice of C (Algorithm 3): Q_k = an orthonormal basis of the
// columns of Chat_k, then Zhat_k = Q_k (Q_k^H Xhat_k). Xh: K x n1 x n2, Ch:
// K x n1 x c.
//  * c <= 64: CholeskyQR applied twice. A column whose Cholesky pivot falls
//    to kProjPivot of the largest is dropped (zero column), so repeated or
//    dependent slices project onto the numerical range: the Gram matrix is
//    float64 in both cases, so dependent columns leave pivots of ~1e-16 of
//    the largest, and 1e-13 drops them; with float32 columns, Q = C R^-1 is
//    formed in float32 and CholeskyQR2 restores orthogonality only up to a
//    condition number of ~1/sqrt(eps_32), so columns below ~3e-4 of the
//    largest singular value (pivot 1e-7) are dropped. (The range finder
//    keeps its own, smaller thresholds: a spurious direction in a sketch
//    basis is harmless, in a projector it is not.)
//  * c > 64 (float32, c <= n1): the block one-sided Jacobi of the
//    thresholding on the rows of Chat_k^H (c rows of length n1) makes them
//    sigma_i u_i^H, u_i the left singular vectors of Chat_k, without
//    squaring the condition number; Q_k = [u_i] for sigma_i above the
//    rounding residue of the rotations, max(n1, c) eps_32 of the largest,
//    and zero columns for the others (directions closer to the residue are
//    not resolved in float32 and would make the projector arbitrary there).
constexpr double kProjPivot64 = 1e-13, kProjPivot32 = 1e-7;
constexpr int64_t kProjJacobiMax = 4096;

// Widths of C the projection handles: any up to 64; beyond, float32 data
// with c <= n1 (more columns than rows span every slice they reach) and
// c <= 4096 (the column selection keeps its norms in LDS).
int check_proj_width(int64_t c, int64_t n1, int dtype) {
  if (c <= kMaxS) return TP_OK;
  if (dtype != TP_F32) return fail(TP_EUNSUPPORTED, "more than 64 lateral slices need float32 data");
  if (c > n1) return fail(TP_EUNSUPPORTED, "more than 64 lateral slices need c <= n1");
  if (c > kProjJacobiMax) return fail(TP_EUNSUPPORTED, "more than 4096 lateral slices");
  return TP_OK;
}
struct ProjLayout {
  RangeFinder rf;  // orthonormalisation workspace (m = n1, n = s = c), c <= 64
  bool wide = false;
  float *xre = nullptr, *xim = nullptr, *qre = nullptr, *qim = nullptr, *ure = nullptr, *uim = nullptr;
  float* ratio = nullptr;
  int* conv = nullptr;
  Spec G, Zh;
  bool carve(Arena& ar, int64_t K, int64_t n1, int64_t n2, int64_t c, int dt, bool real_last) {
    wide = c > kMaxS;
    if (!wide) {
      rf = RangeFinder{K, n1, c, (int)c, dt, real_last};
      rf.carve(ar);
    } else {
      rf = RangeFinder{K, n1, c, 0, dt, real_last};
      xre = ar.take<float>(K * c * n1);
      xim = ar.take<float>(K * c * n1);
      qre = ar.take<float>(K * c * c);
      qim = ar.take<float>(K * c * c);
      ure = ar.take<float>(K * n1 * c);
      uim = ar.take<float>(K * n1 * c);
      ratio = ar.take<float>(svt_ratio_count(K, c));
      conv = ar.take<int>(K);
    }
    G = take(ar, K * c * n2, dt);
    Zh = take(ar, K * n1 * n2, dt);
    return ar.dry() || ar.ok();
  }
  int run(const Spec& Xh, const Spec& Ch, int64_t n1, int64_t n2, int64_t n3, int64_t c, int prec, void* Z,
          hipStream_t st) {
    const int64_t K = rf.K;
    const int dt = rf.dtype;
    Spec Q;
    if (!wide) {
      const double piv = dt == TP_F64 ? kProjPivot64 : kProjPivot32;
      if (int rc = rf.orth(Ch, n1, rf.Q, prec, st, piv)) return rc;
      if (int rc = rf.orth(rf.Q, n1, rf.Y, prec, st, piv)) return rc;
      Q = rf.Y;
    } else {
      if (int rc = spec_conj_transpose((const float*)Ch.re, (const float*)Ch.im, K, n1, c, xre, xim, st)) return rc;
      if (int rc = svt_identity(qre, qim, K, c, st)) return rc;
      if (int rc = svt_jacobi(xre, xim, qre, qim, K, c, n1, rf.real_last, kProjSweeps, kProjTol, ratio, conv, st))
        return rc;
      const double cut = double(std::max(n1, c)) * 1.1920928955078125e-07;
      if (int rc = tsvd_pick(xre, xim, n1, xre, xim, n1, K, c, c, rf.real_last, 2, false, cut, ure, uim, nullptr, st))
        return rc;
      Q.re = ure;
      Q.im = uim;
    }
    if (int rc = mm(Q, 1, n1, c, Xh, 0, n1, n2, G, K, rf.real_last, dt, prec, st)) return rc;
    if (int rc = mm(Q, 0, n1, c, G, 0, c, n2, Zh, K, rf.real_last, dt, prec, st)) return rc;
    return fft_inverse(Zh.re, Zh.im, dt, n3, n1, n2, Z, st);
  }
  static constexpr int kProjSweeps = 30;
  static constexpr double kProjTol = 1e-6;
};

}  // namespace
}  // namespace tp

using namespace tp;

extern "C" {

size_t tp_tsvd_rand_workspace(const tp_tensor* A, int64_t r, int64_t p, const tp_sample* slices, int prec) {
  (void)prec;
  if (!A || A->n1 < 1 || A->n2 < 1 || A->n3 < 1 || r < 1) return 0;
  const int64_t K = half_count(A->n3);
  const int s = tsvd_sketch(A, r, p, slices);
  if (s < 1 || s > kMaxS) return 0;
  Arena dry(nullptr, SIZE_MAX);
  TsvdLayout lay;
  lay.carve(dry, K, A->n1, A->n2, s, r, A->dtype, (A->n3 % 2 == 0) && K > 1);
  return dry.used + 256;
}

int tp_tsvd_rand(const tp_tensor* A, int64_t r, int64_t p, int32_t q, const tp_sample* slices, uint64_t seed,
                 int prec, double* S_out, tp_tensor* U, tp_tensor* V, tp_tensor* Z, double* lev_lateral,
                 double* lev_horizontal, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_tensor(A, "A")) return rc;
  if (int rc = check_prec(A->dtype, prec)) return rc;
  const int64_t n1 = A->n1, n2 = A->n2, n3 = A->n3, K = half_count(n3);
  if (r < 1 || r > std::min(n1, n2)) return fail(TP_EINVAL, "need 1 <= r <= min(n1, n2)");
  if (p < 0 || q < 0) return fail(TP_EINVAL, "oversampling and power iterations must be >= 0");
  if (slices) {
    if (!slices->idx || !slices->scale || !slices->count) return fail(TP_EINVAL, "slices: null idx/scale/count");
    if (slices->cap < r || slices->cap > n2) return fail(TP_EINVAL, "slices: need r <= capacity <= n2");
  }
  const int s = tsvd_sketch(A, r, p, slices);
  if (s > kMaxS) return fail(TP_EUNSUPPORTED, slices ? "more than 64 picked slices" : "r + p above 64");
  struct Out {
    tp_tensor* t;
    int64_t a, b;
    const char* name;
  } outs[3] = {{U, n1, r, "U must be n1 x r x n3"}, {V, n2, r, "V must be n2 x r x n3"}, {Z, n1, n2, "Z must match A"}};
  for (const Out& o : outs)
    if (o.t && (o.t->dtype != A->dtype || o.t->n1 != o.a || o.t->n2 != o.b || o.t->n3 != n3 || !o.t->data))
      return fail(TP_ESHAPE, o.name);
  const size_t need = tp_tsvd_rand_workspace(A, r, p, slices, prec);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "tsvd_rand workspace too small");
  const bool real_last = (n3 % 2 == 0) && K > 1;
  const int dt = A->dtype;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  TsvdLayout lay;
  if (!lay.carve(ar, K, n1, n2, s, r, dt, real_last)) return fail(TP_EWORKSPACE, "tsvd_rand workspace too small");
  Spec &Ah = lay.Ah, &Ub = lay.Ub, &Vs = lay.Vs, &Us = lay.Us;
  RangeFinder& rf = lay.rf;

  TubeGather g;
  g.rows = n1;
  g.cols = n2;
  g.in_cols = n2;
  if (int rc = fft_forward(A->data, dt, n3, g, Ah.re, Ah.im, st)) return rc;
  if (slices) {
    // the basis of the picked lateral slices (t-CX, Definition t-CX and
    // Algorithm 4): Y_k = Chat_k = Ahat_k S D, transformed from the
    // picked tubes (zero columns past the live count)
    TubeGather gc;
    gc.rows = n1;
    gc.cols = s;
    gc.in_cols = n2;
    gc.col_idx = slices->idx;
    gc.col_scale = slices->scale;
    gc.count = slices->count;
    if (int rc = fft_forward(A->data, dt, n3, gc, rf.Y.re, rf.Y.im, st)) return rc;
    if (int rc = rf.finish(Ah, q, prec, st)) return rc;
  } else if (int rc = rf.run(Ah, q, seed, kStreamOmegaA, prec, st)) {
    return rc;
  }
  const double rtol = dt == TP_F64 ? 1e-12 : 1e-6;
  if (S_out)
    if (int rc = singular_values(rf.evals, K, s, (int)r, S_out, st)) return rc;
  // U_B restricted to the leading r eigenvectors
  if (int rc = eig_transform(rf.ure, rf.uim, rf.evals, K, s, (int)r, 1, rtol, 0.0, Ub.re, Ub.im, dt, st)) return rc;
  if (lev_lateral || Z) {
    // V Sigma = Bh U_B: the right singular vectors up to their scales
    if (int rc = mm(rf.Bh, 0, n2, s, Ub, 0, s, r, Vs, K, real_last, dt, prec, st)) return rc;
  }
  if (lev_lateral)
    if (int rc = leverage(Vs.re, Vs.im, dt, K, n2, r, n2 * r, (int)r, real_last, rf.evals, s, rtol, lay.lpart,
                          lev_lateral, st))
      return rc;
  if (lev_horizontal || U || Z) {
    // left singular vectors U = Q U_B
    if (int rc = mm(rf.Q, 0, n1, s, Ub, 0, s, r, Us, K, real_last, dt, prec, st)) return rc;
  }
  if (lev_horizontal)
    if (int rc = leverage(Us.re, Us.im, dt, K, n1, r, n1 * r, (int)r, real_last, nullptr, s, rtol, lay.lpart,
                          lev_horizontal, st))
      return rc;
  if (U)
    if (int rc = fft_inverse(Us.re, Us.im, dt, n3, n1, r, U->data, st)) return rc;
  if (V) {
    // V = Bh U_B diag(1 / sigma)
    if (int rc = eig_transform(rf.ure, rf.uim, rf.evals, K, s, (int)r, 1, rtol, 1.0, lay.Ubs.re, lay.Ubs.im, dt, st))
      return rc;
    if (int rc = mm(rf.Bh, 0, n2, s, lay.Ubs, 0, s, r, lay.Vsc, K, real_last, dt, prec, st)) return rc;
    if (int rc = fft_inverse(lay.Vsc.re, lay.Vsc.im, dt, n3, n2, r, V->data, st)) return rc;
  }
  if (Z) {
    // A_r: Zhat_k = U_k (V_k Sigma_k)^H, into the buffer of A's spectrum
    if (int rc = mm(Us, 0, n1, r, Vs, 1, n2, r, Ah, K, real_last, dt, prec, st)) return rc;
    if (int rc = fft_inverse(Ah.re, Ah.im, dt, n3, n1, n2, Z->data, st)) return rc;
  }
  return TP_OK;
}

size_t tp_tcur_workspace(const tp_tensor* A, int64_t c, int64_t l, int64_t r, int col_kind, int col_mode,
                         int row_kind, int row_mode, int prec) {
  (void)prec;
  if (!A || A->n1 < 1 || A->n2 < 1 || A->n3 < 1 || r < 1 || c < 1 || l < 1) return 0;
  const int64_t K = half_count(A->n3);
  const int64_t capc = col_mode == TP_S_BERNOULLI ? A->n2 : c;
  const int64_t capl = row_mode == TP_S_BERNOULLI ? A->n1 : l;
  Arena dry(nullptr, SIZE_MAX);
  TcurLayout lay;
  lay.carve(dry, K, A->n1, A->n2, A->n3, capc, capl, r, col_kind, row_kind, true, A->dtype,
            (A->n3 % 2 == 0) && K > 1);
  return dry.used + 256;
}

int tp_tcur(const tp_tensor* A, int64_t c, int64_t l, int64_t r, int col_kind, const double* col_w, int col_mode,
            int row_kind, const double* row_w, int row_mode, const tp_mlp* mlp, uint64_t seed, tp_sample* cols,
            tp_sample* rows, tp_spectrum* core, tp_tensor* Z, int prec, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_tensor(A, "A")) return rc;
  if (int rc = check_prec(A->dtype, prec)) return rc;
  const int64_t n1 = A->n1, n2 = A->n2, n3 = A->n3, K = half_count(n3);
  if (c < 1 || c > n2) return fail(TP_EINVAL, "need 1 <= c <= n2");
  if (l < 1 || l > n1) return fail(TP_EINVAL, "need 1 <= l <= n1");
  if (r < 1 || r > std::min(c, l)) return fail(TP_EINVAL, "need 1 <= r <= min(c, l)");
  if (int rc = check_pick_rule(col_kind, col_mode, true)) return rc;
  if (int rc = check_pick_rule(row_kind, row_mode, false)) return rc;
  if (col_kind == TP_P_USER && !col_w) return fail(TP_EINVAL, "column weights are null");
  if (row_kind == TP_P_USER && !row_w) return fail(TP_EINVAL, "row weights are null");
  if (col_kind == TP_P_LEARNED && (!mlp || !mlp->params || !mlp->phi))
    return fail(TP_EINVAL, "TP_P_LEARNED needs the network parameters and Phi");
  if (col_kind == TP_P_LEARNED && (A->dtype != TP_F32 || n3 % 4 != 0))
    return fail(TP_EUNSUPPORTED, "the learned proposal needs float32 data with n3 divisible by 4");
  if (!cols || !rows || !cols->idx || !cols->scale || !cols->count || !rows->idx || !rows->scale || !rows->count)
    return fail(TP_EINVAL, "pick buffers are null");
  const int64_t capc = col_mode == TP_S_BERNOULLI ? n2 : c;
  const int64_t capl = row_mode == TP_S_BERNOULLI ? n1 : l;
  if (cols->cap < capc || rows->cap < capl)
    return fail(TP_EINVAL, "pick capacity must be >= c, l (or n2, n1 for Bernoulli picks)");
  if (Z) {
    if (Z->dtype != A->dtype || Z->n1 != n1 || Z->n2 != n2 || Z->n3 != n3 || !Z->data)
      return fail(TP_ESHAPE, "Z must match A");
  }
  if (core) {
    if (core->dtype != TP_F64 || core->K != K || core->rows != capc || core->cols != capl || !core->re || !core->im)
      return fail(TP_ESHAPE, "core must be a float64 spectrum of K x c x l (n2, n1 for Bernoulli picks)");
  }
  if (sketch_size(r, kOversample, n1, n2) > kMaxS) return fail(TP_EUNSUPPORTED, "r + 10 above 64");
  const size_t need = tp_tcur_workspace(A, c, l, r, col_kind, col_mode, row_kind, row_mode, prec);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "tcur workspace too small");

  const int dt = A->dtype;
  const bool real_last = (n3 % 2 == 0) && K > 1;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  TcurLayout lay;
  if (!lay.carve(ar, K, n1, n2, n3, capc, capl, r, col_kind, row_kind, Z != nullptr || core != nullptr, dt,
                 real_last))
    return fail(TP_EWORKSPACE, "tcur workspace too small");
  const double rtol = dt == TP_F64 ? 1e-12 : 1e-6;

  // 1. column probabilities and picks (Algorithm 5 takes C as an input; it is
  //    drawn here as in Algorithm 4, by lateral leverage, norms, the learned
  //    proposal, uniformly or from caller weights)
  const double* wcol = col_w;
  if (col_kind == TP_P_LEV) {
    if (int rc = col_leverage(lay, A->data, dt, n1, n2, n3, K, r, seed, prec, real_last, rtol, st)) return rc;
    wcol = lay.wbuf;
  } else if (col_kind == TP_P_NORM2) {
    if (int rc = lateral_norms(A->data, dt, n1, n2, n3, lay.wbuf, lay.part, st)) return rc;
    wcol = lay.wbuf;
  } else if (col_kind == TP_P_LEARNED) {
    if (int rc = tp_mlp_proposal(mlp->params, A, mlp->phi, mlp->alpha, lay.wbuf, lay.mlpws, lay.mlp_bytes, stream))
      return rc;
    wcol = lay.wbuf;
  } else if (col_kind == TP_P_UNIFORM) {
    if (int rc = fill_f64(lay.wbuf, n2, 1.0, st)) return rc;
    wcol = lay.wbuf;
  }
  if (int rc = sample_slices(wcol, n2, c, col_mode, seed, kStreamColPick, cols->idx, cols->scale, cols->count,
                             lay.sws, st))
    return rc;

  // 2. Chat_k = Ahat_k S D: the picked lateral slices, scaled, transformed once
  {
    TubeGather g;
    g.rows = n1;
    g.cols = capc;
    g.in_cols = n2;
    g.col_idx = cols->idx;
    g.col_scale = cols->scale;
    g.count = cols->count;
    if (int rc = fft_forward(A->data, dt, n3, g, lay.Ch.re, lay.Ch.im, st)) return rc;
  }

  // 3. row probabilities (horizontal leverage of C, read with the squared
  //    Frobenius norm) and picks
  const double* wrow = row_w;
  if (row_kind == TP_P_LEV) {
    if (int rc = row_leverage(lay, dt, n1, K, r, seed, prec, real_last, rtol, cols->count, st)) return rc;
    wrow = lay.wbuf2;
  } else if (row_kind == TP_P_NORM2) {
    if (int rc = horizontal_norms(A->data, dt, n1, n2, n3, lay.wbuf2, st)) return rc;
    wrow = lay.wbuf2;
  } else if (row_kind == TP_P_UNIFORM) {
    if (int rc = fill_f64(lay.wbuf2, n1, 1.0, st)) return rc;
    wrow = lay.wbuf2;
  }
  if (int rc = sample_slices(wrow, n1, l, row_mode, seed, kStreamRowPick, rows->idx, rows->scale, rows->count,
                             lay.sws, st))
    return rc;
  if (!Z && !core) return TP_OK;

  // 4. Rhat_k = D S^T Ahat_k
  {
    TubeGather g;
    g.rows = capl;
    g.cols = n2;
    g.in_cols = n2;
    g.row_idx = rows->idx;
    g.row_scale = rows->scale;
    g.count = rows->count;
    if (int rc = fft_forward(A->data, dt, n3, g, lay.Rh.re, lay.Rh.im, st)) return rc;
  }

  // 5-6. core Uhat_k = pinv_r(D S^T Chat_k) and Z = ifft(Chat_k Uhat_k Rhat_k)
  return cur_core(lay, n1, n2, n3, K, capc, capl, r, rows->idx, rows->scale, rows->count, seed, dt, prec, real_last,
                  Z ? Z->data : nullptr, core, st);
}

size_t tp_tcur_nn_workspace(const tp_tensor* X, int64_t c, int64_t l, int64_t r, int col_kind, int row_kind,
                            int masked) {
  if (!X || X->n1 < 1 || X->n2 < 1 || X->n3 < 1 || r < 1 || c < 1 || l < 1) return 0;
  const int64_t K = half_count(X->n3);
  Arena dry(nullptr, SIZE_MAX);
  TcurLayout lay;
  lay.carve(dry, K, X->n1, X->n2, X->n3, c, l, r, col_kind, row_kind, true, TP_F32, (X->n3 % 2 == 0) && K > 1);
  CurNNLayout nn;
  nn.carve(dry, X->n1, X->n2, X->n3, c, l, masked != 0);
  return dry.used + 256;
}

int tp_tcur_nn(const tp_tensor* X, const uint8_t* mask, double lambda, int64_t c, int64_t l, int64_t r, int col_kind,
               const double* col_w, int col_mode, int row_kind, const double* row_w, int row_mode, uint64_t seed,
               int32_t iters, double rho, double mu0, double mu_max, tp_sample* cols, tp_sample* rows, tp_tensor* L,
               int prec, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_tensor(X, "X")) return rc;
  if (int rc = check_tensor(L, "L")) return rc;
  if (X->dtype != TP_F32 || L->dtype != TP_F32) return fail(TP_EDTYPE, "CUR t-NN runs on float32 data");
  if (prec != TP_PREC_F32) return fail(TP_EDTYPE, "CUR t-NN supports TP_PREC_F32");
  const int64_t n1 = X->n1, n2 = X->n2, n3 = X->n3, K = half_count(n3);
  if (L->n1 != n1 || L->n2 != n2 || L->n3 != n3) return fail(TP_ESHAPE, "L must match X");
  if (c < 1 || c > n2) return fail(TP_EINVAL, "need 1 <= c <= n2");
  if (l < 1 || l > n1) return fail(TP_EINVAL, "need 1 <= l <= n1");
  if (r < 1 || r > std::min(c, l)) return fail(TP_EINVAL, "need 1 <= r <= min(c, l)");
  if ((col_mode != TP_S_IID && col_mode != TP_S_UNIFORM) || (row_mode != TP_S_IID && row_mode != TP_S_UNIFORM))
    return fail(TP_EINVAL, "CUR t-NN needs exactly c and l picks (TP_S_IID or TP_S_UNIFORM)");
  if (col_kind == TP_P_LEARNED) return fail(TP_EINVAL, "CUR t-NN takes learned weights as TP_P_USER");
  if (int rc = check_pick_rule(col_kind, col_mode, false)) return rc;
  if (int rc = check_pick_rule(row_kind, row_mode, false)) return rc;
  if (col_kind == TP_P_USER && !col_w) return fail(TP_EINVAL, "column weights are null");
  if (row_kind == TP_P_USER && !row_w) return fail(TP_EINVAL, "row weights are null");
  if (!mask && lambda == 0.0) lambda = rpca_default_lambda(X->n1, X->n2, X->n3);
  if (!mask && (!(lambda > 0.0) || !std::isfinite(lambda)))
    return fail(TP_EINVAL, "lambda must be finite and >= 0 (0 selects the default)");
  if (iters < 1) return fail(TP_EINVAL, "need at least one iteration");
  if (!(rho >= 1.0) || !(mu0 > 0.0) || !(mu_max >= mu0) || !std::isfinite(rho) || !std::isfinite(mu_max))
    return fail(TP_EINVAL, "need rho >= 1 and 0 < mu0 <= mu_max");
  if (!cols || !rows || !cols->idx || !cols->scale || !cols->count || !rows->idx || !rows->scale || !rows->count)
    return fail(TP_EINVAL, "pick buffers are null");
  if (cols->cap < c || rows->cap < l) return fail(TP_EINVAL, "pick capacity must be >= c, l");
  if (sketch_size(r, kOversample, n1, n2) > kMaxS) return fail(TP_EUNSUPPORTED, "r + 10 above 64");
  const size_t need = tp_tcur_nn_workspace(X, c, l, r, col_kind, row_kind, mask != nullptr);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "CUR t-NN workspace too small");

  const int dt = TP_F32;
  const bool real_last = (n3 % 2 == 0) && K > 1;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  TcurLayout lay;
  CurNNLayout nn;
  if (!lay.carve(ar, K, n1, n2, n3, c, l, r, col_kind, row_kind, true, dt, real_last) ||
      !nn.carve(ar, n1, n2, n3, c, l, mask != nullptr))
    return fail(TP_EWORKSPACE, "CUR t-NN workspace too small");
  const double rtol = 1e-6;

  // 1. lateral slices C of X by col_kind (eq. cur-col-prob for TP_P_LEV),
  //    taken without rescaling
  const double* wcol = col_w;
  if (col_kind == TP_P_LEV) {
    if (int rc = col_leverage(lay, X->data, dt, n1, n2, n3, K, r, seed, prec, real_last, rtol, st)) return rc;
    wcol = lay.wbuf;
  } else if (col_kind == TP_P_NORM2) {
    if (int rc = lateral_norms(X->data, dt, n1, n2, n3, lay.wbuf, lay.part, st)) return rc;
    wcol = lay.wbuf;
  } else if (col_kind == TP_P_UNIFORM) {
    if (int rc = fill_f64(lay.wbuf, n2, 1.0, st)) return rc;
    wcol = lay.wbuf;
  }
  if (int rc = sample_slices(wcol, n2, c, col_mode, seed, kStreamColPick, cols->idx, cols->scale, cols->count,
                             lay.sws, st))
    return rc;
  if (int rc = gather_slices(X->data, 4, n2, n3, nullptr, cols->idx, cols->count, n1, c, nn.cx, st)) return rc;
  if (mask)
    if (int rc = gather_slices(mask, 1, n2, n3, nullptr, cols->idx, cols->count, n1, c, nn.cm, st)) return rc;

  // 2. Ct = ADMM(C), and its spectrum
  if (int rc = admm_run(nn.cx, nn.cm, lambda, n1, c, n3, iters, rho, mu0, mu_max, 0.0, nn.cl, nn.ce, nn.cy, nullptr,
                        nullptr, nn.admm, nn.admm_bytes, st))
    return rc;
  {
    TubeGather g;
    g.rows = n1;
    g.cols = c;
    g.in_cols = c;
    if (int rc = fft_forward(nn.cl, dt, n3, g, lay.Ch.re, lay.Ch.im, st)) return rc;
  }

  // 3. horizontal slices R of X by row_kind (eq. colprob_rows_exact, the
  //    horizontal leverage of the cleaned Ct, for TP_P_LEV)
  const double* wrow = row_w;
  if (row_kind == TP_P_LEV) {
    if (int rc = row_leverage(lay, dt, n1, K, r, seed, prec, real_last, rtol, nullptr, st)) return rc;
    wrow = lay.wbuf2;
  } else if (row_kind == TP_P_NORM2) {
    if (int rc = horizontal_norms(X->data, dt, n1, n2, n3, lay.wbuf2, st)) return rc;
    wrow = lay.wbuf2;
  } else if (row_kind == TP_P_UNIFORM) {
    if (int rc = fill_f64(lay.wbuf2, n1, 1.0, st)) return rc;
    wrow = lay.wbuf2;
  }
  if (int rc = sample_slices(wrow, n1, l, row_mode, seed, kStreamRowPick, rows->idx, rows->scale, rows->count, lay.sws,
                             st))
    return rc;
  if (int rc = gather_slices(X->data, 4, n2, n3, rows->idx, nullptr, rows->count, l, n2, nn.rx, st)) return rc;
  if (mask)
    if (int rc = gather_slices(mask, 1, n2, n3, rows->idx, nullptr, rows->count, l, n2, nn.rm, st)) return rc;

  // 4. Rt = ADMM(R), and its spectrum
  if (int rc = admm_run(nn.rx, nn.rm, lambda, l, n2, n3, iters, rho, mu0, mu_max, 0.0, nn.rl, nn.re, nn.ry, nullptr,
                        nullptr, nn.admm, nn.admm_bytes, st))
    return rc;
  {
    TubeGather g;
    g.rows = l;
    g.cols = n2;
    g.in_cols = n2;
    if (int rc = fft_forward(nn.rl, dt, n3, g, lay.Rh.re, lay.Rh.im, st)) return rc;
  }

  // 5. W = the picked rows of Ct (unscaled), U = pinv_r(W), L = Ct * U * Rt
  return cur_core(lay, n1, n2, n3, K, c, l, r, rows->idx, nullptr, rows->count, seed, dt, prec, real_last, L->data,
                  nullptr, st);
}

size_t tp_tproject_workspace(const tp_tensor* X, const tp_tensor* C, int prec) {
  (void)prec;
  if (!X || !C || X->n1 < 1 || X->n2 < 1 || X->n3 < 1 || C->n2 < 1) return 0;
  const int64_t K = half_count(X->n3);
  const bool real_last = (X->n3 % 2 == 0) && K > 1;
  Arena dry(nullptr, SIZE_MAX);
  Spec Xh = take(dry, K * X->n1 * X->n2, X->dtype), Ch = take(dry, K * X->n1 * C->n2, X->dtype);
  (void)Xh;
  (void)Ch;
  ProjLayout lay;
  lay.carve(dry, K, X->n1, X->n2, C->n2, X->dtype, real_last);
  return dry.used + 256;
}

int tp_tproject(const tp_tensor* X, const tp_tensor* C, tp_tensor* Z, int prec, void* ws, size_t ws_bytes,
                void* stream) {
  if (int rc = check_tensor(X, "X")) return rc;
  if (int rc = check_tensor(C, "C")) return rc;
  if (int rc = check_tensor(Z, "Z")) return rc;
  if (int rc = check_prec(X->dtype, prec)) return rc;
  if (C->dtype != X->dtype || Z->dtype != X->dtype) return fail(TP_EDTYPE, "X, C and Z must share a dtype");
  if (C->n1 != X->n1 || C->n3 != X->n3) return fail(TP_ESHAPE, "C must be n1 x c x n3 like X");
  if (Z->n1 != X->n1 || Z->n2 != X->n2 || Z->n3 != X->n3) return fail(TP_ESHAPE, "Z must match X");
  if (int rc = check_proj_width(C->n2, X->n1, X->dtype)) return rc;
  const size_t need = tp_tproject_workspace(X, C, prec);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "tproject workspace too small");
  const int64_t n1 = X->n1, n2 = X->n2, n3 = X->n3, c = C->n2, K = half_count(n3);
  const bool real_last = (n3 % 2 == 0) && K > 1;
  const int dt = X->dtype;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  Spec Xh = take(ar, K * n1 * n2, dt), Ch = take(ar, K * n1 * c, dt);
  ProjLayout lay;
  if (!lay.carve(ar, K, n1, n2, c, dt, real_last)) return fail(TP_EWORKSPACE, "tproject workspace too small");
  TubeGather gx;
  gx.rows = n1;
  gx.cols = n2;
  gx.in_cols = n2;
  if (int rc = fft_forward(X->data, dt, n3, gx, Xh.re, Xh.im, st)) return rc;
  TubeGather gc;
  gc.rows = n1;
  gc.cols = c;
  gc.in_cols = c;
  if (int rc = fft_forward(C->data, dt, n3, gc, Ch.re, Ch.im, st)) return rc;
  return lay.run(Xh, Ch, n1, n2, n3, c, prec, Z->data, st);
}

size_t tp_tcx_workspace(const tp_tensor* A, int64_t c, int32_t rounds, int64_t r, int col_kind, int prec) {
  (void)prec;
  if (!A || A->n1 < 1 || A->n2 < 1 || A->n3 < 1 || c < 1 || rounds < 1) return 0;
  if (r < 1) r = 1;
  const int64_t K = half_count(A->n3), cT = c * rounds;
  const bool real_last = (A->n3 % 2 == 0) && K > 1;
  Arena dry(nullptr, SIZE_MAX);
  TcurLayout cur;
  cur.carve(dry, K, A->n1, A->n2, A->n3, cT, 1, r, col_kind, TP_P_UNIFORM, false, A->dtype, real_last);
  if (col_kind != TP_P_LEV) (void)take(dry, K * A->n1 * A->n2, A->dtype);
  (void)dry.take<int64_t>(rounds);
  ProjLayout lay;
  lay.carve(dry, K, A->n1, A->n2, cT, A->dtype, real_last);
  return dry.used + 256;
}

int tp_tcx(const tp_tensor* A, int64_t c, int32_t rounds, int64_t r, int col_kind, const double* col_w, int mode,
           uint64_t seed, tp_sample* cols, tp_tensor* Z, int prec, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_tensor(A, "A")) return rc;
  if (int rc = check_tensor(Z, "Z")) return rc;
  if (int rc = check_prec(A->dtype, prec)) return rc;
  const int64_t n1 = A->n1, n2 = A->n2, n3 = A->n3, K = half_count(n3);
  if (Z->dtype != A->dtype || Z->n1 != n1 || Z->n2 != n2 || Z->n3 != n3) return fail(TP_ESHAPE, "Z must match A");
  if (c < 1 || c > n2) return fail(TP_EINVAL, "need 1 <= c <= n2");
  if (rounds < 1) return fail(TP_EINVAL, "need at least one round");
  if (int rc = check_proj_width(c * (int64_t)rounds, n1, A->dtype)) return rc;
  if (mode != TP_S_IID && mode != TP_S_UNIFORM)
    return fail(TP_EINVAL, "t-CX rounds need exactly c picks (TP_S_IID or TP_S_UNIFORM)");
  if (int rc = check_pick_rule(col_kind, mode, false)) return rc;
  if (col_kind == TP_P_USER && !col_w) return fail(TP_EINVAL, "column weights are null");
  if (col_kind == TP_P_LEV && (r < 1 || r > std::min(n1, n2) || sketch_size(r, kOversample, n1, n2) > kMaxS))
    return fail(TP_EINVAL, "leverage needs 1 <= r <= min(n1, n2) and r + 10 <= 64");
  if (!cols || !cols->idx || !cols->scale || !cols->count) return fail(TP_EINVAL, "pick buffers are null");
  const int64_t cT = c * rounds;
  if (cols->cap < cT) return fail(TP_EINVAL, "pick capacity must be >= c * rounds");
  const int64_t rr = r < 1 ? 1 : r;
  const size_t need = tp_tcx_workspace(A, c, rounds, rr, col_kind, prec);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "tcx workspace too small");

  const int dt = A->dtype;
  const bool real_last = (n3 % 2 == 0) && K > 1;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  TcurLayout cur;
  if (!cur.carve(ar, K, n1, n2, n3, cT, 1, rr, col_kind, TP_P_UNIFORM, false, dt, real_last))
    return fail(TP_EWORKSPACE, "tcx workspace too small");
  Spec Ah = cur.Ah;
  if (col_kind != TP_P_LEV) Ah = take(ar, K * n1 * n2, dt);
  int64_t* counts = ar.take<int64_t>(rounds);
  ProjLayout lay;
  if (!lay.carve(ar, K, n1, n2, cT, dt, real_last)) return fail(TP_EWORKSPACE, "tcx workspace too small");
  const double rtol = dt == TP_F64 ? 1e-12 : 1e-6;

  // 1. probabilities (the leverage path transforms A into Ah on the way)
  const double* wcol = col_w;
  if (col_kind == TP_P_LEV) {
    if (int rc = col_leverage(cur, A->data, dt, n1, n2, n3, K, rr, seed, prec, real_last, rtol, st)) return rc;
    wcol = cur.wbuf;
  } else {
    TubeGather g;
    g.rows = n1;
    g.cols = n2;
    g.in_cols = n2;
    if (int rc = fft_forward(A->data, dt, n3, g, Ah.re, Ah.im, st)) return rc;
    if (col_kind == TP_P_NORM2) {
      if (int rc = lateral_norms(A->data, dt, n1, n2, n3, cur.wbuf, cur.part, st)) return rc;
      wcol = cur.wbuf;
    } else if (col_kind == TP_P_UNIFORM) {
      if (int rc = fill_f64(cur.wbuf, n2, 1.0, st)) return rc;
      wcol = cur.wbuf;
    }
  }
  // 2. independent rounds of c picks (round i draws from stream 16 i of the
  //    seed), kept side by side: the union of all rounds
  for (int32_t i = 0; i < rounds; ++i) {
    if (int rc = sample_slices(wcol, n2, c, mode, seed, kStreamColPick + 16 * (uint64_t)i, cols->idx + i * c,
                               cols->scale + i * c, counts + i, cur.sws, st))
      return rc;
  }
  if (int rc = join_counts(counts, rounds, cols->count, st)) return rc;
  // 3. Chat = the picked lateral slices (unscaled: the projector onto their
  //    span does not depend on the scales), then Z = C * C^+ * A
  {
    TubeGather g;
    g.rows = n1;
    g.cols = cT;
    g.in_cols = n2;
    g.col_idx = cols->idx;
    g.count = cols->count;
    if (int rc = fft_forward(A->data, dt, n3, g, cur.Ch.re, cur.Ch.im, st)) return rc;
  }
  return lay.run(Ah, cur.Ch, n1, n2, n3, cT, prec, Z->data, st);
}

}  // extern "C"
