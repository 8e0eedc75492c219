// C ABI of the per-Fourier-slice singular value thresholding (the
// tensor-nuclear-norm prox, i.e. the L-update of Algorithm 7) and of the
// ADMM loops: Algorithm 7 as stated for robust tensor PCA (eq. tlow7) and
// adapted to the completion problem of eq. tlow6. Validation, workspace
// layout and kernel order only.
#include <algorithm>
#include <cmath>
#include <string>

#include "common.hpp"
#include "svt.hpp"

namespace tp {
namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr double kSvtTol = 1e-6;   // largest |G_st| / max(G_ss, G_tt) of a converged pair
constexpr int kColdSweeps = 30;
constexpr int kWarmSweeps = 20;
// Sweep budget of the warm-started iterations of a fixed-count ADMM other
// than the last. The Jacobi state (U^H) carries over to the next
// iteration, which resumes the rotations from there, so the sweeps of one
// thresholding are spread over consecutive iterations; the last iteration
// runs to convergence, so the returned L is the exact thresholding of the
// last M. On the 256 x 256 x 100 completion workload, against the run that
// converges every iteration (10.7-12.5 ms per warm iteration), two sweeps
// per iteration take 3.8 ms and move L after 100 iterations by 2.9e-4
// (relative Frobenius), three take 5.4 ms and move it by 1.2e-4; the error
// against L* is the same to four digits either way. A looser convergence
// test for the intermediate iterations saves nothing: warm-started sweeps
// do not reach even 1e-3 within three sweeps.
constexpr int kWarmCapSweeps = 2;

struct SvtLayout {
  float *xre = nullptr, *xim = nullptr, *ure = nullptr, *uim = nullptr, *lre = nullptr, *lim = nullptr;
  float* ratio = nullptr;
  int* conv = nullptr;
  double* sig = nullptr;
  float* m = nullptr;  // ADMM only: M = X - E - Y/mu, tube-major
  // ADMM only, for the stop test: the previous L and E, per-workgroup
  // partial maxima and the three stop quantities
  float *lprev = nullptr, *eprev = nullptr, *stop_part = nullptr, *stop_out = nullptr;
  bool carve(Arena& ar, int64_t K, int64_t n1, int64_t n2, int64_t n3, bool completion) {
    xre = ar.take<float>(K * n1 * n2);
    xim = ar.take<float>(K * n1 * n2);
    ure = ar.take<float>(K * n1 * n1);
    uim = ar.take<float>(K * n1 * n1);
    lre = ar.take<float>(K * n1 * n2);
    lim = ar.take<float>(K * n1 * n2);
    ratio = ar.take<float>(svt_ratio_count(K, n1));
    conv = ar.take<int>(K);
    sig = ar.take<double>(K * n1);
    if (completion) {
      const int64_t n = n1 * n2 * n3;
      m = ar.take<float>(n);
      lprev = ar.take<float>(n);
      eprev = ar.take<float>(n);
      stop_part = ar.take<float>(admm_stop_floats(n));
      stop_out = ar.take<float>(4);
    }
    return ar.dry() || ar.ok();
  }
};

// The t-SVT of a tall tensor runs on its t-transpose (mt, lt hold the
// transposed input and result).
struct TsvtLayout {
  SvtLayout svt;
  float *mt = nullptr, *lt = nullptr;
  bool carve(Arena& ar, int64_t n1, int64_t n2, int64_t n3) {
    const int64_t K = half_count(n3);
    if (n1 > n2) {
      mt = ar.take<float>(n1 * n2 * n3);
      lt = ar.take<float>(n1 * n2 * n3);
      return svt.carve(ar, K, n2, n1, n3, false);
    }
    return svt.carve(ar, K, n1, n2, n3, false);
  }
};

// Dense leading-r t-SVD. Near-square slices (longer side at most
// kDirectRatio times the shorter) run the block Jacobi on the slices
// themselves (on A^H for a tall A, through the t-transpose); longer ones on
// the Gram matrix of the shorter side, which is cheaper but squares the
// condition number.
constexpr int64_t kDirectRatio = 4;

inline bool tsvd_direct(int64_t n1, int64_t n2) {
  return std::max(n1, n2) <= kDirectRatio * std::min(n1, n2);
}

// Buffers: the spectrum of A (of A^T on the direct tall path), the Gram
// matrix (then Q G) on the Gram path, the accumulated rotations Q, the V
// columns of the Gram tall path, the left singular planes, and A^T.
struct FullSvdLayout {
  float *are = nullptr, *aim = nullptr, *xre = nullptr, *xim = nullptr, *qre = nullptr, *qim = nullptr;
  float *vre = nullptr, *vim = nullptr, *ure = nullptr, *uim = nullptr, *mt = nullptr;
  float* ratio = nullptr;
  int* conv = nullptr;
  // partial planes of a split contraction of the Gram product
  float *part_re = nullptr, *part_im = nullptr;
  int64_t part = 0;
  bool carve(Arena& ar, int64_t n1, int64_t n2, int64_t n3, int64_t r) {
    const int64_t K = half_count(n3), m = std::min(n1, n2);
    const bool direct = tsvd_direct(n1, n2), tall = n1 > n2;
    are = ar.take<float>(K * n1 * n2);
    aim = ar.take<float>(K * n1 * n2);
    if (!direct) {
      xre = ar.take<float>(K * m * m);
      xim = ar.take<float>(K * m * m);
      part = cgemm_ksplit_floats(K, m, m, std::max(n1, n2));
      if (part) {
        part_re = ar.take<float>(part);
        part_im = ar.take<float>(part);
      }
    }
    qre = ar.take<float>(K * m * m);
    qim = ar.take<float>(K * m * m);
    if (!direct && tall) {
      vre = ar.take<float>(K * m * r);
      vim = ar.take<float>(K * m * r);
    }
    ure = ar.take<float>(K * n1 * r);
    uim = ar.take<float>(K * n1 * r);
    if (direct && tall) mt = ar.take<float>(n1 * n2 * n3);
    ratio = ar.take<float>(svt_ratio_count(K, m));
    conv = ar.take<int>(K);
    return ar.dry() || ar.ok();
  }
};

int check_f32_tensor(const tp_tensor* t, const char* name) {
  if (!t) return fail(TP_EINVAL, std::string(name) + " is null");
  if (t->dtype != TP_F32) return fail(TP_EDTYPE, std::string(name) + ": thresholding runs on float32 data");
  if (t->n1 < 1 || t->n2 < 1 || t->n3 < 1) return fail(TP_ESHAPE, std::string(name) + ": empty tensor");
  if (!t->data) return fail(TP_EINVAL, std::string(name) + ": data is null");
  return TP_OK;
}

// L = ifft(Uh^H D X) after the Jacobi sweeps have made the rows of X
// orthogonal.
int finish_svt(SvtLayout& lay, int64_t K, int64_t n1, int64_t n2, int64_t n3, double tau, bool real_last,
               int32_t* ranks, void* Lout, hipStream_t st) {
  if (int rc = svt_shrink(lay.xre, lay.xim, K, n1, n2, tau, real_last, lay.sig, ranks, st)) return rc;
  CGemm p;
  p.K = K;
  p.M = n1;
  p.N = n2;
  p.Kd = n1;
  p.are = lay.ure;
  p.aim = lay.uim;
  p.bre = lay.xre;
  p.bim = lay.xim;
  p.cre = lay.lre;
  p.cim = lay.lim;
  p.lda = n1;
  p.ldb = n2;
  p.ldc = n2;
  p.sa = n1 * n1;
  p.sb = n1 * n2;
  p.sc = n1 * n2;
  p.op_a = 1;
  p.real_last = real_last;
  if (int rc = cgemm(p, TP_F32, TP_PREC_F32, st)) return rc;
  return fft_inverse(lay.lre, lay.lim, TP_F32, n3, n1, n2, Lout, st);
}

int check_admm(const tp_tensor* X, const tp_tensor* L, const tp_tensor* E, const tp_tensor* Y, int32_t iters,
               double rho, double mu0, double mu_max, int prec) {
  if (int rc = check_f32_tensor(X, "X")) return rc;
  if (int rc = check_f32_tensor(L, "L")) return rc;
  if (int rc = check_f32_tensor(E, "E")) return rc;
  if (int rc = check_f32_tensor(Y, "Y")) return rc;
  if (prec != TP_PREC_F32) return fail(TP_EDTYPE, "the ADMM supports TP_PREC_F32");
  for (const tp_tensor* t : {L, E, Y})
    if (t->n1 != X->n1 || t->n2 != X->n2 || t->n3 != X->n3) return fail(TP_ESHAPE, "L, E, Y must match X");
  if (iters < 1) return fail(TP_EINVAL, "need at least one iteration");
  if (!(rho >= 1.0) || !(mu0 > 0.0) || !(mu_max >= mu0) || !std::isfinite(rho) || !std::isfinite(mu_max))
    return fail(TP_EINVAL, "need rho >= 1 and 0 < mu0 <= mu_max");
  return TP_OK;
}

}  // namespace

namespace {

// The loop of the ADMM on an n1 x n2 x n3 problem with the given layout.
// tol > 0: after every iteration Algorithm 7's check (the infinity norms of
// the changes of L and E and of the residual L + E - X all at most tol) is
// evaluated on the device and read back, and the loop ends at the first
// iteration that meets it; reaching `iters` iterations without it gives
// TP_ENOCONV (the iterates are still written). tol <= 0: exactly `iters`
// iterations with no host synchronisation. *iters_done (host, may be null)
// receives the number of iterations run.
int admm_loop(SvtLayout& lay, const float* x, const uint8_t* mask, double lam, int64_t n1, int64_t n2, int64_t n3,
              int iters, double rho, double mu0, double mu_max, double tol, float* l, float* e, float* y,
              int32_t* ranks, int32_t* iters_done, hipStream_t st) {
  const bool check = tol > 0.0;
  if (iters_done) *iters_done = 0;
  const int64_t K = half_count(n3), n = n1 * n2 * n3;
  const bool real_last = (n3 % 2 == 0) && K > 1;
  // L_0 = E_0 = Y_0 = 0
  if (int rc = zero_f32(e, n, st)) return rc;
  if (int rc = zero_f32(y, n, st)) return rc;
  if (int rc = zero_f32(l, n, st)) return rc;
  if (int rc = svt_identity(lay.ure, lay.uim, K, n1, st)) return rc;
  double mu = mu0;
  TubeGather g;
  g.rows = n1;
  g.cols = n2;
  g.in_cols = n2;
  for (int it = 0; it < iters; ++it) {
    const float inv_mu = (float)(1.0 / mu);
    {
      // M = X - E - Y / mu, then its spectrum
      TraceScope ts("admm.pre_fft", st);
      if (int rc = admm_pre(x, e, y, inv_mu, n, lay.m, st)) return rc;
      if (int rc = fft_forward(lay.m, TP_F32, n3, g, lay.lre, lay.lim, st)) return rc;
    }
    {
      // warm start: rotate the new spectrum by the previous iteration's U^H
      TraceScope ts("admm.rotate", st);
      CGemm p;
      p.K = K;
      p.M = n1;
      p.N = n2;
      p.Kd = n1;
      p.are = lay.ure;
      p.aim = lay.uim;
      p.bre = lay.lre;
      p.bim = lay.lim;
      p.cre = lay.xre;
      p.cim = lay.xim;
      p.lda = n1;
      p.ldb = n2;
      p.ldc = n2;
      p.sa = n1 * n1;
      p.sb = n1 * n2;
      p.sc = n1 * n2;
      p.real_last = real_last;
      if (int rc = cgemm(p, TP_F32, TP_PREC_F32, st)) return rc;
    }
    {
      TraceScope ts("admm.jacobi", st);
      // with the stop test every iteration's thresholding is exact
      const int budget = it == 0 ? kColdSweeps : (check || it == iters - 1) ? kWarmSweeps : kWarmCapSweeps;
      if (int rc = svt_jacobi(lay.xre, lay.xim, lay.ure, lay.uim, K, n1, n2, real_last, budget, kSvtTol, lay.ratio,
                              lay.conv, st))
        return rc;
    }
    if (check) {
      TP_HIP_CHECK(hipMemcpyAsync(lay.lprev, l, n * sizeof(float), hipMemcpyDeviceToDevice, st));
      TP_HIP_CHECK(hipMemcpyAsync(lay.eprev, e, n * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    {
      // L = SVT(M, 1/mu); the shrink leaves X scaled, so the next warm start
      // uses Uh only
      TraceScope ts("admm.shrink_ifft", st);
      int32_t* rk = (check || it == iters - 1) ? ranks : nullptr;
      if (int rc = finish_svt(lay, K, n1, n2, n3, 1.0 / mu, real_last, rk, l, st)) return rc;
    }
    {
      TraceScope ts("admm.post", st);
      if (mask) {
        // E = P_unobs(X - L - Y/mu), Y = Y + mu (L + E - X)
        if (int rc = admm_post(x, mask, l, (float)mu, inv_mu, n, e, y, st)) return rc;
      } else {
        // E = shrink(X - L - Y/mu, lam/mu), Y = Y + mu (L + E - X)
        if (int rc = admm_post_soft(x, l, (float)mu, inv_mu, (float)(lam / mu), n, e, y, st)) return rc;
      }
    }
    mu = std::min(rho * mu, mu_max);
    if (iters_done) *iters_done = it + 1;
    if (check) {
      float q[3] = {0.f, 0.f, 0.f};
      if (int rc = admm_stop(x, l, lay.lprev, e, lay.eprev, n, lay.stop_part, lay.stop_out, st)) return rc;
      TP_HIP_CHECK(hipMemcpyAsync(q, lay.stop_out, sizeof(q), hipMemcpyDeviceToHost, st));
      TP_HIP_CHECK(hipStreamSynchronize(st));
      if (q[0] <= tol && q[1] <= tol && q[2] <= tol) return TP_OK;
    }
  }
  return check ? fail(TP_ENOCONV, "ADMM: the iteration cap was reached before the stop test held") : TP_OK;
}

// Tall problems (n1 > n2) run on the t-transpose: the t-SVT satisfies
// SVT(M^T) = SVT(M)^T (the Fourier slices of M^T are the conjugate
// transposes of those of M), and the l1 term, the mask projection and the
// multiplier update are elementwise, so the iterates of the transposed
// problem are the transposes of the iterates; the row Jacobi then
// orthogonalises min(n1, n2) rows.
struct AdmmLayout {
  SvtLayout svt;
  float *xt = nullptr, *tmp = nullptr;
  uint8_t* mt = nullptr;
  bool carve(Arena& ar, int64_t n1, int64_t n2, int64_t n3, bool masked) {
    const int64_t K = half_count(n3);
    if (n1 > n2) {
      xt = ar.take<float>(n1 * n2 * n3);
      tmp = ar.take<float>(n1 * n2 * n3);
      if (masked) mt = ar.take<uint8_t>(n1 * n2 * n3);
      return svt.carve(ar, K, n2, n1, n3, true);
    }
    return svt.carve(ar, K, n1, n2, n3, true);
  }
};

}  // namespace

size_t admm_workspace(int64_t n1, int64_t n2, int64_t n3) {
  Arena dry(nullptr, SIZE_MAX);
  AdmmLayout lay;
  lay.carve(dry, n1, n2, n3, true);
  return dry.used + 256;
}

int admm_run(const float* x, const uint8_t* mask, double lam, int64_t n1, int64_t n2, int64_t n3, int iters,
             double rho, double mu0, double mu_max, double tol, float* l, float* e, float* y, int32_t* ranks,
             int32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t st) {
  const size_t need = admm_workspace(n1, n2, n3);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "ADMM workspace too small");
  Arena ar(ws, ws_bytes);
  AdmmLayout lay;
  if (!lay.carve(ar, n1, n2, n3, mask != nullptr)) return fail(TP_EWORKSPACE, "ADMM workspace too small");
  if (n1 <= n2)
    return admm_loop(lay.svt, x, mask, lam, n1, n2, n3, iters, rho, mu0, mu_max, tol, l, e, y, ranks, iters_done,
                     st);
  // transposed problem (n2 x n1 x n3), iterates kept in l, e, y, then turned back
  const int64_t n = n1 * n2 * n3;
  if (int rc = ttranspose(x, 4, n1, n2, n3, lay.xt, st)) return rc;
  if (mask)
    if (int rc = ttranspose(mask, 1, n1, n2, n3, lay.mt, st)) return rc;
  const int status = admm_loop(lay.svt, lay.xt, mask ? lay.mt : nullptr, lam, n2, n1, n3, iters, rho, mu0, mu_max,
                               tol, l, e, y, ranks, iters_done, st);
  if (status != TP_OK && status != TP_ENOCONV) return status;
  for (float* b : {l, e, y}) {
    if (int rc = ttranspose(b, 4, n2, n1, n3, lay.tmp, st)) return rc;
    TP_HIP_CHECK(hipMemcpyAsync(b, lay.tmp, n * sizeof(float), hipMemcpyDeviceToDevice, st));
  }
  return status;
}

}  // namespace tp

using namespace tp;

extern "C" {

size_t tp_tsvt_workspace(const tp_tensor* M) {
  if (!M || M->n1 < 1 || M->n2 < 1 || M->n3 < 1) return 0;
  Arena dry(nullptr, SIZE_MAX);
  TsvtLayout lay;
  lay.carve(dry, M->n1, M->n2, M->n3);
  return dry.used + 256;
}

int tp_tsvt(const tp_tensor* M, double tau, tp_tensor* L, int32_t* ranks, int32_t* unconverged, int prec, void* ws,
            size_t ws_bytes, void* stream) {
  if (int rc = check_f32_tensor(M, "M")) return rc;
  if (int rc = check_f32_tensor(L, "L")) return rc;
  if (prec != TP_PREC_F32) return fail(TP_EDTYPE, "thresholding supports TP_PREC_F32");
  if (L->n1 != M->n1 || L->n2 != M->n2 || L->n3 != M->n3) return fail(TP_ESHAPE, "L must match M");
  if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(TP_EINVAL, "tau must be finite and >= 0");
  const size_t need = tp_tsvt_workspace(M);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "tsvt workspace too small");
  const int64_t n1 = M->n1, n2 = M->n2, n3 = M->n3, K = half_count(n3);
  const bool real_last = (n3 % 2 == 0) && K > 1;
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  TsvtLayout lay;
  if (!lay.carve(ar, n1, n2, n3)) return fail(TP_EWORKSPACE, "tsvt workspace too small");
  // a tall problem runs on the t-transpose: SVT(M^T) = SVT(M)^T
  const bool tall = n1 > n2;
  const int64_t r = tall ? n2 : n1, c = tall ? n1 : n2;
  const float* src = (const float*)M->data;
  if (tall) {
    if (int rc = ttranspose(M->data, 4, n1, n2, n3, lay.mt, st)) return rc;
    src = lay.mt;
  }
  TubeGather g;
  g.rows = r;
  g.cols = c;
  g.in_cols = c;
  if (int rc = fft_forward(src, TP_F32, n3, g, lay.svt.xre, lay.svt.xim, st)) return rc;
  if (int rc = svt_identity(lay.svt.ure, lay.svt.uim, K, r, st)) return rc;
  if (int rc = svt_jacobi(lay.svt.xre, lay.svt.xim, lay.svt.ure, lay.svt.uim, K, r, c, real_last, kColdSweeps,
                          kSvtTol, lay.svt.ratio, lay.svt.conv, st))
    return rc;
  if (int rc = svt_count_unconverged(lay.svt.conv, K, unconverged, st)) return rc;
  if (!tall) return finish_svt(lay.svt, K, r, c, n3, tau, real_last, ranks, L->data, st);
  if (int rc = finish_svt(lay.svt, K, r, c, n3, tau, real_last, ranks, lay.lt, st)) return rc;
  return ttranspose(lay.lt, 4, r, c, n3, L->data, st);
}

size_t tp_tsvd_full_workspace(const tp_tensor* A, int64_t r) {
  if (!A || A->n1 < 1 || A->n2 < 1 || A->n3 < 1 || r < 1) return 0;
  Arena dry(nullptr, SIZE_MAX);
  FullSvdLayout lay;
  lay.carve(dry, A->n1, A->n2, A->n3, r);
  return dry.used + 256;
}

int tp_tsvd_full(const tp_tensor* A, int64_t r, tp_tensor* U, double* S_out, int32_t* unconverged, void* ws,
                 size_t ws_bytes, void* stream) {
  if (int rc = check_f32_tensor(A, "A")) return rc;
  if (int rc = check_f32_tensor(U, "U")) return rc;
  const int64_t n1 = A->n1, n2 = A->n2, n3 = A->n3, m = std::min(n1, n2);
  if (r < 1 || r > m) return fail(TP_EINVAL, "need 1 <= r <= min(n1, n2)");
  if (m > kPickMax) return fail(TP_EUNSUPPORTED, "min(n1, n2) above 4096");
  if (U->n1 != n1 || U->n2 != r || U->n3 != n3) return fail(TP_ESHAPE, "U must be n1 x r x n3");
  const size_t need = tp_tsvd_full_workspace(A, r);
  if (!ws || ws_bytes < need) return fail(TP_EWORKSPACE, "tsvd_full workspace too small");
  const int64_t K = half_count(n3);
  const bool real_last = (n3 % 2 == 0) && K > 1;
  const bool tall = n1 > n2, direct = tsvd_direct(n1, n2);
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  FullSvdLayout lay;
  if (!lay.carve(ar, n1, n2, n3, r)) return fail(TP_EWORKSPACE, "tsvd_full workspace too small");
  if (int rc = svt_identity(lay.qre, lay.qim, K, m, st)) return rc;
  // rounding residue: a row the rotations emptied keeps about
  // max(n1, n2) eps_32 sigma_max (the thresholding's cutoff); an
  // eigenvalue of the m x m float32 Gram that is zero keeps about
  // m eps_32 lambda_max. Values at or below these count as zero.
  const double eps32 = 1.1920928955078125e-07;
  const double direct_floor = double(std::max(n1, n2)) * eps32, gram_floor = double(m) * eps32;
  if (direct) {
    // the slices themselves (m rows of length n = the longer side): for a
    // tall A the slices of its t-transpose, A_k^H
    const int64_t n = std::max(n1, n2);
    TubeGather g;
    g.rows = m;
    g.cols = n;
    g.in_cols = n;
    const void* src = A->data;
    if (tall) {
      if (int rc = ttranspose(A->data, 4, n1, n2, n3, lay.mt, st)) return rc;
      src = lay.mt;
    }
    if (int rc = fft_forward(src, TP_F32, n3, g, lay.are, lay.aim, st)) return rc;
    if (int rc = svt_jacobi(lay.are, lay.aim, lay.qre, lay.qim, K, m, n, real_last, kColdSweeps, kSvtTol,
                            lay.ratio, lay.conv, st))
      return rc;
    if (int rc = svt_count_unconverged(lay.conv, K, unconverged, st)) return rc;
    // rows of X are sigma_i times conjugated singular vectors: U from Q
    // (wide, X = U^H A) or from X / sigma (tall, X = Sigma U^H)
    if (tall) {
      if (int rc = tsvd_pick(lay.are, lay.aim, n, lay.are, lay.aim, n, K, m, r, real_last, 2, false, direct_floor,
                             lay.ure, lay.uim, S_out, st))
        return rc;
    } else if (int rc = tsvd_pick(lay.are, lay.aim, n, lay.qre, lay.qim, m, K, m, r, real_last, 0, false,
                                  direct_floor, lay.ure, lay.uim, S_out, st)) {
      return rc;
    }
    return fft_inverse(lay.ure, lay.uim, TP_F32, n3, n1, r, U->data, st);
  }
  TubeGather g;
  g.rows = n1;
  g.cols = n2;
  g.in_cols = n2;
  if (int rc = fft_forward(A->data, TP_F32, n3, g, lay.are, lay.aim, st)) return rc;
  // Gram of the shorter side: A^H A (n2 x n2) for a tall slice, A A^H
  // (n1 x n1) otherwise
  CGemm p;
  p.K = K;
  p.real_last = real_last;
  p.are = lay.are;
  p.aim = lay.aim;
  p.bre = lay.are;
  p.bim = lay.aim;
  p.cre = lay.xre;
  p.cim = lay.xim;
  p.lda = n2;
  p.ldb = n2;
  p.ldc = m;
  p.sa = n1 * n2;
  p.sb = n1 * n2;
  p.sc = m * m;
  p.M = m;
  p.N = m;
  p.Kd = tall ? n1 : n2;
  p.op_a = tall ? 1 : 0;
  p.op_b = tall ? 0 : 1;
  p.part_re = lay.part_re;
  p.part_im = lay.part_im;
  p.part_cap = lay.part;
  if (int rc = cgemm(p, TP_F32, TP_PREC_F32, st)) return rc;
  // its eigenvectors by the block Jacobi of the thresholding (rows of Q G
  // made orthogonal), the r leading ones picked by eigenvalue
  if (int rc = svt_jacobi(lay.xre, lay.xim, lay.qre, lay.qim, K, m, m, real_last, kColdSweeps, kSvtTol, lay.ratio,
                          lay.conv, st))
    return rc;
  if (int rc = svt_count_unconverged(lay.conv, K, unconverged, st)) return rc;
  if (!tall) {
    if (int rc = tsvd_pick(lay.xre, lay.xim, m, lay.qre, lay.qim, m, K, m, r, real_last, 0, true, gram_floor,
                           lay.ure, lay.uim, S_out, st))
      return rc;
    return fft_inverse(lay.ure, lay.uim, TP_F32, n3, n1, r, U->data, st);
  }
  if (int rc = tsvd_pick(lay.xre, lay.xim, m, lay.qre, lay.qim, m, K, m, r, real_last, 1, true, gram_floor, lay.vre,
                         lay.vim, S_out, st))
    return rc;
  // U_r = A V_r Sigma_r^-1 (the picked columns already carry 1 / sigma)
  CGemm u;
  u.K = K;
  u.real_last = real_last;
  u.M = n1;
  u.N = r;
  u.Kd = n2;
  u.are = lay.are;
  u.aim = lay.aim;
  u.bre = lay.vre;
  u.bim = lay.vim;
  u.cre = lay.ure;
  u.cim = lay.uim;
  u.lda = n2;
  u.ldb = r;
  u.ldc = r;
  u.sa = n1 * n2;
  u.sb = n2 * r;
  u.sc = n1 * r;
  if (int rc = cgemm(u, TP_F32, TP_PREC_F32, st)) return rc;
  return fft_inverse(lay.ure, lay.uim, TP_F32, n3, n1, r, U->data, st);
}

size_t tp_tcomplete_workspace(const tp_tensor* X) {
  if (!X || X->n1 < 1 || X->n2 < 1 || X->n3 < 1) return 0;
  return admm_workspace(X->n1, X->n2, X->n3);
}

size_t tp_trpca_workspace(const tp_tensor* X) { return tp_tcomplete_workspace(X); }

int tp_tcomplete(const tp_tensor* X, const uint8_t* mask, int32_t iters, double rho, double mu0, double mu_max,
                 double tol, tp_tensor* L, tp_tensor* E, tp_tensor* Y, int32_t* ranks, int32_t* iters_done, int prec,
                 void* ws, size_t ws_bytes, void* stream) {
  if (iters_done) *iters_done = 0;
  if (!mask) return fail(TP_EINVAL, "mask is null");
  if (int rc = check_admm(X, L, E, Y, iters, rho, mu0, mu_max, prec)) return rc;
  if (std::isnan(tol)) return fail(TP_EINVAL, "tol is NaN");
  return admm_run((const float*)X->data, mask, 0.0, X->n1, X->n2, X->n3, iters, rho, mu0, mu_max, tol,
                  (float*)L->data, (float*)E->data, (float*)Y->data, ranks, iters_done, ws, ws_bytes, S(stream));
}

int tp_trpca(const tp_tensor* X, double lambda, int32_t iters, double rho, double mu0, double mu_max, double tol,
             tp_tensor* L, tp_tensor* E, tp_tensor* Y, int32_t* ranks, int32_t* iters_done, int prec, void* ws,
             size_t ws_bytes, void* stream) {
  if (iters_done) *iters_done = 0;
  if (int rc = check_admm(X, L, E, Y, iters, rho, mu0, mu_max, prec)) return rc;
  if (lambda == 0.0) lambda = rpca_default_lambda(X->n1, X->n2, X->n3);
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(TP_EINVAL, "lambda must be finite and >= 0 (0 selects the default)");
  if (std::isnan(tol)) return fail(TP_EINVAL, "tol is NaN");
  return admm_run((const float*)X->data, nullptr, lambda, X->n1, X->n2, X->n3, iters, rho, mu0, mu_max, tol,
                  (float*)L->data, (float*)E->data, (float*)Y->data, ranks, iters_done, ws, ws_bytes, S(stream));
}

}  // extern "C"
