// Fused t-CUR core for small slices: per Fourier slice k, the truncated
// pseudo-inverse of W_k = D S^T Chat_k (l x c, l, c <= 64) that the core
// step of Algorithm 5 needs, pinv_r(W) = V_r diag(1/sigma) U_r^H, returned
// as the two factors P = V_r diag(1/sigma) (c x r) and U_r (l x r).
//
// The steps are those of the randomized range finder of Halko, Martinsson
// and Tropp used for the larger cores, in float64, inside one 1024-thread
// workgroup per slice with every small matrix in LDS:
//   Y = W Omega, Q = orth(orth(Y)); q times: Z = orth(W^H Q),
//   Q = orth(orth(W Z)); Bh = W^H Q; Bh^H Bh = U_B diag(lambda) U_B^H
//   (Jacobi); P = Bh U_B,r diag(lambda^-1), U_r = Q U_B,r, keeping the
//   leading r with sigma_i > rtol sigma_1.
// orth(X) is CholeskyQR: X^H X = R^H R (pivots at or below 1e-24 of the
// largest diagonal entry dropped), X <- X R^{-1} by forward substitution
// along the rows of X. W (l c <= 3600 entries) is read into LDS once and
// used by every product; the products and Gram matrices run on the float64
// matrix cores from LDS.
#include "common.hpp"
#include "jacobi.hpp"
#include "linalg.hpp"

namespace tp {
namespace {

constexpr int CNT = 1024, CM = 64, CS = 32, LDY = CS, CW = 3600;

// The Gram / Cholesky scratch is dead once the eigensolver starts, so it
// shares its LDS with the solver's state.
struct CoreFactor {
  double gr[CS][CS + 1], gi[CS][CS + 1];  // Gram, then the strict upper triangle of R
};

struct CoreShared {
  double wr[CW], wi[CW];            // W (m x n, m n <= 3600)
  double yr[CM][LDY], yi[CM][LDY];  // Y / Q (m x s)
  double zr[CM][LDY], zi[CM][LDY];  // Omega / Bh / Z (n x s)
  union {
    CoreFactor f;
    JacobiShared<CS, CNT> jac;
  };
  double rd[CS];
  double rinv[CS];  // 1 / R_jj, 0 for a dropped index
  double dmax;
  int order[CS];
};

struct CoreArgs {
  const double *wre, *wim;  // K x m x n
  const double *ore, *oim;  // K x n x s
  int64_t K;
  int m, n, s, r, q;
  int real_last;
  double rtol;  // truncation, relative to sigma_1
  double *p64re, *p64im, *u64re, *u64im;  // K x n x r, K x m x r
  float *p32re, *p32im, *u32re, *u32im;   // optional float32 copies
};

// Products of LDS-resident matrices on the float64 matrix cores
// (v_mfma_f64_16x16x4f64: A lane l = A[l % 16][l / 16], B lane l =
// B[l / 16][l % 16], D lane l register v = D[4 v + l / 16][l % 16]):
// C (M x N) = op(A) B, op(A)[i][k] = A[i lda + k], or conj(A[k lda + i])
// with CA, all row-major, M, N <= 64 (one 16 x 16 output tile per
// wavefront of the 16), entries past M, N or K read as zero. C must not
// overlap A or B.
typedef double cd4 __attribute__((ext_vector_type(4)));

template <bool CA>
__device__ void mm_lds(const double* ar, const double* ai, int lda, const double* br, const double* bi, int ldb,
                       int M, int N, int K, double* cr, double* ci, int ldc) {
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int tn = (N + 15) >> 4, nt = ((M + 15) >> 4) * tn;
  if (w < nt) {
    const int ti = w / tn, tj = w - ti * tn;
    const int i = 16 * ti + (l & 15), j = 16 * tj + (l & 15);
    cd4 accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + (l >> 4);
      double xr = 0.0, xi = 0.0, yr = 0.0, yi = 0.0;
      if (k < K && i < M) {
        const int e = CA ? k * lda + i : i * lda + k;
        xr = ar[e];
        xi = CA ? -ai[e] : ai[e];
      }
      if (k < K && j < N) {
        yr = br[k * ldb + j];
        yi = bi[k * ldb + j];
      }
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yr, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi, yi, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yi, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yr, acci, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * ti + 4 * v + (l >> 4);
      if (row < M && j < N) {
        cr[row * ldc + j] = accr[v];
        ci[row * ldc + j] = acci[v];
      }
    }
  }
  __syncthreads();
}

// Y (m x s) = W Z (Z: n x s in zr / zi)
__device__ void prod_wz(const CoreArgs& a, CoreShared& sh) {
  mm_lds<false>(sh.wr, sh.wi, a.n, &sh.zr[0][0], &sh.zi[0][0], LDY, a.m, a.s, a.n, &sh.yr[0][0], &sh.yi[0][0], LDY);
}

// Bh (n x s, into zr / zi) = W^H Q (Q: m x s in yr / yi)
__device__ void prod_whq(const CoreArgs& a, CoreShared& sh) {
  mm_lds<true>(sh.wr, sh.wi, a.n, &sh.yr[0][0], &sh.yi[0][0], LDY, a.n, a.s, a.m, &sh.zr[0][0], &sh.zi[0][0], LDY);
}

// G (s x s) = X^H X, X rows x s
__device__ void gram_lds(const double (*xr)[LDY], const double (*xi)[LDY], int rows, int s, CoreShared& sh) {
  mm_lds<true>(&xr[0][0], &xi[0][0], LDY, &xr[0][0], &xi[0][0], LDY, s, s, rows, &sh.f.gr[0][0], &sh.f.gi[0][0],
               CS + 1);
}

// R from the Gram matrix in gr / gi: register-resident right-looking
// Cholesky with pivot dropping (entry (tid / 32, tid % 32) per thread). On
// return rd[j] = R_jj (0 for a dropped index) and gr / gi hold the strict
// upper triangle of R (zero rows for dropped indices).
__device__ void chol_lds(int s, double rtol, CoreShared& sh) {
  const int tid = threadIdx.x;
  const int ri = tid / CS, ci = tid % CS;
  const bool mine = ri < s && ci < s && ci >= ri;
  double gr = mine ? sh.f.gr[ri][ci] : 0.0, gi = (mine && ci > ri) ? sh.f.gi[ri][ci] : 0.0;
  if (tid < 64) {
    double mx = tid < s ? sh.f.gr[tid][tid] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (tid == 0) sh.dmax = mx;
  }
  __syncthreads();
  const double tol = rtol * sh.dmax;
  for (int j = 0; j < s; ++j) {
    if (ri == j && ci >= j && ci < s) {
      sh.f.gr[j][ci] = gr;
      sh.f.gi[j][ci] = gi;
    }
    __syncthreads();
    const double d = sh.f.gr[j][j];
    if (d > tol && d > 0.0) {
      // 1 / d: hardware reciprocal refined by two Newton steps
      double inv = __builtin_amdgcn_rcp(d);
      inv = fma(fma(-d, inv, 1.0), inv, inv);
      inv = fma(fma(-d, inv, 1.0), inv, inv);
      if (ri > j && ci >= ri && ci < s) {
        const double ar = sh.f.gr[j][ri], ai = sh.f.gi[j][ri], br = sh.f.gr[j][ci], bi = sh.f.gi[j][ci];
        gr -= (ar * br + ai * bi) * inv;
        gi -= (ar * bi - ai * br) * inv;
      }
    }
  }
  if (tid < CS) {
    const double d = tid < s ? sh.f.gr[tid][tid] : 0.0;
    const bool keep = tid < s && d > tol && d > 0.0;
    const double rd = keep ? sqrt(d) : 0.0;
    sh.rd[tid] = rd;
    sh.rinv[tid] = keep ? 1.0 / rd : 0.0;
  }
  __syncthreads();
  // R: strict upper triangle (zero on dropped rows and past s)
  if (ci > ri) {
    const bool live = ri < s && ci < s && sh.rd[ri] > 0.0;
    sh.f.gr[ri][ci] = live ? gr / sh.rd[ri] : 0.0;
    sh.f.gi[ri][ci] = live ? gi / sh.rd[ri] : 0.0;
  }
  __syncthreads();
}

// X <- X R^{-1} on the kept indices (dropped columns become zero), in place:
// forward substitution along every row of X, Q_j = (X_j - sum_{a<j} Q_a R_aj)
// / R_jj, with 16 lanes per row holding columns tq and tq + 16; the pivot
// value of step j is broadcast from its lane by a 16-wide shuffle, so the
// 32 steps need no workgroup barrier.
__device__ void solve_rows(double (*xr)[LDY], double (*xi)[LDY], int rows, int s, CoreShared& sh) {
  const int tid = threadIdx.x, i = tid >> 4, tq = tid & 15;
  const bool live = i < rows;
  const int ii = live ? i : 0;
  double r0 = 0.0, i0 = 0.0, r1 = 0.0, i1 = 0.0;
  if (live && tq < s) {
    r0 = xr[ii][tq];
    i0 = xi[ii][tq];
  }
  if (live && tq + 16 < s) {
    r1 = xr[ii][tq + 16];
    i1 = xi[ii][tq + 16];
  }
#pragma unroll
  for (int j = 0; j < CS; ++j) {
    if (j >= s) break;
    const bool hi = j >= 16;
    const double vr = __shfl(hi ? r1 : r0, j & 15, 16), vi = __shfl(hi ? i1 : i0, j & 15, 16);
    const double inv = sh.rinv[j];
    const double qr = vr * inv, qi = vi * inv;
    if (tq == (j & 15)) {
      if (hi) {
        r1 = qr;
        i1 = qi;
      } else {
        r0 = qr;
        i0 = qi;
      }
    }
    // x_t -= q R_jt for the columns t > j this lane holds
    if (tq > j) {
      const double rr = sh.f.gr[j][tq], ri = sh.f.gi[j][tq];
      r0 -= qr * rr - qi * ri;
      i0 -= qr * ri + qi * rr;
    }
    if (tq + 16 > j && tq + 16 < s) {
      const double rr = sh.f.gr[j][tq + 16], ri = sh.f.gi[j][tq + 16];
      r1 -= qr * rr - qi * ri;
      i1 -= qr * ri + qi * rr;
    }
  }
  __syncthreads();
  if (live && tq < s) {
    xr[i][tq] = r0;
    xi[i][tq] = i0;
  }
  if (live && tq + 16 < s) {
    xr[i][tq + 16] = r1;
    xi[i][tq + 16] = i1;
  }
  __syncthreads();
}

__device__ void orth_lds(double (*xr)[LDY], double (*xi)[LDY], int rows, int s, CoreShared& sh) {
  gram_lds(xr, xi, rows, s, sh);
  chol_lds(s, 1e-24, sh);
  solve_rows(xr, xi, rows, s, sh);
}

__global__ __launch_bounds__(CNT) void core_pinv_kernel(CoreArgs a) {
  __shared__ CoreShared sh;
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x;
  const bool real = k == 0 || (a.real_last && k == a.K - 1);
  const double* wr = a.wre + k * a.m * a.n;
  const double* wi = a.wim + k * a.m * a.n;
  // W and Omega (imaginary parts of the real slices read as zero)
  for (int e = tid; e < a.m * a.n; e += CNT) {
    sh.wr[e] = wr[e];
    sh.wi[e] = real ? 0.0 : wi[e];
  }
  for (int e = tid; e < a.n * a.s; e += CNT) {
    const int j = e / a.s, t = e - j * a.s;
    sh.zr[j][t] = a.ore[k * a.n * a.s + e];
    sh.zi[j][t] = real ? 0.0 : a.oim[k * a.n * a.s + e];
  }
  __syncthreads();
  prod_wz(a, sh);
  orth_lds(sh.yr, sh.yi, a.m, a.s, sh);
  orth_lds(sh.yr, sh.yi, a.m, a.s, sh);
  for (int it = 0; it < a.q; ++it) {
    prod_whq(a, sh);
    orth_lds(sh.zr, sh.zi, a.n, a.s, sh);
    prod_wz(a, sh);
    orth_lds(sh.yr, sh.yi, a.m, a.s, sh);
    orth_lds(sh.yr, sh.yi, a.m, a.s, sh);
  }
  prod_whq(a, sh);
  // Bh^H Bh into the eigensolver
  gram_lds(sh.zr, sh.zi, a.n, a.s, sh);
  for (int e = tid; e < a.s * a.s; e += CNT) {
    const int p = e / a.s, q = e - p * a.s;
    sh.jac.Hr[p][q] = sh.f.gr[p][q];
    sh.jac.Hi[p][q] = sh.f.gi[p][q];
  }
  __syncthreads();
  jacobi_eig_lds<CS, CNT>(sh.jac, a.s, 40, 1e-15);
  if (tid < a.s) {
    const double lt = sh.jac.Hr[tid][tid];
    int rank = 0;
    for (int j = 0; j < a.s; ++j) {
      const double lj = sh.jac.Hr[j][j];
      if (lj > lt || (lj == lt && j < tid)) ++rank;
    }
    sh.order[rank] = tid;
  }
  __syncthreads();
  // weights of the kept leading columns: 1/lambda for P, 1 for U
  if (tid < a.r) {
    const double l0 = sh.jac.Hr[sh.order[0]][sh.order[0]];
    const double lj = sh.jac.Hr[sh.order[tid]][sh.order[tid]];
    const double s0 = l0 > 0.0 ? sqrt(l0) : 0.0;
    const double sj = lj > 0.0 ? sqrt(lj) : 0.0;
    const bool keep = sj > 0.0 && sj > a.rtol * s0;
    sh.rd[tid] = keep ? 1.0 / (sj * sj) : 0.0;  // P weight; U keeps the same columns with weight 1
  }
  __syncthreads();
  // P = Bh U_B,r diag(w_P) (n x r), U = Q U_B,r diag(w_U) (m x r)
  for (int e = tid; e < (a.n + a.m) * a.r; e += CNT) {
    const bool isp = e < a.n * a.r;
    const int f = isp ? e : e - a.n * a.r;
    const int i = f / a.r, c = f - i * a.r;
    const int col = sh.order[c];
    double vr = 0.0, vi = 0.0;
    for (int t = 0; t < a.s; ++t) {
      const double xr = isp ? sh.zr[i][t] : sh.yr[i][t], xi = isp ? sh.zi[i][t] : sh.yi[i][t];
      const double er = sh.jac.Vr[t][col], ei = sh.jac.Vi[t][col];
      vr += xr * er - xi * ei;
      vi += xr * ei + xi * er;
    }
    const double w = isp ? sh.rd[c] : (sh.rd[c] > 0.0 ? 1.0 : 0.0);
    vr *= w;
    vi *= w;
    if (real) vi = 0.0;
    if (isp) {
      a.p64re[k * a.n * a.r + f] = vr;
      a.p64im[k * a.n * a.r + f] = vi;
      if (a.p32re) {
        a.p32re[k * a.n * a.r + f] = (float)vr;
        a.p32im[k * a.n * a.r + f] = (float)vi;
      }
    } else {
      a.u64re[k * a.m * a.r + f] = vr;
      a.u64im[k * a.m * a.r + f] = vi;
      if (a.u32re) {
        a.u32re[k * a.m * a.r + f] = (float)vr;
        a.u32im[k * a.m * a.r + f] = (float)vi;
      }
    }
  }
}

}  // namespace

bool core_pinv_fits(int64_t m, int64_t n, int s, int64_t r) {
  return m >= 1 && n >= 1 && m <= CM && n <= CM && m * n <= CW && s >= 1 && s <= CS && r >= 1 && r <= s;
}

int core_pinv(const double* wre, const double* wim, const double* ore, const double* oim, int64_t K, int64_t m,
              int64_t n, int s, int64_t r, bool real_last, int q, double rtol, double* p64re, double* p64im,
              double* u64re, double* u64im, float* p32re, float* p32im, float* u32re, float* u32im, hipStream_t st) {
  if (!core_pinv_fits(m, n, s, r))
    return fail(TP_EUNSUPPORTED, "fused core needs l, c <= 64, l c <= 3600 and r <= s <= 32");
  if (K == 0) return TP_OK;
  if (K > 0x7fffffff) return fail(TP_EUNSUPPORTED, "too many Fourier slices");
  CoreArgs a{wre, wim, ore, oim, K, (int)m, (int)n, s, (int)r, q, real_last ? 1 : 0, rtol,
             p64re, p64im, u64re, u64im, p32re, p32im, u32re, u32im};
  hipLaunchKernelGGL(core_pinv_kernel, dim3((unsigned)K), dim3(CNT), 0, st, a);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
