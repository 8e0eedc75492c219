// Small per-Fourier-slice linear algebra for the randomized t-SVD
// (Theorem "t-SVD" and eq. circ1: the t-SVD is one matrix SVD per Fourier
// slice), t-project / t-CX (Algorithms 3-4) and the t-CUR core
// pseudo-inverse (Algorithm 5):
//  * Gaussian test matrices drawn per slice (Philox4x64-10 + Box-Muller);
//  * Gram matrices X^H X of tall slices, accumulated in float64;
//  * a Hermitian eigensolver for s x s Gram matrices (s <= 64): parallel
//    cyclic Jacobi in float64, one workgroup per slice, the matrix and the
//    accumulated rotations held in LDS;
//  * the derived small transforms (orthonormalisation V diag(lambda^-1/2),
//    truncation to the leading r directions with singular-value scaling);
//  * leverage reductions summed over the half spectrum with conjugate
//    weights (1 for the real slices, 2 for the others).
#include <cmath>

#include "common.hpp"
#include "linalg.hpp"

namespace tp {
namespace {

__device__ __forceinline__ uint64_t philox4x64_w01(uint64_t seed, uint64_t stream, uint64_t index, uint64_t* w1) {
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
  *w1 = x1;
  return x0;
}

// Standard complex normal entries (real normal on the real slices).
template <typename T>
__global__ void randn_kernel(T* re, T* im, int64_t K, int64_t per_slice, int real_last, uint64_t seed,
                             uint64_t stream) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * per_slice) return;
  const int64_t k = e / per_slice;
  const bool real = k == 0 || (real_last && k == K - 1);
  uint64_t w1;
  const uint64_t w0 = philox4x64_w01(seed, stream, (uint64_t)e, &w1);
  const double u1 = ((double)(w0 >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)(w1 >> 11) * 0x1.0p-53;         // [0, 1)
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  if (real) {
    re[e] = (T)(rad * cs);
    im[e] = T(0);
  } else {
    re[e] = (T)(rad * cs * 0.7071067811865476);
    im[e] = (T)(rad * sn * 0.7071067811865476);
  }
}

// G_k = X_k^H X_k (s x s, float64) for X_k rows x s (planar, row stride ldx).
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(const T* __restrict__ xre, const T* __restrict__ xim, int64_t K,
                                                   int64_t rows, int s, int64_t ldx, int64_t sx, int real_last,
                                                   double* __restrict__ gre, double* __restrict__ gim) {
  constexpr int CH = 32;
  __shared__ double cr[CH][kMaxS], ci[CH][kMaxS];
  const int64_t k = blockIdx.x;
  const bool real = k == 0 || (real_last && k == K - 1);
  const T* xr = xre + k * sx;
  const T* xi = xim + k * sx;
  const int ne = s * s;
  constexpr int PER = kMaxS * kMaxS / 256;
  double ar[PER], ai[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) ar[q] = ai[q] = 0.0;
  for (int64_t r0 = 0; r0 < rows; r0 += CH) {
    for (int e = threadIdx.x; e < CH * s; e += 256) {
      const int rr = e / s, c = e - rr * s;
      const int64_t row = r0 + rr;
      double vr = 0.0, vi = 0.0;
      if (row < rows) {
        vr = (double)xr[row * ldx + c];
        vi = real ? 0.0 : (double)xi[row * ldx + c];
      }
      cr[rr][c] = vr;
      ci[rr][c] = vi;
    }
    __syncthreads();
    const int nr = (int)((rows - r0) < CH ? (rows - r0) : CH);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e >= ne) continue;
      const int i = e / s, j = e - i * s;
      double sr = ar[q], si = ai[q];
      for (int rr = 0; rr < nr; ++rr) {
        // conj(x_i) * x_j
        sr += cr[rr][i] * cr[rr][j] + ci[rr][i] * ci[rr][j];
        si += cr[rr][i] * ci[rr][j] - ci[rr][i] * cr[rr][j];
      }
      ar[q] = sr;
      ai[q] = si;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (e >= ne) continue;
    gre[k * ne + e] = ar[q];
    gim[k * ne + e] = real ? 0.0 : ai[q];
  }
}

// Parallel cyclic Jacobi for Hermitian s x s matrices (one workgroup per
// slice). Each sweep visits every index pair once through a round-robin
// tournament: in a round the s/2 disjoint pairs are rotated together, rows
// first, then columns, which applies the product of the disjoint rotations.
// For a pair (p, q) with H_pq = |h| e^{i phi}, the rotation is
// J = diag(1, e^{-i phi}) R(theta), R the real Jacobi rotation
// [[c, s], [-s, c]] with t = tan(theta) the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = (H_qq - H_pp) / (2 |h|).
__global__ __launch_bounds__(256) void herm_eig_kernel(const double* __restrict__ gre,
                                                       const double* __restrict__ gim, int s, int max_sweeps,
                                                       double* __restrict__ evals, double* __restrict__ vre,
                                                       double* __restrict__ vim) {
  __shared__ double Hr[kMaxS][kMaxS + 1], Hi[kMaxS][kMaxS + 1];
  __shared__ double Vr[kMaxS][kMaxS + 1], Vi[kMaxS][kMaxS + 1];
  __shared__ double rc[kMaxS / 2], rs[kMaxS / 2], rpr[kMaxS / 2], rpi[kMaxS / 2];
  __shared__ int pp[kMaxS / 2], qq[kMaxS / 2];
  __shared__ int perm[kMaxS + 1];
  __shared__ double red[256];
  __shared__ int sdone;
  const int64_t k = blockIdx.x;
  const int ne = s * s;
  const int tid = threadIdx.x;
  for (int e = tid; e < ne; e += 256) {
    const int i = e / s, j = e - i * s;
    Hr[i][j] = gre[k * ne + e];
    Hi[i][j] = gim[k * ne + e];
    Vr[i][j] = (i == j) ? 1.0 : 0.0;
    Vi[i][j] = 0.0;
  }
  const int n = (s % 2) ? s + 1 : s;  // padded to even; index s is a dummy
  for (int i = tid; i < n; i += 256) perm[i] = i;
  __syncthreads();
  // Hermitian symmetrisation of the input (Gram accumulation is symmetric up
  // to rounding)
  for (int e = tid; e < ne; e += 256) {
    const int i = e / s, j = e - i * s;
    if (i < j) {
      const double ar = 0.5 * (Hr[i][j] + Hr[j][i]), ai = 0.5 * (Hi[i][j] - Hi[j][i]);
      Hr[i][j] = ar;
      Hi[i][j] = ai;
      Hr[j][i] = ar;
      Hi[j][i] = -ai;
    } else if (i == j) {
      Hi[i][i] = 0.0;
    }
  }
  __syncthreads();
  const int npairs = n / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal vs total Frobenius mass
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < ne; e += 256) {
      const int i = e / s, j = e - i * s;
      const double m = Hr[i][j] * Hr[i][j] + Hi[i][j] * Hi[i][j];
      tot += m;
      if (i != j) off += m;
    }
    red[tid] = off;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double offsum = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double totsum = red[0];
    if (tid == 0) sdone = (offsum <= 1e-30 * totsum) || totsum == 0.0;
    __syncthreads();
    if (sdone) break;
    for (int round = 0; round < n - 1; ++round) {
      // tournament pairing: position 0 fixed, the others rotate
      if (tid < npairs) {
        int a = perm[tid], b = perm[n - 1 - tid];
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        pp[tid] = a;
        qq[tid] = b;
        double c = 1.0, sn = 0.0, pr = 1.0, pi = 0.0;
        if (b < s) {
          const double hr = Hr[a][b], hi = Hi[a][b];
          const double habs = sqrt(hr * hr + hi * hi);
          const double diag = fabs(Hr[a][a]) + fabs(Hr[b][b]);
          if (habs > 1e-300 && habs > 1e-18 * diag) {
            const double tau = (Hr[b][b] - Hr[a][a]) / (2.0 * habs);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            pr = hr / habs;  // e^{i phi}
            pi = hi / habs;
          }
        }
        rc[tid] = c;
        rs[tid] = sn;
        rpr[tid] = pr;
        rpi[tid] = pi;
      }
      __syncthreads();
      // rows: H <- J^H H. For column j: x = H_pj, y = H_qj:
      //   H_pj = c x - s e^{i phi} y,  H_qj = s x + c e^{i phi} y
      for (int e = tid; e < npairs * s; e += 256) {
        const int r = e / s, j = e - r * s;
        const int p = pp[r], q = qq[r];
        if (q >= s) continue;
        const double c = rc[r], sn = rs[r], er = rpr[r], ei = rpi[r];
        const double xr = Hr[p][j], xi = Hi[p][j], yr = Hr[q][j], yi = Hi[q][j];
        const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;  // e^{i phi} y
        Hr[p][j] = c * xr - sn * eyr;
        Hi[p][j] = c * xi - sn * eyi;
        Hr[q][j] = sn * xr + c * eyr;
        Hi[q][j] = sn * xi + c * eyi;
      }
      __syncthreads();
      // columns: H <- H J and V <- V J. For row i: x = M_ip, y = M_iq:
      //   M_ip = c x - s e^{-i phi} y,  M_iq = s x + c e^{-i phi} y
      for (int e = tid; e < npairs * s; e += 256) {
        const int r = e / s, i = e - r * s;
        const int p = pp[r], q = qq[r];
        if (q >= s) continue;
        const double c = rc[r], sn = rs[r], er = rpr[r], ei = -rpi[r];
        {
          const double xr = Hr[i][p], xi = Hi[i][p], yr = Hr[i][q], yi = Hi[i][q];
          const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
          Hr[i][p] = c * xr - sn * eyr;
          Hi[i][p] = c * xi - sn * eyi;
          Hr[i][q] = sn * xr + c * eyr;
          Hi[i][q] = sn * xi + c * eyi;
        }
        {
          const double xr = Vr[i][p], xi = Vi[i][p], yr = Vr[i][q], yi = Vi[i][q];
          const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
          Vr[i][p] = c * xr - sn * eyr;
          Vi[i][p] = c * xi - sn * eyi;
          Vr[i][q] = sn * xr + c * eyr;
          Vi[i][q] = sn * xi + c * eyi;
        }
      }
      __syncthreads();
      // rotate the tournament (positions 1..n-1)
      if (tid == 0) {
        const int last = perm[n - 1];
        for (int i = n - 1; i > 1; --i) perm[i] = perm[i - 1];
        perm[1] = last;
      }
      __syncthreads();
    }
  }
  // order eigenvalues descending (ties by index) through ranks
  __shared__ int order[kMaxS];
  if (tid < s) {
    const double lt = Hr[tid][tid];
    int rank = 0;
    for (int j = 0; j < s; ++j) {
      const double lj = Hr[j][j];
      if (lj > lt || (lj == lt && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < ne; e += 256) {
    const int i = e / s, j = e - i * s;  // row i, sorted column j
    const int src = order[j];
    vre[k * ne + e] = Vr[i][src];
    vim[k * ne + e] = Vi[i][src];
  }
  if (tid < s) evals[k * s + tid] = Hr[order[tid]][order[tid]];
}

// Small transforms from an eigen-decomposition G = V diag(lambda) V^H.
// mode 0 (orthonormalise): T = V diag(w), w_i = lambda_i^{-1/2} when
//   lambda_i > rtol * lambda_0 (and > 0), else 0; T is s x s.
// mode 1 (truncate): T = V[:, :r] diag(w), w_i = lambda_i^{-p/2} for the
//   kept i < r with sigma_i = sqrt(lambda_i) > rtol * sigma_0, else 0; T is
//   s x r. p is `power`.
// Output planar in float (Tf) or double (Td).
template <typename T>
__global__ void transform_kernel(const double* __restrict__ vre, const double* __restrict__ vim,
                                 const double* __restrict__ evals, int64_t K, int s, int r, int mode, double rtol,
                                 double power, T* __restrict__ tre, T* __restrict__ tim) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int cols = mode == 0 ? s : r;
  if (e >= K * s * cols) return;
  const int64_t k = e / ((int64_t)s * cols);
  const int rem = (int)(e - k * s * cols);
  const int i = rem / cols, j = rem - i * cols;
  const double l0 = evals[k * s];
  const double lj = evals[k * s + j];
  double w = 0.0;
  if (mode == 0) {
    if (lj > 0.0 && lj > rtol * l0) w = 1.0 / sqrt(lj);
  } else {
    const double s0 = l0 > 0.0 ? sqrt(l0) : 0.0;
    const double sj = lj > 0.0 ? sqrt(lj) : 0.0;
    if (sj > 0.0 && sj > rtol * s0) w = pow(sj, -power);
  }
  const int64_t src = k * (int64_t)s * s + (int64_t)i * s + j;
  tre[e] = (T)(vre[src] * w);
  tim[e] = (T)(vim[src] * w);
}

// out[j] = sum_k w_k sum_{i<r} |X_k[j, i]|^2 * g_k[i], with g_k[i] =
// 1/lambda_k[i] when scaled (so that X_k diag(1/sigma) is normalised), else 1;
// w_k the conjugate weights of the half spectrum.
template <typename T>
__global__ void leverage_kernel(const T* __restrict__ xre, const T* __restrict__ xim, int64_t K, int64_t n,
                                int64_t ldx, int64_t sx, int r, int real_last, const double* __restrict__ evals,
                                int s, double rtol, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double wk = (k == 0 || (real_last && k == K - 1)) ? 1.0 : 2.0;
    const double l0 = evals ? evals[k * s] : 0.0;
    double sk = 0.0;
    for (int i = 0; i < r; ++i) {
      double g = 1.0;
      if (evals) {
        const double li = evals[k * s + i];
        const double si = li > 0 ? sqrt(li) : 0.0, s0 = l0 > 0 ? sqrt(l0) : 0.0;
        g = (si > 0 && si > rtol * s0) ? 1.0 / li : 0.0;
      }
      const double a = (double)xre[k * sx + j * ldx + i], b = (double)xim[k * sx + j * ldx + i];
      sk += (a * a + b * b) * g;
    }
    acc += wk * sk;
  }
  out[j] = acc;
}

__global__ void sqrt_evals_kernel(const double* __restrict__ evals, int64_t K, int s, int r,
                                  double* __restrict__ sv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * r) return;
  const int64_t k = e / r;
  const int i = (int)(e - k * r);
  const double l = evals[k * s + i];
  sv[e] = l > 0 ? sqrt(l) : 0.0;
}

// W[k][t][c] = scale[t] * X[k][idx[t]][c] (row gather of a spectrum, with
// rows at or beyond *count set to zero); converts between float types.
template <typename Ti, typename To>
__global__ void gather_rows_kernel(const Ti* __restrict__ xre, const Ti* __restrict__ xim, int64_t K, int64_t rows,
                                   int64_t cols, const int32_t* __restrict__ idx, const double* __restrict__ scale,
                                   const int64_t* count, int64_t out_rows, To* __restrict__ wre,
                                   To* __restrict__ wim) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * out_rows * cols) return;
  const int64_t k = e / (out_rows * cols);
  const int64_t rem = e - k * out_rows * cols;
  const int64_t t = rem / cols, c = rem - t * cols;
  const int64_t lim = count ? *count : out_rows;
  if (t >= lim) {
    wre[e] = To(0);
    wim[e] = To(0);
    return;
  }
  const double sc = scale ? scale[t] : 1.0;
  const int64_t src = k * rows * cols + (int64_t)idx[t] * cols + c;
  wre[e] = (To)((double)xre[src] * sc);
  wim[e] = (To)((double)xim[src] * sc);
}

template <typename Ti, typename To>
__global__ void convert_kernel(const Ti* __restrict__ a, To* __restrict__ b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (To)a[e];
}

unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int randn_spectrum(void* re, void* im, int dtype, int64_t K, int64_t rows, int64_t cols, bool real_last,
                   uint64_t seed, uint64_t stream_id, hipStream_t st) {
  const int64_t n = K * rows * cols;
  if (n == 0) return TP_OK;
  if (dtype == TP_F64)
    hipLaunchKernelGGL(randn_kernel<double>, dim3(blocks_for(n)), dim3(256), 0, st, (double*)re, (double*)im, K,
                       rows * cols, real_last ? 1 : 0, seed, stream_id);
  else
    hipLaunchKernelGGL(randn_kernel<float>, dim3(blocks_for(n)), dim3(256), 0, st, (float*)re, (float*)im, K,
                       rows * cols, real_last ? 1 : 0, seed, stream_id);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int gram(const void* xre, const void* xim, int dtype, int64_t K, int64_t rows, int s, int64_t ldx, int64_t sx,
         bool real_last, double* gre, double* gim, hipStream_t st) {
  if (s < 1 || s > kMaxS) return fail(TP_EUNSUPPORTED, "Gram size outside 1..64");
  if (dtype == TP_F64)
    hipLaunchKernelGGL(gram_kernel<double>, dim3((unsigned)K), dim3(256), 0, st, (const double*)xre,
                       (const double*)xim, K, rows, s, ldx, sx, real_last ? 1 : 0, gre, gim);
  else
    hipLaunchKernelGGL(gram_kernel<float>, dim3((unsigned)K), dim3(256), 0, st, (const float*)xre,
                       (const float*)xim, K, rows, s, ldx, sx, real_last ? 1 : 0, gre, gim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int herm_eig(const double* gre, const double* gim, int64_t K, int s, double* evals, double* vre, double* vim,
             hipStream_t st) {
  if (s < 1 || s > kMaxS) return fail(TP_EUNSUPPORTED, "eigenproblem size outside 1..64");
  hipLaunchKernelGGL(herm_eig_kernel, dim3((unsigned)K), dim3(256), 0, st, gre, gim, s, 40, evals, vre, vim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int eig_transform(const double* vre, const double* vim, const double* evals, int64_t K, int s, int r, int mode,
                  double rtol, double power, void* tre, void* tim, int out_dtype, hipStream_t st) {
  const int64_t n = K * s * (mode == 0 ? s : r);
  if (n == 0) return TP_OK;
  if (out_dtype == TP_F64)
    hipLaunchKernelGGL(transform_kernel<double>, dim3(blocks_for(n)), dim3(256), 0, st, vre, vim, evals, K, s, r,
                       mode, rtol, power, (double*)tre, (double*)tim);
  else
    hipLaunchKernelGGL(transform_kernel<float>, dim3(blocks_for(n)), dim3(256), 0, st, vre, vim, evals, K, s, r,
                       mode, rtol, power, (float*)tre, (float*)tim);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int leverage(const void* xre, const void* xim, int dtype, int64_t K, int64_t n, int64_t ldx, int64_t sx, int r,
             bool real_last, const double* evals, int s, double rtol, double* out, hipStream_t st) {
  if (n == 0) return TP_OK;
  if (dtype == TP_F64)
    hipLaunchKernelGGL(leverage_kernel<double>, dim3(blocks_for(n)), dim3(256), 0, st, (const double*)xre,
                       (const double*)xim, K, n, ldx, sx, r, real_last ? 1 : 0, evals, s, rtol, out);
  else
    hipLaunchKernelGGL(leverage_kernel<float>, dim3(blocks_for(n)), dim3(256), 0, st, (const float*)xre,
                       (const float*)xim, K, n, ldx, sx, r, real_last ? 1 : 0, evals, s, rtol, out);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int singular_values(const double* evals, int64_t K, int s, int r, double* sv, hipStream_t st) {
  if (K * r == 0) return TP_OK;
  hipLaunchKernelGGL(sqrt_evals_kernel, dim3(blocks_for(K * r)), dim3(256), 0, st, evals, K, s, r, sv);
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int gather_rows(const void* xre, const void* xim, int in_dtype, int64_t K, int64_t rows, int64_t cols,
                const int32_t* idx, const double* scale, const int64_t* count, int64_t out_rows, void* wre,
                void* wim, int out_dtype, hipStream_t st) {
  const int64_t n = K * out_rows * cols;
  if (n == 0) return TP_OK;
  if (in_dtype == TP_F32 && out_dtype == TP_F64)
    hipLaunchKernelGGL((gather_rows_kernel<float, double>), dim3(blocks_for(n)), dim3(256), 0, st,
                       (const float*)xre, (const float*)xim, K, rows, cols, idx, scale, count, out_rows,
                       (double*)wre, (double*)wim);
  else if (in_dtype == TP_F32 && out_dtype == TP_F32)
    hipLaunchKernelGGL((gather_rows_kernel<float, float>), dim3(blocks_for(n)), dim3(256), 0, st,
                       (const float*)xre, (const float*)xim, K, rows, cols, idx, scale, count, out_rows,
                       (float*)wre, (float*)wim);
  else if (in_dtype == TP_F64 && out_dtype == TP_F64)
    hipLaunchKernelGGL((gather_rows_kernel<double, double>), dim3(blocks_for(n)), dim3(256), 0, st,
                       (const double*)xre, (const double*)xim, K, rows, cols, idx, scale, count, out_rows,
                       (double*)wre, (double*)wim);
  else
    return fail(TP_EDTYPE, "gather_rows: unsupported conversion");
  TP_LAUNCH_CHECK();
  return TP_OK;
}

int convert(const void* a, int adt, void* b, int bdt, int64_t n, hipStream_t st) {
  if (n == 0) return TP_OK;
  if (adt == TP_F64 && bdt == TP_F32)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(blocks_for(n)), dim3(256), 0, st, (const double*)a,
                       (float*)b, n);
  else if (adt == TP_F32 && bdt == TP_F64)
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(blocks_for(n)), dim3(256), 0, st, (const float*)a,
                       (double*)b, n);
  else
    return fail(TP_EDTYPE, "convert: unsupported conversion");
  TP_LAUNCH_CHECK();
  return TP_OK;
}

}  // namespace tp
