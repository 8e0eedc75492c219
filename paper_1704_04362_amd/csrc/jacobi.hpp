// Workgroup-level Hermitian Jacobi eigensolver on matrices held in LDS
// (float64). Shared by the batched small eigensolver and the block Jacobi
// SVD of the singular value thresholding.
//
// Parallel cyclic Jacobi: each sweep visits every index pair once through a
// round-robin tournament; in a round the n/2 disjoint pairs are rotated
// together, rows first, then columns (and the accumulated vectors), which
// applies the product of the disjoint rotations. For a pair (p, q) with
// H_pq = |h| e^{i phi} the rotation is J = diag(1, e^{-i phi}) R(theta), R the
// real Jacobi rotation [[c, s], [-s, c]] with t = tan(theta) the smaller root
// of t^2 + 2 tau t - 1 = 0, tau = (H_qq - H_pp) / (2 |h|) (the classical
// symmetric Schur step of Golub and Van Loan, made Hermitian by the phase).
#pragma once

#include <hip/hip_runtime.h>

namespace tp {

template <int MAXN, int NT>
struct JacobiShared {
  double Hr[MAXN][MAXN + 1], Hi[MAXN][MAXN + 1];
  double Vr[MAXN][MAXN + 1], Vi[MAXN][MAXN + 1];
  double rc[MAXN / 2], rs[MAXN / 2], rpr[MAXN / 2], rpi[MAXN / 2];
  int pp[MAXN / 2], qq[MAXN / 2];
  int perm[MAXN + 1];
  double red[NT];
  int done;
};

// Diagonalises the n x n Hermitian matrix in sh.H (n <= MAXN) in place,
// accumulating the unitary in sh.V (initialised here to the identity).
// Stops when the off-diagonal mass is below rel_tol^2 of the total or after
// max_sweeps sweeps. All NT threads of the workgroup must call it.
template <int MAXN, int NT>
__device__ void jacobi_eig_lds(JacobiShared<MAXN, NT>& sh, int n, int max_sweeps, double rel_tol) {
  const int tid = threadIdx.x;
  const int ne = n * n;
  for (int e = tid; e < ne; e += NT) {
    const int i = e / n, j = e - i * n;
    sh.Vr[i][j] = (i == j) ? 1.0 : 0.0;
    sh.Vi[i][j] = 0.0;
  }
  const int m = (n % 2) ? n + 1 : n;  // even count; index n is a dummy
  for (int i = tid; i < m; i += NT) sh.perm[i] = i;
  __syncthreads();
  // exact Hermitian symmetry of the input
  for (int e = tid; e < ne; e += NT) {
    const int i = e / n, j = e - i * n;
    if (i < j) {
      const double ar = 0.5 * (sh.Hr[i][j] + sh.Hr[j][i]), ai = 0.5 * (sh.Hi[i][j] - sh.Hi[j][i]);
      sh.Hr[i][j] = ar;
      sh.Hi[i][j] = ai;
      sh.Hr[j][i] = ar;
      sh.Hi[j][i] = -ai;
    } else if (i == j) {
      sh.Hi[i][i] = 0.0;
    }
  }
  __syncthreads();
  const int npairs = m / 2;
  const double tol2 = rel_tol * rel_tol;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < ne; e += NT) {
      const int i = e / n, j = e - i * n;
      const double v = sh.Hr[i][j] * sh.Hr[i][j] + sh.Hi[i][j] * sh.Hi[i][j];
      tot += v;
      if (i != j) off += v;
    }
    sh.red[tid] = off;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
      if (tid < w) sh.red[tid] += sh.red[tid + w];
      __syncthreads();
    }
    const double offsum = sh.red[0];
    __syncthreads();
    sh.red[tid] = tot;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
      if (tid < w) sh.red[tid] += sh.red[tid + w];
      __syncthreads();
    }
    if (tid == 0) sh.done = (offsum <= tol2 * sh.red[0]) || sh.red[0] == 0.0;
    __syncthreads();
    if (sh.done) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < npairs) {
        int a = sh.perm[tid], b = sh.perm[m - 1 - tid];
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        sh.pp[tid] = a;
        sh.qq[tid] = b;
        double c = 1.0, sn = 0.0, pr = 1.0, pi = 0.0;
        if (b < n) {
          const double hr = sh.Hr[a][b], hi = sh.Hi[a][b];
          const double habs = sqrt(hr * hr + hi * hi);
          const double diag = fabs(sh.Hr[a][a]) + fabs(sh.Hr[b][b]);
          if (habs > 1e-300 && habs > 1e-18 * diag) {
            const double tau = (sh.Hr[b][b] - sh.Hr[a][a]) / (2.0 * habs);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            pr = hr / habs;
            pi = hi / habs;
          }
        }
        sh.rc[tid] = c;
        sh.rs[tid] = sn;
        sh.rpr[tid] = pr;
        sh.rpi[tid] = pi;
      }
      __syncthreads();
      // rows: H <- J^H H; for column j with x = H_pj, y = H_qj:
      //   H_pj = c x - s e^{i phi} y,  H_qj = s x + c e^{i phi} y
      for (int e = tid; e < npairs * n; e += NT) {
        const int r = e / n, j = e - r * n;
        const int p = sh.pp[r], q = sh.qq[r];
        if (q >= n) continue;
        const double c = sh.rc[r], sn = sh.rs[r], er = sh.rpr[r], ei = sh.rpi[r];
        const double xr = sh.Hr[p][j], xi = sh.Hi[p][j], yr = sh.Hr[q][j], yi = sh.Hi[q][j];
        const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
        sh.Hr[p][j] = c * xr - sn * eyr;
        sh.Hi[p][j] = c * xi - sn * eyi;
        sh.Hr[q][j] = sn * xr + c * eyr;
        sh.Hi[q][j] = sn * xi + c * eyi;
      }
      __syncthreads();
      // columns: H <- H J, V <- V J; for row i with x = M_ip, y = M_iq:
      //   M_ip = c x - s e^{-i phi} y,  M_iq = s x + c e^{-i phi} y
      for (int e = tid; e < npairs * n; e += NT) {
        const int r = e / n, i = e - r * n;
        const int p = sh.pp[r], q = sh.qq[r];
        if (q >= n) continue;
        const double c = sh.rc[r], sn = sh.rs[r], er = sh.rpr[r], ei = -sh.rpi[r];
        {
          const double xr = sh.Hr[i][p], xi = sh.Hi[i][p], yr = sh.Hr[i][q], yi = sh.Hi[i][q];
          const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
          sh.Hr[i][p] = c * xr - sn * eyr;
          sh.Hi[i][p] = c * xi - sn * eyi;
          sh.Hr[i][q] = sn * xr + c * eyr;
          sh.Hi[i][q] = sn * xi + c * eyi;
        }
        {
          const double xr = sh.Vr[i][p], xi = sh.Vi[i][p], yr = sh.Vr[i][q], yi = sh.Vi[i][q];
          const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
          sh.Vr[i][p] = c * xr - sn * eyr;
          sh.Vi[i][p] = c * xi - sn * eyi;
          sh.Vr[i][q] = sn * xr + c * eyr;
          sh.Vi[i][q] = sn * xi + c * eyi;
        }
      }
      __syncthreads();
      if (tid == 0) {
        const int last = sh.perm[m - 1];
        for (int i = m - 1; i > 1; --i) sh.perm[i] = sh.perm[i - 1];
        sh.perm[1] = last;
      }
      __syncthreads();
    }
  }
}

}  // namespace tp
