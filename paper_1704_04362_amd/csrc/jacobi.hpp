// Workgroup-level Hermitian Jacobi eigensolver on matrices held in LDS
// (float64). Shared by the batched small eigensolver, the feature whitening
// of the learned proposal and the block Jacobi SVD of the singular value
// thresholding.
//
// Parallel cyclic Jacobi: each sweep visits every index pair once through a
// round-robin tournament (index m-1 fixed, the others rotating; for odd n
// the extra index n is a dummy that pairs with nobody). In a round the m/2
// disjoint pairs are rotated together. Because the rotations are disjoint,
// the two-sided update J^H H J splits into independent 2 x 2 blocks
// (rows of pair u, columns of pair v), so one pass updates H and the
// accumulated vectors without intermediate barriers.
//
// For a pair (p, q) with H_pq = |h| e^{i phi} the rotation is
// J = diag(1, e^{-i phi}) R(theta), R the real Jacobi rotation
// [[c, s], [-s, c]] with t = tan(theta) the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = (H_qq - H_pp) / (2 |h|) (the classical
// symmetric Schur step of Golub and Van Loan, made Hermitian by the phase).
// It is evaluated as t = sign(d) 2 |h| / (|d| + sqrt(d^2 + 4 |h|^2)),
// d = H_qq - H_pp, c = 1 / sqrt(1 + t^2), s = t c, e^{i phi} = h / |h|:
// two square roots side by side, one division and one reciprocal root.
//
// For an even n and several update items per thread, a round's update is
// branch-free and issues all of a thread's LDS reads before its writes.
#pragma once

#include <hip/hip_runtime.h>

namespace tp {

// Rotation of one pair: c, s and the phase e^{i phi} (re, im), read as two
// 16-byte words.
typedef double jrot __attribute__((ext_vector_type(4)));

template <int MAXN, int NT>
struct JacobiShared {
  static_assert(NT % 64 == 0, "whole wavefronts");
  double Hr[MAXN][MAXN + 1], Hi[MAXN][MAXN + 1];
  double Vr[MAXN][MAXN + 1], Vi[MAXN][MAXN + 1];
  jrot rot[MAXN / 2 + 1];
  double red[2][NT / 64];
  int done;
};

// Pair t of round rho in the tournament over m (even) indices. rho < m - 1
// and t < m / 2, so the residues mod m - 1 need one conditional subtraction.
__device__ __forceinline__ void jacobi_pair(int m, int rho, int t, int& p, int& q) {
  int a, b;
  if (t == 0) {
    a = m - 1;
    b = rho;
  } else {
    a = rho + t;
    a = a >= m - 1 ? a - (m - 1) : a;
    b = rho + m - 1 - t;
    b = b >= m - 1 ? b - (m - 1) : b;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Row transform of pair (c, s, e) on a column (x = M_p, y = M_q):
//   M_p = c x - s e y,  M_q = s x + c e y;
// the column transform is the same with conj(e).
__device__ __forceinline__ void jrot_apply(double c, double s, double er, double ei, double& xr, double& xi,
                                           double& yr, double& yi) {
  const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
  const double nxr = c * xr - s * eyr, nxi = c * xi - s * eyi;
  yr = s * xr + c * eyr;
  yi = s * xi + c * eyi;
  xr = nxr;
  xi = nxi;
}

// One round's update H <- J^H H J, V <- V J for an even n (no idle index):
// npairs^2 2 x 2 blocks of H and n x npairs row pairs of V, flat-indexed
// over the workgroup. Every item reads and writes only its own entries, so
// all of a thread's reads are issued before its first write.
template <int MAXN, int NT>
__device__ __forceinline__ void jacobi_update_even(JacobiShared<MAXN, NT>& sh, int n, int rho) {
  constexpr int kP = MAXN / 2;
  constexpr int kTrips = (3 * kP * kP + NT - 1) / NT;
  constexpr int kBatch = 4;  // items held in registers at once (~36 registers each)
  const int tid = threadIdx.x;
  const int npairs = n >> 1, nblk = npairs * npairs, nitems = 3 * nblk;
#pragma unroll
  for (int g0 = 0; g0 < kTrips; g0 += kBatch) {
    constexpr int kB = kTrips < kBatch ? kTrips : kBatch;
    double x[kB][8];
    jrot ru[kB], rv[kB];
    int a0[kB], a1[kB], b0[kB], b1[kB];
#pragma unroll
    for (int t = 0; t < kB; ++t) {
      const int e = tid + (g0 + t) * NT;
      if (g0 + t >= kTrips) break;
      if (e < nblk) {
        const int u = e / npairs, v = e - u * npairs;
        jacobi_pair(n, rho, u, a0[t], a1[t]);
        jacobi_pair(n, rho, v, b0[t], b1[t]);
        x[t][0] = sh.Hr[a0[t]][b0[t]];
        x[t][1] = sh.Hi[a0[t]][b0[t]];
        x[t][2] = sh.Hr[a0[t]][b1[t]];
        x[t][3] = sh.Hi[a0[t]][b1[t]];
        x[t][4] = sh.Hr[a1[t]][b0[t]];
        x[t][5] = sh.Hi[a1[t]][b0[t]];
        x[t][6] = sh.Hr[a1[t]][b1[t]];
        x[t][7] = sh.Hi[a1[t]][b1[t]];
        ru[t] = sh.rot[u];
        rv[t] = sh.rot[v];
      } else if (e < nitems) {
        const int f = e - nblk;
        const int v = f / n, i = f - v * n;
        a0[t] = i;
        jacobi_pair(n, rho, v, b0[t], b1[t]);
        x[t][0] = sh.Vr[i][b0[t]];
        x[t][1] = sh.Vi[i][b0[t]];
        x[t][2] = sh.Vr[i][b1[t]];
        x[t][3] = sh.Vi[i][b1[t]];
        rv[t] = sh.rot[v];
      }
    }
#pragma unroll
    for (int t = 0; t < kB; ++t) {
      const int e = tid + (g0 + t) * NT;
      if (g0 + t >= kTrips) break;
      if (e < nblk) {
        // rows (pair u) on columns b0 and b1, then columns (pair v) on rows a0 and a1
        jrot_apply(ru[t][0], ru[t][1], ru[t][2], ru[t][3], x[t][0], x[t][1], x[t][4], x[t][5]);
        jrot_apply(ru[t][0], ru[t][1], ru[t][2], ru[t][3], x[t][2], x[t][3], x[t][6], x[t][7]);
        jrot_apply(rv[t][0], rv[t][1], rv[t][2], -rv[t][3], x[t][0], x[t][1], x[t][2], x[t][3]);
        jrot_apply(rv[t][0], rv[t][1], rv[t][2], -rv[t][3], x[t][4], x[t][5], x[t][6], x[t][7]);
        sh.Hr[a0[t]][b0[t]] = x[t][0];
        sh.Hi[a0[t]][b0[t]] = x[t][1];
        sh.Hr[a0[t]][b1[t]] = x[t][2];
        sh.Hi[a0[t]][b1[t]] = x[t][3];
        sh.Hr[a1[t]][b0[t]] = x[t][4];
        sh.Hi[a1[t]][b0[t]] = x[t][5];
        sh.Hr[a1[t]][b1[t]] = x[t][6];
        sh.Hi[a1[t]][b1[t]] = x[t][7];
      } else if (e < nitems) {
        jrot_apply(rv[t][0], rv[t][1], rv[t][2], -rv[t][3], x[t][0], x[t][1], x[t][2], x[t][3]);
        const int i = a0[t];
        sh.Vr[i][b0[t]] = x[t][0];
        sh.Vi[i][b0[t]] = x[t][1];
        sh.Vr[i][b1[t]] = x[t][2];
        sh.Vi[i][b1[t]] = x[t][3];
      }
    }
  }
}

// Diagonalises the n x n Hermitian matrix in sh.H (n <= MAXN) in place,
// accumulating the unitary in sh.V (initialised here to the identity).
// Stops when the off-diagonal mass is below rel_tol^2 of the total or after
// max_sweeps sweeps, and returns the number of sweeps made. All NT threads
// of the workgroup must call it.
template <int MAXN, int NT>
__device__ int jacobi_eig_lds(JacobiShared<MAXN, NT>& sh, int n, int max_sweeps, double rel_tol) {
  const int tid = threadIdx.x;
  const int ne = n * n;
  for (int e = tid; e < ne; e += NT) {
    const int i = e / n, j = e - i * n;
    sh.Vr[i][j] = (i == j) ? 1.0 : 0.0;
    sh.Vi[i][j] = 0.0;
  }
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
  const int m = (n % 2) ? n + 1 : n;  // even count; index n is a dummy
  const int npairs = m / 2;
  const int nblk = npairs * npairs;
  const double tol2 = rel_tol * rel_tol;
  // the batched update pays where a thread has several items per round;
  // with one item each it measured slower than the loop below
  constexpr int kP = MAXN / 2;
  constexpr bool kEvenBatched = (3 * kP * kP + NT - 1) / NT > 1 && NT < 1024;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    {
      double off = 0.0, tot = 0.0;
      for (int e = tid; e < ne; e += NT) {
        const int i = e / n, j = e - i * n;
        const double v = sh.Hr[i][j] * sh.Hr[i][j] + sh.Hi[i][j] * sh.Hi[i][j];
        tot += v;
        if (i != j) off += v;
      }
      off = wave_sum(off);
      tot = wave_sum(tot);
      if ((tid & 63) == 0) {
        sh.red[0][tid >> 6] = off;
        sh.red[1][tid >> 6] = tot;
      }
      __syncthreads();
      if (tid == 0) {
        double o = 0.0, t = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
          o += sh.red[0][w];
          t += sh.red[1][w];
        }
        sh.done = (o <= tol2 * t) || t == 0.0;
      }
      __syncthreads();
      if (sh.done) break;
    }
    for (int rho = 0; rho < m - 1; ++rho) {
      // rotation of every pair of the round, from the current H
      if (tid < npairs) {
        int p, q;
        jacobi_pair(m, rho, tid, p, q);
        double c = 1.0, sn = 0.0, pr = 1.0, pi = 0.0;
        if (q < n) {
          const double hr = sh.Hr[p][q], hi = sh.Hi[p][q];
          const double hpp = sh.Hr[p][p], hqq = sh.Hr[q][q];
          const double h2 = hr * hr + hi * hi;
          const double d = hqq - hpp;
          const double ih = rsqrt(h2);
          const double root = sqrt(d * d + 4.0 * h2);
          const double habs = h2 * ih;
          const double t = (d >= 0.0 ? 2.0 : -2.0) * habs / (fabs(d) + root);
          const double ct = rsqrt(1.0 + t * t);
          // rotate only entries that are not negligible (also rules out
          // the infinities of an underflowed h2)
          if (h2 > 1e-300 && habs > 1e-18 * (fabs(hpp) + fabs(hqq))) {
            c = ct;
            sn = t * ct;
            pr = hr * ih;
            pi = hi * ih;
          }
        }
        sh.rot[tid] = jrot{c, sn, pr, pi};
      }
      __syncthreads();
      if constexpr (kEvenBatched) {
        if (!(n & 1)) {
          jacobi_update_even<MAXN, NT>(sh, n, rho);
          __syncthreads();
          continue;
        }
      }
      // H <- J^H H J by 2 x 2 blocks, then V <- V J by row pairs. Row
      // transform of pair u on a column (x = H_pj, y = H_qj):
      //   H_pj = c x - s e^{i phi} y,  H_qj = s x + c e^{i phi} y;
      // column transform of pair v on a row (x = M_ip, y = M_iq):
      //   M_ip = c x - s e^{-i phi} y,  M_iq = s x + c e^{-i phi} y.
      // fixed trip count (MAXN bounds the item count), so the compiler can
      // issue the LDS reads of a thread's items together
      constexpr int kMaxPairs = MAXN / 2 + 1;
      constexpr int kTrips = (kMaxPairs * kMaxPairs + MAXN * kMaxPairs + NT - 1) / NT;
#pragma unroll
      for (int it = 0; it < kTrips; ++it) {
        const int e = tid + it * NT;
        if (e >= nblk + n * npairs) continue;
        if (e < nblk) {
          const int u = e / npairs, v = e - u * npairs;
          int p0, q0, p1, q1;
          jacobi_pair(m, rho, u, p0, q0);
          jacobi_pair(m, rho, v, p1, q1);
          const bool r2 = q0 < n, c2 = q1 < n;
          if (!r2 && !c2) continue;  // 1 x 1 block of two idle indices
          double ar = sh.Hr[p0][p1], ai = sh.Hi[p0][p1];               // (p0, p1)
          double br = c2 ? sh.Hr[p0][q1] : 0.0, bi = c2 ? sh.Hi[p0][q1] : 0.0;  // (p0, q1)
          double cr = r2 ? sh.Hr[q0][p1] : 0.0, ci = r2 ? sh.Hi[q0][p1] : 0.0;  // (q0, p1)
          double dr = (r2 && c2) ? sh.Hr[q0][q1] : 0.0, di = (r2 && c2) ? sh.Hi[q0][q1] : 0.0;
          if (r2) {
            const double c = sh.rot[u][0], s = sh.rot[u][1], er = sh.rot[u][2], ei = sh.rot[u][3];
            // column p1: x = a, y = c
            double eyr = er * cr - ei * ci, eyi = er * ci + ei * cr;
            const double nar = c * ar - s * eyr, nai = c * ai - s * eyi;
            const double ncr = s * ar + c * eyr, nci = s * ai + c * eyi;
            // column q1: x = b, y = d
            eyr = er * dr - ei * di;
            eyi = er * di + ei * dr;
            const double nbr = c * br - s * eyr, nbi = c * bi - s * eyi;
            const double ndr = s * br + c * eyr, ndi = s * bi + c * eyi;
            ar = nar, ai = nai, cr = ncr, ci = nci, br = nbr, bi = nbi, dr = ndr, di = ndi;
          }
          if (c2) {
            const double c = sh.rot[v][0], s = sh.rot[v][1], er = sh.rot[v][2], ei = -sh.rot[v][3];
            // row p0: x = a, y = b
            double eyr = er * br - ei * bi, eyi = er * bi + ei * br;
            const double nar = c * ar - s * eyr, nai = c * ai - s * eyi;
            const double nbr = s * ar + c * eyr, nbi = s * ai + c * eyi;
            // row q0: x = c, y = d
            eyr = er * dr - ei * di;
            eyi = er * di + ei * dr;
            const double ncr = c * cr - s * eyr, nci = c * ci - s * eyi;
            const double ndr = s * cr + c * eyr, ndi = s * ci + c * eyi;
            ar = nar, ai = nai, br = nbr, bi = nbi, cr = ncr, ci = nci, dr = ndr, di = ndi;
          }
          sh.Hr[p0][p1] = ar;
          sh.Hi[p0][p1] = ai;
          if (c2) {
            sh.Hr[p0][q1] = br;
            sh.Hi[p0][q1] = bi;
          }
          if (r2) {
            sh.Hr[q0][p1] = cr;
            sh.Hi[q0][p1] = ci;
          }
          if (r2 && c2) {
            sh.Hr[q0][q1] = dr;
            sh.Hi[q0][q1] = di;
          }
        } else {
          const int f = e - nblk;
          const int v = f / n, i = f - v * n;
          int p, q;
          jacobi_pair(m, rho, v, p, q);
          if (q >= n) continue;
          const double c = sh.rot[v][0], s = sh.rot[v][1], er = sh.rot[v][2], ei = -sh.rot[v][3];
          const double xr = sh.Vr[i][p], xi = sh.Vi[i][p], yr = sh.Vr[i][q], yi = sh.Vi[i][q];
          const double eyr = er * yr - ei * yi, eyi = er * yi + ei * yr;
          sh.Vr[i][p] = c * xr - s * eyr;
          sh.Vi[i][p] = c * xi - s * eyi;
          sh.Vr[i][q] = s * xr + c * eyr;
          sh.Vi[i][q] = s * xi + c * eyi;
        }
      }
      __syncthreads();
    }
  }
  return sweep;
}

}  // namespace tp
