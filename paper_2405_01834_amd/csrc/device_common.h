// device_common.h -- device building blocks shared by the MD kernels:
// the Boys function (Eq. (boys)), the auxiliary integrals [0]^(m) (Eq. (0m))
// and the Hermite recursion (Eq. (r)) into a workgroup's LDS, and the FP64
// matrix-core product used by the Hermite->solid transforms.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mderi {

typedef double d4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x4) * B(4x16) on the FP64 matrix cores.  Operand layout
// (wave64): lane = i + 16 k holds A[i][k]; lane = j + 16 k holds B[k][j];
// register r of lane j + 16 g holds D[4 r + g][j].
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Boys function F_m(T), Eq. (boys), for one m per lane.
//  T < 40: 8-term Taylor expansion about the nearest grid point T_i (spacing
//          1/16, |T - T_i| <= 1/32) using dF_m/dT = -F_{m+1}:
//          F_m(T) = sum_k F_{m+k}(T_i) (T_i - T)^k / k!  (truncation < 3e-17 F_m).
//  T >= 40: F_0 = (1/2) sqrt(pi/T) (erf(sqrt T) rounds to 1) and the upward
//          recursion F_{j+1} = ((2j+1) F_j - e^{-T}) / (2T), stable for
//          2j+1 < 2T.
__device__ __forceinline__ double boys_m(int m, double T, const double *__restrict__ tab) {
  if (T < kBoysTmax) {
    const int i = (int)(T * (double)kBoysGridPerUnit + 0.5);
    const double d = (double)i * (1.0 / kBoysGridPerUnit) - T;
    const double *row = tab + i * kBoysM + m;
    double acc = row[7];
    acc = row[6] + acc * d * (1.0 / 7.0);
    acc = row[5] + acc * d * (1.0 / 6.0);
    acc = row[4] + acc * d * (1.0 / 5.0);
    acc = row[3] + acc * d * (1.0 / 4.0);
    acc = row[2] + acc * d * (1.0 / 3.0);
    acc = row[1] + acc * d * (1.0 / 2.0);
    acc = row[0] + acc * d;
    return acc;
  }
  const double emT = exp(-T);
  const double o2T = 0.5 / T;
  double f = 0.5 * sqrt(3.14159265358979323846 / T);
  for (int j = 0; j < m; ++j) f = ((2 * j + 1) * f - emT) * o2T;
  return f;
}

// Index of (t, u, .) inside the Hermite functions of total degree n, ordered
// t descending then u descending.
__device__ __forceinline__ int deg_index(int n, int t, int u) { return ((n - t) * (n - t + 1) >> 1) + (n - t - u); }

// Builds [r]^(0) for all |r| <= L (Eqs. (0m) and (r)) in the LDS cube
// cube[t*(L+1)^2 + u*(L+1) + v], cooperatively over the workgroup.
//   p, P: bra Hermite exponent and centre; q, Q: ket.
//   lev:  3 rotating level buffers of `levn` doubles each; level n holds
//         [r]^(m) for |r| = n, m = 0..L-n at [m * T_n + deg_index].
// Starts and ends with all threads past a barrier.
__device__ __forceinline__ void build_R(int L, double p, const double *P, double q, const double *Q, double *cube,
                                        double *lev, int levn, const Tables &tab, int tid, int nthr) {
  const double pq = p + q;
  const double rho = p * q / pq;
  const double X = P[0] - Q[0], Y = P[1] - Q[1], Z = P[2] - Q[2];
  const double T = rho * (X * X + Y * Y + Z * Z);
  const int L1 = L + 1;
  const int S1 = L1 * L1;
  if (tid <= L) {
    // Eq. (0m): [0]^(m) = (-2 rho)^m 2 pi^{5/2} / (p q sqrt(p+q)) F_m(T)
    double f = 2.0 * 17.493418327624862 / (p * q * sqrt(pq));  // 17.49.. = pi^{5/2}
    const double m2r = -2.0 * rho;
    for (int j = 0; j < tid; ++j) f *= m2r;
    lev[tid] = f * boys_m(tid, T, tab.boys);
  }
  __syncthreads();
  if (tid == 0) cube[0] = lev[0];
  for (int n = 1; n <= L; ++n) {
    double *cur = lev + (n % 3) * levn;
    const double *pr1 = lev + ((n - 1) % 3) * levn;
    const double *pr2 = lev + ((n + 1) % 3) * levn;  // level n-2
    const int Tn = (n + 1) * (n + 2) / 2, Tn1 = n * (n + 1) / 2, Tn2 = (n - 1) * n / 2;
    const int cnt = (L - n + 1) * Tn;
    const uint32_t *hdeg = tab.herm + (n * (n + 1) * (n + 2)) / 6;
    for (int e = tid; e < cnt; e += nthr) {
      const int m = e / Tn;
      const int i = e - m * Tn;
      const uint32_t h = hdeg[i];
      const int t = h & 0xff, u = (h >> 8) & 0xff, v = (h >> 16) & 0xff;
      double val;
      // Eq. (r): [r+1_i]^(m) = r_i [r-1_i]^(m+1) + (P_i - Q_i) [r]^(m+1)
      if (t > 0) {
        val = X * pr1[(m + 1) * Tn1 + deg_index(n - 1, t - 1, u)];
        if (t > 1) val += (t - 1) * pr2[(m + 1) * Tn2 + deg_index(n - 2, t - 2, u)];
      } else if (u > 0) {
        val = Y * pr1[(m + 1) * Tn1 + deg_index(n - 1, 0, u - 1)];
        if (u > 1) val += (u - 1) * pr2[(m + 1) * Tn2 + deg_index(n - 2, 0, u - 2)];
      } else {
        val = Z * pr1[(m + 1) * Tn1 + deg_index(n - 1, 0, 0)];
        if (v > 1) val += (v - 1) * pr2[(m + 1) * Tn2 + deg_index(n - 2, 0, 0)];
      }
      cur[e] = val;
      if (m == 0) cube[t * S1 + u * L1 + v] = val;
    }
    __syncthreads();
  }
}

// Workgroup id -> work item such that consecutive items land on the same XCD
// (workgroups are dispatched round-robin over the 8 XCDs of MI355X), so the
// output lines shared by neighbouring bra pairs meet in one L2.
__device__ __forceinline__ long xcd_remap(long b, long G) {
  const long nx = 8;
  const long qn = G / nx, rn = G % nx;
  const long x = b % nx, slot = b / nx;
  return (x < rn) ? x * (qn + 1) + slot : rn * (qn + 1) + (x - rn) * qn + slot;
}

}  // namespace mderi
