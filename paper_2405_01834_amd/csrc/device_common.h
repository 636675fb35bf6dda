// device_common.h -- device building blocks shared by the MD kernels:
// the Boys function (Eq. (boys)), the auxiliary integrals [0]^(m) (Eq. (0m))
// and the Hermite recursion (Eq. (r)) into LDS, and the FP64 matrix-core
// product used by the Hermite->solid transforms.
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

// Makes this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void lds_wave_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Builds [r]^(0) for all |r| <= L (Eqs. (0m) and (r)) in the LDS cube
// cube[t*S1 + u*S2 + v] (S2 > L, S1 > L*S2) with a single wave (lanes 0..63)
// and wave-local synchronisation, so the other waves of the workgroup keep
// issuing matrix-core work meanwhile.
//   p, P: bra Hermite exponent and centre; q, Q: ket.
//   herm: LDS copy of the Hermite order (degree-major, t then u descending).
//   lev:  3 rotating level buffers of `levn` doubles each; level n holds
//         [r]^(m) for |r| = n, m = 0..L-n at [m * T_n + deg_index].
// A lane owns whole Hermite functions of a level and runs their m chain, so
// no index division is needed.
__device__ __forceinline__ void build_R_wave(int L, double p, const double *P, double q, const double *Q,
                                             double *cube, int S1, int S2, double *lev, int levn,
                                             const uint32_t *herm, const double *boys, int lane) {
  const double pq = p + q;
  const double rho = p * q / pq;
  const double X = P[0] - Q[0], Y = P[1] - Q[1], Z = P[2] - Q[2];
  const double T = rho * (X * X + Y * Y + Z * Z);
  if (lane <= L) {
    double f = 2.0 * 17.493418327624862 / (p * q * sqrt(pq));  // Eq. (0m), 17.49.. = pi^{5/2}
    const double m2r = -2.0 * rho;
    for (int j = 0; j < lane; ++j) f *= m2r;
    const double v0 = f * boys_m(lane, T, boys);
    lev[lane] = v0;
    if (lane == 0) cube[0] = v0;
  }
  lds_wave_sync();
  for (int n = 1; n <= L; ++n) {
    double *cur = lev + (n % 3) * levn;
    const double *pr1 = lev + ((n - 1) % 3) * levn;
    const double *pr2 = lev + ((n + 1) % 3) * levn;  // level n-2
    const int Tn = (n + 1) * (n + 2) / 2, Tn1 = n * (n + 1) / 2, Tn2 = (n - 1) * n / 2;
    const int M = L - n;  // m = 0..M at this level
    const uint32_t *hdeg = herm + (n * (n + 1) * (n + 2)) / 6;
    for (int i = lane; i < Tn; i += 64) {
      const uint32_t h = hdeg[i];
      const int t = h & 0xff, u = (h >> 8) & 0xff, v = (h >> 16) & 0xff;
      // Eq. (r): [r+1_i]^(m) = r_i [r-1_i]^(m+1) + (P_i - Q_i) [r]^(m+1),
      // raising the first non-zero direction of r
      double xi, ri;
      int i1, i2;
      if (t > 0) {
        xi = X;
        ri = t - 1;
        i1 = deg_index(n - 1, t - 1, u);
        i2 = t > 1 ? deg_index(n - 2, t - 2, u) : -1;
      } else if (u > 0) {
        xi = Y;
        ri = u - 1;
        i1 = deg_index(n - 1, 0, u - 1);
        i2 = u > 1 ? deg_index(n - 2, 0, u - 2) : -1;
      } else {
        xi = Z;
        ri = v - 1;
        i1 = deg_index(n - 1, 0, 0);
        i2 = v > 1 ? deg_index(n - 2, 0, 0) : -1;
      }
      const double *a1 = pr1 + Tn1 + i1;  // m+1 = 1 at m = 0
      const double *a2 = pr2 + Tn2 + (i2 < 0 ? 0 : i2);
      double *o = cur + i;
      double val = xi * a1[0];
      if (i2 >= 0) val += ri * a2[0];
      o[0] = val;
      cube[t * S1 + u * S2 + v] = val;
      for (int m = 1; m <= M; ++m) {
        double w = xi * a1[m * Tn1];
        if (i2 >= 0) w += ri * a2[m * Tn2];
        o[m * Tn] = w;
      }
    }
    lds_wave_sync();
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
