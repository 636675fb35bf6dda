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

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// D(16x16, FP32) += A(16x32) * B(32x16) in BF16 on the matrix cores.  Operand
// layout (wave64): lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] for e = 0..7; register r of lane l holds
// D[4 (l / 16) + r][l % 16].
__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight consecutive BF16 values (16-byte aligned) as an MFMA operand.
__device__ __forceinline__ bf8 load_bf8(const uint16_t *p) {
  return __builtin_bit_cast(bf8, *(const u4 *)p);
}

// 1/x and 1/sqrt(x) for x > 0 (normal): the hardware estimate refined by two
// Newton steps (relative error about one unit in the last place), shorter
// chains than the correctly rounded division and square root.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// x^n for 0 <= n < 32 by binary exponentiation (dependency depth 5 instead of n).
__device__ __forceinline__ double ipow_small(double x, int n) {
  double r = 1.0;
#pragma unroll
  for (int bit = 0; bit < 5; ++bit) {
    r *= (n & 1) ? x : 1.0;
    x *= x;
    n >>= 1;
  }
  return r;
}

// Boys function F_m(T), Eq. (boys), for one m per lane.
//  T < 100: 8-term Taylor expansion about the nearest grid point T_i (spacing
//          1/16, |T - T_i| <= 1/32) using dF_m/dT = -F_{m+1}:
//          F_m(T) = sum_k F_{m+k}(T_i) (T_i - T)^k / k!  (truncation < 3e-17 F_m).
//  T >= 100: F_m = (2m-1)!! / (2T)^m F_0 with F_0 = (1/2) sqrt(pi/T): the
//          terms in e^{-T} of the exact upward recursion are below 1e-18 of
//          F_m there for every m <= 26.
__device__ __forceinline__ double boys_m(int m, double T, const double *__restrict__ tab) {
  if (T < kBoysTmax) {
    const int i = (int)(T * (double)kBoysGridPerUnit + 0.5);
    const double d = (double)i * (1.0 / kBoysGridPerUnit) - T;
    const double *row = tab + i * kBoysM + m;
    // sum_k row[k] d^k / k!, k = 0..7, by Estrin's scheme (dependency depth
    // 4 instead of 14 for Horner's: this runs beside matrix-core work)
    const double d2 = d * d, d4 = d2 * d2;
    const double p01 = fma(row[1], d, row[0]);
    const double p23 = fma(row[3] * (1.0 / 6.0), d, row[2] * 0.5);
    const double p45 = fma(row[5] * (1.0 / 120.0), d, row[4] * (1.0 / 24.0));
    const double p67 = fma(row[7] * (1.0 / 5040.0), d, row[6] * (1.0 / 720.0));
    return fma(fma(p67, d2, p45), d4, fma(p23, d2, p01));
  }
  const double f0 = 0.88622692545275801 * rsqrt_nr(T);  // (1/2) sqrt(pi) = 0.886..
  return f0 * tab[kBoysNgrid * kBoysM + m] * ipow_small(0.5 * rcp_nr(T), m);
}


// Index of (t, u, .) inside the Hermite functions of total degree n, ordered
// t descending then u descending.
__device__ __forceinline__ int deg_index(int n, int t, int u) { return ((n - t) * (n - t + 1) >> 1) + (n - t - u); }

// Value of the next lane (lane i gets lane i+1, lane 63 gets 0) by a DPP
// wavefront shift (gfx9 wave_shl:1): a VALU move, no LDS round trip.
__device__ __forceinline__ double lane_next(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Makes this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void lds_wave_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// One step of Eq. (r) along one direction for a whole m-vector held in
// registers: with a = [.. k ..]^(m) and b = [.. k-1 ..]^(m) (m = 0..LM),
// b <- [.. k+1 ..]^(m) = k [.. k-1 ..]^(m+1) + X [.. k ..]^(m+1).
// Entries past the valid m range carry finite junk that is never stored.
template <int LM>
__device__ __forceinline__ void rr_step(double (&a)[LM + 1], double (&b)[LM + 1], double k, double X) {
#pragma unroll
  for (int m = 0; m < LM; ++m) b[m] = fma(X, a[m + 1], k * b[m + 1]);
  b[LM] = 0.0;
}

// Size (doubles) of the work area of build_R_chains_packed for total L.
__host__ __device__ constexpr int rr_work_size_packed(int L) { return (L + 1) + (L + 1) * (L + 1) + ntil(L); }

// Offset of the (u, v) m-vector in the packed y-stage buffer (pairs ordered
// by u, then v; the vector of (u, v) has L-u-v+1 entries).
__device__ __forceinline__ int uv_base(int L, int u, int v) {
  const int k0 = L + 1, k1 = L + 1 - u;
  const int tet = (k0 * (k0 + 1) * (k0 + 2) - k1 * (k1 + 1) * (k1 + 2)) / 6;
  return tet + v * (L - u + 1) - v * (v - 1) / 2;
}

// Packed-buffer variant of build_R_chains (below) for the long m-vectors of
// L > 18, where fixed-size slots would not fit in LDS beside the cube: the
// m-vectors are stored with their valid lengths only (predicated stores).
// Builds [r]^(0) for all |r| <= L (Eqs. (0m) and (r)) in the LDS cube
// cube[t*S1 + u*S2 + v] (S2 > L, S1 > L*S2) with a single wave and
// wave-local synchronisation, so the other waves of the workgroup keep
// issuing matrix-core work meanwhile.  Eq. (r) is applied direction by
// direction (the same choice of direction as raising the first non-zero
// component of r): z-chain [00v]^(m) on one lane, y-chains [0uv]^(m) with
// one lane per v, x-chains [tuv]^(m) with one lane per (u, v); each lane
// keeps its m-vector in registers (LM >= L at compile time).
//   p, P: bra Hermite exponent and centre; q, Q: ket.
//   work: rr_work_size_packed(L) doubles of LDS; uv: (u | v << 8) of the pairs
//         u+v <= L ordered by u+v (longest chains first).
template <int LM>
__device__ __forceinline__ void build_R_chains_packed(int L, double p, const double *P, double q, const double *Q,
                                               double *cube, int S1, int S2, double *work, const uint32_t *uv,
                                               const double *boys, int lane) {
  const double pq = p + q;
  const double rho = p * q * rcp_nr(pq);
  const double X = P[0] - Q[0], Y = P[1] - Q[1], Z = P[2] - Q[2];
  const double T = rho * (X * X + Y * Y + Z * Z);
  double *f0 = work;                 // [0]^(m), m = 0..L
  double *zb = f0 + (L + 1);         // [00v]^(m) at v*(L+1) + m
  double *yb = zb + (L + 1) * (L + 1);  // [0uv]^(m) at uv_base(u, v) + m
  if (lane <= L) {
    double f = 2.0 * 17.493418327624862 * rcp_nr(p * q) * rsqrt_nr(pq);  // Eq. (0m), 17.49.. = pi^{5/2}
    f *= ipow_small(-2.0 * rho, lane);
    f0[lane] = f * boys_m(lane, T, boys);
  }
  lds_wave_sync();
  double a[LM + 1], b[LM + 1];
  if (lane == 0) {  // z chain
#pragma unroll
    for (int m = 0; m <= LM; ++m) {
      a[m] = m <= L ? f0[m] : 0.0;
      b[m] = 0.0;
    }
#pragma unroll
    for (int m = 0; m <= LM; ++m)
      if (m <= L) zb[m] = a[m];
    for (int v = 0; v < L; v += 2) {
      rr_step<LM>(a, b, (double)v, Z);  // b = level v+1
#pragma unroll
      for (int m = 0; m <= LM; ++m)
        if (m <= L - v - 1) zb[(v + 1) * (L + 1) + m] = b[m];
      if (v + 1 < L) {
        rr_step<LM>(b, a, (double)(v + 1), Z);  // a = level v+2
#pragma unroll
        for (int m = 0; m <= LM; ++m)
          if (m <= L - v - 2) zb[(v + 2) * (L + 1) + m] = a[m];
      }
    }
  }
  lds_wave_sync();
  if (lane <= L) {  // y chains, lane = v
    const int v = lane, M = L - v;
#pragma unroll
    for (int m = 0; m <= LM; ++m) {
      a[m] = m <= M ? zb[v * (L + 1) + m] : 0.0;
      b[m] = 0.0;
    }
#pragma unroll
    for (int m = 0; m <= LM; ++m)
      if (m <= M) yb[uv_base(L, 0, v) + m] = a[m];
    for (int u = 0; u < M; u += 2) {
      rr_step<LM>(a, b, (double)u, Y);
      {
        const int o = uv_base(L, u + 1, v);
#pragma unroll
        for (int m = 0; m <= LM; ++m)
          if (m <= M - u - 1) yb[o + m] = b[m];
      }
      if (u + 1 < M) {
        rr_step<LM>(b, a, (double)(u + 1), Y);
        const int o = uv_base(L, u + 2, v);
#pragma unroll
        for (int m = 0; m <= LM; ++m)
          if (m <= M - u - 2) yb[o + m] = a[m];
      }
    }
  }
  lds_wave_sync();
  const int npair = (L + 1) * (L + 2) / 2;
  for (int pi = lane; pi - lane < npair; pi += 64) {  // x chains, lane = (u, v)
    if (pi < npair) {
      const int u = uv[pi] & 0xff, v = (uv[pi] >> 8) & 0xff, M = L - u - v;
      const int base = uv_base(L, u, v);
#pragma unroll
      for (int m = 0; m <= LM; ++m) {
        a[m] = m <= M ? yb[base + m] : 0.0;
        b[m] = 0.0;
      }
      double *cc = cube + u * S2 + v;
      cc[0] = a[0];
      for (int t = 0; t < M; t += 2) {
        rr_step<LM>(a, b, (double)t, X);
        cc[(t + 1) * S1] = b[0];
        if (t + 1 < M) {
          rr_step<LM>(b, a, (double)(t + 1), X);
          cc[(t + 2) * S1] = a[0];
        }
      }
    }
  }
  lds_wave_sync();
}

// Register length of the producer's m-vectors for total L (the kernels are
// instantiated for these buckets).
__host__ __device__ constexpr int rr_lm_bucket(int L) {
  return L <= 8 ? 8 : L <= 10 ? 10 : L <= 16 ? 16 : L <= 18 ? 18 : L <= 26 ? 26 : -1;
}

// Layout of the y stage of build_R_chains for total L.  The m-vectors
// [0uv]^(m) are computed with one lane per (v, m): the lanes of one v form a
// block of L-v+1 consecutive lanes, blocks are packed whole into groups of at
// most 64 lanes (a group is one register of the wave), and all blocks of a
// group take len = L - (smallest v of the group) steps along u.  The buffer
// is v-major: the vector of (u, v) sits in slot vbase(v) + u (L+1 doubles per
// slot), and every v reserves len + 1 slots of its group, so a lane stores
// level u+1 at a fixed offset from level u whether or not (u+1, v) exists.
//   Returns the number of slots; when v >= 0, *vbase_out = vbase(v).
__host__ __device__ constexpr int ylayout(int L, int v = -1, int *vbase_out = nullptr) {
  int used = 64, len = 0, vb = 0;
  for (int w = 0; w <= L; ++w) {
    const int need = L - w + 1;
    if (used + need > 64) {
      used = 0;
      len = L - w;
    }
    used += need;
    if (w == v && vbase_out) *vbase_out = vb;
    vb += len + 1;
  }
  return vb;
}

__host__ __device__ constexpr int yvbase(int L, int v) {
  int vb = 0;
  (void)ylayout(L, v, &vb);
  return vb;
}

// Number of lane groups of the y stage for total L, and the step count of group j.
__host__ __device__ constexpr int ygroups(int L) {
  int used = 64, ng = 0;
  for (int w = 0; w <= L; ++w) {
    const int need = L - w + 1;
    if (used + need > 64) {
      used = 0;
      ++ng;
    }
    used += need;
  }
  return ng;
}
__host__ __device__ constexpr int ygroup_len(int L, int j) {
  int used = 64, g = -1;
  for (int w = 0; w <= L; ++w) {
    const int need = L - w + 1;
    if (used + need > 64) {
      used = 0;
      if (++g == j) return L - w;
    }
    used += need;
  }
  return 0;
}

// Lane groups the fixed-slot builder provides registers for (every L of the
// bucket fits: ygroups(L) <= 1, 2, 3, 4 for L <= 8, 10, 16, 18).
template <int LM>
__host__ __device__ constexpr int ygroup_regs() {
  return LM <= 9 ? 1 : LM <= 10 ? 2 : LM <= 16 ? 3 : 4;
}

// Size (doubles) of the work area of build_R_chains for total L: the y-stage
// buffer (ylayout slots of L+1 doubles; level u = 0 holds the z chain), then
// a scratch row for the lanes a y group does not use (64 + L (L+1) doubles).
__host__ __device__ constexpr int rr_work_size(int L) {
  return rr_lm_bucket(L) > 18 ? rr_work_size_packed(L) : (ylayout(L) + L) * (L + 1) + 64;
}

// Per-lane state of the y stage, set once per kernel by ylanes_init.
template <int LM>
struct YLanes {
  int addr[ygroup_regs<LM>()];  // slot vbase(v) (L+1) + m of this lane's (v, m) in group j, else scratch row
};

template <int LM>
__device__ __forceinline__ void ylanes_init(int L, int lane, YLanes<LM> &y) {
  constexpr int NG = ygroup_regs<LM>();
  const int W = L + 1;
#pragma unroll
  for (int j = 0; j < NG; ++j) y.addr[j] = ylayout(L) * W + lane;
  int used = 64, g = -1, len = 0, vb = 0;
  for (int w = 0; w <= L; ++w) {
    const int need = L - w + 1;
    if (used + need > 64) {
      used = 0;
      ++g;
      len = L - w;
    }
    if (lane >= used && lane < used + need) {
#pragma unroll
      for (int j = 0; j < NG; ++j)
        if (g == j) y.addr[j] = vb * W + (lane - used);
    }
    used += need;
    vb += len + 1;
  }
}

// x chains of the pairs p0 .. p0+63 (ordered by u+v, so the pass's first
// pair has the longest chain, M0 = L - (u+v of pair p0)): level t+1 of a
// lane's m-vector is valid for m <= M - t - 1 <= M0 - t - 1, so the levels
// shrink; lanes store level t+1 while t < M.
template <int L, int P0>
__device__ __forceinline__ void x_pass(double X, double *cube, int S1, int S2, const double *yb, const uint32_t *uv,
                                       int lane) {
  constexpr int W = L + 1, NPAIR = (L + 1) * (L + 2) / 2;
  if constexpr (P0 < NPAIR) {
    constexpr int S0 = [] {
      int s = 0;
      while ((s + 1) * (s + 2) / 2 <= P0) ++s;
      return s;
    }();
    constexpr int M0 = L - S0;
    const int pi = P0 + lane;
    if (P0 + 64 <= NPAIR || pi < NPAIR) {
      const uint32_t e = uv[pi];
      const int u = e & 0xff, v = (e >> 8) & 0xff, M = L - u - v;
      const double *ys = yb + (e >> 16) * W;
      double a[M0 + 1], b[M0 + 1];
#pragma unroll
      for (int m = 0; m <= M0; ++m) a[m] = ys[m];
      double *cc = cube + u * S2 + v;
      cc[0] = a[0];
#pragma unroll
      for (int t = 0; t < M0; t += 2) {
#pragma unroll
        for (int m = 0; m < M0 - t; ++m) b[m] = t == 0 ? X * a[m + 1] : fma(X, a[m + 1], (double)t * b[m + 1]);
        if (t < M) cc[(t + 1) * S1] = b[0];
        if (t + 1 < M0) {
#pragma unroll
          for (int m = 0; m < M0 - t - 1; ++m) a[m] = fma(X, b[m + 1], (double)(t + 1) * a[m + 1]);
          if (t + 1 < M) cc[(t + 2) * S1] = a[0];
        }
      }
    }
    x_pass<L, P0 + 64>(X, cube, S1, S2, yb, uv, lane);
  }
}

// Builds [r]^(0) for all |r| <= L (Eqs. (0m) and (r)) in the LDS cube
// cube[t*S1 + u*S2 + v] (offsets additive and injective on |r| <= L) with a
// single wave and wave-local synchronisation, so the other waves of the
// workgroup keep issuing matrix-core work meanwhile.  Eq. (r) is applied
// direction by direction (the same choice of direction as raising the first
// non-zero component of r), with L fixed at compile time so every loop is
// unrolled and every LDS offset is an immediate:
//   * [0]^(m) (Eq. (0m)) and the z chain [00v]^(m): one lane per m, the m+1
//     neighbour taken from the next lane by a DPP move;
//   * y chains [0uv]^(m): one lane per (v, m) in the lane groups of ylayout,
//     again with DPP moves, the groups' chains interleaved;
//   * x chains [tuv]^(m): one lane per (u, v) with the m-vector in
//     registers, 64 pairs per pass (x_pass).
// Entries past a vector's valid m range carry junk that only ever feeds
// other junk entries and is never stored in the cube.
//   p, P: bra Hermite exponent and centre; q, Q: ket.
//   work: rr_work_size(L) doubles of LDS; uv: (u | v << 8 | (vbase(v)+u) << 16)
//         of the pairs u+v <= L ordered by u+v (longest chains first).
template <int L, int LM>
__device__ __forceinline__ void build_R_exact(double p, const double *P, double q, const double *Q, double *cube,
                                              int S1, int S2, double *work, const uint32_t *uv, const double *boys,
                                              int lane, const YLanes<LM> &yl) {
  constexpr int W = L + 1, NG = ygroups(L);
  const double pq = p + q;
  const double rho = p * q * rcp_nr(pq);
  const double X = P[0] - Q[0], Y = P[1] - Q[1], Z = P[2] - Q[2];
  const double T = rho * (X * X + Y * Y + Z * Z);
  double *yb = work;  // [0uv]^(m) at (vbase(v) + u) W + m
  // [0]^(m) in lane m, then the z chain: level v+1 from levels v and v-1 at
  // m+1; the level-v-1 neighbour is the previous step's DPP result.  Lanes
  // past L sit out (their DPP reads return 0).
  if (lane <= L) {
    double f = 2.0 * 17.493418327624862 * rcp_nr(p * q) * rsqrt_nr(pq);  // Eq. (0m), 17.49.. = pi^{5/2}
    f *= ipow_small(-2.0 * rho, lane);
    double za = f * boys_m(lane, T, boys), zp = 0.0;
    double *zl = yb + lane;
    zl[0] = za;  // vbase(0) = 0
#pragma unroll
    for (int v = 0; v < L; ++v) {
      const double an = lane_next(za);
      za = v == 0 ? Z * an : fma(Z, an, (double)v * zp);
      zp = an;
      zl[yvbase(L, v + 1) * W] = za;
    }
  }
  lds_wave_sync();
  // y chains: lane (v, m) of group j holds [0uv]^(m); level u+1 lands W
  // doubles after level u
  {
    double ya[NG], yp[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      ya[j] = yb[yl.addr[j]];
      yp[j] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        if (u < ygroup_len(L, j)) {
          const double an = lane_next(ya[j]);
          ya[j] = u == 0 ? Y * an : fma(Y, an, (double)u * yp[j]);
          yp[j] = an;
          yb[yl.addr[j] + (u + 1) * W] = ya[j];
        }
      }
    }
  }
  lds_wave_sync();
  x_pass<L, 0>(X, cube, S1, S2, yb, uv, lane);
  lds_wave_sync();
}

template <int LO, int HI, int LM>
__device__ __forceinline__ void build_R_dispatch(int L, double p, const double *P, double q, const double *Q,
                                                 double *cube, int S1, int S2, double *work, const uint32_t *uv,
                                                 const double *boys, int lane, const YLanes<LM> &yl) {
  if constexpr (HI >= LO) {
    if (L == HI) {
      build_R_exact<HI, LM>(p, P, q, Q, cube, S1, S2, work, uv, boys, lane, yl);
      return;
    }
    build_R_dispatch<LO, HI - 1, LM>(L, p, P, q, Q, cube, S1, S2, work, uv, boys, lane, yl);
  }
}

// [r]^(0) for |r| <= L: the exact-L builder of the bucket LM (L <= 18), the
// packed builder above for larger L.
template <int LM>
__device__ __forceinline__ void build_R_chains(int L, double p, const double *P, double q, const double *Q,
                                               double *cube, int S1, int S2, double *work, const uint32_t *uv,
                                               const double *boys, int lane, const YLanes<LM> &yl) {
  if constexpr (LM > 18) {
    build_R_chains_packed<LM>(L, p, P, q, Q, cube, S1, S2, work, uv, boys, lane);
  } else {
    constexpr int LO = LM <= 8 ? 0 : LM <= 10 ? 9 : LM <= 16 ? 11 : 17;
    build_R_dispatch<LO, LM, LM>(L, p, P, q, Q, cube, S1, S2, work, uv, boys, lane, yl);
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
