// kx_impl.h -- the screened quartet engine: exchange (K) and Coulomb (J)
// builds and the nuclear gradient of E = sum W_abcd (ab|cd), one shell
// quartet at a time per wave (Sec. 6 exchange operator; Sec. 2 for the
// derivative Gaussians).  Instantiated in kx0.hip (digest) and kx1.hip
// (gradient).
//
// Work decomposition.  The pairs of every class are sorted by decreasing
// Schwarz factor on the host, so the B pairs k that pass Q_i Q_k >= tau with
// A pair i form a prefix of B; a block's quartets are numbered
// q = pre[i] + k and cut into fixed-size chunks.  Every wave of the launch
// is independent: it takes the next chunk from a device counter, finds the
// block (binary search over the blocks' first chunks) and the A pair
// (binary search over pre[]), then walks its quartets with k fastest, so
// consecutive quartets share the A pair.  No quartet that fails the
// screening test is ever visited and no workgroup barrier is used.
//
// One quartet by one wave (all in the wave's own LDS region):
//   * [r]^(0) for |r| <= L (Eqs. (0m), (r)) by the wave-level register-chain
//     builder into the cube;
//   * per B column tile ct and A row part (NRT tiles of 16 Hermite rows):
//     X[p][cd] = sum_q [p+q] H_B[q][cd] on the FP64 matrix cores, the A
//     operand gathered from the cube (Eq. (ket-from-hermite), the sign of
//     Eq. (pq) folded into H_B), then
//       digest mode:   V[ab][cd] += sum_p H_A[p][ab] X[p][cd]   (Eq. (bra-from-hermite))
//       gradient mode: X kept transposed, Y^T = S X^T over the tile's columns
//                      and six dot products with the derivative matrices of
//                      the A pair (d/dA, d/dB);
//   * digest mode: each column tile of V is contracted with the staged
//     density blocks into the four exchange images and/or the two Coulomb
//     images (LDS accumulators), which go to K' / J' with one global atomic
//     per image element at the end of the quartet.
// With one primitive quartet per shell quartet (K = 1 shells) R is built
// once and reused by every tile; contracted quartets rebuild it per tile.
#pragma once

#include "device_common.h"

namespace mderi {
namespace kx {

constexpr int kWavesMax = 4;

template <int N>
struct Tiles {
  static constexpr int value = N;
};

// Calls f(Tiles<n>) for the run-time tile count 1 <= n <= NPT.
template <int NPT, class F>
__device__ __forceinline__ void with_tiles(int n, F &f) {
  if constexpr (NPT >= 1) {
    if (n == NPT) {
      f(Tiles<NPT>{});
      return;
    }
    with_tiles<NPT - 1>(n, f);
  }
}

// Block descriptors are read-only for the kernel's lifetime: through the
// constant address space they load with scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(4))) const KxBlock ConstBlock;
typedef __attribute__((address_space(4))) const long ConstLong;
__device__ __forceinline__ long block_chunk0(const KxBlock *b, int i) { return ((ConstBlock *)b)[i].chunk0; }
__device__ __forceinline__ KxBlock block_at(const KxBlock *b, int i) { return ((ConstBlock *)b)[i]; }
__device__ __forceinline__ long pre_at(const long *p, int i) { return ((ConstLong *)p)[i]; }
#else
__device__ __forceinline__ long block_chunk0(const KxBlock *b, int i) { return b[i].chunk0; }
__device__ __forceinline__ KxBlock block_at(const KxBlock *b, int i) { return b[i]; }
__device__ __forceinline__ long pre_at(const long *p, int i) { return p[i]; }
#endif

// Per-block tables of the wave: the (u, v) list of the R builder, the cube
// offsets of the B Hermite rows (zero for padding) and of the A rows (in the
// class's row order; padding rows name valid [r] entries).
__device__ __forceinline__ void block_tables(const KxArgs &g, const KxBlock &a, uint32_t *uvsh, int *offq, int *offp,
                                             uint32_t *shp, int lane) {
  const int L = a.L;
  for (int e = lane; e < (L + 1) * (L + 2) / 2; e += 64) {
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= e) ++s;
    const int u = e - s * (s + 1) / 2, v = s - u;
    int vb = 0;
    (void)ylayout(L, v, &vb);
    uvsh[e] = (uint32_t)u | ((uint32_t)v << 8) | ((uint32_t)(vb + u) << 16);
  }
  for (int q = lane; q < ((a.NhB_pad + 15) & ~15); q += 64) {  // whole 16-row tiles
    const uint32_t h = q < a.NhB ? g.tab.herm[q] : kPadRow;
    offq[q] = (h & kPadRow) ? 0 : (int)(h & 0xff) * a.S1 + (int)((h >> 8) & 0xff) * a.S2 + (int)((h >> 16) & 0xff);
  }
  for (int r = lane; r < a.HA_rows; r += 64) {
    const uint32_t h = a.Aorder[r];
    offp[r] = (int)(h & 0xff) * a.S1 + (int)((h >> 8) & 0xff) * a.S2 + (int)((h >> 16) & 0xff);
    if (a.onev) shp[r] = a.Ashift[r];
  }
  lds_wave_sync();
}

// floor(e / d) for 0 <= e < 2^22 and 1 <= d < 2^16 from inv = fl(1/d): the
// value (e + 1/2)/d lies at least 1/(2d) from an integer and the FP32
// product carries a relative error below 2^-23, so the truncation is exact.
__device__ __forceinline__ int udiv(int e, float inv) { return (int)(((float)e + 0.5f) * inv); }

// Stages one quartet's blocks of D (digest mode) or of the weights
// (gradient mode) in dsh and clears the image accumulators; see quartet.
template <bool GRAD>
__device__ __forceinline__ void stage_quartet(const KxArgs &g, const KxBlock &a, int si, int sj, int sk, int sl,
                                              double *dsh, double *img, int lane) {
  const int na = a.na, nb = a.nb, nc = a.nc, nd = a.nd, nab = na + nb, ncd = nc + nd;
  const int oi = g.ao_off[si], oj = g.ao_off[sj], ok = g.ao_off[sk], ol = g.ao_off[sl];
  const size_t n = (size_t)g.nao;
  auto rowA = [&](int r) { return r < na ? oi + r : oj + (r - na); };
  auto colB = [&](int q) { return q < nc ? ok + q : ol + (q - nc); };
  if (!GRAD) {
    int o = 0, io = 0;
    if (g.kx) {
      // D over rows {a} u {b}, columns {c} u {d}; the exchange images
      // accumulate in img with the same layout
      for (int e = lane; e < nab * ncd; e += 64) {
        const int r = udiv(e, a.inv_ncd), q = e - r * ncd;
        dsh[e] = g.dm[(size_t)rowA(r) * n + colB(q)];
        img[e] = 0.0;
      }
      o = io = nab * ncd;
    }
    if (g.jx) {
      // D_ab (na x nb) and D_cd (nc x nd); Coulomb images over ab and cd
      for (int e = lane; e < a.NA; e += 64) {
        const int x = udiv(e, a.inv_nb);
        dsh[o + e] = g.dm[(size_t)(oi + x) * n + oj + (e - x * nb)];
        img[io + e] = 0.0;
      }
      for (int e = lane; e < a.NB; e += 64) {
        const int x = udiv(e, a.inv_nd);
        dsh[o + a.NA + e] = g.dm[(size_t)(ok + x) * n + ol + (e - x * nd)];
        img[io + a.NA + e] = 0.0;
      }
    }
    return;
  }
  const bool fi = si != sj, fk = sk != sl;
  if (g.pattern == 0) {
    // exchange weights W_abcd = Wl_ac Wr_bd: X1 = Wl and X2 = Wr over rows
    // {a} u {b} and columns {c} u {d}; X3 = Wl and X4 = Wr over rows
    // {c} u {d} and columns {a} u {b} (symmetric Wl = Wr: X1 only)
    const int m = nab * ncd;
    for (int e = lane; e < m; e += 64) {
      const int r = udiv(e, a.inv_ncd), q = e - r * ncd;
      dsh[e] = g.wl[(size_t)rowA(r) * n + colB(q)];
      if (!g.symmetric) {
        dsh[m + e] = g.wr[(size_t)rowA(r) * n + colB(q)];
        const int q2 = e / nab, r2 = e - q2 * nab;
        dsh[2 * m + e] = g.wl[(size_t)colB(q2) * n + rowA(r2)];
        dsh[3 * m + e] = g.wr[(size_t)colB(q2) * n + rowA(r2)];
      }
    }
  } else {
    // Coulomb weights W_abcd = Wl_ab Wr_cd: u1 = Wl_ab + [i!=j] Wl_ba,
    // u4 = Wr_ab + [i!=j] Wr_ba over ab; u2 = Wr_cd + [k!=l] Wr_dc,
    // u3 = Wl_cd + [k!=l] Wl_dc over cd
    const int NA = a.NA, NB = a.NB;
    double *u1 = dsh, *u4 = dsh + NA, *u2 = dsh + 2 * NA, *u3 = dsh + 2 * NA + NB;
    for (int e = lane; e < NA; e += 64) {
      const int x = udiv(e, a.inv_nb), y = e - x * nb;
      const size_t f = (size_t)(oi + x) * n + oj + y, r = (size_t)(oj + y) * n + oi + x;
      u1[e] = g.wl[f] + (fi ? g.wl[r] : 0.0);
      u4[e] = g.wr[f] + (fi ? g.wr[r] : 0.0);
    }
    for (int e = lane; e < NB; e += 64) {
      const int x = udiv(e, a.inv_nd), y = e - x * nd;
      const size_t f = (size_t)(ok + x) * n + ol + y, r = (size_t)(ol + y) * n + ok + x;
      u2[e] = g.wr[f] + (fk ? g.wr[r] : 0.0);
      u3[e] = g.wl[f] + (fk ? g.wl[r] : 0.0);
    }
  }
}

// Gradient weights of one B column tile, S[ab][16 ct + cl] into
// v[ab * 16 + cl] (zero outside NA x NB), from the staged blocks: the summed
// weights of every ordering of the four shells that maps onto this visit,
// S = Wbar(A,B)[ab][cd] + Wbar(B,A)[cd][ab], with Wbar(A,B) collecting the
// orderings (ab|cd), (ba|cd), (ab|dc), (ba|dc) of distinct shells.
__device__ __forceinline__ void grad_weights(const KxArgs &g, const KxBlock &a, int si, int sj, int sk, int sl, int ct,
                                             double wscale, const double *dsh, double *v, int lane) {
  const int na = a.na, nb = a.nb, nc = a.nc, nd = a.nd, nab = na + nb, ncd = nc + nd;
  const int NA = a.NA, NB = a.NB;
  const double ffi = si != sj ? 1.0 : 0.0, ffk = sk != sl ? 1.0 : 0.0;
  for (int e = lane; e < a.NA_pad * 16; e += 64) {
    const int ab = e >> 4, cd = ct * 16 + (e & 15);
    double s = 0.0;
    if (ab < NA && cd < NB) {
      if (g.pattern == 0) {
        const int m = nab * ncd;
        const double *X1 = dsh, *X2 = g.symmetric ? dsh : dsh + m;
        const int x = udiv(ab, a.inv_nb), y = ab - x * nb, cc = udiv(cd, a.inv_nd), dd = cd - cc * nd;
        const int ra = x, rb = na + y, qc = cc, qd = nc + dd;
        s = X1[ra * ncd + qc] * X2[rb * ncd + qd];
        s = fma(ffi * X1[rb * ncd + qc], X2[ra * ncd + qd], s);
        s = fma(ffk * X1[ra * ncd + qd], X2[rb * ncd + qc], s);
        s = fma(ffi * ffk * X1[rb * ncd + qd], X2[ra * ncd + qc], s);
        if (g.symmetric) {
          s *= 2.0;  // Wbar(B,A)[cd][ab] = Wbar(A,B)[ab][cd] when Wl = Wr is symmetric
        } else {
          const double *X3 = dsh + 2 * m, *X4 = dsh + 3 * m;
          s = fma(X3[qc * nab + ra], X4[qd * nab + rb], s);
          s = fma(ffk * X3[qd * nab + ra], X4[qc * nab + rb], s);
          s = fma(ffi * X3[qc * nab + rb], X4[qd * nab + ra], s);
          s = fma(ffi * ffk * X3[qd * nab + rb], X4[qc * nab + ra], s);
        }
      } else {
        const double *u1 = dsh, *u4 = dsh + NA, *u2 = dsh + 2 * NA, *u3 = dsh + 2 * NA + NB;
        s = fma(u1[ab], u2[cd], u3[cd] * u4[ab]);
      }
    }
    v[e] = wscale * s;
  }
}

// Digest (digest mode).  Exchange: with K_ac = sum_bd (ab|cd) D_bd the
// permutations of a unique quartet give
//   K_ac += v D_bd, K_bc += v D_ad, K_ad += v D_bc, K_bd += v D_ac
// and their transposes (added once at the end, K = K' + K'^T); a quartet
// stands for its whole permutation orbit, so every image carries
// w = 2^-(#coincidences among i=j, k=l, ij=kl).  Coulomb: J_ab +=
// (1 + [k!=l]) sum_cd v D_cd into block (i, j) and J_cd += (1 + [i!=j])
// sum_ab v D_ab into block (k, l) (skipped when ij = kl), halved on a
// diagonal shell block because J = J' + J'^T doubles it.
// digest_tile: every lane takes elements of one B column tile of the
// shellset, v[ab * 16 + cl] = (ab|cd), cd = 16 ct + cl, and adds their
// contributions to the images in LDS (atomic LDS adds).
__device__ __forceinline__ void digest_tile(const KxArgs &g, const KxBlock &a, int ct, const double *v,
                                            const double *dsh, double *img, int lane) {
  const int na = a.na, nb = a.nb, nc = a.nc, nd = a.nd, nab = na + nb, ncd = nc + nd, NA = a.NA, NB = a.NB;
  const int ko = g.kx ? nab * ncd : 0;  // offset of the Coulomb blocks / images
  const double *dab = dsh + ko, *dcd = dsh + ko + NA;
  double *jab = img + ko, *jcd = img + ko + NA;
  for (int e = lane; e < NA * 16; e += 64) {
    const int ab = e >> 4, cd = ct * 16 + (e & 15);
    if (cd >= NB) continue;
    const double x = v[e];
    if (g.kx) {
      const int xa = udiv(ab, a.inv_nb), yb = ab - xa * nb, cc = udiv(cd, a.inv_nd), dd = cd - cc * nd;
      const int ra = xa * ncd, rb = (na + yb) * ncd, qc = cc, qd = nc + dd;
      atomicAdd(&img[ra + qc], x * dsh[rb + qd]);  // K_ac += v D_bd
      atomicAdd(&img[rb + qc], x * dsh[ra + qd]);  // K_bc += v D_ad
      atomicAdd(&img[ra + qd], x * dsh[rb + qc]);  // K_ad += v D_bc
      atomicAdd(&img[rb + qd], x * dsh[ra + qc]);  // K_bd += v D_ac
    }
    if (g.jx) {
      atomicAdd(&jab[ab], x * dcd[cd]);
      atomicAdd(&jcd[cd], x * dab[ab]);
    }
  }
}

// Adds v to element e of a K' / J' matrix: an FP64 atomic, or in the
// deterministic mode v * sc as the fixed-point pair (floor, rounded fraction
// 2^32) by two 64-bit integer atomics (pairs that are zero are skipped).
__device__ __forceinline__ void image_add(double *m, size_t e, double v, bool fixed, double sc) {
  if (!fixed) {
    atomicAdd(&m[e], v);
    return;
  }
  const double y = v * sc, h = floor(y);
  const long long hi = (long long)h, lo = (long long)rint((y - h) * 0x1p32);
  unsigned long long *p = (unsigned long long *)m + 2 * e;
  if (hi) atomicAdd(p, (unsigned long long)hi);
  if (lo) atomicAdd(p + 1, (unsigned long long)lo);
}

// Adds v to element e of the wave's gradient copy: an FP64 atomic, or in the
// deterministic mode |v| 2^80 as four 32-bit digits (weights 2^(32 k - 80),
// k = 0..3: |v| < 2^47 in steps of 2^-80), each added with v's sign to its
// own 64-bit word by an integer atomic; integer sums do not depend on the
// order of the adds (digits that are zero are skipped).
__device__ __forceinline__ void grad_add(const KxArgs &g, size_t e, double v) {
  if (!g.gfixed) {
    atomicAdd(&g.grad[e], v);
    return;
  }
  unsigned long long *p = (unsigned long long *)g.grad + 4 * e;
  const double t = fabs(v) * 0x1p-16;
  const double d3 = floor(t);
  double r = (t - d3) * 0x1p32;  // exact: 0 <= t - d3 < 1
  const double d2 = floor(r);
  r = (r - d2) * 0x1p32;
  const double d1 = floor(r);
  r = (r - d1) * 0x1p32;
  const double d0 = rint(r);
  const long long sg = v < 0.0 ? -1 : 1;
  if (d3 != 0.0) atomicAdd(p + 3, (unsigned long long)(sg * (long long)d3));
  if (d2 != 0.0) atomicAdd(p + 2, (unsigned long long)(sg * (long long)d2));
  if (d1 != 0.0) atomicAdd(p + 1, (unsigned long long)(sg * (long long)d1));
  if (d0 != 0.0) atomicAdd(p, (unsigned long long)(sg * (long long)d0));
}

// The images of one quartet into K' / J' (one global atomic per element).
__device__ __forceinline__ void digest_flush(const KxArgs &g, const KxBlock &a, int i, int k, int si, int sj, int sk,
                                             int sl, const double *img, int lane) {
  const int na = a.na, nb = a.nb, nc = a.nc, nd = a.nd, nab = na + nb, ncd = nc + nd, NA = a.NA, NB = a.NB;
  const int oi = g.ao_off[si], oj = g.ao_off[sj], ok = g.ao_off[sk], ol = g.ao_off[sl];
  const size_t n = (size_t)g.nao;
  const bool same_pair = a.same && i == k;
  const int ko = g.kx ? nab * ncd : 0;
  const bool fixed = g.fixed != 0;
  const double sc = fixed ? g.fscale[0] : 1.0;
  if (g.kx) {
    const int neq = (si == sj) + (sk == sl) + (same_pair ? 1 : 0);
    const double w = neq == 0 ? 1.0 : neq == 1 ? 0.5 : neq == 2 ? 0.25 : 0.125;
    for (int o = lane; o < nab * ncd; o += 64) {
      const int r = udiv(o, a.inv_ncd), q = o - r * ncd;
      const int row = r < na ? oi + r : oj + (r - na), col = q < nc ? ok + q : ol + (q - nc);
      image_add(g.kx, (size_t)row * n + col, w * img[o], fixed, sc);
    }
  }
  if (g.jx) {
    const double wb = ((sk != sl) ? 2.0 : 1.0) * ((si == sj) ? 0.5 : 1.0);
    const double wk = ((si != sj) ? 2.0 : 1.0) * ((sk == sl) ? 0.5 : 1.0);
    for (int ab = lane; ab < NA; ab += 64) {
      const int x = udiv(ab, a.inv_nb);
      image_add(g.jx, (size_t)(oi + x) * n + oj + (ab - x * nb), wb * img[ko + ab], fixed, sc);
    }
    if (!same_pair)
      for (int cd = lane; cd < NB; cd += 64) {
        const int x = udiv(cd, a.inv_nd);
        image_add(g.jx, (size_t)(ok + x) * n + ol + (cd - x * nd), wk * img[ko + NA + cd], fixed, sc);
      }
  }
}

constexpr int kBufferWord3 = 0x00020000;  // buffer resource word 3 for gfx9-family raw loads

// Derivative contraction of the gradient: gpart[m] += sum_p,ab H^(m0+m)[p][ab]
// Y[p][ab], m < NM, over one 16 x 16 tile of Y^T (register r of lane c + 16 g
// holds Y^T[ab = 16 at + 4 r + g][p = row c of the tile]); the matrices are
// stored transposed, [ab][p].  They are read by buffer loads: the lane's
// part of the offset (vo, bytes) in a VGPR, the (matrix, row) part in an
// SGPR, so no per-element addresses stay live.
template <int NM>
__device__ __forceinline__ void grad_dots(__amdgpu_buffer_rsrc_t hrs, int vo, int mstride, int HA_rows, int m0,
                                          const d4 &y, double (&gpart)[6]) {
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int so = 8 * ((m0 + m) * mstride + 4 * r * HA_rows);
      const double h = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(hrs, vo, so, 0));
      gpart[m] = fma(y[r], h, gpart[m]);
    }
}

// One shell quartet (A pair i, B pair k) by one wave.
template <int NRT, int LM, int MODE>
__device__ __forceinline__ void quartet(const KxArgs &g, const KxBlock &a, int i, int k, double *base,
                                        const uint32_t *uvsh, const int *offq, const int *offp, const uint32_t *shp,
                                        const YLanes<LM> &yl, double (&gpart)[6], double (&dpa)[3]) {
  constexpr bool GRAD = MODE == 1;
  const int lane = threadIdx.x & 63, gq = lane >> 4, c = lane & 15;
  double *cube = base, *work = base + g.o_work, *vsh = base + g.o_v, *dsh = base + g.o_d, *img = base + g.o_img;
  double *gsh = base + g.o_g;
  const int ap0 = a.A_off[i], nap = a.A_off[i + 1] - ap0;
  const int bp0 = a.B_off[k], nbp = a.B_off[k + 1] - bp0;
  const int nsteps = nap * nbp;
  const int si = a.A_sh[2 * i], sj = a.A_sh[2 * i + 1], sk = a.B_sh[2 * k], sl = a.B_sh[2 * k + 1];
  for (int e = lane; e < 4 * nap; e += 64) gsh[e] = a.A_G[4 * (size_t)ap0 + e];
  for (int e = lane; e < 4 * nbp; e += 64) gsh[4 * nap + e] = a.B_G[4 * (size_t)bp0 + e];
  stage_quartet<GRAD>(g, a, si, sj, sk, sl, dsh, img, lane);
  lds_wave_sync();

  auto build = [&](int ia, int ib) {
    const double *Ga = gsh + 4 * ia, *Gb = gsh + 4 * (nap + ib);
    const double P[3] = {Ga[1], Ga[2], Ga[3]};
    const double Q[3] = {Gb[1], Gb[2], Gb[3]};
    build_R_chains<LM>(a.L, Ga[0], P, Gb[0], Q, cube, a.S1, a.S2, work, uvsh, g.tab.boys, lane, yl);
  };
  // single-step quartets build R once; v (one column tile of V or of the
  // weights) may then share the builder's work area, which is free after it
  if (nsteps == 1) build(0, 0);

  const int nks = a.NhB_pad >> 2;
  const int ntiles = (a.NhA + 15) >> 4;
  const int nat = a.NA_pad >> 4;
  double rq[3] = {0.0, 0.0, 0.0};  // one-visit: derivative along C - D of the B pair
  double dp[3] = {0.0, 0.0, 0.0};  // one-visit: derivative along P (the A pair moved as a whole)
  // S is the weight of (ab|cd) summed over both assignments of the two
  // pairs; a one-visit quartet whose two pairs are the same pair takes all
  // four centres' derivatives of an integral that appears once, so half
  const double wscale = (GRAD && a.onev && a.same && i == k) ? 0.5 * g.scale : g.scale;
  for (int ct = 0; ct < a.nct; ++ct) {
    const int col = ct * 16 + c;  // this lane's B column cd
    if (GRAD) grad_weights(g, a, si, sj, sk, sl, ct, wscale, dsh, vsh, lane);
    else
      for (int e = lane; e < a.NA_pad * 16; e += 64) vsh[e] = 0.0;
    lds_wave_sync();
    for (int part = 0; part < a.nparts; ++part) {
      const int t0 = part * NRT;
      const int ntw = min(NRT, ntiles - t0);
      int op[NRT];
#pragma unroll
      for (int pt = 0; pt < NRT; ++pt) op[pt] = offp[(t0 + pt) * 16 + c];
      for (int ia = 0; ia < nap; ++ia) {
        d4 xacc[NRT];
#pragma unroll
        for (int pt = 0; pt < NRT; ++pt) xacc[pt] = d4{0.0, 0.0, 0.0, 0.0};
        for (int ib = 0; ib < nbp; ++ib) {
          if (nsteps > 1) {
            lds_wave_sync();  // the previous step's gathers are done with the cube
            build(ia, ib);
          }
          const double *Hk = a.B_H + (size_t)(bp0 + ib) * a.B_mats * a.NhB_pad * a.NB_pad + col;
          // X[p][cd] += sum_q [p+q] H_B[q][cd] in blocks of four k-steps:
          // the H_B values of the next block are loaded before this block's
          // gathers and products (indices clamped, so every load is
          // unconditional; the steps past nks are skipped)
          auto hload = [&](int ks) { return Hk[(size_t)(4 * min(ks, nks - 1) + gq) * a.NB_pad]; };
          auto ket = [&](auto ntc) {
            constexpr int NT = decltype(ntc)::value;
            double h[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) h[j] = hload(j);
#pragma unroll 1
            for (int k0 = 0; k0 < nks; k0 += 4) {
              double hn[4];
#pragma unroll
              for (int j = 0; j < 4; ++j) hn[j] = hload(k0 + 4 + j);
              int oq[4];
#pragma unroll
              for (int j = 0; j < 4; ++j) oq[j] = offq[4 * min(k0 + j, nks - 1) + gq];
              double av[4][NT];
#pragma unroll
              for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int pt = 0; pt < NT; ++pt) av[j][pt] = cube[op[pt] + oq[j]];
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (k0 + j < nks) {
#pragma unroll
                  for (int pt = 0; pt < NT; ++pt)
                    xacc[pt] = GRAD ? mfma16x16x4(h[j], av[j][pt], xacc[pt]) : mfma16x16x4(av[j][pt], h[j], xacc[pt]);
                }
#pragma unroll
              for (int j = 0; j < 4; ++j) h[j] = hn[j];
            }
          };
          with_tiles<NRT>(ntw, ket);
        }
        if constexpr (!GRAD) {
          // V[ab][cd] += sum_p H_A[p][ab] X[p][cd]: X's accumulator layout
          // is the B operand (rows 4r+g of a tile in register r)
          const double *Hb = a.A_H + (size_t)(ap0 + ia) * a.HA_rows * a.NA_pad + (size_t)t0 * 16 * a.NA_pad +
                             (size_t)gq * a.NA_pad + c;
          auto bra = [&](auto ntc) {
            constexpr int NT = decltype(ntc)::value;
#pragma unroll 1
            for (int at = 0; at < nat; ++at) {
              const double *Ht = Hb + at * 16;
              d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int pt = 0; pt < NT; ++pt) {
                double h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) h[r] = Ht[(size_t)(pt * 16 + 4 * r) * a.NA_pad];
                acc0 = mfma16x16x4(h[0], xacc[pt][0], acc0);
                acc1 = mfma16x16x4(h[1], xacc[pt][1], acc1);
                acc0 = mfma16x16x4(h[2], xacc[pt][2], acc0);
                acc1 = mfma16x16x4(h[3], xacc[pt][3], acc1);
              }
#pragma unroll
              for (int r = 0; r < 4; ++r) vsh[(at * 16 + 4 * r + gq) * 16 + c] += acc0[r] + acc1[r];
            }
          };
          with_tiles<NRT>(ntw, bra);
        } else {
          // X is held transposed: register r of lane c + 16 g holds
          // X^T[cd = 16 ct + 4 r + g][p = row c of tile pt].  With Y = X S^T
          // the weighted derivative sum_ab,cd S[ab][cd] sum_p H^(m)[p][ab]
          // X[p][cd] is sum_p,ab H^(m)[p][ab] Y[p][ab]: Y^T = S X^T over the
          // tile's 16 columns on the matrix cores, then six dot products
          // with the derivative matrices ([m][ab][p], p fastest).  In
          // accumulating blocks Y^T adds into the wave's LDS accumulator
          // instead and the dot products wait for the end of the A pair's run.
          const int mstride = a.HA_rows * a.NA_pad;  // doubles per derivative matrix
          if (a.onev) {
            // X^T of this part for the one-visit d/dP (row p at p * 17)
            double *xs = base + g.o_x;
#pragma unroll
            for (int pt = 0; pt < NRT; ++pt)
#pragma unroll
              for (int r = 0; r < 4; ++r) xs[((t0 + pt) * 16 + c) * 17 + 4 * r + gq] = xacc[pt][r];
          }
          if (a.yacc) {
            // tile (p tile t, ab tile at) of primitive pair ia at
            // ((ia ntA + t) nat + at) 256, register r of every lane at r 64 + lane
            double *yb = base + g.o_y + (size_t)ia * (a.HA_rows >> 4) * nat * 256 + lane;
            auto gry = [&](auto ntc) {
              constexpr int NT = decltype(ntc)::value;
#pragma unroll 1
              for (int at = 0; at < nat; ++at) {
                double w[4];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) w[s4] = vsh[(at * 16 + c) * 16 + gq + 4 * s4];
#pragma unroll
                for (int pt = 0; pt < NT; ++pt) {
                  double *yt = yb + ((t0 + pt) * nat + at) * 256;
                  d4 y = d4{yt[0], yt[64], yt[128], yt[192]};
#pragma unroll
                  for (int s4 = 0; s4 < 4; ++s4) y = mfma16x16x4(w[s4], xacc[pt][s4], y);
#pragma unroll
                  for (int r = 0; r < 4; ++r) yt[64 * r] = y[r];
                }
              }
            };
            with_tiles<NRT>(ntw, gry);
          } else {
            const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.A_H + (size_t)(ap0 + ia) * a.A_mats * mstride), (short)0, a.A_mats * mstride * 8,
                kBufferWord3);
            auto grd = [&](auto ntc) {
              constexpr int NT = decltype(ntc)::value;
#pragma unroll 1
              for (int at = 0; at < nat; ++at) {
                double w[4];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) w[s4] = vsh[(at * 16 + c) * 16 + gq + 4 * s4];
                // this lane's element of the [m][ab][p] matrices: ab = 16 at + g
                // (+ 4 r), p = 16 (t0 + pt) + c
                const int vo = 8 * ((at * 16 + gq) * a.HA_rows + t0 * 16 + c);
#pragma unroll
                for (int pt = 0; pt < NT; ++pt) {
                  d4 y = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                  for (int s4 = 0; s4 < 4; ++s4) y = mfma16x16x4(w[s4], xacc[pt][s4], y);
                  // y[r] = Y^T[ab = 16 at + 4 r + g][p = row c of tile pt]; one-visit
                  // blocks take the relative coordinate A - B (d/dP comes with d/dQ)
                  if (a.onev) grad_dots<3>(hrs, vo + 8 * 16 * pt, mstride, a.HA_rows, a.A_rel, y, gpart);
                  else grad_dots<6>(hrs, vo + 8 * 16 * pt, mstride, a.HA_rows, 0, y, gpart);
                }
              }
            };
            with_tiles<NRT>(ntw, grd);
          }
        }
      }
    }
    if (GRAD && a.onev) {
      // B-pair centres (one-visit blocks, single primitives): with
      // T[p][cd] = sum_ab H_A[p][ab] S[ab][cd] and Z[q][cd] =
      // sum_p [p+q] T[p][cd], the derivative of sum S (ab|cd) along the
      // relative coordinate C - D of the B pair is
      // sum_q,cd dH_B/d(C-D)[q][cd] Z[q][cd], and along P (the A pair moved
      // as a whole, d/dP [p+q] = [p+e+q]) it is sum_p,cd T[p][cd] X[p+e][cd];
      // T stays in the accumulator layout, which is Z's B operand
      lds_wave_sync();  // X^T of every part staged
      const int mstride = a.HA_rows * a.NA_pad;
      const double *Ha = a.A_H + ((size_t)ap0 * a.A_mats + a.A_plain) * mstride;
      const int mB = a.NhB_pad * a.NB_pad;
      const double *Hr = a.B_H + (size_t)bp0 * a.B_mats * mB + mB;  // the three d/d(C-D) matrices
      const double *xs = base + g.o_x;
      for (int part = 0; part < a.nparts; ++part) {
        const int t0 = part * NRT;
        const int ntw = min(NRT, ntiles - t0);
        auto zb = [&](auto ntc) {
          constexpr int NT = decltype(ntc)::value;
          d4 T[NT];
#pragma unroll
          for (int pt = 0; pt < NT; ++pt) T[pt] = d4{0.0, 0.0, 0.0, 0.0};
          // four k-steps per pass: the H_A loads of a pass are issued together
#pragma unroll 1
          for (int k4 = 0; k4 < (a.NA_pad >> 2); k4 += 4) {
            double ha[4][NT], sb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int ks = k4 + j;  // NA_pad is a multiple of 16: ks < NA_pad / 4
              sb[j] = vsh[(4 * ks + gq) * 16 + c];  // B[k = ab][j = cd] = S[4 ks + k][16 ct + j]
#pragma unroll
              for (int pt = 0; pt < NT; ++pt)
                ha[j][pt] = Ha[(size_t)((t0 + pt) * 16 + c) * a.NA_pad + 4 * ks + gq];  // A[i = p][k = ab]
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int pt = 0; pt < NT; ++pt) T[pt] = mfma16x16x4(ha[j][pt], sb[j], T[pt]);
          }
          // T[pt][r] = T[p = 16 (t0 + pt) + 4 r + g][cd = 16 ct + c]
#pragma unroll
          for (int pt = 0; pt < NT; ++pt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint32_t sh = shp[(t0 + pt) * 16 + 4 * r + gq];
              dp[0] = fma(T[pt][r], xs[(int)(sh & 1023u) * 17 + c], dp[0]);
              dp[1] = fma(T[pt][r], xs[(int)((sh >> 10) & 1023u) * 17 + c], dp[1]);
              dp[2] = fma(T[pt][r], xs[(int)((sh >> 20) & 1023u) * 17 + c], dp[2]);
            }
#pragma unroll 1
          for (int qt = 0; qt < (a.NhB_pad + 15) >> 4; ++qt) {
            // the tile's d/d(C-D) elements are loaded before its products
            // (rows past NhB_pad read row 0 and are dropped)
            double hr[4][3];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int q = qt * 16 + 4 * r + gq;
              const size_t o = (size_t)(q < a.NhB_pad ? q : 0) * a.NB_pad + col;
#pragma unroll
              for (int x = 0; x < 3; ++x) hr[r][x] = q < a.NhB_pad ? Hr[x * (size_t)mB + o] : 0.0;
            }
            const int oqr = offq[qt * 16 + c];
            d4 z = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int pt = 0; pt < NT; ++pt)
#pragma unroll
              for (int r = 0; r < 4; ++r) z = mfma16x16x4(cube[oqr + offp[(t0 + pt) * 16 + 4 * r + gq]], T[pt][r], z);
            // z[r] = Z[q = 16 qt + 4 r + g][cd = 16 ct + c]
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int x = 0; x < 3; ++x) rq[x] = fma(z[r], hr[r][x], rq[x]);
          }
        };
        with_tiles<NRT>(ntw, zb);
      }
    }
    if (!GRAD) {
      lds_wave_sync();
      digest_tile(g, a, ct, vsh, dsh, img, lane);
    }
    lds_wave_sync();  // the next tile overwrites v
  }
  if constexpr (!GRAD) digest_flush(g, a, i, k, si, sj, sk, sl, img, lane);
  if (GRAD && a.onev) {
    // the B pair's centres of this quartet: d/dQ = -d/dP (R depends on
    // P - Q only), split as d/dC = (zeta_c/q) d/dQ + d/d(C-D) and d/dD =
    // (zeta_d/q) d/dQ - d/d(C-D); d/dP adds to the A pair's run (its split
    // needs only the A pair's exponents)
    double v[6] = {dp[0], dp[1], dp[2], rq[0], rq[1], rq[2]};
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[m] += __shfl_xor(v[m], off);
#pragma unroll
    for (int x = 0; x < 3; ++x) dpa[x] += v[x];
    if (lane < 6) {
      const int x = lane % 3;
      double P = v[0], r = v[3];
#pragma unroll
      for (int y = 1; y < 3; ++y)
        if (x == y) {
          P = v[y];
          r = v[3 + y];
        }
      const PrimPair pr = a.B_pp[bp0];
      const double zc = g.exps[pr.pa], zd = g.exps[pr.pb], dq = -P;
      const double val = lane < 3 ? fma(zc / (zc + zd), dq, r) : fma(zd / (zc + zd), dq, -r);
      grad_add(g, (size_t)(blockIdx.x % g.gcopies) * g.gstride + 3 * g.atom[lane < 3 ? sk : sl] + x, val);
    }
  }
  lds_wave_sync();  // the next quartet may overwrite the wave's LDS
}

// Adds the wave's partial derivatives of the A pair's two centres to its
// gradient copy and clears them.
__device__ __forceinline__ void flush_grad(const KxArgs &g, int si, int sj, double (&gpart)[6], int lane) {
  double tot[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double x = gpart[m];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    tot[m] = x;
    gpart[m] = 0.0;
  }
  if (lane < 6) {
    double val = tot[0];
#pragma unroll
    for (int m = 1; m < 6; ++m)
      if (lane == m) val = tot[m];
    const int at = g.atom[lane < 3 ? si : sj];
    grad_add(g, (size_t)(blockIdx.x % g.gcopies) * g.gstride + 3 * at + (lane % 3), val);
  }
}

// End of an A pair's run of quartets (gradient mode): the accumulated Y
// (accumulating blocks) meets the derivative matrices of every primitive
// pair of A pair i (the six centre derivatives, or the three along A - B in
// one-visit blocks), then the derivatives of the pair's two centres go to
// the gradient copy; the accumulators are left at zero.
__device__ __forceinline__ void flush_run(const KxArgs &g, const KxBlock &a, int i, double *ybase,
                                          double (&gpart)[6], double (&dpa)[3], int lane) {
  if (a.yacc) {
    const int gq = lane >> 4, c = lane & 15;
    const int ap0 = a.A_off[i], nap = a.A_off[i + 1] - ap0;
    const int ntiles = (a.NhA + 15) >> 4, nat = a.NA_pad >> 4, ntA = a.HA_rows >> 4;
    const int mstride = a.HA_rows * a.NA_pad;
    for (int ia = 0; ia < nap; ++ia) {
      const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(a.A_H + (size_t)(ap0 + ia) * a.A_mats * mstride), (short)0, a.A_mats * mstride * 8, kBufferWord3);
#pragma unroll 1
      for (int t = 0; t < ntiles; ++t)
#pragma unroll 1
        for (int at = 0; at < nat; ++at) {
          double *yt = ybase + ((ia * ntA + t) * nat + at) * 256 + lane;
          const d4 y = d4{yt[0], yt[64], yt[128], yt[192]};
#pragma unroll
          for (int r = 0; r < 4; ++r) yt[64 * r] = 0.0;
          const int vo = 8 * ((at * 16 + gq) * a.HA_rows + t * 16 + c);
          if (a.onev) grad_dots<3>(hrs, vo, mstride, a.HA_rows, a.A_rel, y, gpart);
          else grad_dots<6>(hrs, vo, mstride, a.HA_rows, 0, y, gpart);
        }
    }
  }
  const int si = a.A_sh[2 * i], sj = a.A_sh[2 * i + 1];
  if (!a.onev) {
    flush_grad(g, si, sj, gpart, lane);
    return;
  }
  // one-visit (single primitive pair): d/dA = (zeta_a/p) d/dP + d/d(A-B),
  // d/dB = (zeta_b/p) d/dP - d/d(A-B); dpa holds the run's d/dP (the same in
  // every lane), gpart[0..2] the lanes' parts of d/d(A-B)
  double r3[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    double v = gpart[x];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    r3[x] = v;
  }
  if (lane < 6) {
    const int x = lane % 3;
    double P = dpa[0], r = r3[0];
#pragma unroll
    for (int y = 1; y < 3; ++y)
      if (x == y) {
        P = dpa[y];
        r = r3[y];
      }
    const PrimPair pr = a.A_pp[a.A_off[i]];
    const double za = g.exps[pr.pa], zb = g.exps[pr.pb];
    const double val = lane < 3 ? fma(za / (za + zb), P, r) : fma(zb / (za + zb), P, -r);
    grad_add(g, (size_t)(blockIdx.x % g.gcopies) * g.gstride + 3 * g.atom[lane < 3 ? si : sj] + x, val);
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) gpart[m] = 0.0;
#pragma unroll
  for (int x = 0; x < 3; ++x) dpa[x] = 0.0;
}

template <int NRT, int LM, int MODE>
__global__ void __launch_bounds__(64 * kWavesMax, 2) kx_kernel(KxArgs g) {
  constexpr bool GRAD = MODE == 1;
  extern __shared__ double smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *base = smem + (size_t)wave * g.wave_doubles;
  uint32_t *uvsh = (uint32_t *)(base + g.o_tab);
  int *offq = (int *)(uvsh + g.uv_max);
  int *offp = offq + g.oq_max;
  uint32_t *shp = (uint32_t *)(offp + g.op_max);
  double *ybase = base + g.o_y;
  int cur = -1;
  KxBlock a{};
  YLanes<LM> yl;
  double gpart[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double dpa[3] = {0.0, 0.0, 0.0};
  int yi = -1;  // A pair (of block cur) whose run the wave's Y and gpart hold
  if (GRAD) {
    for (int e = lane; e < g.o_x - g.o_y; e += 64) ybase[e] = 0.0;
  }
  for (;;) {
    unsigned long long ch = 0;
    if (lane == 0) ch = atomicAdd(g.counter, 1ull);
    const unsigned lo32 = __builtin_amdgcn_readfirstlane((unsigned)(ch & 0xffffffffu));
    const unsigned hi32 = __builtin_amdgcn_readfirstlane((unsigned)(ch >> 32));
    const long chunk = (long)(((unsigned long long)hi32 << 32) | lo32);
    if (chunk >= g.nchunk) break;
    int lo = 0, hi = g.nblk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (block_chunk0(g.blocks, mid) <= chunk) lo = mid;
      else hi = mid - 1;
    }
    if (lo != cur) {
      if (GRAD && yi >= 0) {
        flush_run(g, a, yi, ybase, gpart, dpa, lane);
        yi = -1;
      }
      a = block_at(g.blocks, lo);
      cur = lo;
      block_tables(g, a, uvsh, offq, offp, shp, lane);
      if constexpr (LM <= 18) ylanes_init<LM>(a.L, lane, yl);
    }
    long q = (chunk - a.chunk0) * (long)a.chunk;
    const long qend = min(q + (long)a.chunk, a.nq);
    int i0 = 0, i1 = a.nA - 1;  // the A pair holding quartet q: last i with pre[i] <= q
    while (i0 < i1) {
      const int mid = (i0 + i1 + 1) >> 1;
      if (pre_at(a.pre, mid) <= q) i0 = mid;
      else i1 = mid - 1;
    }
    int i = i0;
    long pend = pre_at(a.pre, i + 1);
    int k = (int)(q - pre_at(a.pre, i));
    for (; q < qend; ++q) {
      if (GRAD && i != yi) {
        if (yi >= 0) flush_run(g, a, yi, ybase, gpart, dpa, lane);
        yi = i;
      }
      quartet<NRT, LM, MODE>(g, a, i, k, base, uvsh, offq, offp, shp, yl, gpart, dpa);
      ++k;
      if (q + 1 == pend && q + 1 < qend) {  // next A pair that has quartets
        do {
          ++i;
          pend = pre_at(a.pre, i + 1);
        } while (pend == q + 1);
        k = 0;
      }
    }
  }
  if (GRAD && yi >= 0) flush_run(g, a, yi, ybase, gpart, dpa, lane);
}

template <int NRT, int LM, int MODE>
hipError_t launch_t(const KxArgs &a, int waves, size_t lds, int grid, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)kx_kernel<NRT, LM, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((kx_kernel<NRT, LM, MODE>), dim3((unsigned)grid), dim3(64 * waves), lds, s, a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const KxArgs &a, int npt, int Lmax, int waves, size_t lds, int grid, hipStream_t s) {
  const int lm = rr_lm_bucket(Lmax);
#define KX_CASE(NRT, LM) \
  if (npt == NRT && lm == LM) return launch_t<NRT, LM, MODE>(a, waves, lds, grid, s);
  KX_CASE(1, 8) KX_CASE(2, 8)
  KX_CASE(1, 10) KX_CASE(2, 10)
  KX_CASE(1, 16) KX_CASE(2, 16)
  KX_CASE(1, 18) KX_CASE(2, 18)
  if constexpr (MODE == 0) {  // the gradient plans at most two row tiles per part
    KX_CASE(4, 8) KX_CASE(4, 10) KX_CASE(4, 16) KX_CASE(4, 18)
  }
#undef KX_CASE
  return hipErrorInvalidValue;
}

}  // namespace kx
}  // namespace mderi
