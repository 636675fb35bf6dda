// eri4.hip -- fused 4-centre MD kernel on the FP64 matrix cores.
//
// One workgroup evaluates one shell quartet (ij, kl).  It runs
//   * one producer wave that builds [r]^(0) (Eqs. (0m), (r)) for the primitive
//     quartets one after another into a double-buffered LDS cube, one quartet
//     ahead of the consumers, and
//   * nct * nps consumer waves: each owns the 16 ket components cd in
//     [16 ct, 16 ct + 16) of one column tile ct and the bra Hermite rows p of
//     one part (up to npt 16-row tiles).  Waves run on SIMD (wave mod 4), and
//     on MI355X a wave that issues FP64 MFMAs back to back holds off every
//     VALU instruction of the other waves of its SIMD, so the parts with the
//     fewest tiles go to the producer's SIMD (eri4_fill_wtask).
// For each bra primitive pair a consumer computes
//   X[p][cd]  = sum_{ket prims} sum_q [p|q] H_ket[q][cd]        Eq. (ket-from-hermite)
//   V[ab][cd] += sum_p H_bra[p][ab] X[p][cd]                      Eq. (bra-from-hermite)
// with [p|q] = (-1)^{|q|} [p+q]^(0) (Eq. (pq); the sign lives in H_ket)
// gathered straight from the LDS cube as the A operand of a 16x16x4 FP64
// MFMA, so the Ñ_bra x Ñ_ket matrix [p|q] is never stored.  X stays in
// registers: the accumulator tile of the ket step is exactly the B operand of
// the bra step (rows 4r..4r+3 of a 16-row tile sit in register r), so the two
// transforms are chained without leaving the wave.  The bra step runs one
// 16-row ab tile at a time and adds it into an LDS copy of V[ab][cd]
// (FP64 LDS atomics, since the nps row parts share columns), which is written
// to V[ij,ab,cd,kl] (Sec. 3, ij fastest) at the end; with one row part and
// single-primitive bra pairs a wave holds complete elements and stores them
// from registers (vdirect).
// Quartet runs: when every pair has one primitive pair, a quartet is a single
// step, so the producer would have nothing to build ahead; a workgroup then
// takes nrun quartets (ij, kl0 + m) in a row as its steps, and the producer
// builds quartet m+1's [r] while the consumers transform quartet m.
#include <algorithm>
#include <vector>

#include "device_common.h"

namespace mderi {

namespace {

constexpr int kMaxWaves = kMaxWavesArgs;
constexpr int kBufferWord3 = 0x00020000;  // buffer resource word 3 for gfx9-family raw loads

template <int N>
struct Tiles {
  static constexpr int value = N;
};

// Calls f(Tiles<n>) for the run-time tile count 1 <= n <= NPT (nothing for 0).
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

// One shell quartet (ij, kl) by the whole workgroup.  Waves beyond the
// block's nct * nps consumers and its producer (a task-list launch sizes the
// workgroup for its largest block) only take part in the barriers.
template <int NPT, int LM, int MODE>
__device__ __forceinline__ void eri4_quartet(const Eri4Args &a, int ij, int kl, int slab, double *smem, uint32_t tk,
                                             int nq = 1) {
  constexpr bool SPLIT = MODE >= 2;  // split-precision bra transform with S = MODE + 3 slices
  constexpr bool SINGLE = MODE == 1;  // single-primitive pairs: quartet runs / V from registers
  constexpr int S = MODE + 3;
  const int L = a.L;
  // column slab: this workgroup owns ket columns [c0, c0 + 16 nct); V keeps
  // only those columns (row stride vstride) when the quartet is split
  const int c0 = slab * a.nct * 16;
  const int vstride = a.nslab > 1 ? a.nct * 16 : a.Nk;
  const int vcols = min(a.Nk - c0, a.nct * 16);
  const int S1 = a.S1, S2 = a.S2;
  const int cube_sz = a.cube_sz;
  double *cube0 = smem;
  double *cube1 = a.dbuf ? smem + cube_sz : smem;
  double *work = smem + (a.dbuf ? 2 : 1) * cube_sz;  // R-chain work area of the producer
  double *gsh = work + rr_work_size(L);              // G of this quartet's bra then ket primitive pairs
  double *vsh = gsh + 4 * a.maxpp;                   // V[ab][cd] of this quartet (none when vdirect)
  uint32_t *uvsh = (uint32_t *)(vsh + (SINGLE && a.vdirect ? 0 : a.Nb * vstride));  // (u, v, y slot) of the pairs u+v <= L
  int *offq = (int *)(uvsh + (L + 1) * (L + 2) / 2);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c = lane & 15;
  const int ncons = a.nct * a.nps;

  // run: steps n = 0 .. nq-1 are the quartets (ij, kl + n), one primitive
  // pair each side (the ket index ik of a step is then the quartet)
  const bool run = SINGLE && a.nrun > 1, vd = SINGLE && a.vdirect != 0;
  const int bp0 = a.bra_off[ij], bp1 = a.bra_off[ij + 1];
  const int kp0 = a.ket_off[kl], kp1 = a.ket_off[kl + 1];
  const int nbp = bp1 - bp0, nkp = run ? nq : kp1 - kp0;
  const int nsteps = nbp * nkp;

  for (int e = tid; e < 4 * nbp; e += blockDim.x) gsh[e] = a.bra_G[4 * (size_t)bp0 + e];
  if (run) {
    for (int e = tid; e < 4 * nq; e += blockDim.x) gsh[4 * nbp + e] = a.ket_G[4 * (size_t)a.ket_off[kl + (e >> 2)] + (e & 3)];
  } else {
    for (int e = tid; e < 4 * nkp; e += blockDim.x) gsh[4 * nbp + e] = a.ket_G[4 * (size_t)kp0 + e];
  }
  for (int e = tid; e < (L + 1) * (L + 2) / 2; e += blockDim.x) {
    // e-th pair in the order s = u+v ascending, u ascending
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= e) ++s;
    const int u = e - s * (s + 1) / 2, v = s - u;
    int vb = 0;
    (void)ylayout(L, v, &vb);
    uvsh[e] = (uint32_t)u | ((uint32_t)v << 8) | ((uint32_t)(vb + u) << 16);
  }
  if (!vd)
    for (int e = tid; e < a.Nb * vstride; e += blockDim.x) vsh[e] = 0.0;
  for (int q = tid; q < a.Nhk_pad; q += blockDim.x) {
    int o = 0;
    const uint32_t h = a.korder ? a.korder[q] : (q < a.Nhk ? a.tab.herm[q] : kPadRow);
    if (!(h & kPadRow)) o = (int)(h & 0xff) * S1 + (int)((h >> 8) & 0xff) * S2 + (int)((h >> 16) & 0xff);
    offq[q] = o;
  }
  __syncthreads();

  // V of quartet (ij, kl + m) at V[ij + nbra (ab + Nb cd)] from this base
  auto vbase = [&](int m) -> size_t { return (size_t)ij + (size_t)a.nbra * (size_t)a.Nb * (size_t)a.Nk * (kl + m); };
  // run with an LDS copy of V: after step m every wave waits for the row
  // parts' adds, the workgroup writes quartet m out and clears the copy (the
  // next step's barrier orders the clearing before its adds)
  const bool flushes = run && !vd;
  auto flush = [&](int m) {
    __syncthreads();
    const size_t base = vbase(m);
    for (int e = tid; e < a.Nb * vcols; e += blockDim.x) {
      const int cl = e / a.Nb, ab = e - cl * a.Nb;  // column c0 + cl of this workgroup's slab
      a.V[base + (size_t)a.nbra * ((size_t)ab + (size_t)a.Nb * (c0 + cl))] = vsh[ab * vstride + cl];
      vsh[ab * vstride + cl] = 0.0;
    }
  };

  if (wave == ncons) {
    // ---------------- producer: [r] one primitive quartet ahead ----------------
    // the producer shares its SIMD with consumer waves that keep the matrix
    // core busy; top issue priority keeps its VALU chains from being starved
    __builtin_amdgcn_s_setprio(3);
    YLanes<LM> yl;
    if constexpr (LM <= 18) ylanes_init<LM>(L, lane, yl);
    auto build = [&](int n, double *cube) {
      const int ib = n / nkp, ik = n - ib * nkp;
      const double *Gb = gsh + 4 * ib;
      const double *Gk = gsh + 4 * (nbp + ik);
      const double P[3] = {Gb[1], Gb[2], Gb[3]};
      const double Q[3] = {Gk[1], Gk[2], Gk[3]};
      build_R_chains<LM>(L, Gb[0], P, Gk[0], Q, cube, S1, S2, work, uvsh, a.tab.boys, lane, yl);
    };
    // one build site: step n is built while the consumers work on step n-1
    // (two cubes) or after they are done with the single cube
    for (int n = 0; n < nsteps; ++n) {
      if (!a.dbuf && n > 0) __syncthreads();  // consumers are done with the single cube
      build(n, (a.dbuf && (n & 1)) ? cube1 : cube0);
      if (flushes && n > 0) {
        __builtin_amdgcn_s_setprio(0);
        flush(n - 1);
        __builtin_amdgcn_s_setprio(3);
      }
      __syncthreads();  // [r] of step n published
    }
    __builtin_amdgcn_s_setprio(0);
    if (flushes) flush(nsteps - 1);
  } else if (wave > ncons) {
    // ---------------- surplus waves: barriers only ----------------
    for (int n = 0; n < nsteps; ++n) {
      if (!a.dbuf && n > 0) __syncthreads();
      if (flushes && n > 0) flush(n - 1);
      __syncthreads();
    }
    if (flushes) flush(nsteps - 1);
  } else {
    // ---------------- consumers ----------------
    // this wave's ket column tile ct and bra row tiles [t0, t0 + ntw); the
    // tiles t0 + ntw .. t0 + NPT - 1 are zero rows and are skipped by the ket
    // product (their X stays zero)
    const int ct = (int)(tk & 0xff), t0 = (int)((tk >> 8) & 0xff), ntw = (int)((tk >> 16) & 0xff);
    const int col = c0 + ct * 16 + c;  // this lane's ket column cd
    int offp[NPT];
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      // rows are permuted per class so the 16 rows of a tile sit in distinct LDS banks
      const uint32_t h = a.border[(t0 + pt) * 16 + c];
      offp[pt] = (int)(h & 0xff) * S1 + (int)((h >> 8) & 0xff) * S2 + (int)((h >> 16) & 0xff);
    }
    const int nks = a.Nhk_pad >> 2;  // even: Nhk_pad is a multiple of 8
    const int klo = g * a.Nk_pad + col, kstep = 4 * a.Nk_pad;
    const int blo = g * a.Nb_pad + c;
    const int nat = a.Nb_pad >> 4;
    d4 xacc[NPT];
    for (int n = 0; n < nsteps; ++n) {
      if (!a.dbuf && n > 0) __syncthreads();
      if (flushes && n > 0) flush(n - 1);
      const int ib = n / nkp, ik = n - ib * nkp;
      // ket transform: X[p][cd] += sum_q [p+q] H_ket[q][cd].  Two register
      // sets of LDS gathers ping-pong one k-step ahead of the MFMAs (the
      // scheduling barriers keep that order); the H_ket values come from
      // global memory and are loaded two k-steps further ahead (hC, hD) so
      // an L2 or last-level-cache round trip hides behind two k-steps of
      // MFMAs.  Prefetch indices are clamped so every load is unconditional;
      // nks is even (Nhk_pad is a multiple of 8).
      const double *Hk = a.ket_H + (size_t)(run ? a.ket_off[kl + ik] : kp0 + ik) * a.Nhk_pad * a.Nk_pad;
      // H_ket reads as buffer loads: the lane part of the offset sits in a
      // VGPR set once, the k-step part in an SGPR, so the loop spends no
      // vector instructions on addresses (and never rewrites a register an
      // in-flight MFMA still has to read)
      const __amdgpu_buffer_rsrc_t hks = __builtin_amdgcn_make_buffer_rsrc(
          (void *)Hk, (short)0, a.Nhk_pad * a.Nk_pad * 8, kBufferWord3);
      auto hload = [&](int k) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(hks, klo * 8, k * kstep * 8, 0));
      };
      // the first four k-steps of H_ket do not depend on [r]: their loads
      // are issued before the wait for the producer, which hides them
      const double h0 = hload(0), h1 = hload(min(1, nks - 1));
      const double h2 = hload(min(2, nks - 1)), h3 = hload(min(3, nks - 1));
      __syncthreads();  // [r] of step n published
      const double *cube = (a.dbuf && (n & 1)) ? cube1 : cube0;
      if (run || ik == 0) {
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt) xacc[pt] = d4{0.0, 0.0, 0.0, 0.0};
      }
      // the product over NT = ntw row tiles (compiled for every NT <= NPT)
      auto ket = [&](auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        double aA[NT], aB[NT];
        double hA, hB, hC, hD;
        // ket offsets of the k-steps ks+1, ks+2 sit in registers; those of the
        // next iteration are read from LDS before this iteration's MFMAs, so
        // the gathers never wait on a just-issued LDS read
        int oq1, oq2;
        {
          const int oq = offq[g];
#pragma unroll
          for (int pt = 0; pt < NT; ++pt) aA[pt] = cube[offp[pt] + oq];
          oq1 = offq[4 * min(1, nks - 1) + g];
          oq2 = offq[4 * min(2, nks - 1) + g];
          hA = h0;
          hB = h1;
          hC = h2;
          hD = h3;
        }
        // The matrix core of a SIMD serves its waves oldest first, so without
        // help the first wave finishes well before the last, which then runs
        // alone and cannot keep the pipe busy through its load latencies.
        // Issue priority falls with progress (2, 1, 0 over the thirds of the
        // k range), so the waves of a SIMD finish close together.
        const int k1 = (nks / 3) & ~1, k2 = (2 * nks / 3) & ~1;
        __builtin_amdgcn_s_setprio(2);
#pragma unroll 1
        for (int ks = 0; ks < nks; ks += 2) {
          if (ks == k1) __builtin_amdgcn_s_setprio(1);
          if (ks == k2) __builtin_amdgcn_s_setprio(0);
#pragma unroll
          for (int pt = 0; pt < NT; ++pt) aB[pt] = cube[offp[pt] + oq1];
          const int on1 = offq[4 * min(ks + 3, nks - 1) + g];
          const int on2 = offq[4 * min(ks + 4, nks - 1) + g];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int pt = 0; pt < NT; ++pt)
            xacc[pt] = mfma16x16x4(aA[pt], hA, xacc[pt]);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int pt = 0; pt < NT; ++pt) aA[pt] = cube[offp[pt] + oq2];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int pt = 0; pt < NT; ++pt)
            xacc[pt] = mfma16x16x4(aB[pt], hB, xacc[pt]);
          __builtin_amdgcn_sched_barrier(0);
          oq1 = on1;
          oq2 = on2;
          hA = hC;
          hB = hD;
          hC = hload(min(ks + 4, nks - 1));
          hD = hload(min(ks + 5, nks - 1));
        }
      };
      if (ntw == NPT) ket(Tiles<NPT>{});
      else with_tiles<NPT - 1>(ntw, ket);
      if (SPLIT && ik == nkp - 1) {
        // Split-precision bra transform on the BF16 matrix cores.  After row
        // balancing, with a power-of-two exponent per column of X over this
        // wave's rows (fx)
        // and per column ab of H over all rows (pair data), both scaled
        // operands are sums of S slices of 7-bit integers,
        // X 2^-fx = sum_j x_j 128^-j, H 2^-E = sum_i h_i 128^-i.  Every
        // BF16 product h_i x_j is an integer of at most 2^14 and the FP32
        // accumulation of one level i+j over a 32-row block stays below
        // 2^24, so the matrix cores add exactly; levels i+j > S+1 are
        // dropped (35-bit operands), the levels are combined in FP64.
        // rows balanced with the pair data's row exponents (X row p times
        // 2^k_p, H row p times 2^-k_p: products unchanged)
        const int *Kr = a.bra_Hrow + (size_t)(bp0 + ib) * a.Hs_rows + t0 * 16 + g;
        double mx = 0.0;
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            xacc[pt][r] = ldexp(xacc[pt][r], Kr[pt * 16 + 4 * r]);
            mx = fmax(mx, fabs(xacc[pt][r]));
          }
        mx = fmax(mx, __shfl_xor(mx, 16));
        mx = fmax(mx, __shfl_xor(mx, 32));
        int fx = 0;
        if (mx > 0.0) (void)frexp(mx, &fx);
        // B operands: k slot 8 g + e of block b = row 4 (e % 4) + g of tile
        // 2 b + e / 4; one 32-row block at a time (slices of one block live)
        constexpr int NB = NPT / 2;
        const uint16_t *Hs =
            a.bra_Hs + (size_t)(bp0 + ib) * S * a.Nb_pad * a.Hs_rows + (size_t)(t0 / 2) * 32 + 8 * g;
        const int *Ex = a.bra_Hexp + (size_t)(bp0 + ib) * a.Nb_pad;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          bf8 xb[S];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            double rr = ldexp(xacc[2 * b + (e >> 2)][e & 3], -fx);
#pragma unroll
            for (int sl = 0; sl < S; ++sl) {
              const double v = rr * 128.0;
              const double t = rint(v);
              rr = v - t;
              xb[sl][e] = (__bf16)(float)t;
            }
          }
#pragma unroll 1
          for (int at = 0; at < nat; ++at) {
            f4 acc[S];
#pragma unroll
            for (int l = 0; l < S; ++l) acc[l] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < S; ++i) {
              const bf8 ha = load_bf8(Hs + ((size_t)i * a.Nb_pad + at * 16 + c) * a.Hs_rows + b * 32);
#pragma unroll
              for (int j = 0; i + j < S; ++j) acc[i + j] = mfma_bf16(ha, xb[j], acc[i + j]);
            }
            if (col < a.Nk) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int ab = at * 16 + 4 * g + r;  // D[4 g + r][c] in register r
                if (ab < a.Nb) {
                  double v = 0.0;
#pragma unroll
                  for (int l = S - 1; l >= 0; --l) v = fma(v, 1.0 / 128.0, (double)acc[l][r]);
                  atomicAdd(&vsh[ab * vstride + (col - c0)], ldexp(v, Ex[ab] + fx - 14));  // level l: 128^-(l+2)
                }
              }
            }
          }
        }
      } else if (!SPLIT && (run || ik == nkp - 1)) {
        // bra transform: V[ab][cd] += sum_p H_bra[p][ab] X[p][cd], one ab tile
        // at a time (two accumulators), summed into the LDS copy of V or
        // (vdirect) stored to this step's quartet by buffer stores: the
        // quartet's base in the resource, the lane's part of the offset
        // (column cd, row 4 r + g of the tile) in a VGPR, the tile's part in
        // an SGPR (the host keeps one quartet's nbra Nb Nk doubles below 2 GiB)
        const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.V + (vd ? vbase(run ? ik : 0) : 0)), (short)0, a.nbra * a.Nb * a.Nk * 8, kBufferWord3);
        const int vlane = 8 * a.nbra * (g + a.Nb * col);
        const double *Hb = a.bra_H + (size_t)(bp0 + ib) * a.Hb_rows * a.Nb_pad + (size_t)t0 * 16 * a.Nb_pad;
#pragma unroll 1
        for (int at = 0; at < nat; ++at) {
          const double *Ht = Hb + at * 16 + blo;
          d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
          double h[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) h[r] = Ht[(4 * r) * a.Nb_pad];
#pragma unroll
          for (int pt = 0; pt < NPT; ++pt) {
            double hn[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) hn[r] = (pt + 1 < NPT) ? Ht[((pt + 1) * 16 + 4 * r) * a.Nb_pad] : 0.0;
            acc0 = mfma16x16x4(h[0], xacc[pt][0], acc0);
            acc1 = mfma16x16x4(h[1], xacc[pt][1], acc1);
            acc0 = mfma16x16x4(h[2], xacc[pt][2], acc0);
            acc1 = mfma16x16x4(h[3], xacc[pt][3], acc1);
#pragma unroll
            for (int r = 0; r < 4; ++r) h[r] = hn[r];
          }
          if (col < a.Nk) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ab = at * 16 + 4 * r + g;
              if (ab < a.Nb) {
                if (vd) {
                  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
                  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, acc0[r] + acc1[r]), vrs, vlane,
                                                        8 * a.nbra * (at * 16 + 4 * r), 0);
                } else {
                  atomicAdd(&vsh[ab * vstride + (col - c0)], acc0[r] + acc1[r]);
                }
              }
            }
          }
        }
      }
    }
    if (flushes) flush(nsteps - 1);
  }
  __syncthreads();  // V complete in LDS
  if (vd || run) return;  // stored from registers, or flushed quartet by quartet

  if (a.diag) {
    // (ab|ab) for the ab that fall in this workgroup's column slab
    for (int cl = tid; cl < vcols; cl += blockDim.x) {
      const int ab = c0 + cl;
      if (ab < a.Nb) a.V[(size_t)ij * a.Nb + ab] = vsh[ab * vstride + cl];
    }
    return;
  }
  if (a.orow) {
    // matrix output: (ab, cd) of quartet (ij, kl) at V[orow[ij] + ab + ld (ocol[kl] + cd)]
    const long r0 = a.orow[ij], q0 = a.ocol[kl];
    for (int e = tid; e < a.Nb * vcols; e += blockDim.x) {
      const int cl = e / a.Nb, ab = e - cl * a.Nb;
      a.V[r0 + ab + a.ld * (q0 + c0 + cl)] = vsh[ab * vstride + cl];
    }
    return;
  }
  const size_t base = (size_t)ij + (size_t)a.nbra * (size_t)a.Nb * (size_t)a.Nk * kl;
  for (int e = tid; e < a.Nb * vcols; e += blockDim.x) {
    const int cl = e / a.Nb, ab = e - cl * a.Nb;
    a.V[base + (size_t)a.nbra * ((size_t)ab + (size_t)a.Nb * (c0 + cl))] = vsh[ab * vstride + cl];
  }
}

// One workgroup per quartet of one class batch.
template <int NPT, int LM, int MODE>
__global__ void __launch_bounds__(64 * kMaxWaves) eri4_kernel(Eri4Args a) {
  extern __shared__ double smem[];
  const int nr = a.nrun > 1 ? a.nrun : 1, nkr = (a.nket + nr - 1) / nr;  // ket runs
  const long G = (a.diag ? (long)a.nbra : (long)a.nbra * nkr) * a.nslab;
  const long v0 = xcd_remap(blockIdx.x, G);
  const int slab = (int)(v0 % a.nslab);  // slabs of one quartet are neighbours (shared bra data)
  const long v = v0 / a.nslab;
  const int ij = (int)(v % a.nbra), kl = a.diag ? ij : (int)(v / a.nbra) * nr;
  eri4_quartet<NPT, LM, MODE>(a, ij, kl, slab, smem, a.wtask[threadIdx.x >> 6], min(nr, a.nket - kl));
}

// Persistent task-list kernel: the workgroups stride over tasks (block id,
// quartet index ij + nbra kl), sorted by the host by decreasing cost, of any
// number of class blocks that share the register tile NPT and the producer
// length LM; the workgroup holds the largest block's waves and LDS.
// OCC: waves per SIMD the kernel is compiled for (4: any workgroup up to
// kMaxWaves waves, 128 VGPRs; 5 or 6: workgroups of at most 4 waves, 96 or
// 80 VGPRs, see eri4_tasks_occupancy).
template <int NPT, int LM, int OCC>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, OCC == 4 ? 64 * kMaxWaves : 256),
                               amdgpu_waves_per_eu(OCC == 4 ? 1 : OCC)))
    eri4_tasks_kernel(const Eri4Args *__restrict__ blocks, const int2 *__restrict__ tasks, int ntask) {
  extern __shared__ double smem[];
  for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
    // wave-uniform by construction; readfirstlane lets the block's arguments
    // be fetched with scalar loads
    const int bi = __builtin_amdgcn_readfirstlane(tasks[t].x);
    const int q = __builtin_amdgcn_readfirstlane(tasks[t].y);
    // the descriptors are read-only for the kernel's lifetime: viewed through
    // the constant address space they load with scalar loads and can be
    // reloaded instead of being kept live
#if defined(__HIP_DEVICE_COMPILE__)
    typedef __attribute__((address_space(4))) const Eri4Args ConstArgs;
    const Eri4Args a = ((ConstArgs *)(blocks))[bi];
    const uint32_t tk = blocks[bi].wtask[threadIdx.x >> 6];
#else
    const Eri4Args a = blocks[bi];  // host pass: the kernel is never run there
    const uint32_t tk = 0;
#endif
    const int ij = q % a.nbra, kl = q / a.nbra;
    __syncthreads();  // the previous task is done with LDS
    eri4_quartet<NPT, LM, 0>(a, ij, kl, 0, smem, tk);
  }
}

template <int NPT, int LM, int MODE>
hipError_t launch_t(const Eri4Args &a, hipStream_t s) {
  const int waves = a.nct * a.nps + 1;
  const size_t lds = eri4_lds_bytes(a);
  const int nr = a.nrun > 1 ? a.nrun : 1;
  const long G = (a.diag ? (long)a.nbra : (long)a.nbra * ((a.nket + nr - 1) / nr)) * a.nslab;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)eri4_kernel<NPT, LM, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((eri4_kernel<NPT, LM, MODE>), dim3((unsigned)G), dim3(64 * waves), lds, s, a);
  return hipGetLastError();
}

__global__ void schwarz_reduce_kernel(int npair, int Nab, const double *__restrict__ D, const int *__restrict__ idx,
                                      double *__restrict__ Q) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= npair) return;
  double mx = 0.0;
  for (int ab = 0; ab < Nab; ++ab) mx = fmax(mx, fabs(D[(size_t)n * Nab + ab]));
  Q[idx[n]] = sqrt(mx);
}

// p tiles per consumer wave that are built.
const int kTiles[] = {1, 2, 3, 4, 6};

__global__ void symmetrize_kernel(int n, const double *__restrict__ in, double *__restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const size_t r = e / n, c = e - r * n;
  out[e] = in[e] + in[c * n + r];
}

__global__ void sum_copies_kernel(int n, int copies, const double *__restrict__ in, double *__restrict__ out,
                                  int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int c = 0; c < copies; ++c) acc += in[(size_t)c * n + i];
  out[i] = accumulate ? out[i] + acc : acc;
}

// part[b] = sum of a[e] b1[e] (and a[e] b2[e]) over this block's stride of e
// (fixed order per block: the traces are deterministic)
constexpr int kDotBlocks = 512;
__global__ void __launch_bounds__(256) dot_partial_kernel(size_t n, const double *__restrict__ a,
                                                          const double *__restrict__ b1, const double *__restrict__ b2,
                                                          double *__restrict__ part) {
  __shared__ double s1[256], s2[256];
  double x1 = 0.0, x2 = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    if (b1) x1 = fma(a[e], b1[e], x1);
    if (b2) x2 = fma(a[e], b2[e], x2);
  }
  s1[threadIdx.x] = x1;
  s2[threadIdx.x] = x2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] += s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1[0];
    part[kDotBlocks + blockIdx.x] = s2[0];
  }
}

__global__ void dot_final_kernel(const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double s[2][kDotBlocks];
  for (int e = threadIdx.x; e < 2 * kDotBlocks; e += blockDim.x) s[e / kDotBlocks][e % kDotBlocks] = part[e];
  __syncthreads();
  if (threadIdx.x < 2) {
    double acc = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) acc += s[threadIdx.x][b];
    out[threadIdx.x] = acc;
  }
}

__global__ void zero_kernel(size_t n, double *__restrict__ x) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

}  // namespace

hipError_t launch_symmetrize(int n, const double *in, double *out, hipStream_t s) {
  const size_t tot = (size_t)n * n;
  if (!tot) return hipSuccess;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}

hipError_t launch_sum_copies(int n, int copies, const double *in, double *out, hipStream_t s, int accumulate) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_copies_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, copies, in, out, accumulate);
  return hipGetLastError();
}

size_t dot2_work_doubles() { return 2 * kDotBlocks; }

hipError_t launch_dot2(size_t n, const double *a, const double *b1, const double *b2, double *work, double *out,
                       hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks), dim3(256), 0, s, n, a, b1, b2, work);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(64), 0, s, (const double *)work, out);
  return hipGetLastError();
}

hipError_t launch_zero(size_t n, double *x, hipStream_t s) {
  if (!n) return hipSuccess;
  const size_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, x);
  return hipGetLastError();
}

hipError_t launch_schwarz_reduce(int npair, int Nab, const double *D, const int *idx, double *Q, hipStream_t s) {
  if (npair <= 0) return hipSuccess;
  hipLaunchKernelGGL(schwarz_reduce_kernel, dim3((npair + 255) / 256), dim3(256), 0, s, npair, Nab, D, idx, Q);
  return hipGetLastError();
}

static size_t cube_region(int cube_sz, int ncube) { return sizeof(double) * (size_t)cube_sz * ncube; }

static size_t side_bytes(int L, int maxpp, int Nhk_pad, int Nb, int Nk) {
  return sizeof(double) * ((size_t)rr_work_size(L) + 4 * (size_t)maxpp + (size_t)Nb * Nk) +
         sizeof(uint32_t) * (size_t)((L + 1) * (L + 2) / 2) + sizeof(int) * (size_t)Nhk_pad;
}

size_t eri4_lds_bytes(const Eri4Args &a) {
  const int vcols = a.vdirect ? 0 : a.nslab > 1 ? a.nct * 16 : a.Nk;
  return cube_region(a.cube_sz, a.dbuf ? 2 : 1) + side_bytes(a.L, a.maxpp, a.Nhk_pad, a.Nb, vcols);
}

void eri4_fill_wtask(Eri4Args &a) {
  // parts of the bra row tiles that hold real rows: part ph covers tiles
  // [ph npt, ph npt + npt) of which the first min(npt, need - ph npt) are
  // computed (split precision pairs tiles and computes all of them)
  const int need = round16(a.Nhb) / 16, ncons = a.nct * a.nps;
  struct Task {
    int ct, t0, nt;
  };
  std::vector<Task> tasks;
  for (int ph = 0; ph < a.nps; ++ph)
    for (int ct = 0; ct < a.nct; ++ct) {
      const int t0 = ph * a.npt;
      tasks.push_back({ct, t0, a.bra_Hs ? a.npt : std::max(0, std::min(a.npt, need - t0))});
    }
  // the waves sharing the producer's SIMD take the lightest parts, the other
  // SIMDs the rest, heaviest first onto the least loaded SIMD
  std::stable_sort(tasks.begin(), tasks.end(), [](const Task &x, const Task &y) { return x.nt < y.nt; });
  const int psimd = ncons % 4;
  std::vector<int> slot_of(ncons, -1);  // task index per wave
  size_t next = 0;
  for (int w = psimd; w < ncons; w += 4) slot_of[w] = (int)(next++);
  int load[4] = {0, 0, 0, 0};
  for (size_t k = ncons; k-- > next;) {
    int best = -1;
    for (int sm = 0; sm < 4; ++sm) {
      if (sm == psimd) continue;
      bool free = false;
      for (int w = sm; w < ncons; w += 4) free = free || slot_of[w] < 0;
      if (free && (best < 0 || load[sm] < load[best])) best = sm;
    }
    for (int w = best; w < ncons; w += 4)
      if (slot_of[w] < 0) {
        slot_of[w] = (int)k;
        break;
      }
    load[best] += tasks[k].nt;
  }
  for (int w = 0; w < kMaxWaves; ++w) a.wtask[w] = 0;
  for (int w = 0; w < ncons; ++w) {
    const Task &t = tasks[slot_of[w]];
    a.wtask[w] = (uint32_t)t.ct | ((uint32_t)t.t0 << 8) | ((uint32_t)t.nt << 16);
  }
}

bool eri4_plan(int Nhb, int Nb, int Nk, int L, int cube_sz, int Nhk_pad, int maxpp, bool slabs, Eri4Plan *p) {
  if (L > 26) return false;
  const int need_p = round16(Nhb) / 16, nct_all = round16(Nk) / 16;
  const size_t lds_budget = 160 * 1024;
  // Preferred: all ket columns in one workgroup, bra rows split over `parts`
  // waves of at most 6 tiles each.  When that does not fit the wave or LDS
  // limits and `slabs` is allowed, the ket columns are split into slabs of
  // nct tiles handled by separate workgroups.
  for (int nslab = 1; nslab <= (slabs ? nct_all : 1); ++nslab) {
    const int nct = (nct_all + nslab - 1) / nslab;
    if (nslab > 1 && (nct_all + nct - 1) / nct != nslab) continue;  // same split as a smaller nslab
    {
      const int maxt = 6;
      int parts = 1;
      while ((need_p + parts - 1) / parts > maxt) ++parts;
      const int per = (need_p + parts - 1) / parts;
      if (nct * parts + 1 > kMaxWaves) continue;
      int npt = 0;
      for (int t : kTiles)
        if (t >= per) {
          npt = t;
          break;
        }
      if (!npt) continue;
      const size_t rest = side_bytes(L, maxpp, Nhk_pad, Nb, nslab > 1 ? nct * 16 : Nk);
      int dbuf;
      if (cube_region(cube_sz, 2) + rest <= lds_budget) dbuf = 1;
      else if (cube_region(cube_sz, 1) + rest <= lds_budget) dbuf = 0;
      else continue;
      p->npt = npt;
      p->nps = parts;
      p->dbuf = dbuf;
      p->nct = nct;
      p->nslab = nslab;
      return true;
    }
  }
  return false;
}

template <int LM, int MODE>
hipError_t launch_lm(const Eri4Args &a, hipStream_t s) {
  if constexpr (MODE >= 2) {  // split precision pairs row tiles: even npt only
    switch (a.npt) {
      case 2: return launch_t<2, LM, MODE>(a, s);
      case 4: return launch_t<4, LM, MODE>(a, s);
      case 6: return launch_t<6, LM, MODE>(a, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.npt) {
      case 1: return launch_t<1, LM, MODE>(a, s);
      case 2: return launch_t<2, LM, MODE>(a, s);
      case 3: return launch_t<3, LM, MODE>(a, s);
      case 4: return launch_t<4, LM, MODE>(a, s);
      case 6: return launch_t<6, LM, MODE>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
}

template <int NPT, int LM, int OCC>
hipError_t launch_tasks_o(const Eri4Args *b, const int2 *t, int n, int waves, size_t lds, int grid, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)eri4_tasks_kernel<NPT, LM, OCC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((eri4_tasks_kernel<NPT, LM, OCC>), dim3((unsigned)grid), dim3(64 * waves), lds, s, b, t, n);
  return hipGetLastError();
}

template <int NPT, int LM>
hipError_t launch_tasks_t(const Eri4Args *b, const int2 *t, int n, int waves, size_t lds, int grid, hipStream_t s) {
  const int occ = eri4_tasks_occupancy(NPT, LM, waves);
  if constexpr (LM <= 10 && NPT == 1)
    if (occ == 6) return launch_tasks_o<NPT, LM, 6>(b, t, n, waves, lds, grid, s);
  if constexpr (LM <= 10 && NPT == 2)
    if (occ == 5) return launch_tasks_o<NPT, LM, 5>(b, t, n, waves, lds, grid, s);
  return launch_tasks_o<NPT, LM, 4>(b, t, n, waves, lds, grid, s);
}

template <int LM>
hipError_t launch_tasks_lm(const Eri4Args *b, const int2 *t, int n, int npt, int waves, size_t lds, int grid,
                           hipStream_t s) {
  switch (npt) {
    case 1: return launch_tasks_t<1, LM>(b, t, n, waves, lds, grid, s);
    case 2: return launch_tasks_t<2, LM>(b, t, n, waves, lds, grid, s);
    case 3: return launch_tasks_t<3, LM>(b, t, n, waves, lds, grid, s);
    case 4: return launch_tasks_t<4, LM>(b, t, n, waves, lds, grid, s);
    case 6: return launch_tasks_t<6, LM>(b, t, n, waves, lds, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
hipError_t launch_g(const Eri4Args &a, hipStream_t s) {
  // register length of the producer's m-vectors: smallest bound >= L
  if (a.L <= 8) return launch_lm<8, MODE>(a, s);
  if (a.L <= 10) return launch_lm<10, MODE>(a, s);
  if (a.L <= 16) return launch_lm<16, MODE>(a, s);
  if (a.L <= 18) return launch_lm<18, MODE>(a, s);
  if (a.L <= 26) return launch_lm<26, MODE>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_eri4(const Eri4Args &a0, hipStream_t s) {
  if (a0.nbra <= 0 || a0.nket <= 0) return hipSuccess;
  if (a0.nct * a0.nps + 1 > kMaxWaves) return hipErrorInvalidValue;
  Eri4Args a = a0;
  eri4_fill_wtask(a);
  if (a.bra_Hs) {
    switch (a.split) {  // mode = slices - 3
      case 5: return launch_g<2>(a, s);
      case 6: return launch_g<3>(a, s);
      case 7: return launch_g<4>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  return (a.nrun > 1 || a.vdirect) ? launch_g<1>(a, s) : launch_g<0>(a, s);
}

int eri4_lm_bucket(int L) { return rr_lm_bucket(L); }

// The one- and two-tile shapes with short R chains (L <= 10) fit 80 / 96
// VGPRs without spilling, so their task-list workgroups (at most 4 waves)
// can sit 6 / 5 to a SIMD side by side: more producer waves per CU for the
// 3-centre task lists, whose [r] builds bound them.
int eri4_tasks_occupancy(int npt, int Lmax, int waves) {
  if (waves > 4 || rr_lm_bucket(Lmax) > 10) return 4;
  return npt == 1 ? 6 : npt == 2 ? 5 : 4;
}

hipError_t launch_eri4_tasks(const Eri4Args *d_blocks, const int2 *d_tasks, int ntask, int npt, int Lmax, int waves,
                             size_t lds, int grid, hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (waves < 2 || waves > kMaxWaves || grid <= 0) return hipErrorInvalidValue;
  switch (eri4_lm_bucket(Lmax)) {
    case 8: return launch_tasks_lm<8>(d_blocks, d_tasks, ntask, npt, waves, lds, grid, s);
    case 10: return launch_tasks_lm<10>(d_blocks, d_tasks, ntask, npt, waves, lds, grid, s);
    case 16: return launch_tasks_lm<16>(d_blocks, d_tasks, ntask, npt, waves, lds, grid, s);
    case 18: return launch_tasks_lm<18>(d_blocks, d_tasks, ntask, npt, waves, lds, grid, s);
    case 26: return launch_tasks_lm<26>(d_blocks, d_tasks, ntask, npt, waves, lds, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mderi
