// eri4.hip -- fused 4-centre MD kernel on the FP64 matrix cores.
//
// One workgroup evaluates one shell quartet (ij, kl); wave w owns the 16
// ket components cd in [16w, 16w+16) for every bra component ab.  For each
// bra primitive pair:
//   X[p][cd]  = sum_{ket prims} sum_q [p|q] H_ket[q][cd]        Eq. (ket-from-hermite)
//   V[ab][cd] += sum_p H_bra[p][ab] X[p][cd]                      Eq. (bra-from-hermite)
// with [p|q] = (-1)^{|q|} [p+q]^(0) (Eq. (pq); the sign lives in H_ket)
// gathered straight from the LDS copy of [r]^(0) (Eqs. (0m), (r)) as the A
// operand of a 16x16x4 FP64 MFMA, so the Ñ_bra x Ñ_ket matrix [p|q] is never
// stored.  X stays in registers: the accumulator tile of the ket step is
// exactly the B operand of the bra step (rows 4r..4r+3 of a 16-row tile sit
// in register r), so the two transforms are chained without leaving the
// wave.  Output goes to V[ij,ab,cd,kl] (Sec. 3), ij fastest.
#include "device_common.h"

namespace mderi {

namespace {

constexpr int kMaxWaves = 6;

template <int NPT, int NAT>
__global__ void __launch_bounds__(64 * kMaxWaves) eri4_kernel(Eri4Args a) {
  extern __shared__ double smem[];
  const int L = a.L;
  const int L1 = L + 1, S1 = L1 * L1;
  double *cube = smem;
  double *lev = cube + S1 * L1;
  int *offq = (int *)(lev + 3 * a.levn);

  const long G = a.diag ? (long)a.nbra : (long)a.nbra * a.nket;
  const long v = xcd_remap(blockIdx.x, G);
  const int ij = (int)(v % a.nbra), kl = a.diag ? ij : (int)(v / a.nbra);

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c = lane & 15;

  for (int q = tid; q < a.Nhk_pad; q += nthr) {
    int o = 0;
    if (q < a.Nhk) {
      const uint32_t h = a.tab.herm[q];
      o = (int)(h & 0xff) * S1 + (int)((h >> 8) & 0xff) * L1 + (int)((h >> 16) & 0xff);
    }
    offq[q] = o;
  }
  int offp[NPT];
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt) {
    const int p = pt * 16 + c;
    int o = 0;
    if (p < a.Nhb) {
      const uint32_t h = a.tab.herm[p];
      o = (int)(h & 0xff) * S1 + (int)((h >> 8) & 0xff) * L1 + (int)((h >> 16) & 0xff);
    }
    offp[pt] = o;
  }

  d4 vacc[NAT];
#pragma unroll
  for (int at = 0; at < NAT; ++at) vacc[at] = d4{0.0, 0.0, 0.0, 0.0};

  const int bp0 = a.bra_off[ij], bp1 = a.bra_off[ij + 1];
  const int kp0 = a.ket_off[kl], kp1 = a.ket_off[kl + 1];
  const int nks = a.Nhk_pad >> 2;
  const int col = wave * 16 + c;  // this lane's ket column cd

  for (int bp = bp0; bp < bp1; ++bp) {
    d4 xacc[NPT];
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) xacc[pt] = d4{0.0, 0.0, 0.0, 0.0};
    const double pz = a.bra_G[4 * (size_t)bp];
    const double P[3] = {a.bra_G[4 * (size_t)bp + 1], a.bra_G[4 * (size_t)bp + 2], a.bra_G[4 * (size_t)bp + 3]};

    for (int kp = kp0; kp < kp1; ++kp) {
      const double qz = a.ket_G[4 * (size_t)kp];
      const double Q[3] = {a.ket_G[4 * (size_t)kp + 1], a.ket_G[4 * (size_t)kp + 2], a.ket_G[4 * (size_t)kp + 3]};
      __syncthreads();  // previous [r] consumed by every wave
      build_R(L, pz, P, qz, Q, cube, lev, a.levn, a.tab, tid, nthr);

      // ket transform: X[p][cd] += sum_q [p+q] H_ket[q][cd]
      const double *Hk = a.ket_H + (size_t)kp * a.Nhk_pad * a.Nk_pad + col;
      double bnext = Hk[(size_t)g * a.Nk_pad];
#pragma unroll 1
      for (int ks = 0; ks < nks; ++ks) {
        const double bcur = bnext;
        if (ks + 1 < nks) bnext = Hk[(size_t)(4 * (ks + 1) + g) * a.Nk_pad];
        const int oq = offq[4 * ks + g];
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt) xacc[pt] = mfma16x16x4(cube[offp[pt] + oq], bcur, xacc[pt]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // bra transform: V[ab][cd] += sum_p H_bra[p][ab] X[p][cd]
    const double *Hb = a.bra_H + (size_t)bp * a.Nhb_pad * a.Nb_pad + c;
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double *row = Hb + (size_t)(pt * 16 + 4 * r + g) * a.Nb_pad;
#pragma unroll
        for (int at = 0; at < NAT; ++at) vacc[at] = mfma16x16x4(row[at * 16], xacc[pt][r], vacc[at]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  if (a.diag) {
#pragma unroll
    for (int at = 0; at < NAT; ++at)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ab = at * 16 + 4 * r + g;
        if (ab == col && ab < a.Nb) a.V[(size_t)ij * a.Nb + ab] = vacc[at][r];
      }
    return;
  }
  if (col < a.Nk) {
    const size_t base = (size_t)ij + (size_t)a.nbra * (size_t)a.Nb * ((size_t)col + (size_t)a.Nk * kl);
#pragma unroll
    for (int at = 0; at < NAT; ++at)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ab = at * 16 + 4 * r + g;
        if (ab < a.Nb) a.V[base + (size_t)a.nbra * ab] = vacc[at][r];
      }
  }
}

template <int NPT, int NAT>
hipError_t launch_t(const Eri4Args &a, hipStream_t s) {
  const int waves = a.Nk_pad / 16;
  const size_t lds = eri4_lds_bytes(a.L, a.Nhk_pad, a.levn);
  const long G = a.diag ? (long)a.nbra : (long)a.nbra * a.nket;
  hipLaunchKernelGGL((eri4_kernel<NPT, NAT>), dim3((unsigned)G), dim3(64 * waves), lds, s, a);
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

}  // namespace

hipError_t launch_schwarz_reduce(int npair, int Nab, const double *D, const int *idx, double *Q, hipStream_t s) {
  if (npair <= 0) return hipSuccess;
  hipLaunchKernelGGL(schwarz_reduce_kernel, dim3((npair + 255) / 256), dim3(256), 0, s, npair, Nab, D, idx, Q);
  return hipGetLastError();
}

int rr_level_stride(int L) {
  int mx = L + 1;
  for (int n = 1; n <= L; ++n) {
    const int e = (L - n + 1) * (n + 1) * (n + 2) / 2;
    if (e > mx) mx = e;
  }
  return mx;
}

size_t eri4_lds_bytes(int L, int Nhk_pad, int levn) {
  const size_t L1 = (size_t)L + 1;
  return sizeof(double) * (L1 * L1 * L1 + 3 * (size_t)levn) + sizeof(int) * (size_t)Nhk_pad;
}

// Register tiles built: (p tiles, ab tiles) of the bra side.  The host pads
// the bra transform matrices to the chosen tile so the kernel has no
// partial tiles.
static const int kTiles[][2] = {{1, 1}, {2, 1}, {3, 1}, {3, 2}, {4, 2}, {4, 3}, {6, 3}, {6, 4}, {8, 4}, {11, 6}};

bool eri4_pick_tiles(int npt, int nat, int *NPT, int *NAT) {
  for (const auto &t : kTiles)
    if (t[0] >= npt && t[1] >= nat) {
      *NPT = t[0];
      *NAT = t[1];
      return true;
    }
  return false;
}

hipError_t launch_eri4(const Eri4Args &a, hipStream_t s) {
  if (a.nbra <= 0 || a.nket <= 0) return hipSuccess;
  if (a.Nk_pad / 16 > kMaxWaves) return hipErrorInvalidValue;
#define MDERI_TILE(P, A) \
  if (a.npt == P && a.nat == A) return launch_t<P, A>(a, s);
  MDERI_TILE(1, 1) MDERI_TILE(2, 1) MDERI_TILE(3, 1) MDERI_TILE(3, 2) MDERI_TILE(4, 2)
  MDERI_TILE(4, 3) MDERI_TILE(6, 3) MDERI_TILE(6, 4) MDERI_TILE(8, 4) MDERI_TILE(11, 6)
#undef MDERI_TILE
  return hipErrorInvalidValue;
}

}  // namespace mderi
