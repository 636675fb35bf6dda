// internal.h -- definitions shared by the host code and the HIP kernels of
// libmderi (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mderi.h"

namespace mderi {

constexpr int kLmax = MDERI_LMAX;       // largest shell l
constexpr int kLshell = kLmax + 1;      // l+1 shells appear in derivatives
constexpr int kSplitMin = 5, kSplitMax = 7, kSplitDefault = 6;  // 7-bit slices per operand in split precision
constexpr int kLtotMax = 4 * kLshell;   // largest total L = la+lb+lc+ld
constexpr int kNtilMax = (kLtotMax + 1) * (kLtotMax + 2) * (kLtotMax + 3) / 6;

// Boys-function interpolation table: F_m(T_i), T_i = i/16 for i = 0..1600
// (T <= 100), m = 0..33, stored row-major [i][m], then one row holding the
// double factorials (2m-1)!! of the large-T form.  Evaluated on the host in
// long double from the positive-term series of F_mmax and downward
// recursion; see boys_table() in host.hip.
constexpr int kBoysM = 34;
constexpr int kBoysGridPerUnit = 16;
constexpr double kBoysTmax = 100.0;
constexpr int kBoysNgrid = 1601;
constexpr int kBoysTaylor = 8;  // Taylor terms around the nearest grid point

// Number of Hermite functions of total degree <= l.
__host__ __device__ constexpr int ntil(int l) { return (l + 1) * (l + 2) * (l + 3) / 6; }
// Number of solid harmonics of one shell.
__host__ __device__ constexpr int nsph(int l) { return 2 * l + 1; }
__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int round16(int n) { return (n + 15) & ~15; }

// Waves per workgroup of the 4-centre kernels (consumers + producer + idle).
constexpr int kMaxWavesArgs = 16;

// Packed Hermite / Cartesian triple.
__host__ __device__ inline uint32_t pack3(int t, int u, int v) {
  return (uint32_t)t | ((uint32_t)u << 8) | ((uint32_t)v << 16);
}
// Flag of a padding row in a Hermite row order: the row of H is zero, while
// its (t,u,v) still names a valid [r] entry for the matrix-core gather.
constexpr uint32_t kPadRow = 0x80000000u;

// Constant device tables owned by a context.
struct Tables {
  double *boys = nullptr;        // [kBoysNgrid + 1][kBoysM]
  uint32_t *herm = nullptr;      // [kNtilMax] (t,u,v), ordered by degree, then t desc, then u desc
  int *solid_start = nullptr;    // [(kLshell+1)*(2*kLshell+1) + 1]: nonzeros of (l, m) start at
                                 //   solid_start[l*(2*kLshell+1) + (m+l)]
  double *solid_coef = nullptr;  // nonzero Cartesian->solid coefficients
  uint32_t *solid_cart = nullptr;// matching Cartesian exponents (packed)
};
__host__ __device__ inline int solid_slot(int l, int m) { return l * (2 * kLshell + 1) + (m + l); }
constexpr int kSolidSlots = (kLshell + 1) * (2 * kLshell + 1) + 1;

// Primitive-pair descriptor built on the host for a class batch.
struct PrimPair {
  int sa, sb;  // shell indices
  int pa, pb;  // global primitive indices (into the basis exponent / coefficient arrays)
};

// Device copy of a basis.
struct DevBasis {
  int nshell = 0, nprim = 0;
  int *l = nullptr, *K = nullptr, *poff = nullptr, *atom = nullptr;
  int *ao_off = nullptr;      // first AO of every shell
  double *centers = nullptr;  // [nshell][3]
  double *exps = nullptr;     // [nprim]
  double *coefs = nullptr;    // [nprim], normalised contraction coefficients
};

// Arguments of the pair-data kernel (Sec. 3: pair data G and transform
// matrices H, stored contiguously per (pair, primitive)).
struct PairArgs {
  int npp;
  const PrimPair *pp;
  DevBasis basis;
  int la, lb;
  int Nh, N, Nh_pad, N_pad;
  int ket_sign;  // fold (-1)^{|q|} of Eq. (pq) into a ket transform matrix
  int one_centre;  // single shells (lb ignored): Eqs. (E1rr)-(E1-aa), zeta_p = zeta_a, P = A
  int deriv;       // write the six centre-derivative matrices d/dA_x, d/dB_x (see pairs.hip)
                   // transposed, H[6][N_pad][Nh_pad] (rows then span |p| <= la+lb+1), before
                   // the plain matrix [Nh_pad][N_pad]
  int rderiv;      // after the plain matrix, the three derivatives with respect to the
                   // relative coordinate A - B at fixed P, each [Nh_pad][N_pad] ([N_pad][Nh_pad]
                   // with rtrans); per primitive pair 6 deriv + 1 + 3 rderiv matrices
  int rtrans;
  // split precision: also write the matrix as `split` BF16 slices of
  // 7-bit integers relative to a power-of-two exponent per column ab (see
  // pairs.hip), rows in the k order of the BF16 matrix-core operand
  int split;      // 0, or the number of slices (kSplitMin..kSplitMax)
  uint16_t *Hs;   // [npp][split][N_pad][Hs_rows] (BF16 bit patterns)
  int *Hexp;      // [npp][N_pad] column exponents
  int *Hrow;      // [npp][Hs_rows] row balancing exponents
  int Hs_rows;    // Nh_pad rounded up to 32
  const uint32_t *order;  // row order (Nh_pad packed (t,u,v); kPadRow set = zero row), or
                          // nullptr for the global Hermite order with Nh real rows
  Tables tab;
  double *G;  // [npp][4] : zeta_p, P_x, P_y, P_z
  double *H;  // [npp][Nh_pad][N_pad]
};

// Arguments of the fused 4-centre kernel.
struct Eri4Args {
  int nbra, nket;
  int L, Nhb, Nhk, Nb, Nk;
  int Nhb_pad, Nhk_pad, Nb_pad, Nk_pad;
  int Hb_rows;   // rows allocated per bra transform matrix (>= Nhb_pad; its stride)
  int npt;       // p tiles held by a consumer wave
  int nps;       // bra Hermite rows split over nps waves (Nhb_pad = 16 npt nps)
  int nct;       // ket column tiles per workgroup
  int nslab;     // workgroups per quartet (ket column slabs of nct tiles; Nk_pad >= 16 nct nslab)
  int dbuf;      // double-buffered [r] cube
  int S1, S2;    // [r] cube strides: [r] sits at t*S1 + u*S2 + v
  int cube_sz;   // doubles per cube
  int maxpp;     // largest (bra + ket) primitive-pair count of one quartet
  const uint32_t *border;  // bra Hermite row order (Nhb_pad entries, see PairArgs::order)
  const uint32_t *korder;  // ket Hermite row order (Nhk_pad entries), or nullptr for the global order
  int diag;      // Schwarz mode: quartets (ij|ij) only, V receives the diagonal [ij][ab]
  // quartet runs (single-primitive pairs on both sides, two [r] cubes): a
  // workgroup takes the nrun ket pairs kl0 .. kl0 + nrun - 1 of one bra pair
  // as consecutive steps, the producer building the next quartet's [r] while
  // the consumers transform the current one (0 or 1: one quartet)
  int nrun;
  // V leaves the consumer registers straight for global memory (single
  // primitive bra pairs and one row part, so a wave holds complete
  // elements): no LDS copy of V
  int vdirect;
  // matrix output (orow != nullptr): (ab, cd) of quartet (ij, kl) goes to
  // V[orow[ij] + ab + ld * (ocol[kl] + cd)] instead of the class-batch layout
  const long *orow, *ocol;
  long ld;
  const int *bra_off, *ket_off;  // [n+1] primitive-pair offsets per shell pair
  const double *bra_G, *ket_G;
  const double *bra_H, *ket_H;
  // split-precision bra transform (precision 1): BF16 slices of the bra
  // matrices and their per-ab exponents (PairArgs::Hs, Hexp)
  const uint16_t *bra_Hs;
  const int *bra_Hexp, *bra_Hrow;
  int Hs_rows;
  int split;     // number of slices (kernel mode follows it)
  Tables tab;
  double *V;
  // work of consumer wave w (set by eri4_fill_wtask): ket column tile
  // (bits 0-7), first bra row tile (bits 8-15), row tiles computed (bits 16-23)
  uint32_t wtask[kMaxWavesArgs];
};

// One class block of the screened quartet engine (kx.hip: K and J builds and
// the nuclear gradient).  Side A holds shell pairs (a, b) of one class, side
// B pairs (c, d) of one class, each sorted by decreasing Schwarz factor, so
// the B pairs that pass Q_A Q_B >= tau with A pair i are a prefix of B: the
// block's quartets are (i, k) with k < cnt(i) = pre[i+1] - pre[i] (same-list
// blocks of the K and J builds keep k <= i as well).  A's Hermite functions
// are the matrix-core rows of the ket product; B's are contracted.
struct KxBlock {
  long chunk0;            // first global chunk index of the block
  long nq;                // quartets of the block
  int chunk;              // quartets per chunk
  const long *pre;        // [nA + 1] first quartet of every A pair
  int nA;
  int L;                  // Hermite degree of R (l_a+l_b+l_c+l_d, +1 in gradient mode)
  int S1, S2;             // [r] cube strides
  int NhA, HA_rows;       // A Hermite rows used, rows allocated per A matrix (multiple of 16)
  int nparts;             // A row parts of NRT tiles
  int NhB, NhB_pad;       // B Hermite rows, padded to a multiple of 8
  int NA, NB, NA_pad, NB_pad, nct;  // solid components per side (padded to 16), B column tiles
  int na, nb, nc, nd;     // N(l) of the four shells
  int same;               // A and B are the same pair list
  int A_mats, B_mats;     // matrices stored per primitive pair (A: 1, or 7 in gradient mode; B: 1 or 4)
  int onev;               // gradient: one visit per quartet supplies all four centres (single-
                          // primitive pairs; B side through Z = [p+q]^T (H_A S) and dH_B/d(C-D))
  int yacc;               // gradient: Y = sum_k X S^T of one A pair's run of quartets accumulates in
                          // LDS and meets the derivative matrices once per run
  const uint32_t *Ashift; // one-visit: rows of (t+1,u,v), (t,u+1,v), (t,u,v+1) for every A row
                          // (10 bits each; any valid row where the shifted function is absent)
  const PrimPair *A_pp, *B_pp;  // primitive pairs (exponents of the one-visit splits)
  int A_plain, A_rel;     // A role: index of the plain matrix and of the first d/d(A-B) matrix
  float inv_nb, inv_nd, inv_NB, inv_ncd;  // 1/nb, 1/nd, 1/NB, 1/(nc + nd) for index decoding
  const uint32_t *Aorder; // A Hermite row order (HA_rows entries, see PairArgs::order)
  const int *A_off, *B_off;            // primitive-pair offsets per pair [n + 1]
  const double *A_G, *B_G, *A_H, *B_H; // pair data (A: derivative matrices in gradient mode)
  const int *A_sh, *B_sh;              // shells of every pair [n][2]
};

// Arguments shared by every block of one launch of the quartet engine.
struct KxArgs {
  const KxBlock *blocks;  // device array, sorted by chunk0
  int nblk;
  long nchunk;            // chunks over all blocks
  unsigned long long *counter;  // next chunk to take (zero before the launch)
  Tables tab;
  const int *ao_off;      // first AO of every shell
  int nao;
  // digest mode: K' += the four exchange images, J' += the two Coulomb
  // images (either may be null); K = K' + K'^T, J = J' + J'^T afterwards
  const double *dm;       // density D [nao][nao] (symmetric)
  double *kx, *jx;
  // deterministic digest: kx / jx then point at [nao][nao][2] 64-bit integer
  // pairs (floor, fraction 2^32) of the images times *fscale
  int fixed;
  const double *fscale;
  // gradient mode: E = sum W_abcd (ab|cd) with W = Wl_ac Wr_bd (pattern 0) or
  // Wl_ab Wr_cd (pattern 1), times scale; dE/dR of the A centres added to
  // grad copy (workgroup % gcopies) at [atom][xyz]
  const double *wl, *wr;
  int pattern;
  int symmetric;          // Wl = Wr and symmetric (caller's guarantee): one staged weight block
  double scale;
  double *grad;
  int gcopies, gstride;
  int gfixed;             // deterministic: grad holds four 64-bit digit words per element (see grad_add)
  const int *atom;
  const double *exps;     // basis exponents
  // per-wave LDS layout (offsets in doubles from the wave's base)
  int wave_doubles, o_work, o_v, o_d, o_img, o_g, o_tab;
  int o_y, o_x;           // gradient: Y accumulator, one-visit X staging (rows of 17 doubles)
  int uv_max, oq_max, op_max;  // entries of the (u, v) table, the B and the A offset tables
};

// Launchers (defined in the .hip files).
// density-fitted Coulomb (df.hip)
hipError_t launch_df_dvec(int nrow, const int2 *ab, const double *w, const double *D, int nao, double *dvec,
                          hipStream_t s);
hipError_t launch_df_gamma(int nrow, int ncol, const double *B, const double *dvec, double *gamma, hipStream_t s);
hipError_t launch_df_j(int nrow, int ncol, const double *B, const double *c, const int2 *ab, double *J, int nao,
                       hipStream_t s);
hipError_t launch_df_expand(int nrow, int ncol, const double *B, const int2 *ab, const double *w, int nao, double *Bt,
                            hipStream_t s);
hipError_t launch_df_scatter(int na, int Na, int nc, int Nc, const double *V, const int *shells_a, const int *shells_c,
                             const int *ao_off, double *M, int n, hipStream_t s);
hipError_t launch_pairs(const PairArgs &a, hipStream_t s);
hipError_t launch_eri4(const Eri4Args &a, hipStream_t s);
// Q[idx[n]] = sqrt(max_ab |D[n][ab]|) for n < npair (Schwarz factors).
hipError_t launch_schwarz_reduce(int npair, int Nab, const double *D, const int *idx, double *Q, hipStream_t s);
// K = K' + K'^T (in place would race, so out != in), n x n.
hipError_t launch_symmetrize(int n, const double *in, double *out, hipStream_t s);
// Deterministic accumulation (det.hip): scale[0] = 2^(62 - ceil(log2 B)),
// B = 4 qmax^2 sum_e |D[e]| (1 when B is 0 or not finite), summed in a fixed
// order over n elements; work holds det_scale_work_doubles().
size_t det_scale_work_doubles();
hipError_t launch_det_scale(size_t n, const double *D, double qmax, double *work, double *scale, hipStream_t s);
// out = K' + K'^T with K' the fixed-point pairs of in[n][n][2] divided by *scale.
hipError_t launch_symmetrize_fixed(int n, const unsigned long long *in, const double *scale, double *out,
                                   hipStream_t s);
// x[0..n) = 0 for 64-bit integers.
hipError_t launch_zero_u64(size_t n, unsigned long long *x, hipStream_t s);
// out[i] (+)= the sum over c < copies of the fixed-point values in[c n + i]
// (four digit words each, value = sum_k W_k 2^(32 k - 80)), summed as integers.
hipError_t launch_sum_copies_fixed(int n, int copies, const unsigned long long *in, double *out, int accumulate,
                                   hipStream_t s);
// x[0..n) = 0 with a plain kernel (no memset node, capture-safe).
hipError_t launch_zero(size_t n, double *x, hipStream_t s);
// out[i] = sum_c in[c n + i] for i < n, c < copies (added to out[i] when accumulate).
hipError_t launch_sum_copies(int n, int copies, const double *in, double *out, hipStream_t s, int accumulate = 0);
// out[0] = sum a[e] b1[e], out[1] = sum a[e] b2[e] over e < n (either b may be
// null: its sum is 0), in a fixed order; work holds dot2_work_doubles().
size_t dot2_work_doubles();
hipError_t launch_dot2(size_t n, const double *a, const double *b1, const double *b2, double *work, double *out,
                       hipStream_t s);
// Work split of the fused kernel for one class.
struct Eri4Plan {
  int npt;    // bra row tiles per consumer wave
  int nps;    // bra row parts (waves per column tile)
  int dbuf;   // double-buffered [r] cube
  int nct;    // ket column tiles per workgroup
  int nslab;  // workgroups per quartet (column slabs)
};
// Chooses the split of the 4-centre kernel; false if the class does not
// fit.  slabs admits splitting the ket columns over workgroups (plain output
// only).
bool eri4_plan(int Nhb, int Nb, int Nk, int L, int cube_sz, int Nhk_pad, int maxpp, bool slabs, Eri4Plan *p);
// Launches the quartet engine for blocks sharing the row tile count npt
// (1, 2 or 4) and the producer bucket of Lmax; grad selects gradient mode.
hipError_t launch_kx(const KxArgs &a, int npt, int Lmax, bool grad, int waves, size_t lds, int grid, hipStream_t s);
// Persistent task-list launch over class blocks that share npt and the
// producer length bucket of Lmax: d_blocks[nblk] device copies of the blocks'
// arguments, d_tasks[ntask] = (block, ij + nbra kl); the workgroup has
// `waves` waves and `lds` bytes (the largest block's), the grid `grid`
// workgroups.
hipError_t launch_eri4_tasks(const Eri4Args *d_blocks, const int2 *d_tasks, int ntask, int npt, int Lmax, int waves,
                             size_t lds, int grid, hipStream_t s);
// The producer length bucket (m-vector registers) used for total L.
int eri4_lm_bucket(int L);
// LDS bytes needed by one 4-centre workgroup.
size_t eri4_lds_bytes(const Eri4Args &a);
// Waves per SIMD the task-list kernel of this shape is built for (4, 5 or 6).
int eri4_tasks_occupancy(int npt, int Lmax, int waves);
// Fills a.wtask from nct, nps, npt, Nhb and split (see eri4.hip).
void eri4_fill_wtask(Eri4Args &a);

}  // namespace mderi
