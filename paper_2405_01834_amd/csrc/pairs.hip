// pairs.hip -- primitive-pair data G and Hermite->solid transform matrices H
// for one class batch of shell pairs (or of single shells, for the auxiliary
// side of 3-centre integrals).
//
// For each primitive pair of shells (a, b) with exponents za, zb:
//   zeta_p = za + zb, P = (za A + zb B) / zeta_p                  (Sec. 2)
//   E^t_{ij} per axis by Eqs. (E2rr1)-(E2-abp), E^0_00 = exp(-mu X_AB^2)
//   H[p][ab] = c_a c_b sum_{a,b Cartesian} C_{l_a m_a}^a C_{l_b m_b}^b
//              E^{t}_{a_x b_x} E^{u}_{a_y b_y} E^{v}_{a_z b_z}   Eq. (solid2herm-2)
// with p = (t,u,v) in the global Hermite order.  For a ket pair the sign
// (-1)^{|q|} of Eq. (pq) is folded into H.  Rows p >= Nh and columns
// ab >= N are zero padding up to multiples of 16 (the matrix-core tiles).
#include "device_common.h"

namespace mderi {

namespace {

constexpr int kPairThreads = 256;
constexpr int kEmaxA = kLshell + 1;            // la+1
constexpr int kEmaxT = 2 * kLshell + 2;        // la+lb+2 (one spare for t+1 reads)

__global__ void __launch_bounds__(kPairThreads) pair_kernel(PairArgs a) {
  const int pp = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double E[3][kEmaxA][kEmaxA][kEmaxT];
  __shared__ double sc[2];

  const PrimPair d = a.pp[pp];
  const double za = a.basis.exps[d.pa], zb = a.one_centre ? 0.0 : a.basis.exps[d.pb];
  const double *A = a.basis.centers + 3 * d.sa;
  const double *B = a.one_centre ? A : a.basis.centers + 3 * d.sb;
  const double p = za + zb;
  const double mu = za * zb / p;
  const int la = a.la, lb = a.one_centre ? 0 : a.lb;

  for (int e = tid; e < 3 * kEmaxA * kEmaxA * kEmaxT; e += kPairThreads) (&E[0][0][0][0])[e] = 0.0;
  __syncthreads();
  if (tid < 3) {
    const int x = tid;
    const double Px = (za * A[x] + zb * B[x]) / p;
    const double XPA = Px - A[x], XPB = Px - B[x], XAB = A[x] - B[x];
    const double o2p = 0.5 / p;
    double(*Ex)[kEmaxA][kEmaxT] = E[x];
    // Eq. (E2-000); a single Gaussian has E^0_0 = 1 and, with zeta_b = 0 and
    // P = A, Eq. (E2rr1) reduces to Eq. (E1rr)
    Ex[0][0][0] = exp(-mu * XAB * XAB);
    const int up = (a.deriv || a.rderiv) ? 1 : 0;
    const int lae = la + up, lbe = lb + up;  // one more on each centre for derivatives
    for (int i = 0; i < lae; ++i)  // Eq. (E2rr1), b = 0
      for (int t = 0; t <= i + 1; ++t)
        Ex[i + 1][0][t] = (t > 0 ? o2p * Ex[i][0][t - 1] : 0.0) + XPA * Ex[i][0][t] + (t + 1) * Ex[i][0][t + 1];
    for (int i = 0; i <= lae; ++i)  // Eq. (E2rr2)
      for (int j = 0; j < lbe; ++j)
        for (int t = 0; t <= i + j + 1; ++t)
          Ex[i][j + 1][t] = (t > 0 ? o2p * Ex[i][j][t - 1] : 0.0) + XPB * Ex[i][j][t] + (t + 1) * Ex[i][j][t + 1];
    if (x == 0) sc[0] = a.basis.coefs[d.pa] * (a.one_centre ? 1.0 : a.basis.coefs[d.pb]);
  }
  if (tid == 0) {
    double *G = a.G + 4 * (size_t)pp;
    G[0] = p;
    G[1] = (za * A[0] + zb * B[0]) / p;
    G[2] = (za * A[1] + zb * B[1]) / p;
    G[3] = (za * A[2] + zb * B[2]) / p;
  }
  __syncthreads();
  const double cab = sc[0];
  const int Nbb = nsph(lb);
  if (a.deriv) {
    // d/dA_x (x_A^{a} e^{-za r_A^2}) = 2 za x_A^{a+1x} e^{..} - a_x x_A^{a-1x} e^{..},
    // the same for B: H^(X,x)[p][ab] = c_a c_b sum C C [2 z E^{(a+1x) b}_p - a_x E^{(a-1x) b}_p]
    // stored transposed, [mat][ab][p] with p fastest (the gradient stage of
    // the quartet engine reads 16 consecutive p per lane group)
    double *H = a.H + (size_t)pp * (7 + (a.rderiv ? 3 : 0)) * a.Nh_pad * a.N_pad;
    const int total = 6 * a.Nh_pad * a.N_pad;
    for (int e = tid; e < total; e += kPairThreads) {
      const int mat = e / (a.Nh_pad * a.N_pad);
      const int rem = e - mat * (a.Nh_pad * a.N_pad);
      const int ab = rem / a.Nh_pad;
      const int ph = rem - ab * a.Nh_pad;
      const int cen = mat / 3, dir = mat - 3 * cen;  // cen 0 = A, 1 = B
      double h = 0.0;
      const uint32_t hp = a.order[ph];
      if (!(hp & kPadRow) && ab < a.N) {
        const int tq[3] = {(int)(hp & 0xff), (int)((hp >> 8) & 0xff), (int)((hp >> 16) & 0xff)};
        const int ma = ab / Nbb - la, mb = ab % Nbb - lb;
        const int s0 = a.tab.solid_start[solid_slot(la, ma)], s1 = a.tab.solid_start[solid_slot(la, ma) + 1];
        const int r0 = a.tab.solid_start[solid_slot(lb, mb)], r1 = a.tab.solid_start[solid_slot(lb, mb) + 1];
        const double z2 = 2.0 * (cen == 0 ? za : zb);
        for (int s_ = s0; s_ < s1; ++s_) {
          const uint32_t ca = a.tab.solid_cart[s_];
          const int av[3] = {(int)(ca & 0xff), (int)((ca >> 8) & 0xff), (int)((ca >> 16) & 0xff)};
          double inner = 0.0;
          for (int r = r0; r < r1; ++r) {
            const uint32_t cb = a.tab.solid_cart[r];
            int bv[3] = {(int)(cb & 0xff), (int)((cb >> 8) & 0xff), (int)((cb >> 16) & 0xff)};
            int up[3] = {av[0], av[1], av[2]}, vp[3] = {bv[0], bv[1], bv[2]};
            // raised / lowered component on the differentiated centre
            int *sh = cen == 0 ? up : vp;
            const int n0 = sh[dir];
            double term = 0.0;
            sh[dir] = n0 + 1;
            if (tq[0] <= up[0] + vp[0] && tq[1] <= up[1] + vp[1] && tq[2] <= up[2] + vp[2])
              term += z2 * E[0][up[0]][vp[0]][tq[0]] * E[1][up[1]][vp[1]][tq[1]] * E[2][up[2]][vp[2]][tq[2]];
            if (n0 > 0) {
              sh[dir] = n0 - 1;
              if (tq[0] <= up[0] + vp[0] && tq[1] <= up[1] + vp[1] && tq[2] <= up[2] + vp[2])
                term -= n0 * E[0][up[0]][vp[0]][tq[0]] * E[1][up[1]][vp[1]][tq[1]] * E[2][up[2]][vp[2]][tq[2]];
            }
            inner += a.tab.solid_coef[r] * term;
          }
          h += a.tab.solid_coef[s_] * inner;
        }
        h *= cab;
      }
      H[e] = h;
    }
    // the plain matrix follows the six derivative matrices ([p][ab], no sign)
  }
  const size_t mats = (a.deriv ? 6 : 0) + 1 + (a.rderiv ? 3 : 0);
  double *H = a.H + (size_t)pp * mats * a.Nh_pad * a.N_pad + (a.deriv ? 6 * (size_t)a.Nh_pad * a.N_pad : 0);
  const int total = a.Nh_pad * a.N_pad;
  for (int e = tid; e < total; e += kPairThreads) {
    const int ph = e / a.N_pad;
    const int ab = e - ph * a.N_pad;
    double h = 0.0;
    const uint32_t hp = a.order ? a.order[ph] : (ph < a.Nh ? a.tab.herm[ph] : kPadRow);
    if (!(hp & kPadRow) && ab < a.N) {
      const int t = hp & 0xff, u = (hp >> 8) & 0xff, v = (hp >> 16) & 0xff;
      const int ma = ab / Nbb - la, mb = ab % Nbb - lb;
      const int s0 = a.tab.solid_start[solid_slot(la, ma)], s1 = a.tab.solid_start[solid_slot(la, ma) + 1];
      const int r0 = a.tab.solid_start[solid_slot(lb, mb)], r1 = a.tab.solid_start[solid_slot(lb, mb) + 1];
      for (int s = s0; s < s1; ++s) {
        const uint32_t ca = a.tab.solid_cart[s];
        const int ax = ca & 0xff, ay = (ca >> 8) & 0xff, az = (ca >> 16) & 0xff;
        double inner = 0.0;
        for (int r = r0; r < r1; ++r) {
          const uint32_t cb = a.tab.solid_cart[r];
          const int bx = cb & 0xff, by = (cb >> 8) & 0xff, bz = (cb >> 16) & 0xff;
          if (t <= ax + bx && u <= ay + by && v <= az + bz)
            inner += a.tab.solid_coef[r] * E[0][ax][bx][t] * E[1][ay][by][u] * E[2][az][bz][v];
        }
        h += a.tab.solid_coef[s] * inner;
      }
      h *= cab;
      if (a.ket_sign && ((t + u + v) & 1)) h = -h;
    }
    H[e] = h;
  }
  if (a.rderiv) {
    // derivatives with respect to the relative coordinate R = A - B at fixed
    // P (ket pairs: d/dC = (zeta_c/q) d/dQ + d/dR); with Lambda_t the
    // derivatives of exp(-p x_P^2) with respect to P_x (so d/dP Lambda_t =
    // Lambda_{t+1}) and d/dA x_A^i = 2 za x_A^{i+1} - i x_A^{i-1}, the
    // coefficient of Lambda_t in d/dR_x of x_A^i x_B^j e^{..} is
    //   2 za E^{i+1,j}_t - i E^{i-1,j}_t - (za / p) E^{ij}_{t-1};
    // matrices 1..3 after the plain one, [x][p][ab] ([x][ab][p] with
    // rtrans), ket sign included
    const double za_p = za / p;
    double *Hr = H + (size_t)a.Nh_pad * a.N_pad;
    for (int e = tid; e < 3 * total; e += kPairThreads) {
      const int dir = e / total, rem = e - dir * total;
      const int ph = rem / a.N_pad, ab = rem - ph * a.N_pad;
      double h = 0.0;
      const uint32_t hp = a.order ? a.order[ph] : (ph < a.Nh ? a.tab.herm[ph] : kPadRow);
      if (!(hp & kPadRow) && ab < a.N) {
        const int tq[3] = {(int)(hp & 0xff), (int)((hp >> 8) & 0xff), (int)((hp >> 16) & 0xff)};
        const int ma = ab / Nbb - la, mb = ab % Nbb - lb;
        const int s0 = a.tab.solid_start[solid_slot(la, ma)], s1 = a.tab.solid_start[solid_slot(la, ma) + 1];
        const int r0 = a.tab.solid_start[solid_slot(lb, mb)], r1 = a.tab.solid_start[solid_slot(lb, mb) + 1];
        for (int s_ = s0; s_ < s1; ++s_) {
          const uint32_t ca = a.tab.solid_cart[s_];
          const int av[3] = {(int)(ca & 0xff), (int)((ca >> 8) & 0xff), (int)((ca >> 16) & 0xff)};
          double inner = 0.0;
          for (int r = r0; r < r1; ++r) {
            const uint32_t cb = a.tab.solid_cart[r];
            const int bv[3] = {(int)(cb & 0xff), (int)((cb >> 8) & 0xff), (int)((cb >> 16) & 0xff)};
            double f = 1.0;
            for (int x = 0; x < 3 && f != 0.0; ++x) {
              const int i = av[x], j = bv[x], t = tq[x];
              if (x != dir) {
                f *= t <= i + j ? E[x][i][j][t] : 0.0;
              } else {
                double d = 2.0 * za * (t <= i + j + 1 ? E[x][i + 1][j][t] : 0.0);
                if (i > 0 && t <= i + j - 1) d -= i * E[x][i - 1][j][t];
                if (t > 0 && t - 1 <= i + j) d -= za_p * E[x][i][j][t - 1];
                f *= d;
              }
            }
            inner += a.tab.solid_coef[r] * f;
          }
          h += a.tab.solid_coef[s_] * inner;
        }
        h *= cab;
        if (a.ket_sign && ((tq[0] + tq[1] + tq[2]) & 1)) h = -h;
      }
      Hr[a.rtrans ? (size_t)dir * total + (size_t)ab * a.Nh_pad + ph : (size_t)e] = h;
    }
  }
  if (!a.split) return;
  // Split precision.  Rows are balanced first: row p of H is scaled by
  // 2^-k_p (k_p: exponent of its largest |H[p][ab]|) and the fused kernel
  // scales row p of [p|ket] by 2^+k_p, which leaves the products unchanged
  // and exact.  Then per column ab an exponent E with |H~[p][ab]| < 2^E over
  // all rows, and H~ 2^-E = sum_s h_s 128^-s with integers |h_1| <= 128 and
  // |h_s| <= 64 (s > 1), each exact in BF16.  Slices are stored in the k
  // order of the BF16 16x16x32 operand: position 32 b + 8 g + e of a column
  // holds row 32 b + 16 (e / 4) + 4 (e % 4) + g (two 16-row tiles per block;
  // lane group g of the consumer wave holds rows 4 r + g of each tile).
  __syncthreads();  // H of this primitive pair written by the whole workgroup
  int *Kr = a.Hrow + (size_t)pp * a.Hs_rows;
  for (int ph = tid; ph < a.Hs_rows; ph += kPairThreads) {
    double mx = 0.0;
    if (ph < a.Nh_pad)
      for (int ab = 0; ab < a.N_pad; ++ab) mx = fmax(mx, fabs(H[(size_t)ph * a.N_pad + ab]));
    // mx = f 2^ex, f in [0.5, 1); a zero row (padding, or a Hermite function
    // the pair does not use) sends its [p|ket] row to zero (2^-2000 underflows)
    // so that it cannot set the column exponents of the kernel's operand
    int ex = -2000;
    if (mx > 0.0) (void)frexp(mx, &ex);
    Kr[ph] = ex;
  }
  __syncthreads();
  int *Ex = a.Hexp + (size_t)pp * a.N_pad;
  for (int ab = tid; ab < a.N_pad; ab += kPairThreads) {
    double mx = 0.0;
    for (int ph = 0; ph < a.Nh_pad; ++ph) mx = fmax(mx, fabs(ldexp(H[(size_t)ph * a.N_pad + ab], -Kr[ph])));
    int ex = 0;
    if (mx > 0.0) (void)frexp(mx, &ex);
    Ex[ab] = ex;
  }
  __syncthreads();
  uint16_t *Hs = a.Hs + (size_t)pp * a.split * a.N_pad * a.Hs_rows;
  for (int e = tid; e < a.N_pad * a.Hs_rows; e += kPairThreads) {
    const int ab = e / a.Hs_rows, pos = e - ab * a.Hs_rows;
    const int blk = pos >> 5, g = (pos >> 3) & 3, ee = pos & 7;
    const int row = 32 * blk + 16 * (ee >> 2) + 4 * (ee & 3) + g;
    double r = row < a.Nh_pad ? ldexp(H[(size_t)row * a.N_pad + ab], -Kr[row] - Ex[ab]) : 0.0;
    for (int sl = 0; sl < a.split; ++sl) {
      const double v = r * 128.0;
      const double t = rint(v);
      r = v - t;
      // |t| <= 128: an integer of at most 8 significant bits, exact in BF16
      // (the upper half of its FP32 pattern)
      const float tf = (float)t;
      Hs[((size_t)sl * a.N_pad + ab) * a.Hs_rows + pos] = (uint16_t)(__float_as_uint(tf) >> 16);
    }
  }
}

}  // namespace

hipError_t launch_pairs(const PairArgs &a, hipStream_t s) {
  if (a.npp <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_kernel, dim3(a.npp), dim3(kPairThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace mderi
