/*
 * oracle.c -- plain FP64 CPU oracle for McMurchie-Davidson two-electron
 * integrals.  TEST INFRASTRUCTURE ONLY (see oracle.h): loaded by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg, never by the
 * GPU library.
 *
 * Every step follows Sec. 2 ("Formalism") of Asadchev & Valeev in the
 * paper's order and notation, written out as plain nested sums:
 *   Eq. (boys)        Boys function F_m(x)                  -> oracle_boys
 *   Eqs. (E2rr1/2), (E2-000), (E2-abp)   2-centre E         -> oracle_E2
 *   Eqs. (E1rr), (E1-00), (E1-aa)        1-centre E         -> oracle_E1
 *   Eqs. (0m), (r)    auxiliary integrals [r]^(m)           -> oracle_R
 *   Eq. (pq) and Eqs. (ket-from-hermite), (bra-from-hermite) in Cartesian
 *                     sum form                              -> prim_cart
 *   Eqs. (solid2herm-1/2): Cartesian -> real solid harmonics,
 *                     applied after contraction             -> oracle_solid
 *   Sec. 6 exchange operator, brute force                  -> oracle_kbuild
 *   Coulomb operator (the J half of the Fock build)        -> oracle_jbuild
 *   selected shell blocks of K or J                        -> oracle_fock_blocks
 *   2-centre Coulomb metric (P|Q)                          -> oracle_eri2
 *   gradient of sum W (ab|cd), exchange or Coulomb weights -> oracle_grad_pattern
 * Nuclear derivatives use d/dA_x [x_A^a e^{-z r_A^2}] =
 * 2 z x_A^{a+1} e^{..} - a x_A^{a-1} e^{..} on Cartesian primitives.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846
static const long double PI_L = 3.141592653589793238462643383279502884L;

typedef struct {
  int l, K;
  double A[3];
  double z[ORACLE_KMAX];
  double c[ORACLE_KMAX]; /* normalised contraction coefficients */
} oshell;

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int nsph(int l) { return 2 * l + 1; }

/* Cartesian components of a shell: lx descending, then ly descending. */
static void cart_list(int l, int (*out)[3]) {
  int k = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      out[k][0] = lx;
      out[k][1] = ly;
      out[k][2] = l - lx - ly;
      ++k;
    }
}

static int cart_index(int lx, int ly, int lz) {
  int l = lx + ly + lz;
  int r = l - lx; /* components before this lx block: sum_{k<r} (k+1) */
  return r * (r + 1) / 2 + (r - ly);
}

/* ------------------------------------------------------------------ */
/* Boys function, Eq. (boys): F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy.   */
/* Small x: the all-positive series                                     */
/*   F_m(x) = e^{-x} sum_k (2x)^k / [(2m+1)(2m+3)...(2m+2k+1)]          */
/* for m = mmax, then the stable downward recursion                     */
/*   F_m = (2x F_{m+1} + e^{-x}) / (2m+1).                              */
/* Large x: F_0 = (1/2) sqrt(pi/x) erf(sqrt x) and the upward recursion */
/*   F_{m+1} = ((2m+1) F_m - e^{-x}) / (2x),                            */
/* which is stable once x exceeds 2*mmax+30.  Long double throughout.   */
/* ------------------------------------------------------------------ */
void oracle_boys(int mmax, double T, double *F) {
  long double t = T > 0 ? (long double)T : 0.0L;
  long double et = expl(-t);
  if (t < 2.0L * mmax + 30.0L) {
    long double term = 1.0L / (2 * mmax + 1), sum = term;
    for (int k = 1; k < 100000; ++k) {
      term *= 2.0L * t / (2 * mmax + 2 * k + 1);
      sum += term;
      if (k > t && term < 1e-22L * sum) break;
    }
    long double f = et * sum;
    F[mmax] = (double)f;
    for (int m = mmax - 1; m >= 0; --m) {
      f = (2.0L * t * f + et) / (2 * m + 1);
      F[m] = (double)f;
    }
  } else {
    long double f = 0.5L * sqrtl(PI_L / t) * erfl(sqrtl(t));
    F[0] = (double)f;
    for (int m = 0; m < mmax; ++m) {
      f = ((2 * m + 1) * f - et) / (2.0L * t);
      F[m + 1] = (double)f;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Hermite expansion coefficients                                      */
/* ------------------------------------------------------------------ */
void oracle_E2(int la, int lb, double za, double zb, double Ax, double Bx, double *E) {
  const int nt = la + lb + 1;
  const double p = za + zb;
  const double P = (za * Ax + zb * Bx) / p;
  const double mu = za * zb / p;
  const double XPA = P - Ax, XPB = P - Bx, XAB = Ax - Bx;
  const double o2p = 0.5 / p;
#define E2AT(i, j, t) E[((i) * (lb + 1) + (j)) * nt + (t)]
  memset(E, 0, sizeof(double) * (size_t)(la + 1) * (lb + 1) * nt);
  E2AT(0, 0, 0) = exp(-mu * XAB * XAB); /* Eq. (E2-000) */
  /* Eq. (E2rr1) with b = 0; terms outside t in [0, i+j] vanish, Eq. (E2-abp) */
  for (int i = 0; i < la; ++i)
    for (int t = 0; t <= i + 1; ++t) {
      double v = 0.0;
      if (t >= 1) v += o2p * E2AT(i, 0, t - 1);
      if (t <= i) v += XPA * E2AT(i, 0, t);
      if (t + 1 <= i) v += (t + 1) * E2AT(i, 0, t + 1);
      E2AT(i + 1, 0, t) = v;
    }
  /* Eq. (E2rr2) */
  for (int i = 0; i <= la; ++i)
    for (int j = 0; j < lb; ++j)
      for (int t = 0; t <= i + j + 1; ++t) {
        double v = 0.0;
        if (t >= 1) v += o2p * E2AT(i, j, t - 1);
        if (t <= i + j) v += XPB * E2AT(i, j, t);
        if (t + 1 <= i + j) v += (t + 1) * E2AT(i, j, t + 1);
        E2AT(i, j + 1, t) = v;
      }
#undef E2AT
}

void oracle_E1(int la, double za, double *E) {
  const int nt = la + 1;
  memset(E, 0, sizeof(double) * (size_t)(la + 1) * nt);
  E[0] = 1.0; /* Eq. (E1-00) */
  /* Eq. (E1rr); entries outside [0, a] vanish, Eq. (E1-aa) */
  for (int i = 0; i < la; ++i)
    for (int t = 0; t <= i + 1; ++t) {
      double v = 0.0;
      if (t >= 1) v += E[i * nt + t - 1] / (2.0 * za);
      if (t + 1 <= i) v += (t + 1) * E[i * nt + t + 1];
      E[(i + 1) * nt + t] = v;
    }
}

/* ------------------------------------------------------------------ */
/* Auxiliary integrals, Eqs. (0m) and (r)                               */
/* ------------------------------------------------------------------ */
static void R_work(int L, double rho, const double PQ[3], double pref, double *R, double *W, double *F) {
  const size_t n1 = (size_t)L + 1;
#define RW(n, t, u, v) W[(((size_t)(n) * n1 + (t)) * n1 + (u)) * n1 + (v)]
  oracle_boys(L, rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]), F);
  double f = pref;
  for (int n = 0; n <= L; ++n) { /* Eq. (0m): [0]^(n) = (-2 rho)^n pref F_n */
    RW(n, 0, 0, 0) = f * F[n];
    f *= -2.0 * rho;
  }
  /* Eq. (r): [r + 1_i]^(m) = r_i [r - 1_i]^(m+1) + (P_i - Q_i) [r]^(m+1),
   * raising the first non-zero Cartesian direction of each target. */
  for (int lev = 1; lev <= L; ++lev)
    for (int n = 0; n <= L - lev; ++n)
      for (int t = 0; t <= lev; ++t)
        for (int u = 0; u <= lev - t; ++u) {
          int v = lev - t - u;
          double val;
          if (t > 0) {
            val = PQ[0] * RW(n + 1, t - 1, u, v);
            if (t > 1) val += (t - 1) * RW(n + 1, t - 2, u, v);
          } else if (u > 0) {
            val = PQ[1] * RW(n + 1, t, u - 1, v);
            if (u > 1) val += (u - 1) * RW(n + 1, t, u - 2, v);
          } else {
            val = PQ[2] * RW(n + 1, t, u, v - 1);
            if (v > 1) val += (v - 1) * RW(n + 1, t, u, v - 2);
          }
          RW(n, t, u, v) = val;
        }
  memset(R, 0, sizeof(double) * n1 * n1 * n1);
  for (int t = 0; t <= L; ++t)
    for (int u = 0; u <= L - t; ++u)
      for (int v = 0; v <= L - t - u; ++v) R[(t * n1 + u) * n1 + v] = RW(0, t, u, v);
#undef RW
}

void oracle_R(int L, double rho, const double PQ[3], double pref, double *R) {
  const size_t n1 = (size_t)L + 1;
  double *W = (double *)calloc(n1 * n1 * n1 * n1, sizeof(double));
  double *F = (double *)malloc(sizeof(double) * n1);
  R_work(L, rho, PQ, pref, R, W, F);
  free(W);
  free(F);
}

/* ------------------------------------------------------------------ */
/* Cartesian -> real solid harmonics (the C of Eqs. (solid2herm-1/2)), */
/* written from the closed form of the real regular solid harmonics   */
/*   S_lm = N_lm sum_{t,u,v} C^{lm}_{tuv}                              */
/*          x^{2t+|m|-2(u+v)} y^{2(u+v)} z^{l-2t-|m|}                  */
/*   C^{lm}_{tuv} = (-1)^{t+v-vm} 4^{-t} binom(l,t) binom(l-t,|m|+t)   */
/*                  binom(t,u) binom(|m|,2v),                           */
/*   N_lm = sqrt(2 (l+|m|)! (l-|m|)! / 2^{delta_m0}) / (2^|m| l!),      */
/* with vm = 0 (m >= 0) or 1/2 (m < 0) and v running over vm, vm+1, .. */
/* This normalisation gives S_lm the same norm on the sphere as x^l.   */
/* ------------------------------------------------------------------ */
static double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  return fact(n) / (fact(k) * fact(n - k));
}

void oracle_solid(int l, double *C) {
  const int nc = ncart(l);
  memset(C, 0, sizeof(double) * (size_t)nsph(l) * nc);
  for (int m = -l; m <= l; ++m) {
    const int am = m < 0 ? -m : m;
    const double Nlm = sqrt(2.0 * fact(l + am) * fact(l - am) / (m == 0 ? 2.0 : 1.0)) / (pow(2.0, am) * fact(l));
    /* 2v is an integer: twov = 0,2,4,.. (m >= 0) or 1,3,5,.. (m < 0) */
    const int twovm = m < 0 ? 1 : 0;
    for (int t = 0; t <= (l - am) / 2; ++t)
      for (int u = 0; u <= t; ++u)
        for (int twov = twovm; twov <= am; twov += 2) {
          /* v - vm = (twov - twovm)/2 */
          const int sgnexp = t + (twov - twovm) / 2;
          const double coef = (sgnexp % 2 ? -1.0 : 1.0) * pow(0.25, t) * binom(l, t) * binom(l - t, am + t) *
                              binom(t, u) * binom(am, twov);
          const int ypow = 2 * u + twov; /* 2(u+v) */
          const int xpow = 2 * t + am - ypow;
          const int zpow = l - 2 * t - am;
          if (xpow < 0 || zpow < 0) continue;
          C[(m + l) * nc + cart_index(xpow, ypow, zpow)] += Nlm * coef;
        }
  }
}

/* ------------------------------------------------------------------ */
/* Normalisation of contracted shells                                  */
/* ------------------------------------------------------------------ */
static double dfact_odd(int n) { /* n!! for odd n >= -1 */
  double r = 1.0;
  for (int i = n; i > 1; i -= 2) r *= i;
  return r;
}

void oracle_norm_coefs(int l, int K, const double *z, const double *c, int normalize, double *out) {
  if (!normalize) {
    for (int k = 0; k < K; ++k) out[k] = c[k];
    return;
  }
  /* norm of the contraction of unit-normalised primitives x^l exp(-z r^2),
   * whose pairwise overlap on one centre is (2 sqrt(z z')/(z+z'))^{l+3/2} */
  double S = 0.0;
  for (int k = 0; k < K; ++k)
    for (int kk = 0; kk < K; ++kk) S += c[k] * c[kk] * pow(2.0 * sqrt(z[k] * z[kk]) / (z[k] + z[kk]), l + 1.5);
  const double s = 1.0 / sqrt(S);
  /* primitive normalisation (2z/pi)^{3/4} (4z)^{l/2} / sqrt((2l-1)!!) */
  for (int k = 0; k < K; ++k)
    out[k] = s * c[k] * pow(2.0 * z[k] / PI_D, 0.75) * pow(4.0 * z[k], 0.5 * l) / sqrt(dfact_odd(2 * l - 1));
}

/* ------------------------------------------------------------------ */
/* Basis handling                                                       */
/* ------------------------------------------------------------------ */
static int build_shells(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                        const double *centers, int normalize, int lmax, oshell **out) {
  oshell *s = (oshell *)calloc((size_t)(nshell > 0 ? nshell : 1), sizeof(oshell));
  int off = 0;
  for (int i = 0; i < nshell; ++i) {
    if (l[i] < 0 || l[i] > lmax || nprim[i] < 1 || nprim[i] > ORACLE_KMAX) {
      free(s);
      return -1;
    }
    s[i].l = l[i];
    s[i].K = nprim[i];
    for (int x = 0; x < 3; ++x) s[i].A[x] = centers[3 * i + x];
    for (int k = 0; k < nprim[i]; ++k) {
      s[i].z[k] = exps[off + k];
      if (!(exps[off + k] > 0.0)) {
        free(s);
        return -1;
      }
    }
    oracle_norm_coefs(l[i], nprim[i], exps + off, coefs + off, normalize, s[i].c);
    off += nprim[i];
  }
  *out = s;
  return 0;
}

/* Per-thread scratch, sized for shells up to ORACLE_LMAX. */
typedef struct {
  double *R, *RW, *F, *W, *E[6];
  int *hidx;
} scratch;

#define LTOT_MAX (4 * ORACLE_LMAX)
static void scratch_init(scratch *s) {
  const size_t n1 = LTOT_MAX + 1;
  s->R = (double *)malloc(sizeof(double) * n1 * n1 * n1);
  s->RW = (double *)calloc(n1 * n1 * n1 * n1, sizeof(double));
  s->F = (double *)malloc(sizeof(double) * n1);
  /* W[hermite of bra][cart c][cart d] */
  const size_t nh = (size_t)(2 * ORACLE_LMAX + 1) * (2 * ORACLE_LMAX + 2) * (2 * ORACLE_LMAX + 3) / 6;
  s->W = (double *)malloc(sizeof(double) * nh * ncart(ORACLE_LMAX) * ncart(ORACLE_LMAX));
  for (int x = 0; x < 6; ++x)
    s->E[x] = (double *)malloc(sizeof(double) * (ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (2 * ORACLE_LMAX + 1));
  s->hidx = (int *)malloc(sizeof(int) * (2 * ORACLE_LMAX + 1) * (2 * ORACLE_LMAX + 1) * (2 * ORACLE_LMAX + 1));
}
static void scratch_free(scratch *s) {
  free(s->R);
  free(s->RW);
  free(s->F);
  free(s->W);
  for (int x = 0; x < 6; ++x) free(s->E[x]);
  free(s->hidx);
}

/*
 * Primitive Cartesian integrals, accumulated as out += w * [ab|cd] for all
 * Cartesian components (row-major [a][b][c][d]).  lb/ld may be zero-exponent
 * placeholders only through the 3-centre path below.  onecentre != 0 makes the
 * ket a single Gaussian (exponent zc at C, Eqs. (E1rr)-(E1-aa)); ld and zd are
 * then ignored.
 */
static void prim_cart(int la, int lb, int lc, int ld, double za, const double *A, double zb, const double *B,
                      double zc, const double *C, double zd, const double *D, int onecentre, double w, double *out,
                      scratch *s) {
  const double p = za + zb;
  const double q = onecentre ? zc : zc + zd;
  double P[3], Q[3], PQ[3];
  for (int x = 0; x < 3; ++x) {
    P[x] = (za * A[x] + zb * B[x]) / p;
    Q[x] = onecentre ? C[x] : (zc * C[x] + zd * D[x]) / q;
    PQ[x] = P[x] - Q[x];
  }
  if (onecentre) ld = 0;
  const double rho = p * q / (p + q);
  const double pref = 2.0 * pow(PI_D, 2.5) / (p * q * sqrt(p + q)); /* Eq. (0m) */
  const int Lab = la + lb, Lcd = lc + ld, L = Lab + Lcd;
  const int nab = Lab + 1, ncd = Lcd + 1;
  const size_t n1 = (size_t)L + 1;

  double *Eab[3] = {s->E[0], s->E[1], s->E[2]};
  double *Ecd[3] = {s->E[3], s->E[4], s->E[5]};
  for (int x = 0; x < 3; ++x) {
    oracle_E2(la, lb, za, zb, A[x], B[x], Eab[x]);
    if (onecentre)
      oracle_E1(lc, zc, Ecd[x]);
    else
      oracle_E2(lc, ld, zc, zd, C[x], D[x], Ecd[x]);
  }
#define EAB(x, i, j, t) Eab[x][((i) * (lb + 1) + (j)) * nab + (t)]
#define ECD(x, i, j, t) (onecentre ? Ecd[x][(i) * (lc + 1) + (t)] : Ecd[x][((i) * (ld + 1) + (j)) * ncd + (t)])
  R_work(L, rho, PQ, pref, s->R, s->RW, s->F);
#define RR(t, u, v) s->R[((t) * n1 + (u)) * n1 + (v)]

  int ca[64][3], cb[64][3], cc[64][3], cd[64][3];
  cart_list(la, ca);
  cart_list(lb, cb);
  cart_list(lc, cc);
  cart_list(ld, cd);
  const int Na = ncart(la), Nb = ncart(lb), Nc = ncart(lc), Nd = ncart(ld);

  /* bra Hermite functions p = (t,u,v), |p| <= la+lb */
  int nh = 0;
  for (int t = 0; t <= Lab; ++t)
    for (int u = 0; u <= Lab - t; ++u)
      for (int v = 0; v <= Lab - t - u; ++v) s->hidx[(t * nab + u) * nab + v] = nh++;

  /* Ket side: Eq. (pq) [p|q] = (-1)^{|q|} [p+q]^(0), summed against the ket
   * Hermite expansion of each Cartesian ket product (Eq. (ket-from-hermite)
   * before the solid-harmonic contraction). */
  for (int t = 0; t <= Lab; ++t)
    for (int u = 0; u <= Lab - t; ++u)
      for (int v = 0; v <= Lab - t - u; ++v) {
        double *Wp = s->W + (size_t)s->hidx[(t * nab + u) * nab + v] * Nc * Nd;
        for (int ic = 0; ic < Nc; ++ic)
          for (int id = 0; id < Nd; ++id) {
            double sum = 0.0;
            for (int tau = 0; tau <= cc[ic][0] + cd[id][0]; ++tau)
              for (int nu = 0; nu <= cc[ic][1] + cd[id][1]; ++nu)
                for (int phi = 0; phi <= cc[ic][2] + cd[id][2]; ++phi) {
                  const double sgn = ((tau + nu + phi) & 1) ? -1.0 : 1.0;
                  sum += sgn * ECD(0, cc[ic][0], cd[id][0], tau) * ECD(1, cc[ic][1], cd[id][1], nu) *
                         ECD(2, cc[ic][2], cd[id][2], phi) * RR(t + tau, u + nu, v + phi);
                }
            Wp[ic * Nd + id] = sum;
          }
      }
  /* Bra side, Eq. (bra-from-hermite) before the solid-harmonic contraction. */
  for (int ia = 0; ia < Na; ++ia)
    for (int ib = 0; ib < Nb; ++ib) {
      double *o = out + ((size_t)ia * Nb + ib) * Nc * Nd;
      for (int t = 0; t <= ca[ia][0] + cb[ib][0]; ++t)
        for (int u = 0; u <= ca[ia][1] + cb[ib][1]; ++u)
          for (int v = 0; v <= ca[ia][2] + cb[ib][2]; ++v) {
            const double e = w * EAB(0, ca[ia][0], cb[ib][0], t) * EAB(1, ca[ia][1], cb[ib][1], u) *
                             EAB(2, ca[ia][2], cb[ib][2], v);
            const double *Wp = s->W + (size_t)s->hidx[(t * nab + u) * nab + v] * Nc * Nd;
            for (int k = 0; k < Nc * Nd; ++k) o[k] += e * Wp[k];
          }
    }
#undef EAB
#undef ECD
#undef RR
}

/* Contracted Cartesian 4-centre shell quartet: out[a][b][c][d]. */
static void shell_cart4(const oshell *a, const oshell *b, const oshell *c, const oshell *d, double *out,
                        scratch *s) {
  const size_t n = (size_t)ncart(a->l) * ncart(b->l) * ncart(c->l) * ncart(d->l);
  memset(out, 0, sizeof(double) * n);
  for (int ka = 0; ka < a->K; ++ka)
    for (int kb = 0; kb < b->K; ++kb)
      for (int kc = 0; kc < c->K; ++kc)
        for (int kd = 0; kd < d->K; ++kd)
          prim_cart(a->l, b->l, c->l, d->l, a->z[ka], a->A, b->z[kb], b->A, c->z[kc], c->A, d->z[kd], d->A, 0,
                    a->c[ka] * b->c[kb] * c->c[kc] * d->c[kd], out, s);
}

/* Contracted Cartesian 3-centre shell triple (ab|c): out[a][b][c]. */
static void shell_cart3(const oshell *a, const oshell *b, const oshell *c, double *out, scratch *s) {
  const size_t n = (size_t)ncart(a->l) * ncart(b->l) * ncart(c->l);
  memset(out, 0, sizeof(double) * n);
  for (int ka = 0; ka < a->K; ++ka)
    for (int kb = 0; kb < b->K; ++kb)
      for (int kc = 0; kc < c->K; ++kc)
        prim_cart(a->l, b->l, c->l, 0, a->z[ka], a->A, b->z[kb], b->A, c->z[kc], c->A, 0.0, c->A, 1,
                  a->c[ka] * b->c[kb] * c->c[kc], out, s);
}

/* Transform index `which` (0..nidx-1) of a row-major tensor with dims
 * dim[] from Cartesian to solid harmonics (dim[which] changes to 2l+1). */
static void solid_index(double *in, double *outb, int nidx, int *dim, int which, int l) {
  double C[(2 * ORACLE_LMAX + 1) * ((ORACLE_LMAX + 1) * (ORACLE_LMAX + 2) / 2)];
  oracle_solid(l, C);
  const int nc = ncart(l), ns = nsph(l);
  size_t outer = 1, inner = 1;
  for (int i = 0; i < which; ++i) outer *= dim[i];
  for (int i = which + 1; i < nidx; ++i) inner *= dim[i];
  for (size_t o = 0; o < outer; ++o)
    for (int m = 0; m < ns; ++m)
      for (size_t in_ = 0; in_ < inner; ++in_) {
        double acc = 0.0;
        for (int k = 0; k < nc; ++k) acc += C[m * nc + k] * in[(o * nc + k) * inner + in_];
        outb[(o * ns + m) * inner + in_] = acc;
      }
  dim[which] = ns;
}

/* Full solid transform of a 4-index (or 3-index) Cartesian tensor.
 * buf and tmp must each hold the Cartesian size; the result ends in res. */
static void solid_all(double *buf, double *tmp, int nidx, const int *ls, double *res) {
  int dim[4];
  for (int i = 0; i < nidx; ++i) dim[i] = ncart(ls[i]);
  double *src = buf, *dst = tmp;
  for (int i = 0; i < nidx; ++i) {
    solid_index(src, dst, nidx, dim, i, ls[i]);
    double *t = src;
    src = dst;
    dst = t;
  }
  size_t n = 1;
  for (int i = 0; i < nidx; ++i) n *= dim[i];
  memcpy(res, src, sizeof(double) * n);
}

static size_t cart4_size(int a, int b, int c, int d) {
  return (size_t)ncart(a) * ncart(b) * ncart(c) * ncart(d);
}

/* ------------------------------------------------------------------ */
/* Public API                                                           */
/* ------------------------------------------------------------------ */
int oracle_eri4_cart(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                     const double *centers, int normalize, int i, int j, int k, int m, double *out) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  if (i < 0 || j < 0 || k < 0 || m < 0 || i >= nshell || j >= nshell || k >= nshell || m >= nshell) {
    free(sh);
    return -1;
  }
  scratch s;
  scratch_init(&s);
  shell_cart4(&sh[i], &sh[j], &sh[k], &sh[m], out, &s);
  scratch_free(&s);
  free(sh);
  return 0;
}

static void shell_solid4(const oshell *a, const oshell *b, const oshell *c, const oshell *d, double *res,
                         double *buf, double *tmp, scratch *s) {
  shell_cart4(a, b, c, d, buf, s);
  const int ls[4] = {a->l, b->l, c->l, d->l};
  solid_all(buf, tmp, 4, ls, res);
}

static int max_threads(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

int oracle_eri4(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                const double *centers, int normalize, int nbra, const int *bra, int nket, const int *ket,
                double *V, int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  if (nbra <= 0 || nket <= 0) {
    free(sh);
    return 0;
  }
  for (int n = 0; n < nbra; ++n)
    if (bra[2 * n] < 0 || bra[2 * n] >= nshell || bra[2 * n + 1] < 0 || bra[2 * n + 1] >= nshell ||
        sh[bra[2 * n]].l != sh[bra[0]].l || sh[bra[2 * n + 1]].l != sh[bra[1]].l) {
      free(sh);
      return -2;
    }
  for (int n = 0; n < nket; ++n)
    if (ket[2 * n] < 0 || ket[2 * n] >= nshell || ket[2 * n + 1] < 0 || ket[2 * n + 1] >= nshell ||
        sh[ket[2 * n]].l != sh[ket[0]].l || sh[ket[2 * n + 1]].l != sh[ket[1]].l) {
      free(sh);
      return -2;
    }
  const int la = sh[bra[0]].l, lb = sh[bra[1]].l, lc = sh[ket[0]].l, ld = sh[ket[1]].l;
  const int Nab = nsph(la) * nsph(lb), Ncd = nsph(lc) * nsph(ld);
  const size_t ncartq = cart4_size(la, lb, lc, ld);
  const long nq = (long)nbra * nket;
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * ncartq);
    double *tmp = (double *)malloc(sizeof(double) * ncartq);
    double *res = (double *)malloc(sizeof(double) * ncartq);
#pragma omp for schedule(dynamic, 1)
    for (long q = 0; q < nq; ++q) {
      const int ij = (int)(q % nbra), kl = (int)(q / nbra);
      shell_solid4(&sh[bra[2 * ij]], &sh[bra[2 * ij + 1]], &sh[ket[2 * kl]], &sh[ket[2 * kl + 1]], res, buf, tmp,
                   &s);
      for (int ab = 0; ab < Nab; ++ab)
        for (int cd = 0; cd < Ncd; ++cd)
          V[ij + (size_t)nbra * (ab + (size_t)Nab * (cd + (size_t)Ncd * kl))] = res[(size_t)ab * Ncd + cd];
    }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  free(sh);
  return 0;
}

int oracle_eri3(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                const double *centers, int naux_shell, const int *al, const int *anprim, const double *aexps,
                const double *acoefs, const double *acenters, int normalize, int npair, const int *pairs, int naux,
                const int *aux, double *V, int nthreads) {
  oshell *sh, *ax;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  if (build_shells(naux_shell, al, anprim, aexps, acoefs, acenters, normalize, ORACLE_LMAX - 1, &ax)) {
    free(sh);
    return -1;
  }
  if (npair <= 0 || naux <= 0) {
    free(sh);
    free(ax);
    return 0;
  }
  for (int n = 0; n < npair; ++n)
    if (pairs[2 * n] < 0 || pairs[2 * n] >= nshell || pairs[2 * n + 1] < 0 || pairs[2 * n + 1] >= nshell ||
        sh[pairs[2 * n]].l != sh[pairs[0]].l || sh[pairs[2 * n + 1]].l != sh[pairs[1]].l) {
      free(sh);
      free(ax);
      return -2;
    }
  for (int n = 0; n < naux; ++n)
    if (aux[n] < 0 || aux[n] >= naux_shell || ax[aux[n]].l != ax[aux[0]].l) {
      free(sh);
      free(ax);
      return -2;
    }
  const int la = sh[pairs[0]].l, lb = sh[pairs[1]].l, lc = ax[aux[0]].l;
  const int Nab = nsph(la) * nsph(lb), Nc = nsph(lc);
  const size_t ncart3 = (size_t)ncart(la) * ncart(lb) * ncart(lc);
  const long nq = (long)npair * naux;
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * ncart3);
    double *tmp = (double *)malloc(sizeof(double) * ncart3);
    double *res = (double *)malloc(sizeof(double) * ncart3);
#pragma omp for schedule(dynamic, 1)
    for (long q = 0; q < nq; ++q) {
      const int ij = (int)(q % npair), k = (int)(q / npair);
      shell_cart3(&sh[pairs[2 * ij]], &sh[pairs[2 * ij + 1]], &ax[aux[k]], buf, &s);
      const int ls[3] = {la, lb, lc};
      solid_all(buf, tmp, 3, ls, res);
      for (int ab = 0; ab < Nab; ++ab)
        for (int c = 0; c < Nc; ++c)
          V[ij + (size_t)npair * (ab + (size_t)Nab * (c + (size_t)Nc * k))] = res[(size_t)ab * Nc + c];
    }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  free(sh);
  free(ax);
  return 0;
}

/* 2-centre Coulomb integral of two primitive Cartesian shells (a|c), both
 * expanded in Hermite Gaussians about their own centres with the 1-centre
 * coefficients of Eqs. (E1rr)-(E1-aa):
 *   (a|c) = 2 pi^{5/2} / (za zc sqrt(za+zc)) sum_t sum_tau E^a_t E^c_tau
 *           (-1)^{|tau|} R_{t+tau}(rho, A - C),   rho = za zc / (za + zc),
 * the one-centre bra and ket of Eqs. (0m), (r) and (pq).  Adds w * (a|c) to
 * out[ia][ic] (Cartesian components). */
static void prim_cart2(int la, int lc, double za, const double *A, double zc, const double *C, double w,
                       double *out, scratch *s) {
  const double rho = za * zc / (za + zc);
  const double pref = 2.0 * pow(PI_D, 2.5) / (za * zc * sqrt(za + zc));
  const double AC[3] = {A[0] - C[0], A[1] - C[1], A[2] - C[2]};
  const int L = la + lc;
  const size_t n1 = (size_t)L + 1;
  double *Ea = s->E[0], *Ec = s->E[3];
  oracle_E1(la, za, Ea);
  oracle_E1(lc, zc, Ec);
  R_work(L, rho, AC, pref, s->R, s->RW, s->F);
  int ca[64][3], cc[64][3];
  cart_list(la, ca);
  cart_list(lc, cc);
  for (int ia = 0; ia < ncart(la); ++ia)
    for (int ic = 0; ic < ncart(lc); ++ic) {
      double sum = 0.0;
      for (int t = 0; t <= ca[ia][0]; ++t)
        for (int u = 0; u <= ca[ia][1]; ++u)
          for (int v = 0; v <= ca[ia][2]; ++v) {
            const double ea = Ea[ca[ia][0] * (la + 1) + t] * Ea[ca[ia][1] * (la + 1) + u] * Ea[ca[ia][2] * (la + 1) + v];
            if (ea == 0.0) continue;
            for (int tau = 0; tau <= cc[ic][0]; ++tau)
              for (int nu = 0; nu <= cc[ic][1]; ++nu)
                for (int phi = 0; phi <= cc[ic][2]; ++phi) {
                  const double ec = Ec[cc[ic][0] * (lc + 1) + tau] * Ec[cc[ic][1] * (lc + 1) + nu] *
                                    Ec[cc[ic][2] * (lc + 1) + phi];
                  const double sgn = ((tau + nu + phi) & 1) ? -1.0 : 1.0;
                  sum += ea * sgn * ec * s->R[((t + tau) * n1 + (u + nu)) * n1 + (v + phi)];
                }
          }
      out[(size_t)ia * ncart(lc) + ic] += w * sum;
    }
}

int oracle_eri2(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                const double *centers, int normalize, int na, const int *as, int nc, const int *cs, double *V,
                int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  if (na <= 0 || nc <= 0) {
    free(sh);
    return 0;
  }
  for (int n = 0; n < na; ++n)
    if (as[n] < 0 || as[n] >= nshell || sh[as[n]].l != sh[as[0]].l) {
      free(sh);
      return -2;
    }
  for (int n = 0; n < nc; ++n)
    if (cs[n] < 0 || cs[n] >= nshell || sh[cs[n]].l != sh[cs[0]].l) {
      free(sh);
      return -2;
    }
  const int la = sh[as[0]].l, lc = sh[cs[0]].l;
  const int Na = nsph(la), Nc = nsph(lc);
  const size_t ncart2 = (size_t)ncart(la) * ncart(lc);
  const long nq = (long)na * nc;
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * ncart2);
    double *tmp = (double *)malloc(sizeof(double) * ncart2);
    double *res = (double *)malloc(sizeof(double) * ncart2);
#pragma omp for schedule(dynamic, 1)
    for (long q = 0; q < nq; ++q) {
      const int i = (int)(q % na), k = (int)(q / na);
      const oshell *a = &sh[as[i]], *c = &sh[cs[k]];
      memset(buf, 0, sizeof(double) * ncart2);
      for (int ka = 0; ka < a->K; ++ka)
        for (int kc = 0; kc < c->K; ++kc) prim_cart2(la, lc, a->z[ka], a->A, c->z[kc], c->A, a->c[ka] * c->c[kc], buf, &s);
      const int ls[2] = {la, lc};
      solid_all(buf, tmp, 2, ls, res);
      for (int ma = 0; ma < Na; ++ma)
        for (int mc = 0; mc < Nc; ++mc) V[i + (size_t)na * (ma + (size_t)Na * (mc + (size_t)Nc * k))] = res[(size_t)ma * Nc + mc];
    }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  free(sh);
  return 0;
}

/* Schwarz factor of one pair from its diagonal quartet (ab|ab). */
static double pair_q(const oshell *a, const oshell *b, double *res, double *buf, double *tmp, scratch *s) {
  shell_solid4(a, b, a, b, res, buf, tmp, s);
  const int Nab = nsph(a->l) * nsph(b->l);
  double mx = 0.0;
  for (int ab = 0; ab < Nab; ++ab) {
    const double v = fabs(res[(size_t)ab * Nab + ab]);
    if (v > mx) mx = v;
  }
  return sqrt(mx);
}

int oracle_schwarz(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                   const double *centers, int normalize, int npair, const int *pairs, double *Q, int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  for (int n = 0; n < npair; ++n)
    if (pairs[2 * n] < 0 || pairs[2 * n] >= nshell || pairs[2 * n + 1] < 0 || pairs[2 * n + 1] >= nshell) {
      free(sh);
      return -2;
    }
  const size_t nmax = cart4_size(ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1);
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * nmax);
    double *tmp = (double *)malloc(sizeof(double) * nmax);
    double *res = (double *)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
    for (int n = 0; n < npair; ++n) Q[n] = pair_q(&sh[pairs[2 * n]], &sh[pairs[2 * n + 1]], res, buf, tmp, &s);
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  free(sh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Nuclear derivatives                                                  */
/* ------------------------------------------------------------------ */

/* Cartesian derivative integrals of a contracted quartet with respect to
 * centre `which` (0..3): out[xyz][a][b][c][d] with the shells' own l. */
static void shell_cart4_deriv(const oshell *sh4[4], int which, double *out, double *plus, double *minus,
                              scratch *s) {
  int ls[4], lp[4], lm[4];
  for (int i = 0; i < 4; ++i) ls[i] = lp[i] = lm[i] = sh4[i]->l;
  lp[which] += 1;
  lm[which] -= 1;
  const size_t n = cart4_size(ls[0], ls[1], ls[2], ls[3]);
  memset(out, 0, sizeof(double) * 3 * n);
  int cl[64][3];
  cart_list(ls[which], cl);
  /* strides of the `which` index in the shifted tensors */
  size_t inner = 1, outer = 1;
  for (int i = which + 1; i < 4; ++i) inner *= ncart(ls[i]);
  for (int i = 0; i < which; ++i) outer *= ncart(ls[i]);
  const int nw = ncart(ls[which]), nwp = ncart(lp[which]), nwm = lm[which] >= 0 ? ncart(lm[which]) : 0;
  const oshell *a = sh4[0], *b = sh4[1], *c = sh4[2], *d = sh4[3];
  for (int ka = 0; ka < a->K; ++ka)
    for (int kb = 0; kb < b->K; ++kb)
      for (int kc = 0; kc < c->K; ++kc)
        for (int kd = 0; kd < d->K; ++kd) {
          const double w = a->c[ka] * b->c[kb] * c->c[kc] * d->c[kd];
          const double zs[4] = {a->z[ka], b->z[kb], c->z[kc], d->z[kd]};
          memset(plus, 0, sizeof(double) * cart4_size(lp[0], lp[1], lp[2], lp[3]));
          prim_cart(lp[0], lp[1], lp[2], lp[3], zs[0], a->A, zs[1], b->A, zs[2], c->A, zs[3], d->A, 0, 1.0, plus, s);
          if (lm[which] >= 0) {
            memset(minus, 0, sizeof(double) * cart4_size(lm[0], lm[1], lm[2], lm[3]));
            prim_cart(lm[0], lm[1], lm[2], lm[3], zs[0], a->A, zs[1], b->A, zs[2], c->A, zs[3], d->A, 0, 1.0, minus,
                      s);
          }
          const double zw = zs[which];
          for (size_t o = 0; o < outer; ++o)
            for (int k = 0; k < nw; ++k)
              for (int x = 0; x < 3; ++x) {
                int up[3] = {cl[k][0], cl[k][1], cl[k][2]};
                up[x] += 1;
                const int kp = cart_index(up[0], up[1], up[2]);
                int km = -1;
                if (cl[k][x] > 0) {
                  int dn[3] = {cl[k][0], cl[k][1], cl[k][2]};
                  dn[x] -= 1;
                  km = cart_index(dn[0], dn[1], dn[2]);
                }
                double *dst = out + (size_t)x * n + (o * nw + k) * inner;
                const double *sp = plus + (o * nwp + kp) * inner;
                for (size_t in_ = 0; in_ < inner; ++in_) dst[in_] += w * 2.0 * zw * sp[in_];
                if (km >= 0) {
                  const double *sm = minus + (o * nwm + km) * inner;
                  for (size_t in_ = 0; in_ < inner; ++in_) dst[in_] -= w * cl[k][x] * sm[in_];
                }
              }
        }
}

typedef struct {
  double *out3, *plus, *minus, *buf, *tmp;
} dscratch;

static void dscratch_init(dscratch *d) {
  const size_t np = cart4_size(ORACLE_LMAX, ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1);
  d->out3 = (double *)malloc(sizeof(double) * 3 * np);
  d->plus = (double *)malloc(sizeof(double) * np);
  d->minus = (double *)malloc(sizeof(double) * np);
  d->buf = (double *)malloc(sizeof(double) * np);
  d->tmp = (double *)malloc(sizeof(double) * np);
}
static void dscratch_free(dscratch *d) {
  free(d->out3);
  free(d->plus);
  free(d->minus);
  free(d->buf);
  free(d->tmp);
}

/* Solid-harmonic derivative quartet: res[centre][xyz][ma][mb][mc][md]. */
static void shell_solid4_deriv(const oshell *sh4[4], double *res, dscratch *ds, scratch *s) {
  const int ls[4] = {sh4[0]->l, sh4[1]->l, sh4[2]->l, sh4[3]->l};
  const size_t n = cart4_size(ls[0], ls[1], ls[2], ls[3]);
  const size_t ns = (size_t)nsph(ls[0]) * nsph(ls[1]) * nsph(ls[2]) * nsph(ls[3]);
  for (int w = 0; w < 4; ++w) {
    shell_cart4_deriv(sh4, w, ds->out3, ds->plus, ds->minus, s);
    for (int x = 0; x < 3; ++x) {
      memcpy(ds->buf, ds->out3 + (size_t)x * n, sizeof(double) * n);
      solid_all(ds->buf, ds->tmp, 4, ls, res + ((size_t)w * 3 + x) * ns);
    }
  }
}

int oracle_eri4_deriv(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                      const double *centers, int normalize, int i, int j, int k, int m, double *out) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  if (i < 0 || j < 0 || k < 0 || m < 0 || i >= nshell || j >= nshell || k >= nshell || m >= nshell) {
    free(sh);
    return -1;
  }
  scratch s;
  scratch_init(&s);
  dscratch ds;
  dscratch_init(&ds);
  const oshell *sh4[4] = {&sh[i], &sh[j], &sh[k], &sh[m]};
  shell_solid4_deriv(sh4, out, &ds, &s);
  dscratch_free(&ds);
  scratch_free(&s);
  free(sh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Exchange operator (Sec. 6) and its nuclear gradient, brute force     */
/* ------------------------------------------------------------------ */
static int basis_offsets(int nshell, const oshell *sh, int *off) {
  int n = 0;
  for (int i = 0; i < nshell; ++i) {
    off[i] = n;
    n += nsph(sh[i].l);
  }
  return n;
}

/* Q over all ordered shell pairs (i,j), row-major nshell x nshell. */
static void all_pair_q(int nshell, const oshell *sh, double *Q, int nthreads) {
  const size_t nmax = cart4_size(ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1);
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * nmax);
    double *tmp = (double *)malloc(sizeof(double) * nmax);
    double *res = (double *)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
    for (long ij = 0; ij < (long)nshell * nshell; ++ij) {
      const int i = (int)(ij / nshell), j = (int)(ij % nshell);
      Q[ij] = pair_q(&sh[i], &sh[j], res, buf, tmp, &s);
    }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
}

int oracle_kbuild(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                  const double *centers, int normalize, const double *D, double tau, double *K, int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  int *off = (int *)malloc(sizeof(int) * (size_t)(nshell > 0 ? nshell : 1));
  const int nao = basis_offsets(nshell, sh, off);
  double *Q = (double *)malloc(sizeof(double) * (size_t)nshell * nshell + 8);
  all_pair_q(nshell, sh, Q, nthreads);
  memset(K, 0, sizeof(double) * (size_t)nao * nao);
  const size_t nmax = cart4_size(ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1);
  /* each thread owns the K rows of shell i (index a), so no update races */
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * nmax);
    double *tmp = (double *)malloc(sizeof(double) * nmax);
    double *res = (double *)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < nshell; ++i)
      for (int j = 0; j < nshell; ++j)
        for (int k = 0; k < nshell; ++k)
          for (int m = 0; m < nshell; ++m) {
            if (Q[(size_t)i * nshell + j] * Q[(size_t)k * nshell + m] < tau) continue;
            shell_solid4(&sh[i], &sh[j], &sh[k], &sh[m], res, buf, tmp, &s);
            const int Na = nsph(sh[i].l), Nb = nsph(sh[j].l), Nc = nsph(sh[k].l), Nd = nsph(sh[m].l);
            for (int a = 0; a < Na; ++a)
              for (int c = 0; c < Nc; ++c) {
                double acc = 0.0;
                for (int b = 0; b < Nb; ++b)
                  for (int d = 0; d < Nd; ++d)
                    acc += res[((size_t)(a * Nb + b) * Nc + c) * Nd + d] * D[(size_t)(off[j] + b) * nao + off[m] + d];
                K[(size_t)(off[i] + a) * nao + off[k] + c] += acc;
              }
          }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  free(Q);
  free(off);
  free(sh);
  return 0;
}

int oracle_exchange_grad(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                         const double *centers, int normalize, const int *atom_of_shell, int natom, const double *D,
                         double tau, double *grad, int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  for (int i = 0; i < nshell; ++i)
    if (atom_of_shell[i] < 0 || atom_of_shell[i] >= natom) {
      free(sh);
      return -1;
    }
  int *off = (int *)malloc(sizeof(int) * (size_t)(nshell > 0 ? nshell : 1));
  const int nao = basis_offsets(nshell, sh, off);
  double *Q = (double *)malloc(sizeof(double) * (size_t)nshell * nshell + 8);
  all_pair_q(nshell, sh, Q, nthreads);
  const int nthr = max_threads(nthreads);
  double *gthr = (double *)calloc((size_t)nthr * natom * 3, sizeof(double));
  const size_t ns4max = (size_t)nsph(ORACLE_LMAX - 1) * nsph(ORACLE_LMAX - 1) * nsph(ORACLE_LMAX - 1) *
                        nsph(ORACLE_LMAX - 1);
#pragma omp parallel num_threads(nthr)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    scratch s;
    scratch_init(&s);
    dscratch ds;
    dscratch_init(&ds);
    double *res = (double *)malloc(sizeof(double) * 12 * ns4max);
    double *g = gthr + (size_t)tid * natom * 3;
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < nshell; ++i)
      for (int j = 0; j < nshell; ++j)
        for (int k = 0; k < nshell; ++k)
          for (int m = 0; m < nshell; ++m) {
            if (Q[(size_t)i * nshell + j] * Q[(size_t)k * nshell + m] < tau) continue;
            const oshell *sh4[4] = {&sh[i], &sh[j], &sh[k], &sh[m]};
            shell_solid4_deriv(sh4, res, &ds, &s);
            const int Na = nsph(sh[i].l), Nb = nsph(sh[j].l), Nc = nsph(sh[k].l), Nd = nsph(sh[m].l);
            const size_t ns = (size_t)Na * Nb * Nc * Nd;
            const int atoms[4] = {atom_of_shell[i], atom_of_shell[j], atom_of_shell[k], atom_of_shell[m]};
            for (int w = 0; w < 4; ++w)
              for (int x = 0; x < 3; ++x) {
                const double *r = res + ((size_t)w * 3 + x) * ns;
                double acc = 0.0;
                /* W_abcd = D_ac D_bd */
                for (int a = 0; a < Na; ++a)
                  for (int b = 0; b < Nb; ++b)
                    for (int c = 0; c < Nc; ++c)
                      for (int d = 0; d < Nd; ++d)
                        acc += r[((size_t)(a * Nb + b) * Nc + c) * Nd + d] *
                               D[(size_t)(off[i] + a) * nao + off[k] + c] * D[(size_t)(off[j] + b) * nao + off[m] + d];
                g[atoms[w] * 3 + x] += acc;
              }
          }
    free(res);
    dscratch_free(&ds);
    scratch_free(&s);
  }
  memset(grad, 0, sizeof(double) * (size_t)natom * 3);
  for (int t = 0; t < nthr; ++t)
    for (int a = 0; a < natom * 3; ++a) grad[a] += gthr[(size_t)t * natom * 3 + a];
  free(gthr);
  free(Q);
  free(off);
  free(sh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Coulomb matrix (the other half of the Fock build, Sec. 1 and Sec. 6), */
/* brute force over every ordered shell quartet like oracle_kbuild:      */
/*   J_ab = sum_cd (ab|cd) D_cd.                                         */
/* ------------------------------------------------------------------ */
int oracle_jbuild(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                  const double *centers, int normalize, const double *D, double tau, double *J, int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  int *off = (int *)malloc(sizeof(int) * (size_t)(nshell > 0 ? nshell : 1));
  const int nao = basis_offsets(nshell, sh, off);
  double *Q = (double *)malloc(sizeof(double) * (size_t)nshell * nshell + 8);
  all_pair_q(nshell, sh, Q, nthreads);
  memset(J, 0, sizeof(double) * (size_t)nao * nao);
  const size_t nmax = cart4_size(ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1);
  /* one bra pair (i, j) per iteration: each thread owns the J block (i, j) */
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * nmax);
    double *tmp = (double *)malloc(sizeof(double) * nmax);
    double *res = (double *)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
    for (long ij = 0; ij < (long)nshell * nshell; ++ij) {
      const int i = (int)(ij / nshell), j = (int)(ij % nshell);
      for (int k = 0; k < nshell; ++k)
        for (int m = 0; m < nshell; ++m) {
          if (Q[(size_t)i * nshell + j] * Q[(size_t)k * nshell + m] < tau) continue;
          shell_solid4(&sh[i], &sh[j], &sh[k], &sh[m], res, buf, tmp, &s);
          const int Na = nsph(sh[i].l), Nb = nsph(sh[j].l), Nc = nsph(sh[k].l), Nd = nsph(sh[m].l);
          for (int a = 0; a < Na; ++a)
            for (int b = 0; b < Nb; ++b) {
              double acc = 0.0;
              for (int c = 0; c < Nc; ++c)
                for (int d = 0; d < Nd; ++d)
                  acc += res[((size_t)(a * Nb + b) * Nc + c) * Nd + d] * D[(size_t)(off[k] + c) * nao + off[m] + d];
              J[(size_t)(off[i] + a) * nao + off[j] + b] += acc;
            }
        }
    }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  free(Q);
  free(off);
  free(sh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Selected shell blocks of K and J, for checks on systems whose full   */
/* brute force is out of reach.  Block n is the pair (s0, s1) =         */
/* blocks[2n], blocks[2n+1]:                                             */
/*   which = 0 (K): out_n[a][c] = sum_{j,m} sum_{b,d} (s0 j|s1 m)_{a b c d} D_bd, */
/*   which = 1 (J): out_n[a][b] = sum_{k,m} sum_{c,d} (s0 s1|k m)_{a b c d} D_cd, */
/* over the quartets with Q_ij Q_km >= tau (Q from the diagonal          */
/* quartets, as everywhere in the oracle).  out holds the blocks one     */
/* after another, each row-major N(l_s0) x N(l_s1).                      */
/* ------------------------------------------------------------------ */
int oracle_fock_blocks(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                       const double *centers, int normalize, const double *D, double tau, int which, int nblk,
                       const int *blocks, double *out, int nthreads) {
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  if (which != 0 && which != 1) {
    free(sh);
    return -2;
  }
  for (int n = 0; n < nblk; ++n)
    if (blocks[2 * n] < 0 || blocks[2 * n] >= nshell || blocks[2 * n + 1] < 0 || blocks[2 * n + 1] >= nshell) {
      free(sh);
      return -2;
    }
  int *off = (int *)malloc(sizeof(int) * (size_t)(nshell > 0 ? nshell : 1));
  const int nao = basis_offsets(nshell, sh, off);
  size_t *bo = (size_t *)malloc(sizeof(size_t) * (size_t)(nblk + 1));
  bo[0] = 0;
  for (int n = 0; n < nblk; ++n) bo[n + 1] = bo[n] + (size_t)nsph(sh[blocks[2 * n]].l) * nsph(sh[blocks[2 * n + 1]].l);
  memset(out, 0, sizeof(double) * bo[nblk]);
  const size_t nmax = cart4_size(ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1, ORACLE_LMAX - 1);
  /* Schwarz factors of every pair that can appear: all (x, y) with x a
   * block shell (K: both s0 and s1 lead a pair; J: s0 leads the bra pair)
   * and, for J, all ket pairs (k, m) */
  double *Q = (double *)malloc(sizeof(double) * (size_t)nshell * nshell + 8);
  char *need = (char *)calloc((size_t)nshell, 1);
  for (int n = 0; n < nblk; ++n) {
    need[blocks[2 * n]] = 1;
    if (which == 0) need[blocks[2 * n + 1]] = 1;
  }
  if (which == 1) {
    all_pair_q(nshell, sh, Q, nthreads);
  } else {
#pragma omp parallel num_threads(max_threads(nthreads))
    {
      scratch s;
      scratch_init(&s);
      double *buf = (double *)malloc(sizeof(double) * nmax);
      double *tmp = (double *)malloc(sizeof(double) * nmax);
      double *res = (double *)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
      for (long ij = 0; ij < (long)nshell * nshell; ++ij) {
        const int i = (int)(ij / nshell), j = (int)(ij % nshell);
        if (need[i]) Q[ij] = pair_q(&sh[i], &sh[j], res, buf, tmp, &s);
      }
      free(buf);
      free(tmp);
      free(res);
      scratch_free(&s);
    }
  }
  /* work items: (block, inner shell) -> a private partial, summed in order */
  const long nwork = (long)nblk * nshell;
  double *part = (double *)calloc((size_t)nshell * (bo[nblk] > 0 ? bo[nblk] : 1), sizeof(double));
#pragma omp parallel num_threads(max_threads(nthreads))
  {
    scratch s;
    scratch_init(&s);
    double *buf = (double *)malloc(sizeof(double) * nmax);
    double *tmp = (double *)malloc(sizeof(double) * nmax);
    double *res = (double *)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
    for (long w = 0; w < nwork; ++w) {
      const int n = (int)(w / nshell), x = (int)(w % nshell);
      const int s0 = blocks[2 * n], s1 = blocks[2 * n + 1];
      double *o = part + (size_t)x * bo[nblk] + bo[n];
      const int N0 = nsph(sh[s0].l), N1 = nsph(sh[s1].l);
      for (int y = 0; y < nshell; ++y) {
        if (which == 0) {
          /* quartet (s0 x | s1 y): j = x, m = y */
          if (Q[(size_t)s0 * nshell + x] * Q[(size_t)s1 * nshell + y] < tau) continue;
          shell_solid4(&sh[s0], &sh[x], &sh[s1], &sh[y], res, buf, tmp, &s);
          const int Nb = nsph(sh[x].l), Nd = nsph(sh[y].l);
          for (int a = 0; a < N0; ++a)
            for (int c = 0; c < N1; ++c) {
              double acc = 0.0;
              for (int b = 0; b < Nb; ++b)
                for (int d = 0; d < Nd; ++d)
                  acc += res[((size_t)(a * Nb + b) * N1 + c) * Nd + d] * D[(size_t)(off[x] + b) * nao + off[y] + d];
              o[a * N1 + c] += acc;
            }
        } else {
          /* quartet (s0 s1 | x y): k = x, m = y */
          if (Q[(size_t)s0 * nshell + s1] * Q[(size_t)x * nshell + y] < tau) continue;
          shell_solid4(&sh[s0], &sh[s1], &sh[x], &sh[y], res, buf, tmp, &s);
          const int Nc = nsph(sh[x].l), Nd = nsph(sh[y].l);
          for (int a = 0; a < N0; ++a)
            for (int b = 0; b < N1; ++b) {
              double acc = 0.0;
              for (int c = 0; c < Nc; ++c)
                for (int d = 0; d < Nd; ++d)
                  acc += res[((size_t)(a * N1 + b) * Nc + c) * Nd + d] * D[(size_t)(off[x] + c) * nao + off[y] + d];
              o[a * N1 + b] += acc;
            }
        }
      }
    }
    free(buf);
    free(tmp);
    free(res);
    scratch_free(&s);
  }
  for (int x = 0; x < nshell; ++x)
    for (size_t e = 0; e < bo[nblk]; ++e) out[e] += part[(size_t)x * bo[nblk] + e];
  free(part);
  free(need);
  free(Q);
  free(bo);
  free(off);
  free(sh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Nuclear gradient of a general weighted sum of integrals               */
/*   E = sum_abcd W_abcd (ab|cd),                                        */
/*   pattern 0 (exchange type): W_abcd = Wl_ac Wr_bd  (E = tr(Wl K[Wr])),*/
/*   pattern 1 (Coulomb type):  W_abcd = Wl_ab Wr_cd  (E = tr(Wl J[Wr])),*/
/* brute force over every ordered quartet with Q_ij Q_km >= tau, each    */
/* differentiated on all four centres (grad is [natom][3], overwritten). */
/* Wl and Wr need not be symmetric.                                      */
/* ------------------------------------------------------------------ */
int oracle_grad_pattern(int nshell, const int *l, const int *nprim, const double *exps, const double *coefs,
                        const double *centers, int normalize, const int *atom_of_shell, int natom, int pattern,
                        const double *Wl, const double *Wr, double tau, double *grad, int nthreads) {
  if (pattern != 0 && pattern != 1) return -2;
  oshell *sh;
  if (build_shells(nshell, l, nprim, exps, coefs, centers, normalize, ORACLE_LMAX - 1, &sh)) return -1;
  for (int i = 0; i < nshell; ++i)
    if (atom_of_shell[i] < 0 || atom_of_shell[i] >= natom) {
      free(sh);
      return -1;
    }
  int *off = (int *)malloc(sizeof(int) * (size_t)(nshell > 0 ? nshell : 1));
  const int nao = basis_offsets(nshell, sh, off);
  double *Q = (double *)malloc(sizeof(double) * (size_t)nshell * nshell + 8);
  all_pair_q(nshell, sh, Q, nthreads);
  const int nthr = max_threads(nthreads);
  double *gthr = (double *)calloc((size_t)nthr * natom * 3, sizeof(double));
  const size_t ns4max = (size_t)nsph(ORACLE_LMAX - 1) * nsph(ORACLE_LMAX - 1) * nsph(ORACLE_LMAX - 1) *
                        nsph(ORACLE_LMAX - 1);
#pragma omp parallel num_threads(nthr)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    scratch s;
    scratch_init(&s);
    dscratch ds;
    dscratch_init(&ds);
    double *res = (double *)malloc(sizeof(double) * 12 * ns4max);
    double *g = gthr + (size_t)tid * natom * 3;
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < nshell; ++i)
      for (int j = 0; j < nshell; ++j)
        for (int k = 0; k < nshell; ++k)
          for (int m = 0; m < nshell; ++m) {
            if (Q[(size_t)i * nshell + j] * Q[(size_t)k * nshell + m] < tau) continue;
            const oshell *sh4[4] = {&sh[i], &sh[j], &sh[k], &sh[m]};
            shell_solid4_deriv(sh4, res, &ds, &s);
            const int Na = nsph(sh[i].l), Nb = nsph(sh[j].l), Nc = nsph(sh[k].l), Nd = nsph(sh[m].l);
            const size_t ns = (size_t)Na * Nb * Nc * Nd;
            const int atoms[4] = {atom_of_shell[i], atom_of_shell[j], atom_of_shell[k], atom_of_shell[m]};
            for (int w = 0; w < 4; ++w)
              for (int x = 0; x < 3; ++x) {
                const double *r = res + ((size_t)w * 3 + x) * ns;
                double acc = 0.0;
                for (int a = 0; a < Na; ++a)
                  for (int b = 0; b < Nb; ++b)
                    for (int c = 0; c < Nc; ++c)
                      for (int d = 0; d < Nd; ++d) {
                        const int A = off[i] + a, B = off[j] + b, C = off[k] + c, Dd = off[m] + d;
                        const double wt = pattern == 0 ? Wl[(size_t)A * nao + C] * Wr[(size_t)B * nao + Dd]
                                                       : Wl[(size_t)A * nao + B] * Wr[(size_t)C * nao + Dd];
                        acc += r[((size_t)(a * Nb + b) * Nc + c) * Nd + d] * wt;
                      }
                g[atoms[w] * 3 + x] += acc;
              }
          }
    free(res);
    dscratch_free(&ds);
    scratch_free(&s);
  }
  memset(grad, 0, sizeof(double) * (size_t)natom * 3);
  for (int t = 0; t < nthr; ++t)
    for (int a = 0; a < natom * 3; ++a) grad[a] += gthr[(size_t)t * natom * 3 + a];
  free(gthr);
  free(Q);
  free(off);
  free(sh);
  return 0;
}
