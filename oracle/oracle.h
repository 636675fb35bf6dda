/*
 * oracle.h -- plain FP64 CPU oracle for McMurchie-Davidson (MD) 3- and
 * 4-centre two-electron Coulomb integrals over contracted real solid-harmonic
 * Gaussians (Asadchev & Valeev, "3-center and 4-center 2-particle Gaussian AO
 * integrals on modern accelerated processors", Sec. 2 "Formalism").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU library; the GPU product never links
 * or calls it.
 *
 * Everything is scalar FP64 in the textbook *sum* form of the MD expansion
 * (Cartesian Hermite expansion, Hermite integrals, Cartesian contraction, then
 * the Cartesian -> solid-harmonic transform), except the Boys function, which
 * is evaluated in long double so that it is never the limiting error.
 *
 * Basis convention (shared with the GPU library by specification only):
 *   - a shell is (l, K, exponents[K], coefficients[K], centre[3]);
 *   - with normalize=1 the user coefficients multiply unit-normalised
 *     primitive x^l Gaussians and the contracted shell is then rescaled to unit
 *     norm; with normalize=0 the coefficients multiply the bare primitives
 *     x^a y^b z^c exp(-zeta r^2);
 *   - real solid harmonics are ordered m = -l..l and have the same norm on the
 *     sphere as x^l (so p shells come out as y, z, x).
 *
 * Error returns: 0 on success, negative on invalid input (unsupported l,
 * mixed classes in a class batch, K above ORACLE_KMAX).
 */
#ifndef MDERI_ORACLE_H
#define MDERI_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_LMAX 9  /* shells up to l=9 (l=8 plus one for derivatives) */
#define ORACLE_KMAX 16 /* primitives per shell */

/* Boys function F_m(T), m = 0..mmax, Eq. (boys). */
void oracle_boys(int mmax, double T, double *F);

/* 1-D Hermite expansion coefficients of a Gaussian product, Eqs.
 * (E2rr1)-(E2-abp): E[i][j][t], i<=la, j<=lb, t<=la+lb, stored densely with
 * strides (lb+1)*(la+lb+1) and (la+lb+1). */
void oracle_E2(int la, int lb, double za, double zb, double Ax, double Bx, double *E);

/* 1-D Hermite expansion coefficients of one Gaussian, Eqs. (E1rr)-(E1-aa):
 * E[i][t], i<=la, t<=la, stride la+1. */
void oracle_E1(int la, double za, double *E);

/* Hermite Coulomb integrals [r]^(0), Eqs. (0m) and (r), for all r=(t,u,v)
 * with t+u+v <= L, written densely as R[t][u][v] with strides (L+1)^2, L+1.
 * pref multiplies [0]^(m) (the 2 pi^{5/2}/(p q sqrt(p+q)) factor of Eq. (0m)
 * when called from the integral code; tests pass 1). */
void oracle_R(int L, double rho, const double PQ[3], double pref, double *R);

/* Cartesian -> real solid harmonic coefficients C[m+l][cart], m=-l..l, with
 * Cartesian components ordered lx descending, then ly descending. */
void oracle_solid(int l, double *C);

/* Normalised contraction coefficients (see the basis convention above). */
void oracle_norm_coefs(int l, int K, const double *z, const double *c, int normalize, double *out);

/* Contracted Cartesian (ab|cd) for one shell quartet (no solid transform):
 * out[a][b][c][d] over Cartesian components. */
int oracle_eri4_cart(int nshell, const int *l, const int *nprim, const double *exps,
                     const double *coefs, const double *centers, int normalize,
                     int i, int j, int k, int m, double *out);

/* Class batch of 4-centre integrals in solid harmonics, layout
 * V[ij, ab, cd, kl] column-major (ij fastest), ab = ma*N(lb)+mb,
 * cd = mc*N(ld)+md.  Every bra pair must share (la,lb) and every ket pair
 * (lc,ld).  pairs are int32 [n][2] shell indices. */
int oracle_eri4(int nshell, const int *l, const int *nprim, const double *exps,
                const double *coefs, const double *centers, int normalize,
                int nbra, const int *bra, int nket, const int *ket, double *V, int nthreads);

/* 3-centre (ab|P): pairs from the primary basis, single shells from the
 * auxiliary basis; layout V[ij, ab, mP, k] (ij fastest). */
int oracle_eri3(int nshell, const int *l, const int *nprim, const double *exps,
                const double *coefs, const double *centers,
                int naux_shell, const int *al, const int *anprim, const double *aexps,
                const double *acoefs, const double *acenters, int normalize,
                int npair, const int *pairs, int naux, const int *aux, double *V, int nthreads);

/* 2-centre Coulomb integrals (a|c) (the density-fitting metric): single
 * shells as[na] (one l) against single shells cs[nc] (one l) of one basis;
 * layout V[i, ma, mc, k] (i fastest). */
int oracle_eri2(int nshell, const int *l, const int *nprim, const double *exps,
                const double *coefs, const double *centers, int normalize,
                int na, const int *as, int nc, const int *cs, double *V, int nthreads);

/* Schwarz factors Q_ij = sqrt(max_{ab} |(ab|ab)|) for each pair. */
int oracle_schwarz(int nshell, const int *l, const int *nprim, const double *exps,
                   const double *coefs, const double *centers, int normalize,
                   int npair, const int *pairs, double *Q, int nthreads);

/* Derivatives of one solid-harmonic shell quartet with respect to the four
 * shell centres: out[centre 0..3][xyz][ma][mb][mc][md]. */
int oracle_eri4_deriv(int nshell, const int *l, const int *nprim, const double *exps,
                      const double *coefs, const double *centers, int normalize,
                      int i, int j, int k, int m, double *out);

/* Brute-force exchange matrix K_ac = sum_bd (ab|cd) D_bd over all shell
 * quartets with Q_ij*Q_kl >= tau (no permutational symmetry used).  D, K are
 * row-major nao x nao over AOs in shell order. */
int oracle_kbuild(int nshell, const int *l, const int *nprim, const double *exps,
                  const double *coefs, const double *centers, int normalize,
                  const double *D, double tau, double *K, int nthreads);

/* Brute-force gradient of E = sum_abcd D_ac D_bd (ab|cd) (= tr(D K)) with
 * respect to atom positions, over the same screened quartets as
 * oracle_kbuild.  grad is [natom][3] and is overwritten. */
int oracle_exchange_grad(int nshell, const int *l, const int *nprim, const double *exps,
                         const double *coefs, const double *centers, int normalize,
                         const int *atom_of_shell, int natom,
                         const double *D, double tau, double *grad, int nthreads);

/* Brute-force Coulomb matrix J_ab = sum_cd (ab|cd) D_cd over every ordered
 * shell quartet with Q_ij*Q_kl >= tau (the other half of the Fock build).
 * D, J are row-major nao x nao. */
int oracle_jbuild(int nshell, const int *l, const int *nprim, const double *exps,
                  const double *coefs, const double *centers, int normalize,
                  const double *D, double tau, double *J, int nthreads);

/* Selected shell blocks of K (which = 0) or J (which = 1) by the same brute
 * force, restricted to the quartets that feed them: block n is the shell
 * pair (blocks[2n], blocks[2n+1]) and receives, row-major,
 *   K: out[a][c] = sum (s0 j|s1 m) D_jm over all shells j, m,
 *   J: out[a][b] = sum (s0 s1|k m) D_km over all shells k, m.
 * Blocks are stored one after another. */
int oracle_fock_blocks(int nshell, const int *l, const int *nprim, const double *exps,
                       const double *coefs, const double *centers, int normalize,
                       const double *D, double tau, int which, int nblk, const int *blocks,
                       double *out, int nthreads);

/* Brute-force gradient of E = sum_abcd W_abcd (ab|cd) with respect to atom
 * positions, W_abcd = Wl_ac Wr_bd (pattern 0, exchange: E = tr(Wl K[Wr]))
 * or Wl_ab Wr_cd (pattern 1, Coulomb: E = tr(Wl J[Wr])); Wl, Wr need not be
 * symmetric.  grad is [natom][3] and is overwritten. */
int oracle_grad_pattern(int nshell, const int *l, const int *nprim, const double *exps,
                        const double *coefs, const double *centers, int normalize,
                        const int *atom_of_shell, int natom, int pattern,
                        const double *Wl, const double *Wr, double tau, double *grad, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
