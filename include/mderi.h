/*
 * mderi.h -- C ABI of libmderi, an MI355X (gfx950) implementation of the
 * McMurchie-Davidson (MD) evaluation of 3-centre (ab|P) and 4-centre (ab|cd)
 * two-electron Coulomb integrals over contracted real solid-harmonic
 * Gaussians (Asadchev & Valeev, "3-center and 4-center 2-particle Gaussian AO
 * integrals on modern accelerated processors").
 *
 * General rules for every entry point:
 *  - extern "C"; only plain integers, doubles and pointers cross the ABI.
 *  - Pointers named *_host are host memory and are read (or copied) before
 *    the call returns; pointers named *_dev are device memory owned by the
 *    caller; the library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work of a call is enqueued on that stream and the call returns
 *    without waiting for it, except where stated.
 *  - A context owns per-device workspace (pair data, scratch), the Boys
 *    interpolation table and the constant tables; calls that share a context
 *    must be issued from one host thread at a time and on one stream at a
 *    time (workspace is reused in stream order).
 *  - Validation happens before anything is enqueued: on any error nothing is
 *    enqueued, the status is returned and mderi_last_error() describes it.
 *    HIP launch failures return MDERI_EDEVICE.
 *
 * Basis convention (Sec. 2 "Formalism"): a shell is (l, K, exponents[K],
 * coefficients[K], centre[3] in bohr).  With normalize=1 the coefficients
 * multiply unit-normalised primitive x^l Gaussians and the contracted shell
 * is rescaled to unit norm; with normalize=0 they multiply bare primitives
 * x^a y^b z^c exp(-zeta r^2).  Real solid harmonics are ordered m = -l..l
 * and carry the norm of x^l on the sphere (p shells come out as y, z, x).
 */
#ifndef MDERI_H
#define MDERI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MDERI_OK = 0,
  MDERI_EINVAL = -1,       /* bad argument (range, null pointer, mixed classes, ...) */
  MDERI_ENOMEM = -2,       /* device workspace could not be allocated */
  MDERI_EUNSUPPORTED = -3, /* valid request outside what is built (l, K, class) */
  MDERI_EDEVICE = -4,      /* HIP runtime / launch failure */
  MDERI_ESIZE = -5         /* output buffer too small */
} mderi_status;

#define MDERI_LMAX 8  /* largest shell angular momentum */
#define MDERI_KMAX 16 /* largest number of primitives per shell */

typedef struct mderi_ctx *mderi_ctx_t;
typedef struct mderi_basis *mderi_basis_t;

/* Arithmetic of the Hermite->solid transforms (mderi_opts.precision). */
#define MDERI_FP64 0       /* everything in FP64 */
#define MDERI_SPLIT_BF16 1 /* bra transform on the BF16 matrix cores with operands split into 7-bit
                              integer slices (see mderi_eri4); all else FP64 */
#define MDERI_SPLIT_FP32 2 /* not built: every call returns MDERI_EUNSUPPORTED.  The FP32 matrix
                              rate of MI355X (157.3 TFLOP/s) is twice the FP64 rate, and an FP32
                              split with exact sums needs 12-bit slices, three per 35-bit operand,
                              so at least six slice products: more matrix work than FP64 itself */

/* Options shared by the compute calls; NULL means defaults. */
typedef struct {
  int precision;      /* MDERI_FP64 (all entry points) or MDERI_SPLIT_BF16 (mderi_eri4) */
  double schwarz_tau; /* screening threshold for the K build (default 1e-12) */
  int flags;          /* MDERI_FLAG_* (mderi_eri3_batch; mderi_eri4 takes MDERI_FLAG_AUTOTUNE;
                         mderi_kbuild_grad takes MDERI_FLAG_SYMMETRIC) */
  int split_slices;   /* MDERI_SPLIT_BF16: 7-bit slices per operand, 5..7 (0 = default 6) */
  int tile_variant;   /* mderi_eri4, FP64: 0 = the planned (or tuned) work split; v > 0 = the v-th of
                         the splits mderi_eri4_tile_variants counts for the batch */
  int deterministic;  /* mderi_jkbuild / mderi_kbuild / mderi_kbuild_grad: 1 = bitwise repeatable
                         results (fixed-point integer accumulation, see those calls); 0 = FP64
                         atomics (default) */
} mderi_opts;

#define MDERI_FLAG_GRAPH 1    /* capture the call's launches in a hipGraph, replay it on identical calls */
#define MDERI_FLAG_AUTOTUNE 2 /* choose each class block's kernel tiles by timing the candidates */
#define MDERI_FLAG_SYMMETRIC 4 /* mderi_kbuild_grad: Wl_dev == Wr_dev and the matrix is symmetric (the
                                  caller's guarantee); the weights are then gathered from one block */

/* Creates a context on HIP device `device`: uploads the Boys-function
 * interpolation table and the constant Hermite / solid-harmonic tables.
 * *out receives the handle. */
mderi_status mderi_create(int device, mderi_ctx_t *out);

/* Releases the context and all library-owned device memory.  NULL is a no-op. */
void mderi_destroy(mderi_ctx_t ctx);

/* Text of the last failure on the calling host thread ("" if none). */
const char *mderi_last_error(void);

/* Copies a shell list to the device (Sec. 2; see the basis convention
 * above).  Arrays: l_host[nshell] (0..MDERI_LMAX), nprim_host[nshell]
 * (1..MDERI_KMAX), exps_host / coefs_host concatenated over shells
 * (sum(nprim) entries, exponents finite and > 0), centers_host[nshell][3].
 * atom_host[nshell] maps shells to atoms (may be NULL: shell i -> atom i).
 * Host arrays are copied before return; the call synchronises the device. */
mderi_status mderi_basis_upload(mderi_ctx_t ctx, int nshell, const int *l_host, const int *nprim_host,
                                const double *exps_host, const double *coefs_host, const double *centers_host,
                                const int *atom_host, int normalize, mderi_basis_t *out);

/* Releases a basis.  NULL is a no-op. */
void mderi_basis_free(mderi_basis_t basis);

/* Number of shells / AOs of a basis (AOs: sum of 2l+1 in shell order). */
int mderi_basis_nshell(mderi_basis_t basis);
int mderi_basis_nao(mderi_basis_t basis);

/*
 * Class batch of 4-centre integrals (Sec. 3 "MD Algorithm Variants": output
 * layout V[ij,ab,cd,kl], column-major, ij fastest).
 *
 * bra_host[nbra][2] and ket_host[nket][2] are int32 shell-index pairs.  All
 * bra pairs must share (l_a, l_b) and all ket pairs (l_c, l_d); contraction
 * degrees may differ from pair to pair.  The call evaluates every quartet
 * (ij, kl) of the two lists -- pair data and the Hermite->solid transform
 * matrices H of Eqs. (solid2herm-2) included -- and writes
 *     V_dev[ij + nbra*(ab + Nab*(cd + Ncd*kl))],
 * ab = m_a*N(l_b) + m_b, cd = m_c*N(l_d) + m_d (0-based component indices,
 * N(l) = 2l+1).  V_elems is the capacity of V_dev in doubles and must be at
 * least nbra*Nab*Ncd*nket.  Contracted over all primitive quartets in FP64.
 * opts->precision = MDERI_SPLIT_BF16 runs the bra transform (Eq.
 * bra-from-hermite) on the BF16 matrix cores: the rows of H_bra and [p|ket]
 * are balanced by powers of two, both operands are scaled by a power of two
 * per column and split into S = opts->split_slices 7-bit integer slices;
 * the slice products are exact in BF16, their FP32 sums over 32-row blocks
 * are exact, products of total order above S+1 are dropped (7S-bit
 * operands) and the rest is combined in FP64.  Boys, R, the ket transform
 * and the accumulation of V stay FP64.  The error per shellset relative to
 * its largest element grows with the cancellation in the bra sum (see the
 * split-precision tests for measured bounds per class and S).
 * opts->flags may hold MDERI_FLAG_AUTOTUNE: the first call of a class
 * signature (l_a, l_b, l_c, l_d and the largest primitive-pair counts) times
 * every work split the kernel supports on this batch, synchronising the
 * stream, and keeps the fastest in the context for later calls.
 */
mderi_status mderi_eri4(mderi_ctx_t ctx, mderi_basis_t basis, int nbra, const int32_t *bra_host, int nket,
                        const int32_t *ket_host, double *V_dev, size_t V_elems, const mderi_opts *opts,
                        void *stream);

/*
 * Number of work splits (row tiles per wave, row parts, single or double
 * [r] buffer) the fused kernel supports for the class batch of mderi_eri4
 * with these pair lists: the candidates MDERI_FLAG_AUTOTUNE times and
 * opts->tile_variant selects (0 when the class runs on column slabs, where
 * the split is fixed).  Validation as for mderi_eri4; nothing is enqueued.
 */
mderi_status mderi_eri4_tile_variants(mderi_ctx_t ctx, mderi_basis_t basis, int nbra, const int32_t *bra_host,
                                      int nket, const int32_t *ket_host, int *count);

/*
 * Allocation-free variant of mderi_eri4, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Arguments, output layout and
 * results are those of mderi_eri4 (FP64 only; opts->precision must be
 * MDERI_FP64 and opts->flags 0).  Every device region the call needs (pair
 * lists, primitive-pair data and transform matrices of both sides) is a
 * slice of a fixed 64 MiB device array compiled into the library, and its
 * metadata goes through one 4 MiB slot of the pinned staging buffer that
 * mderi_create allocates (four slots, used by successive calls in turn); the
 * call itself calls no allocating routine.  A batch that needs more scratch
 * or staging than that returns MDERI_ESIZE with nothing enqueued.  All calls on one GPU share that GPU's array (contexts
 * included), which keeps the last call's contents: calls that overlap on
 * one GPU (different streams, or different host threads) race and must be
 * serialised by the caller.
 */
mderi_status mderi_eri4_noalloc(mderi_ctx_t ctx, mderi_basis_t basis, int nbra, const int32_t *bra_host, int nket,
                                const int32_t *ket_host, double *V_dev, size_t V_elems, const mderi_opts *opts,
                                void *stream);

/*
 * Class batch of 2-centre Coulomb integrals (P|Q), the metric of density
 * fitting (Sec. 1 motivates 3-centre integrals by it; Sec. 2: both shells
 * expanded with the 1-centre Hermite coefficients of Eqs. (E1rr)-(E1-aa),
 * then Eqs. (0m), (r), (pq) and the two transforms, as for (ab|P) with a
 * 1-centre bra).
 *
 * shells_a_host[na] and shells_c_host[nc] are int32 shell indices of `basis`,
 * each list of one l (l_a, l_c).  Writes
 *     V_dev[i + na*(ma + N(l_a)*(mc + N(l_c)*k))]
 * (i fastest).  V_elems must be at least na*N(l_a)*N(l_c)*nc.  FP64;
 * opts may be NULL or carry MDERI_FLAG_AUTOTUNE.  EINVAL for bad shells or
 * mixed l within a list, ESIZE for a short output.
 */
mderi_status mderi_eri2(mderi_ctx_t ctx, mderi_basis_t basis, int na, const int32_t *shells_a_host, int nc,
                        const int32_t *shells_c_host, double *V_dev, size_t V_elems, const mderi_opts *opts,
                        void *stream);

/*
 * Density-fitted Coulomb matrix (the use of 3-centre integrals Sec. 1
 * motivates): the pair density sum_cd D_cd (cd| is fitted in the Coulomb
 * metric of the auxiliary basis,
 *     gamma_Q = sum_cd (Q|cd) D_cd,  M_PQ = (P|Q),  c = M^{-1} gamma,
 *     J_ab = sum_P (ab|P) c_P,
 * with (ab|P) over every canonical shell pair of `basis` and every shell of
 * `aux` (mderi_eri3_batch), M from mderi_eri2's class batches, and the
 * Cholesky solve by rocSOLVER on the stream.  D_dev, J_dev: [nao][nao]
 * row-major FP64 on the device, D symmetric; J is written in full.  The
 * metric must be positive definite (a linearly dependent fitting set is the
 * caller's to prune; the solve does not report it and J is then undefined).
 * Device workspace grows to hold the npairrow x naux (ab|P) matrix and the
 * naux x naux metric.  The (ab|P) plan's first call synchronises the stream.
 * The context keeps these factors for the next mderi_dfj / mderi_dfk call:
 * when it has the same two bases and neither was moved since
 * (mderi_basis_set_centers), the 3-centre integrals, the metric and its
 * factorisation are not recomputed, so the calls of an SCF's later rounds
 * are a few matrix-vector products (after a mderi_dfk they use the B L^-T
 * that call left in place of B, which gives the same J without the solve).
 * Another basis pair or mderi_set_workspace_limit drops them.
 */
mderi_status mderi_dfj(mderi_ctx_t ctx, mderi_basis_t basis, mderi_basis_t aux, const double *D_dev, double *J_dev,
                       int nao, const mderi_opts *opts, void *stream);

/*
 * Density-fitted exchange matrix (the exchange operator of Sec. 6 over
 * integrals fitted with the 3-centre integrals Sec. 1 motivates): every pair
 * product is fitted in the Coulomb metric of `aux`,
 *     (ab|cd)_fit = sum_PQ (ab|P) [M^{-1}]_PQ (Q|cd) = sum_Q B'_ab,Q B'_cd,Q,
 *     B' = B L^{-T},  M = (P|Q) = L L^T,
 *     K_ac = sum_bd (ab|cd)_fit D_bd = sum_Q (B'_Q D B'_Q^T)_ac,
 * with B the (ab|P) matrix of mderi_dfj, the Cholesky factor and the
 * triangular solve by rocSOLVER / rocBLAS, B'_Q spread over all AO pairs and
 * the two contractions as two rocBLAS GEMMs (2 nao^3 naux FLOPs each), all on
 * the stream.  D_dev, K_dev: [nao][nao] row-major FP64 on the device, D
 * symmetric; K is written in full and exactly symmetric.  Any D is allowed
 * (no orbital factorisation is assumed), so the work space holds two
 * nao x nao x naux arrays besides those of mderi_dfj: MDERI_ENOMEM when they
 * do not fit.  Metric, synchronisation and the kept factors as for
 * mderi_dfj; a repeated call on the same bases also keeps B' spread over
 * the AO pairs, so it is the two GEMMs and the symmetrisation alone.
 */
mderi_status mderi_dfk(mderi_ctx_t ctx, mderi_basis_t basis, mderi_basis_t aux, const double *D_dev, double *K_dev,
                       int nao, const mderi_opts *opts, void *stream);

/*
 * Class batch of 3-centre integrals (ab|P) (Sec. 2: the 1-centre Hermite
 * expansion of Eqs. (E1rr)-(E1-aa); the paper writes them [P|ab]).
 *
 * pairs_host[npair][2] are int32 shell-index pairs of `basis`, all of one
 * class (l_a, l_b); aux_host[naux] are int32 shell indices of `aux` (another
 * uploaded basis, e.g. a fitting basis), all of one l_P.  Writes
 *     V_dev[ij + npair*(ab + Nab*(mP + N(l_P)*k))]
 * (ij fastest, ab = m_a*N(l_b) + m_b).  V_elems must be at least
 * npair*Nab*N(l_P)*naux.  Contracted over all primitives in FP64.
 */
mderi_status mderi_eri3(mderi_ctx_t ctx, mderi_basis_t basis, mderi_basis_t aux, int npair, const int32_t *pairs_host,
                        int naux, const int32_t *aux_host, double *V_dev, size_t V_elems, const mderi_opts *opts,
                        void *stream);

/*
 * 3-centre integrals (ab|P) over pairs and auxiliary shells of ANY classes in
 * one call (the class-batched form of mderi_eri3 generalised to a task list).
 * pairs_host[npair][2] index `basis`, aux_host[naux] index `aux`.  Output is
 * the matrix B with rows = the AO pairs of the pair list (pair i contributes
 * N(l_a)N(l_b) rows, ab = m_a N(l_b) + m_b, in list order) and columns = the
 * AOs of the aux list (aux k contributes N(l_k) columns), column-major:
 *     V_dev[(rowoff_i + ab) + nrow * (coloff_k + m)],
 * nrow = sum_i N(l_a)N(l_b); V_elems >= nrow * ncol.
 * The call groups the triplets by class block (pair class x aux l), sorts
 * them by the cost of Table md-scheme and runs one persistent launch per
 * kernel shape; the plan (pair data, block descriptors, task lists) stays on
 * the device, keyed by (bases, lists, V_dev, flags), and an identical later
 * call only relaunches it.  opts->flags: MDERI_FLAG_GRAPH captures the
 * launches in a hipGraph on the first call and replays it afterwards;
 * MDERI_FLAG_AUTOTUNE times every candidate tile shape of a new class
 * signature on the first call (results are kept in the context).  The first
 * call of a plan synchronises the stream.
 */
mderi_status mderi_eri3_batch(mderi_ctx_t ctx, mderi_basis_t basis, mderi_basis_t aux, int npair,
                              const int32_t *pairs_host, int naux, const int32_t *aux_host, double *V_dev,
                              size_t V_elems, const mderi_opts *opts, void *stream);

/*
 * Schwarz factors Q_ij = sqrt(max_ab |(ab|ab)|) of shell pairs, from the
 * diagonal quartets (ij|ij) evaluated by the same MD path as mderi_eri4.
 * Screening (not defined in the paper beyond the remark in Sec. 3 that
 * screening makes pair lists sparse) keeps a pair when Q_ij * Q_max >= tau
 * and a quartet when Q_ij * Q_kl >= tau.
 * pairs_host[npair][2] are int32 shell indices of any mix of classes;
 * Q_dev[npair] (device, doubles) receives the factors in input order.
 */
mderi_status mderi_schwarz(mderi_ctx_t ctx, mderi_basis_t basis, int npair, const int32_t *pairs_host, double *Q_dev,
                           void *stream);

/*
 * Coulomb and exchange matrices of a symmetric density D (Sec. 6: the
 * exchange operator K_ac = sum_bd (ab|cd) D_bd, written K_bc = sum_ad
 * [ab|cd] D_ad there, the same operator for symmetric D; the Coulomb matrix
 * J_ab = sum_cd (ab|cd) D_cd is the other half of the Fock build):
 * every shell quartet of `basis` that survives Schwarz screening (Q_ij Q_kl
 * >= tau, opts->schwarz_tau, default 1e-12; Q over canonical shell pairs,
 * pairs kept when Q_ij Q_max >= tau) is evaluated once, as a
 * symmetry-unique quartet, and digested into the permutational images of
 * both matrices.  D_dev, J_dev and K_dev are row-major nao x nao device
 * matrices over the AOs in shell order (nao must equal mderi_basis_nao);
 * J_dev or K_dev may be NULL (that matrix is not built), not both; the
 * matrices built are overwritten.  energy_dev (device, may be NULL)
 * receives {tr(D J), tr(D K)} (a NULL matrix gives 0).
 * The first call for a basis, geometry and tau computes the Schwarz
 * factors of all canonical shell pairs on the stream and synchronises it
 * once, to sort the significant pairs of each class by Q on the host (so
 * the admissible partners of every pair are a prefix of the sorted list);
 * the context keeps that selection for the two most recent (basis,
 * geometry, tau) keys, so later calls on an unchanged basis (the rounds of
 * an SCF) do not synchronise at all.  Everything after the selection is
 * enqueued asynchronously.  mderi_basis_set_centers starts a new geometry
 * (the next call selects again).  Work space grows with the number of significant pairs
 * (pair data of every class in both roles).  By default the sums of the
 * images use FP64 atomics, so the last bits of J and K vary from run to run.
 * With opts->deterministic = 1 every image is scaled by 2^e and added as a
 * fixed-point number with 32 fraction bits, held in two 64-bit integers
 * (the floor and the rounded fraction), by integer atomics, whose sums do
 * not depend on the order of the adds; J and K are then the same bits on
 * every run with the same inputs on the same device.  e = 62 -
 * ceil(log2 B), B = 4 Q_max^2 sum|D| (computed on the device), so no sum
 * of magnitudes reaching one element can overflow; each image is rounded
 * to B 2^-95, far below FP64 rounding of J and K themselves.  This mode
 * takes 16 bytes per element of each matrix built as work space and two
 * integer atomics per image instead of one.
 */
mderi_status mderi_jkbuild(mderi_ctx_t ctx, mderi_basis_t basis, const double *D_dev, double *J_dev, double *K_dev,
                           int nao, double *energy_dev, const mderi_opts *opts, void *stream);

/* mderi_jkbuild for K alone (J_dev = NULL, no energies). */
mderi_status mderi_kbuild(mderi_ctx_t ctx, mderi_basis_t basis, const double *D_dev, double *K_dev, int nao,
                          const mderi_opts *opts, void *stream);

/* Replaces the shell centres of a basis by centers_dev[nshell][3] (device,
 * bohr), copied on `stream` (asynchronous, the caller keeps centers_dev
 * alive until the stream reaches the copy).  Later calls on that stream
 * see the new geometry; shells, exponents, coefficients and the atom map
 * stay.  The pair selections the context cached for this basis are
 * dropped. */
mderi_status mderi_basis_set_centers(mderi_basis_t basis, const double *centers_dev, void *stream);

/*
 * Kernel timing (measurement support, not part of the method).  While
 * enabled, every launch of the fused integral kernel (eri4, eri3, Schwarz,
 * K build and gradient all use it) is bracketed by two HIP events recorded on
 * the launch stream.  mderi_kernel_times waits for the recorded launches,
 * writes the durations in milliseconds, in launch order, to ms_host[0..cap)
 * and stores the number recorded in *count; if cap >= *count the records are
 * cleared, otherwise they are kept so the call can be repeated with a larger
 * buffer.
 */
mderi_status mderi_kernel_timing(mderi_ctx_t ctx, int enable);
mderi_status mderi_kernel_times(mderi_ctx_t ctx, double *ms_host, int cap, int *count);

/*
 * Progress report (measurement support, not part of the method).  While
 * enabled, the J/K builds and the gradient enqueue a host function after each
 * launch group of the screened quartet engine; it prints one line to stderr
 * when the group's kernel has finished (group index, total degree, quartets,
 * seconds since the call).  Meant for long calls on large systems.  EINVAL
 * for a NULL context.
 */
mderi_status mderi_progress(mderi_ctx_t ctx, int enable);

/*
 * Caps the device workspace the context may hold (the sum over its work
 * slots: pair data, intermediate matrices, partial results; not the
 * constant tables, the pinned staging buffer, the cached task-list plans of
 * mderi_eri3_batch or the library handle of the density-fitting solve) at
 * `bytes`; 0 removes the cap.  The call synchronises the device
 * and releases the workspace held so far.  A later call that would grow it
 * past the cap returns MDERI_ENOMEM, exactly as when hipMalloc fails; as
 * with a failed hipMalloc, work of that call enqueued before the failing
 * request (Schwarz factors, pair data) may already be on the stream, and
 * its outputs are then undefined.  The context stays usable: after the cap
 * is raised or removed, the same call succeeds.  Serves callers that share
 * the GPU with other memory users, and tests of the ENOMEM paths.
 */
mderi_status mderi_set_workspace_limit(mderi_ctx_t ctx, size_t bytes);

/*
 * Persistent autotune cache.  mderi_tune_save writes the tile choices the
 * context's autotuner has made (MDERI_FLAG_AUTOTUNE of mderi_eri4,
 * mderi_eri2 and mderi_eri3_batch, one per class signature: l of the four
 * centres and the largest primitive-pair counts of the two sides) to the
 * text file path_host, headed by the device's architecture name;
 * mderi_tune_load reads such a file into a context, so that later calls use
 * the stored choices without timing candidates again.  Loading checks the
 * header and every entry before it changes anything: a file that does not
 * parse, or that was written on another architecture, gives MDERI_EINVAL
 * and leaves the context as it was.  Loaded entries replace those of the
 * same signature; a stored choice that is not among a class's candidates
 * when the class runs is ignored.  Host-only; nothing is enqueued.
 */
mderi_status mderi_tune_save(mderi_ctx_t ctx, const char *path_host);
mderi_status mderi_tune_load(mderi_ctx_t ctx, const char *path_host);

/* Weight patterns of mderi_kbuild_grad. */
#define MDERI_EXCHANGE 0 /* W_abcd = Wl_ac Wr_bd: E = tr(Wl^T K[Wr]) */
#define MDERI_COULOMB 1  /* W_abcd = Wl_ab Wr_cd: E = tr(Wl^T J[Wr]) */

/*
 * Nuclear gradient of E = scale * sum_abcd W_abcd (ab|cd) over every AO
 * quadruple of the screened quartets of mderi_jkbuild, W given by
 * `pattern` from the row-major nao x nao device matrices Wl_dev and Wr_dev
 * (need not be symmetric).  The paper gives no gradient; the derivative
 * follows from differentiating the Gaussians of Sec. 2: d/dA_x of
 * x_A^{a} e^{-zeta r_A^2} is 2 zeta x_A^{a+1} e^{..} minus a_x x_A^{a-1}
 * e^{..}, so the MD path runs with A-side Hermite degree l_a+l_b+1 and R up
 * to L+1 and W held fixed.  Each quartet of canonical shell pairs is
 * visited once per orientation and supplies the derivatives of its first
 * pair's two centres, weighted by the summed weights of every AO ordering
 * that maps onto it.  grad_dev[natom][3] (device, row-major) receives
 * dE/dR_atom summed over the shells of each atom (the atom map given to
 * mderi_basis_upload; natom must exceed every atom index); accumulate = 0
 * overwrites it, 1 adds to it.  The exchange energy of mderi_jkbuild,
 * tr(D K[D]), is pattern MDERI_EXCHANGE with Wl = Wr = D and scale 1; its
 * Coulomb energy tr(D J[D]) is MDERI_COULOMB with Wl = Wr = D.
 * Synchronisation and screening as for mderi_jkbuild.  By default the
 * gradient sums use FP64 atomics (last bits vary from run to run).  With
 * opts->deterministic = 1 every contribution v is added as |v| 2^80 in four
 * 32-bit digits (weights 2^(32k-80), so |v| < 2^47 in steps of 2^-80), each
 * with v's sign into its own 64-bit word by integer atomics; the words are
 * summed over the partial copies as integers and the total rounded once, so
 * the result is the same bits on every run (work space four times larger).
 */
mderi_status mderi_kbuild_grad(mderi_ctx_t ctx, mderi_basis_t basis, int pattern, const double *Wl_dev,
                               const double *Wr_dev, int nao, double scale, double *grad_dev, int natom, int accumulate,
                               const mderi_opts *opts, void *stream);

#ifdef __cplusplus
}
#endif
#endif
