/*
 * dmlmc.h -- C ABI of the deflated multigrid multilevel Monte Carlo library (gfx950).
 *
 * Computes tr(D^-1) for the 2D Wilson-Schwinger operator D by multigrid multilevel
 * Monte Carlo with exact deflation of the coarsest term (Frommer & Ramirez-Hidalgo,
 * "Deflated Multigrid Multilevel Monte Carlo", Lattice 2022: eq. 11 with eqs. 4-7).
 *
 * Conventions shared by every call
 * --------------------------------
 * Status:      every call returns dmlmc_status (0 = OK, < 0 = error) and never throws
 *              or aborts across the ABI.  dmlmc_last_error() gives the message.
 * Validation:  arguments are checked on the host before any device work; a rejected
 *              call returns DMLMC_EINVAL and leaves every output untouched.
 * Streams:     all device work of a context is enqueued on the context's stream; every
 *              call returns after that stream is synchronised (results are ready).
 * Ownership:   the caller owns every buffer it passes.  Host inputs are copied before
 *              the call returns.  Device buffers (B, X, ...) are caller-allocated, must
 *              not alias each other, and are only read/written during the call.  The
 *              library owns contexts, hierarchies and deflations together with their
 *              device memory; each is released only by its destroy/free call.  A
 *              hierarchy or deflation belongs to the context that created it.
 * Threads:     a context is not thread-safe; distinct contexts are independent.
 * Complex:     interleaved (re, im) pairs: complex128 = 2 doubles, complex64 = 2 floats
 *              (the layout of numpy/torch complex arrays).
 * Index:       a vector at level l with lattice Lx_l x Lt_l and d_l dofs per site has
 *              n_l = Lx_l * Lt_l * d_l entries; entry d_l * (x + Lx_l * t) + dof.
 *              Fine level: d_1 = 2 spin components.  Coarse level: the first half of a
 *              site's dofs has chirality +, the second half chirality -.
 * Blocks of RHS: nrhs vectors stored one after another with leading dimension ld >= n_l
 *              (vector r starts at element r * ld).
 * Levels:      1-based, l = 1 is the fine lattice, l = L the coarsest.
 */
#ifndef DMLMC_H
#define DMLMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DMLMC_OK = 0,
  DMLMC_EINVAL = -1,   /* invalid argument (shape, level, size, null pointer)        */
  DMLMC_ENOMEM = -2,   /* device or host allocation failed                            */
  DMLMC_EHIP = -3,     /* a HIP runtime call failed; message holds the HIP error      */
  DMLMC_ENOCONV = -4,  /* solver stopped at maxiter; outputs hold the best iterate    */
  DMLMC_ENUMERIC = -5, /* NaN or Inf detected in a residual norm                      */
  DMLMC_ESTATE = -6    /* object used with a context it does not belong to            */
} dmlmc_status;

typedef enum { DMLMC_FP64 = 0, DMLMC_MIXED = 1 } dmlmc_precision;

typedef struct dmlmc_ctx dmlmc_ctx;
typedef struct dmlmc_hier dmlmc_hier;
typedef struct dmlmc_defl dmlmc_defl;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  hip_stream: a hipStream_t to enqueue on,
 * or NULL for a stream the context creates (default priority) and owns. */
dmlmc_status dmlmc_create(dmlmc_ctx **out, int device, void *hip_stream);
void dmlmc_destroy(dmlmc_ctx *ctx);
/* Message of the last failed call on ctx (or of the last failed dmlmc_create when ctx
 * is NULL); owned by the library, valid until the next call on ctx. */
const char *dmlmc_last_error(const dmlmc_ctx *ctx);
/* Library version string. */
const char *dmlmc_version(void);

/* ---------------------------------------------------------------- hierarchy
 * The operator (Sec. 1 and 4.3: the 2D Wilson-Schwinger model; Gamma5-hermitian,
 * Sec. 2 before eq. 7), with Wilson parameter 1 and two spin components:
 *   (D psi)(x) = (m0+2) psi(x) - 1/2 sum_mu [ (1 - s_mu) U_mu(x) psi(x+mu)
 *                                       + (1 + s_mu) conj(U_mu(x-mu)) psi(x-mu) ],
 * s_x = sigma_1, s_t = sigma_2, Gamma5 = sigma_3; periodic in x, antiperiodic in t when
 * antiperiodic_t != 0.  U_mu(x, t) = exp(i theta[mu][t][x]).
 *
 * The multigrid hierarchy (Sec. 3.1, eq. 8 and the Petrov-Galerkin coarse operator
 * D_{l+1} = P_l^H D_l P_l; spin-preserving aggregation, eq. 14): level l is coarsened
 * by agg[l-1] = {ax, at} site blocks with ntv[l-1] test vectors per chirality.  The
 * test vectors are V = MGS(D_l^-1 ... MGS(D_l^-1 V0)) (n_inv steps, solves to relative
 * residual 1e-12) from Z4 start vectors V0 drawn by the SplitMix64 counter hash with
 * `seed`; P_l is the QR factor (positive real diagonal) of V on every
 * (aggregate, chirality) block.  import_tv, when not NULL, gives per coarsening step
 * l (0-based) host complex128 test vectors [ntv][n_l] (vector k at k * n_l) that
 * replace the inverse iteration (P_l is then the local QR of the imported vectors). */
typedef struct {
  int Lx, Lt;
  double m0;
  int antiperiodic_t;
  const double *theta; /* host, [2][Lt][Lx]; copied */
} dmlmc_lattice;

typedef struct {
  int nlevels;          /* L >= 1 (1 = fine level only, no coarsening) */
  int agg[7][2];        /* {ax, at} per coarsening step */
  int ntv[7];           /* test vectors per chirality per coarsening step */
  int n_inv;            /* inverse-iteration steps of the test-vector setup (>= 1) */
  uint64_t seed;        /* seed of the Z4 start vectors */
  const void *const *import_tv; /* NULL or nlevels-1 host pointers (see above) */
} dmlmc_mg_params;

/* Builds the hierarchy.  Errors: EINVAL when a lattice extent is not divisible by its
 * aggregate, a coarse extent would be < 2, ntv exceeds the rows of an
 * (aggregate, chirality) block, or nlevels is outside 1..8. */
dmlmc_status dmlmc_build_hierarchy(dmlmc_ctx *ctx, const dmlmc_lattice *lat,
                                   const dmlmc_mg_params *mg, dmlmc_hier **out);
void dmlmc_free_hierarchy(dmlmc_hier *h);

/* Level geometry: lattice extents and dofs per site of level `level`. */
dmlmc_status dmlmc_level_info(const dmlmc_hier *h, int level, int *Lx, int *Lt, int *dofs);

/* Stride (in complex entries) between consecutive right-hand sides of the solver's
 * internal work vectors on level `level`: the level size n, plus 256 below the coarsest
 * level once n >= 4096 (at power-of-two level sizes the same entry of consecutive RHS
 * would otherwise fall on the same HBM channels).  Vectors passed through this interface
 * are [nrhs][n] unless an entry point takes strides.  Errors: EINVAL. */
dmlmc_status dmlmc_work_stride(const dmlmc_hier *h, int level, int64_t *ld);

/* Copies level data to host buffers (any of them may be NULL):
 *   P_host:  complex128 [n_level][n_{level+1}] dense row-major interpolator P_level
 *            (level < L; zero outside the aggregate blocks);
 *   Dc_host: complex128 [sites][5][d][d] block stencil of level `level` >= 2
 *            (directions self, +x, -x, +t, -t; where an extent is 2 the +mu block holds
 *            the whole coupling and the -mu block is zero);
 *   tv_host: complex128 [ntv][n_level] test vectors used for P_level (level < L). */
dmlmc_status dmlmc_export_level(dmlmc_ctx *ctx, const dmlmc_hier *h, int level, void *P_host,
                                void *Dc_host, void *tv_host);

/* ---------------------------------------------------------------- deflation
 * Exact deflation at level `level` (normally L) by the k eigenpairs of
 * Q = Gamma5 D_level with the smallest |lambda| (ties: lambda ascending), which are the
 * k smallest singular triplets of D_level (eq. 7: U = Gamma5 X sign(Lambda), V = X,
 * Sigma = |Lambda|).  The projector is Pi = W W^H with W = Gamma5 X_k (eq. 4) and the
 * small trace term tr(D^-1 Pi) = sum_i x_i^H Gamma5 x_i / lambda_i (eq. 6) is returned in
 * tr_defl_out.  The eigensolver is Chebyshev-filtered subspace iteration on Q^2 with
 * Rayleigh-Ritz on Q, run until every residual ||Q x_i - lambda_i x_i|| <= eig_rtol *
 * ||Q||_est.  import_X (host complex128 [k][n_level]) and import_lambda (host double
 * [k]), when not NULL, replace the eigensolve.  Errors: EINVAL for k < 1 or k > n_level
 * / 4; ENOCONV when the eigensolver stops at its iteration limit (outputs still set). */
dmlmc_status dmlmc_deflate(dmlmc_ctx *ctx, dmlmc_hier *h, int level, int k, double eig_rtol,
                           const void *import_X, const double *import_lambda,
                           dmlmc_defl **out, double *tr_defl_out);
void dmlmc_free_deflation(dmlmc_defl *d);
/* Eigensolver statistics: outer subspace iterations, Chebyshev degrees summed over them
 * (Q^2 applications per subspace vector) and the final max ||Q x_i - lambda_i x_i|| /
 * ||Q||_bound (all zero for an imported deflation).  Any pointer may be NULL. */
dmlmc_status dmlmc_deflation_info(const dmlmc_defl *d, int *iters, int64_t *degree_sum,
                                  double *max_residual);
/* Copies the deflation to the host: X_host complex128 [k][n_level] eigenvectors of Q,
 * lambda_host double [k]; either may be NULL. */
dmlmc_status dmlmc_export_deflation(dmlmc_ctx *ctx, const dmlmc_defl *d, void *X_host,
                                    double *lambda_host);

/* ---------------------------------------------------------------- solves
 * Solves D_level X = B for nrhs right-hand sides (Sec. 3.1: multigrid-preconditioned
 * Krylov solves; the paper solves each sample to a relative residual, Sec. 4.3).
 * Right-preconditioned FGMRES with per-RHS Krylov spaces, FP64 Arnoldi (Gram-Schmidt
 * with reorthogonalisation) and a V-cycle (eq. 8, applied recursively) as
 * preconditioner; stops when ||B_r - D X_r|| <= rtol ||B_r|| for every r, the residual
 * computed in FP64.  prec = DMLMC_FP64: everything in FP64.  prec = DMLMC_MIXED: the
 * V-cycle, its smoother and coarse solves and the operator inside the Krylov solver run
 * in complex FP32; an outer FP64 iterative refinement recomputes the residual in FP64.
 * When proj != NULL (a deflation of this level) B is replaced by (I - W W^H) B.
 * A right-hand side whose root-mean-square entry lies outside 2^-8 .. 2^8 is solved as
 * 2^-e B_r (2^e its root mean square, exact in every precision) and its solution scaled
 * back, so the complex-FP32 bulk neither underflows nor overflows.
 * B, X: device complex128, [nrhs][ld]; X is overwritten (initial guess zero).
 * maxiter bounds the total Krylov iterations per RHS.  Errors: EINVAL (level, nrhs < 1,
 * ld < n_level, null pointers), ENOCONV (rtol not met; X holds the last iterate),
 * ENUMERIC (NaN/Inf residual). */
typedef struct {
  int iters;        /* Krylov iterations (max over RHS, summed over refinement steps) */
  int ir_steps;     /* FP64 refinement steps (1 in FP64 mode) */
  int converged;    /* 1 if every RHS met rtol */
  double relres_max;/* max_r ||B_r - D X_r|| / ||B_r|| in FP64 */
} dmlmc_solve_stats;

dmlmc_status dmlmc_solve_multi_rhs(dmlmc_ctx *ctx, const dmlmc_hier *h, int level,
                                   const dmlmc_defl *proj, const void *B, void *X, int nrhs,
                                   int64_t ld, dmlmc_precision prec, double rtol, int maxiter,
                                   dmlmc_solve_stats *stats);

/* ---------------------------------------------------------------- trace
 * MGMLMC estimate of tr(D^-1) (eq. 11) with exact deflation of the coarsest term
 * (eq. 5): samples of difference level l < L are s = x^H D_l^-1 x - y^H D_{l+1}^-1 y with
 * y = P_l^H x; samples of level L are s = x^H D_L^-1 (x - W W^H x); x is the real Z2
 * vector of sample i of level l, entry j = 1 - 2 bit_j(SplitMix64 hash of
 * (noise_seed, l, i, j / 64)).  Samples are drawn in blocks of rhs_block indices; the
 * estimate is Re(sum_l mean_l) + tr_defl with relative error sqrt(sum_l var_l / N_l) /
 * |estimate|.  Sample counts start at n0[l] (rounded up to rhs_block) and follow the
 * multilevel allocation N_l = ceil(eps^-2 T^-2 sqrt(V_l / C_l) sum_j sqrt(V_j C_j))
 * (C_l: a fixed per-level work proxy) until the error is <= eps, unless fixed_counts.
 * rhs_block = 0 takes the block size chosen by dmlmc_tune_rhs_block for this hierarchy
 * (ESTATE if it was never tuned).
 * samples_out[l-1], when not NULL, receives max_samples[l-1] complex128 sample values
 * (host).  Errors: EINVAL, ENOCONV (a solve failed; result holds the samples so far). */
typedef struct {
  double eps;
  uint64_t noise_seed;
  int n0[8];
  int64_t max_samples[8];
  int rhs_block;
  dmlmc_precision prec;
  double rtol;
  int fixed_counts;
  int maxiter;
  double *samples_out[8];
  /* skip[l-1] != 0 leaves hierarchy level l out of the telescoping sum, so that a term
   * joins level l-1 to level l+1 through the composite P_{l-1} P_l (eq. 12; levels 1 and
   * L are always kept).  Results, n0, max_samples and samples_out stay indexed by the
   * level a term starts at; skipped levels report N = 0. */
  int skip[8];
  /* term_defl[a-1]: exact deflation of the difference term that starts at level a
   * (dmlmc_deflate_difference for that term), or NULL; its trace term is added to the
   * estimate and to tr_defl of the result. */
  const dmlmc_defl *term_defl[8];
} dmlmc_mlmc_params;

typedef struct {
  double trace, trace_imag, rel_err;   /* tr_defl below is included in trace */
  int64_t N[8];
  double mean_re[8], mean_im[8], var[8];
  double cost_s[8];       /* wall seconds spent per level */
  double tr_defl;
  double t_trace_s;       /* wall seconds of the whole estimate */
  int64_t iters[8];       /* Krylov iterations summed over the level's solves */
} dmlmc_trace_result;

dmlmc_status dmlmc_mlmc_trace(dmlmc_ctx *ctx, const dmlmc_hier *h, const dmlmc_defl *coarsest,
                              const dmlmc_mlmc_params *p, dmlmc_trace_result *out);

/* ---------------------------------------------------------------- deflated Hutchinson
 * Plain (single-level) Hutchinson estimate of tr(D^-1) at the fine level (Sec. 1, eq. 1)
 * with exact deflation (Sec. 2, eqs. 4-7; the comparison method of Table 1): samples
 * s = x^H D_1^-1 (x - W W^H x), x the Z2 vector of sample i of level 1 (the noise stream
 * of the multilevel estimator's first level), W from fine = dmlmc_deflate at level 1
 * (k up to n_1 / 4), or fine = NULL for no deflation.  Estimate Re(mean) + tr_defl(fine),
 * relative error sqrt(var / N) / |estimate|; N starts at n0[0] (rounded up to the RHS
 * block) and grows to ceil(var / (eps T)^2) until the error is <= eps, unless
 * fixed_counts.  The solves use the hierarchy's V-cycles; coarsest (NULL allowed) is
 * attached to their coarsest solve for the call (for a one-level hierarchy, fine is).
 * p as for dmlmc_mlmc_trace with only index 0 of n0, max_samples and samples_out used;
 * skip and term_defl must be zero.  out: index 0 of the per-level arrays.
 * Errors: EINVAL, ESTATE, ENOCONV. */
dmlmc_status dmlmc_hutchinson_trace(dmlmc_ctx *ctx, const dmlmc_hier *h, const dmlmc_defl *fine,
                                    const dmlmc_defl *coarsest, const dmlmc_mlmc_params *p,
                                    dmlmc_trace_result *out);

/* ---------------------------------------------------------------- difference-level deflation
 * Exact deflation of the term (a, b) of the telescoping sum (Sec. 4.2):
 * M_ab = D_a^-1 - P_ab D_b^-1 P_ab^H with P_ab = P_a ... P_{b-1} (b = a + 1, or further
 * when the levels in between are skipped, eq. 12).  The k eigenpairs of largest |lambda|
 * (ties: lambda descending) of the Hermitian J_ab = M_ab Gamma5 = Q_a^-1 - P_ab Q_b^-1 P_ab^H
 * (eqs. 15-16) give the k largest singular triplets of M_ab, with right singular vectors
 * V = Gamma5 X.  Samples of the term then project x - V V^H x, and the estimate adds
 * tr(M_ab V V^H) = sum_i lambda_i x_i^H Gamma5 x_i (returned in *corr_out and kept as
 * tr_defl of the handle).  Each application of J solves with D_a and D_b in precision
 * prec to relative residual solve_rtol; the block Davidson eigensolver stops when
 * max_i ||J x_i - lambda_i x_i|| <= eig_rtol max_i |lambda_i| (ENOCONV after 400 steps,
 * handle still returned).  The V-cycles inside use the coarsest deflation attached with
 * dmlmc_set_deflation, if any.  import_X (host [k][n_a] complex128, orthonormal) and
 * import_lambda (host [k]) replace the eigensolver.
 * Inexact deflation (Sec. 3.2, here for M_ab): with corr_rtol > 0 the small term is not
 * taken from the eigenpairs but evaluated for the vectors at hand,
 * Re sum_i x_i^H Gamma5 (J_ab x_i), with k more applications of J solved to corr_rtol; the
 * split then holds for approximate vectors (a loose eig_rtol / solve_rtol, e.g. 1e-1 /
 * 1e-3).  corr_rtol <= 0: sum_i lambda_i x_i^H Gamma5 x_i (exact eigenpairs).
 * Errors: EINVAL (1 <= a < b <= L, 1 <= k, 4 k <= n_a), ENOCONV, ENOMEM, EHIP.  The handle
 * is freed by dmlmc_free_deflation. */
dmlmc_status dmlmc_deflate_difference(dmlmc_ctx *ctx, dmlmc_hier *h, int a, int b, int k, double eig_rtol,
                                      double solve_rtol, dmlmc_precision prec, const void *import_X,
                                      const double *import_lambda, double corr_rtol, dmlmc_defl **out,
                                      double *corr_out);

/* ---------------------------------------------------------------- direct coarsest solve
 * enable = 1 or 2: the complex-FP32 coarsest solves (inside every mixed-precision V-cycle,
 * and so the preconditioner of solves at the coarsest level) apply the explicit inverse
 * D_L^-1 instead of the fixed-count GMRES; the paper's coarsest level is likewise solved
 * directly.  The inverse is computed once, column by column from multi-RHS solves of
 * D_L X = I (1024 columns per solve) refined in FP64 to a residual of 1e-8 for
 * enable = 1 and 1e-6 for the FP16 and 8-bit copies, far below the rounding of the copy
 * applied (coarsest, if given, deflates their V-cycles); an inverse built to the looser
 * tolerance is rebuilt when enable = 1 asks for the tighter one.  It is kept in complex
 * FP32: n_L^2 * 8 bytes (2.1 GB at n_L = 16384).
 *   enable = 1: applied in FP32 on the matrix cores (exact to FP32 rounding);
 *   enable = 2: applied from a complex-FP16 copy (n_L^2 * 4 more bytes, made on first
 *               use; one power-of-two scale for the matrix and one per RHS, FP32
 *               accumulation): each coarsest solve is then accurate to ~1e-3 relative,
 *               half the bytes and half the matrix-core instructions of enable = 1;
 *   enable = 3: applied from an 8-bit copy (n_L^2 * 2 more bytes, made on first use):
 *               each component is a byte of sign, 4 exponent bits (bias 7) and 3
 *               mantissa bits, nearest with ties to even, after its row is scaled by a
 *               power of two that brings the row's largest component below 256.  In the
 *               kernel a byte is widened exactly to FP16, and the products run as for
 *               enable = 2.  Each coarsest solve is then accurate to a few percent
 *               (2^-4 relative rounding per entry), with a quarter of the bytes of
 *               enable = 1.
 * Every solve still stops at its FP64 residual tolerance, so the precision changes
 * iteration counts only.  enable = 0 returns to the iterative coarsest solve and frees
 * every inverse.  Needs a coarse coarsest level with 16 dofs per site and
 * n_L <= 65536, n_L a multiple of 256 (EINVAL otherwise); ENOCONV if a column solve
 * fails, ENUMERIC if the inverse holds NaN/Inf.  The FP64 solver path is unaffected. */
dmlmc_status dmlmc_coarsest_direct(dmlmc_ctx *ctx, dmlmc_hier *h, const dmlmc_defl *coarsest, int enable);

/* ---------------------------------------------------------------- RHS block autotuner
 * Batching is this library's own design choice (the method is indifferent to how many
 * noise vectors one launch carries), so the block size is measured, not derived: for
 * each of the ncand candidate sizes, one block of samples of every level is drawn and
 * solved (twice; the second, warm pass is timed) exactly as dmlmc_mlmc_trace would with
 * precision prec and tolerance rtol, using sample indices from 2^62 on, so no estimate's
 * samples are touched.  The candidate with the least wall time per sample summed over
 * the levels is stored in the hierarchy (used by dmlmc_mlmc_trace with rhs_block = 0)
 * and returned in *best; sec_per_sample (nullable, host [ncand]) receives the sums.
 * candidates: host [ncand], each in 1..512, ncand in 1..16.  coarsest: as for
 * dmlmc_mlmc_trace.  Errors: EINVAL, ENOCONV (a solve failed). */
dmlmc_status dmlmc_tune_rhs_block(dmlmc_ctx *ctx, dmlmc_hier *h, const dmlmc_defl *coarsest,
                                  const int *candidates, int ncand, dmlmc_precision prec, double rtol,
                                  uint64_t noise_seed, int *best, double *sec_per_sample);

/* ---------------------------------------------------------------- launch-variant autotuner
 * The hot complex-FP32 kernels of the V-cycles each come in launch variants that divide
 * the same work differently over threads and wavefronts; the arithmetic of every output
 * entry is the same in all of them, so a choice changes timing only, never a result bit.
 * Kernel ids and their values (0 always selects the built-in rule):
 *   DMLMC_KV_WILSON_RB     fine stencil, RHS per thread: 1, 2, 4, 8
 *   DMLMC_KV_COARSE_SPLIT  coarse block stencil (16 dofs/site): wavefronts per site, 1 or 2;
 *                          3: one wavefront per site, blocks and vectors read and results
 *                          written by whole 128-byte lines staged through LDS (the rule)
 *   DMLMC_KV_SAP_RB        SAP colour sweep, RHS per thread: 1, 2, 4, 8
 *   DMLMC_KV_GS_SPLIT      coarse Gauss-Seidel (FP16 blocks): wavefronts per site, 1 or 2;
 *                          3: one wavefront per site with two 16-RHS tiles' loads in flight;
 *                          4: one wavefront per site, vectors read and written by whole
 *                          128-byte lines staged through LDS
 *   DMLMC_KV_RESTRICT_UT   matrix-core restriction: tiles per batch of loads, 1, 2, 4
 *   DMLMC_KV_PROLONG_MT    matrix-core prolongation: tiles per wavefront, 1, 2, 4 (a value
 *                          that does not divide the level's tile count falls back to the rule)
 *   DMLMC_KV_PROLONG_STAGED  prolongation onto a level with 16 dofs per site, or whose
 *                          aggregate rows are half a 128-byte line (a_x x dofs = 8, an even
 *                          number of aggregates in x): 1 = direct loads and stores, 2 = whole
 *                          128-byte lines staged through LDS (the rule from 16384 fine sites on)
 *   DMLMC_KV_RESTRICT_STAGED  restriction from a level whose aggregate rows are half a line
 *                          (as above, a_t <= 4): 1 = direct, 2 = whole lines staged through
 *                          LDS, one wavefront per pair of aggregates adjacent in x (the rule
 *                          from 16384 fine sites on)
 * dmlmc_tune_kernels times, on every level of h, each variant of each kernel that runs
 * there at that level's real shape (nrhs right-hand sides at the solver's work stride,
 * reps launches per variant after one warm-up, HIP events on the context stream) and
 * keeps the fastest if it beats the built-in rule by more than 2 % (else the rule).  Choices are cached in the process by (GPU
 * architecture, kernel, level shape, nrhs, stride); cache_path (nullable) names a text
 * file read before and rewritten after tuning ("key value" per line), so a later process
 * reuses them without timing.  picks (nullable, host int [levels][DMLMC_KV_COUNT])
 * receives each choice (-1: the kernel does not run on that level); best_us and
 * default_us (nullable, host double, same shape) the time per launch of the choice and
 * of the rule (both 0 when the choice came from the cache).  Temporary vectors are
 * allocated and freed inside the call.  Errors: EINVAL (nrhs not in 1..512, reps not in
 * 1..1000, cache file not writable), EHIP. */
enum { DMLMC_KV_WILSON_RB = 0, DMLMC_KV_COARSE_SPLIT = 1, DMLMC_KV_SAP_RB = 2, DMLMC_KV_GS_SPLIT = 3,
       DMLMC_KV_RESTRICT_UT = 4, DMLMC_KV_PROLONG_MT = 5, DMLMC_KV_PROLONG_STAGED = 6,
       DMLMC_KV_RESTRICT_STAGED = 7, DMLMC_KV_COUNT = 8 };
dmlmc_status dmlmc_tune_kernels(dmlmc_ctx *ctx, dmlmc_hier *h, int nrhs, int reps, const char *cache_path,
                                int *picks, double *best_us, double *default_us);
/* Sets (or reads) one kernel's variant on one level (1-based) by hand; EINVAL for an
 * unknown kernel id, a level out of range or a value not listed above.  Recorded HIP
 * graphs of earlier launches are re-recorded on their next use. */
dmlmc_status dmlmc_set_kernel_variant(dmlmc_hier *h, int level, int kernel, int value);
dmlmc_status dmlmc_get_kernel_variant(const dmlmc_hier *h, int level, int kernel, int *value);

/* ---------------------------------------------------------------- single operators
 * Applies one operator of level `level` to nrhs device vectors (for parity checks and
 * kernel timing).  in/out: device, complex128 when prec = DMLMC_FP64 and complex64
 * when prec = DMLMC_MIXED, [nrhs][ld_in] / [nrhs][ld_out] with ld = n of the vector's
 * level:
 *   DMLMC_OP_D         out = D_level in
 *   DMLMC_OP_RESTRICT  out (level+1) = P_level^H in (level)
 *   DMLMC_OP_PROLONG   out (level) = P_level in (level+1)
 *   DMLMC_OP_SMOOTH    out = smoother sweeps(out; b = in), out is the initial guess
 *   DMLMC_OP_VCYCLE    out = V-cycle(in) (one preconditioner application)
 *   DMLMC_OP_DEFL_C    out ([nrhs][k]) = W^H in                 (needs dmlmc_set_deflation)
 *   DMLMC_OP_DEFL_P    out = in - W (W^H in)                    (needs dmlmc_set_deflation)
 *                      (both take complex128 in/out; DMLMC_FP64 selects FP64 kernels,
 *                      DMLMC_MIXED the complex-FP32 matrix-core kernels with FP64
 *                      accumulation of W^H in)
 *   DMLMC_OP_GAMMA5_D  out = Gamma5 D_level in
 * `arg` is the number of smoother sweeps for DMLMC_OP_SMOOTH and unused otherwise. */
enum {
  DMLMC_OP_D = 0, DMLMC_OP_RESTRICT = 1, DMLMC_OP_PROLONG = 2, DMLMC_OP_SMOOTH = 3,
  DMLMC_OP_VCYCLE = 4, DMLMC_OP_DEFL_C = 6, DMLMC_OP_DEFL_P = 7, DMLMC_OP_GAMMA5_D = 8
};
dmlmc_status dmlmc_apply(dmlmc_ctx *ctx, const dmlmc_hier *h, int op, int level, const void *in,
                         void *out, int nrhs, dmlmc_precision prec, uint64_t arg);

/* dmlmc_apply with the vectors' strides given: RHS r of in at r * ld_in, of out at
 * r * ld_out (complex entries; 0 stands for n of the vector's level).  Entries between n
 * and the stride are neither read nor written.  Strides must be even and at least n;
 * DMLMC_OP_SMOOTH and DMLMC_OP_VCYCLE need ld_in == ld_out (and DMLMC_OP_VCYCLE on the
 * coarsest level unpadded vectors), the DMLMC_OP_DEFL_* operators unpadded vectors.
 * Errors: as dmlmc_apply. */
dmlmc_status dmlmc_apply_strided(dmlmc_ctx *ctx, const dmlmc_hier *h, int op, int level, const void *in,
                                 int64_t ld_in, void *out, int64_t ld_out, int nrhs, dmlmc_precision prec,
                                 uint64_t arg);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): out = in - W (W^H in) for nrhs
 * unpadded complex128 vectors [nrhs][n] of the deflation's level (n = n_level), computed
 * exactly as dmlmc_apply(DMLMC_OP_DEFL_P, DMLMC_MIXED) computes it (complex-FP32 matrix-core
 * products, FP64 sums across K-chunks).  It calls no device allocation: the K-chunk
 * partials and the coefficients W^H in live in a 16 MiB array that each GPU holds from
 * library load until the process ends; a call needs 16 * k * nrhs * (ceil(n / 256) + 1)
 * bytes of it (n = 16384, k = 128: up to 124 RHS).  All calls on one GPU share that array,
 * so calls that overlap in time on one GPU (other contexts or threads) race and must be
 * serialised by the caller; nothing in it needs to persist between calls.  in and out are
 * device buffers owned by the caller and must not overlap; d need not be attached.
 * Returns after the context stream is synchronised.  Errors: EINVAL (NULL arguments,
 * nrhs < 1, overlapping buffers, a size beyond the array), ESTATE (d from another
 * context), EHIP. */
dmlmc_status dmlmc_deflate_project_noalloc(dmlmc_ctx *ctx, const dmlmc_defl *d, const void *in, void *out,
                                           int nrhs);

/* Writes the real Z2 noise vectors of samples sample0 .. sample0 + nrhs - 1 of level
 * `level` (length n each, [nrhs][n], device, complex128 for DMLMC_FP64 / complex64 for
 * DMLMC_MIXED): entry j = 1 - 2 * bit (j % 64) of SM(SM(SM(SM(seed) + level) + i) + j / 64)
 * with SM one SplitMix64 step (Steele, Lea & Flood 2014); Z2 noise as in Sec. 2, eq. 2. */
dmlmc_status dmlmc_z2_noise(dmlmc_ctx *ctx, int64_t n, uint64_t seed, int level, int64_t sample0,
                            int nrhs, void *out, dmlmc_precision prec);

/* Attaches (or with d = NULL detaches) a deflation used by DMLMC_OP_DEFL_* and, when it is
 * of the coarsest level, by the coarsest solve inside every V-cycle (exact inverse on the
 * deflation space, GMRES on the projected rest).  The caller keeps d alive while attached.
 * dmlmc_mlmc_trace attaches its coarsest deflation for the duration of the call. */
dmlmc_status dmlmc_set_deflation(dmlmc_hier *h, const dmlmc_defl *d);

/* ---------------------------------------------------------------- solver parameters
 * Parameters of the solver that change iteration counts and speed but not the solution
 * (every solve still stops at its FP64 residual tolerance): SAP local minimal-residual
 * iterations (default 2), pre/post smoothing sweeps of the V-cycle (nu_pre 0, nu_post 2
 * on the fine level, nu_post_coarse 2 on the coarse levels; every level must smooth at
 * least once), fixed GMRES iterations of the coarsest solve without / with an attached
 * coarsest deflation (24 / 8), the FGMRES restart length (16, at most 31), and
 * use_graphs: 1 (default) replays each complex-FP32 FGMRES iteration (preconditioner,
 * operator, Gram-Schmidt) as a recorded HIP graph after its first two runs with the same
 * shapes, 0 launches every kernel directly (results are bitwise the same).  Values < 0
 * keep the current setting; a rejected call (EINVAL) changes nothing. */
typedef struct {
  int sap_mr_iters, nu_pre, nu_post, coarsest_iters, coarsest_iters_defl, restart, use_graphs, nu_post_coarse;
  /* mixed precision: each complex-FP32 FGMRES cycle stops once it has reduced the FP64
   * residual it started from by this factor (0 < inner_rtol < 1, default 1e-2), after
   * which the residual is recomputed in FP64 and a new cycle starts; < 0 keeps it */
  double inner_rtol;
  /* 1 (default): the coarse-level block Gauss-Seidel sweeps of the complex-FP32 V-cycles
   * read complex-FP16 copies of the hop and inverse self blocks (half the block bytes;
   * the products and vectors stay FP32; a preconditioner, so iteration counts only; a
   * level with a block entry beyond the FP16 range keeps its FP32 blocks);
   * 0: the FP32 blocks; < 0 keeps the setting */
  int smoother_half;
} dmlmc_solver_params;
dmlmc_status dmlmc_set_solver_params(dmlmc_hier *h, const dmlmc_solver_params *p);
dmlmc_status dmlmc_get_solver_params(const dmlmc_hier *h, dmlmc_solver_params *p);

/* ---------------------------------------------------------------- progress lines
 * level > 0: long phases of this context (each outer iteration of the eigensolvers, the
 * device Rayleigh-Ritz factorisations) print one progress line each to stderr; 0 (the
 * default): silent. */
dmlmc_status dmlmc_set_verbose(dmlmc_ctx *ctx, int level);

/* ---------------------------------------------------------------- kernel timing
 * When enabled, the library brackets every launch of the named kernel classes with HIP
 * events on the context stream and accumulates their durations.  Classes:
 * "wilson", "coarse", "sap", "coarse_gs", "restrict", "prolong", "gs_dots", "gs_update",
 * "gs_fused" (the single-workgroup Arnoldi step of small levels), "defl_gemm",
 * "coarse_direct" (the FP32 explicit-inverse coarsest solve) and "coarse_direct16" (its
 * FP16 form: RHS scaling, product and reduction as one timed unit).
 * dmlmc_timing_get returns (launches, total milliseconds, work summed over launches) for
 * a class: algorithmic bytes, except flops for "defl_gemm" and "coarse_direct".
 * dmlmc_timing_select restricts the bracketing to a comma-separated list of classes
 * (NULL or "" = every class), so that a timed run carries events only around the kernels
 * it measures.  Unknown names are accepted and simply never match.  The colour sweeps of
 * one smoother call ("sap", "coarse_gs") run back to back and are bracketed by one event
 * pair; each of them counts as one launch of the class, with its own bytes. */
dmlmc_status dmlmc_timing_enable(dmlmc_ctx *ctx, int enable);
dmlmc_status dmlmc_timing_select(dmlmc_ctx *ctx, const char *classes);
dmlmc_status dmlmc_timing_reset(dmlmc_ctx *ctx);
dmlmc_status dmlmc_timing_get(dmlmc_ctx *ctx, const char *cls, int64_t *launches, double *ms,
                              double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* DMLMC_H */
