/*
 * krr.h -- C ABI of the MI355X (gfx950) kernel-ridge-regression library.
 *
 * The library computes the three phases of the paper's multivariate-GWAS
 * KRR driver (arXiv 2409.01712, Algorithm 1) on one GPU:
 *
 *   Build     K_ij = exp(-gamma * ||g_i - g_j||^2) over all training patient
 *             pairs (Algorithm 2 with the Gaussian kernel of Algorithm 5),
 *             the squared distances formed as an INT8 Gram product
 *             d_ij = n_i + n_j - 2 g_i . g_j (subsection "Engaging INT8
 *             Tensor Cores for Distance Calculations"), exponentiated per
 *             tile before the tile is released ("TC-based Distance
 *             Computations").
 *   Associate factor K + lambda*I = L L^T with a tile Cholesky whose
 *             trailing updates run in FP32, FP16 or FP8 per tile
 *             ("Deploying a Four-Precision Cholesky-Based Solver"), then
 *             solve for the weights W with triangular solves (Algorithm 3),
 *             refined against an FP64 residual.
 *   Predict   K_test = Build(gamma, T, G) and P = K_test W (Algorithm 4).
 *
 * Names: the paper's N_P1 is n, N_S is m, N_Ph is nrhs, P_h is Y, W is X,
 * P_r is P.  The paper's regularisation parameter (alpha in Algorithms 1
 * and 3) is called lambda here.
 *
 * Conventions for every entry point:
 *   - Pointers to matrices (G, T, Y, X, P, diagnostic destinations) are
 *     DEVICE pointers on the context's device, owned by the caller.
 *   - G and T are int8 row-major (one patient per row, SNPs contiguous) with
 *     values in {0, 1, 2}; ldg/ldt is the row pitch in bytes, a multiple of
 *     16 and >= m, and the base pointer is 16-byte aligned.
 *   - Y, X, P are FP64 column-major (one phenotype per column), leading
 *     dimension >= the number of rows.
 *   - Work is ordered on the context's HIP stream.  Calls that must read a
 *     device result (krr_factor, krr_solve, status-returning checks) wait
 *     on that stream; the others return after enqueueing.
 *   - Errors are returned as krr_status codes; nothing aborts or throws
 *     across the ABI.  On error no output handle is created.
 *   - One context must not be used from two host threads at once.
 */
#ifndef KRR_H
#define KRR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum krr_status {
  KRR_SUCCESS = 0,
  KRR_ERROR_INVALID_VALUE = 1,         /* bad argument (null, size, ld, gamma <= 0, lambda < 0) */
  KRR_ERROR_BAD_GENOTYPE = 2,          /* a genotype value outside {0, 1, 2} */
  KRR_ERROR_OUT_OF_MEMORY = 3,         /* device allocation failed or exceeds the workspace cap */
  KRR_ERROR_NOT_POSITIVE_DEFINITE = 4, /* Cholesky breakdown that promotion could not cure */
  KRR_ERROR_NOT_CONVERGED = 5,         /* refinement hit max_iters; X still written, info filled */
  KRR_ERROR_HIP = 6,                   /* a HIP runtime call failed */
  KRR_ERROR_NOT_SUPPORTED = 7,         /* option combination not implemented */
  KRR_ERROR_SCRATCH_TOO_SMALL = 8      /* krr_predict_noalloc: input larger than its fixed scratch */
} krr_status;

typedef struct krr_context_s *krr_context;
typedef struct krr_kernel_s *krr_kernel;
typedef struct krr_factor_s *krr_factorization;

/* Device allocator a caller may supply (both functions or neither): alloc
 * returns device memory of at least `bytes` on the context's device (NULL on
 * failure, reported as KRR_ERROR_OUT_OF_MEMORY); free gets back exactly what
 * alloc returned, with the same size.  The library keeps freed blocks in its
 * per-context cache and returns them through free when the cache is flushed
 * (krr_destroy, or an allocation failure). */
typedef void *(*krr_alloc_fn)(uint64_t bytes, void *user);
typedef void (*krr_free_fn)(void *ptr, uint64_t bytes, void *user);

/* Context options. */
typedef struct krr_options {
  int32_t tile;             /* Cholesky tile size nb: 256 or 512 (0 = 512) */
  int32_t verbose;          /* 0 = silent; 1 = per-call summary on stderr */
  int64_t workspace_limit;  /* max bytes the library may allocate (0 = no cap) */
  krr_alloc_fn device_alloc;/* NULL: hipMalloc */
  krr_free_fn device_free;  /* NULL: hipFree */
  void *alloc_user;         /* passed to both */
} krr_options;

/* Operand precisions of a trailing-matrix update. */
enum { KRR_PREC_FP32 = 0, KRR_PREC_FP16 = 1, KRR_PREC_FP8 = 2 };

/* Factorization precision policies. */
enum {
  KRR_POLICY_FP32 = 0,      /* every update in FP32 (the plain single-precision path) */
  KRR_POLICY_ADAPTIVE = 1,  /* per-update precision from operand (or tile) norms */
  KRR_POLICY_FIXED = 2,     /* every off-diagonal update of panels >= high_panels in fixed_prec */
  KRR_POLICY_FIXED_MAP = 3  /* the caller's map gives every off-diagonal update's precision */
};

/* ADAPTIVE precision rules (krr_precision_policy.rule). */
enum {
  KRR_RULE_OPERAND = 0, /* u_p ||L_IK||_F ||L_JK||_F <= eps ||A||_F / NT (default) */
  KRR_RULE_TILE = 1,    /* u_p ||A_IJ||_F <= eps ||A||_F / NT, ||A_IJ|| from the build */
  KRR_RULE_BOTH = 2     /* both must hold: the tile rule is a ceiling on the operand rule */
};

/*
 * Precision policy for krr_factor ("Deploying a Four-Precision
 * Cholesky-Based Solver"; the rule below is this library's reading of the
 * tile-centric adaptive precision the paper cites).
 *
 * ADAPTIVE: the update A_IJ -= L_IK L_JK^T (I > J > K) uses the lowest
 * allowed precision p with  u_p * ||L_IK||_F * ||L_JK||_F <= eps * ||A||_F / NT,
 * u_FP8 = 2^-4, u_FP16 = 2^-11; otherwise FP32 (rule KRR_RULE_OPERAND; see
 * KRR_RULE_* for the tile-norm variants).  Updates of diagonal tiles and of
 * panels K < high_panels are always FP32.  FP8 operands carry a per-tile
 * power-of-two scale (unless no_fp8_scale); accumulation is FP32.
 *
 * FIXED_MAP: fixed_map (HOST memory, fixed_map_count = NT * NT(NT+1)/2
 * bytes in the layout krr_factor_precision_map returns, NT = ceil(n / tile))
 * gives KRR_PREC_* for the update of tile (I, J) by panel K; entries of
 * diagonal tiles and values > KRR_PREC_FP8 mean FP32.  Replaying a map that
 * krr_factor_precision_map exported reproduces that factor bit for bit.
 *
 * Promotion (allow_promotion): after a non-positive pivot in tile row B,
 * every panel K < B may use one precision level less than before (FP8 ->
 * FP16 -> FP32) and the factorization is redone from the stored distances;
 * when all those panels are FP32 already, the diagonal POTRF moves to FP64;
 * when that is done too, KRR_ERROR_NOT_POSITIVE_DEFINITE.
 * A zero-initialised struct with mode and eps set is a valid policy.
 */
typedef struct krr_precision_policy {
  int32_t mode;            /* KRR_POLICY_* */
  int32_t allowed;         /* bit mask of (1 << KRR_PREC_FP16) | (1 << KRR_PREC_FP8) */
  double eps;              /* ADAPTIVE threshold (default 1.0) */
  int32_t high_panels;     /* panels K < high_panels update in FP32 (default 1) */
  int32_t fixed_prec;      /* FIXED mode: KRR_PREC_FP16 or KRR_PREC_FP8 */
  int32_t allow_promotion; /* on breakdown, promote the panels before it and refactor */
  int32_t diag_fp64;       /* 1: diagonal-tile POTRF in FP64; 0: in FP32 */
  int32_t rule;            /* ADAPTIVE: KRR_RULE_* (0 = operand norms) */
  int32_t no_fp8_scale;    /* 1: FP8 operands without the per-tile power-of-two scale */
  const uint8_t *fixed_map;/* FIXED_MAP only (host), else NULL */
  int64_t fixed_map_count; /* bytes at fixed_map */
} krr_precision_policy;

/* Refinement methods for krr_solve. */
enum {
  KRR_REFINE_NONE = 0, /* one pair of FP32 triangular solves, no FP64 residual */
  KRR_REFINE_IR = 1,   /* iterative refinement with an FP64 residual */
  KRR_REFINE_PCG = 2,  /* conjugate gradients on K + lambda I preconditioned by the factor
                          (A p from the FP64 residual kernel); iters counts CG steps.
                          krr_solve only: krr_solve_batched returns
                          KRR_ERROR_NOT_SUPPORTED */
  KRR_REFINE_AUTO = 3  /* IR while each iteration at least halves the bound, then PCG
                          from the current X (krr_solve_batched: IR) */
};

typedef struct krr_refine_opts {
  int32_t method;    /* KRR_REFINE_* */
  int32_t max_iters; /* default 30 */
  double tol;        /* stop when max_j ||r_j||_2 / (lambda ||x_j||_2) <= tol (default 1e-6) */
} krr_refine_opts;

typedef struct krr_solve_info {
  int32_t iters;        /* refinement iterations performed */
  int32_t converged;    /* 1 if the tolerance was met */
  double fwd_err_bound; /* max_j ||r_j|| / (lambda ||x_j||): a bound on the relative
                           forward error, since lambda_min(K + lambda I) >= lambda */
  double backward_err;  /* max_j ||r_j|| / (||A||_F ||x_j|| + ||y_j||) */
  double first_bound;   /* fwd_err_bound after the unrefined solve */
} krr_solve_info;

typedef struct krr_factor_info {
  int64_t updates[3];     /* tile updates performed in FP32, FP16, FP8 */
  int32_t promotions;     /* refactorizations after breakdown */
  int64_t breakdown_col;  /* first failing column of the last breakdown, -1 if none */
  int32_t nt;             /* tiles per dimension */
  int32_t tile;           /* tile size nb */
  double norm_a;          /* ||K + lambda I||_F */
} krr_factor_info;

/* Create a context on HIP device `device`, ordering work on `stream` (a
 * hipStream_t; NULL = the default stream).  opts may be NULL. */
krr_status krr_create(krr_context *ctx, int device, void *stream, const krr_options *opts);
/* Destroy a context.  If kernel or factor handles created on it are still
 * alive, the context is freed when the last of them is released; it accepts
 * no new work meanwhile. */
krr_status krr_destroy(krr_context ctx);
krr_status krr_set_stream(krr_context ctx, void *stream);

/*
 * Build (Algorithm 2, Gaussian kernel): computes and keeps, on the device,
 * the exact int32 squared distances and the FP32 matrix K + lambda*I over
 * the lower triangle of nb x nb tiles (n padded to a multiple of nb with
 * identity rows).  G (n x m, ldg) must stay valid and unchanged until the
 * kernel handle is released: predict and refactorization re-read it.
 * Returns KRR_ERROR_BAD_GENOTYPE (and no handle) if G has a value > 2.
 */
krr_status krr_build_kernel(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                            double gamma, double lambda, krr_kernel *out);
krr_status krr_kernel_release(krr_kernel K);

/* Kernel types of Algorithm 5. */
enum {
  KRR_KERNEL_GAUSSIAN = 0, /* K_ij = exp(-gamma (d_ij + dc_ij)), dc from the confounders (if any) */
  KRR_KERNEL_IBS = 1,      /* K_ij = (alleles shared identical by state) / (2m); gamma unused */
  KRR_KERNEL_LINEAR = 2    /* K_ij = g_i . g_j (exact int32; FP32 exact below 2^24); gamma
                              unused.  krr_kernel_copy_distances returns the inner products */
};

/*
 * Optional description of the kernel for krr_build_kernel_ex.
 *
 * IBS (Algorithm 5, IBS branch; the SKAT kernel of the state-of-the-art
 * survey): for genotypes a, b in {0, 1, 2} the alleles shared identical by
 * state are 2 - |a - b|; summed over the m SNPs and divided by the 2m
 * alleles of a patient (the text's normalisation; the algorithm's listing
 * divides by m).  Computed exactly as 1 - d/(2m) with d = sum_k |g_ik - g_jk|,
 * the squared distance of thermometer-encoded rows ([g >= 1], [g >= 2])
 * through the same INT8 Gram.  The library keeps the encoded copy (n x
 * 2 round_up(m, 16) bytes); krr_kernel_copy_distances returns d.
 *
 * Confounders (subsection "Engaging INT8 Tensor Cores for Distance
 * Calculations": real-valued covariates whose squared distances are added to
 * the integer genotype distances before the exponential): C is n x q FP64
 * row-major (one patient per row, leading dimension ldc >= q, q <= 32), a
 * DEVICE array copied at build time.  dc_ij = sum_k (c_ik - c_jk)^2 in FP64;
 * the library keeps exp(-gamma dc_ij) in FP64 (8 bytes per stored entry) for
 * the FP64 residual and multiplies it into the FP32 matrix.  Gaussian only;
 * Predict then needs the test rows' confounders (krr_predict_ex); the
 * batched solve and predict return KRR_ERROR_NOT_SUPPORTED for such kernels.
 */
typedef struct krr_kernel_desc {
  int32_t kind;     /* KRR_KERNEL_* */
  int32_t reserved; /* 0 */
  const double *C;  /* confounders (device), or NULL */
  int64_t q;        /* confounders per patient */
  int64_t ldc;      /* row pitch of C in elements */
} krr_kernel_desc;

/* Build with a kernel description (NULL = Gaussian without confounders, the
 * same as krr_build_kernel).  Errors as krr_build_kernel, plus
 * KRR_ERROR_INVALID_VALUE for an unknown kind or bad confounder sizes and
 * KRR_ERROR_NOT_SUPPORTED for q > 32. */
krr_status krr_build_kernel_ex(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                               double gamma, double lambda, const krr_kernel_desc *desc,
                               krr_kernel *out);

/*
 * Factorize (Algorithm 3, first half): L L^T = K + lambda*I under the
 * precision policy (NULL = ADAPTIVE defaults).  The first factorization of
 * a kernel handle consumes its FP32 matrix in place; later ones re-expand
 * it from the stored distances.  Blocks until the breakdown check is done.
 * Returns KRR_ERROR_NOT_POSITIVE_DEFINITE if a pivot is not positive and
 * promotion is off or exhausted.
 */
krr_status krr_factor(krr_context ctx, krr_kernel K, const krr_precision_policy *policy,
                      krr_factorization *out);
/* The kernel handle must outlive its factors (solves read its distances). */
krr_status krr_factor_release(krr_factorization F);
krr_status krr_factor_get_info(krr_factorization F, krr_factor_info *info);

/*
 * Solve (Algorithm 3, second half): X = (K + lambda*I)^{-1} Y for nrhs
 * phenotype columns, by FP32 forward/back substitution with the factor and
 * refinement against an FP64 residual recomputed from the exact distances
 * (classical refinement or preconditioned conjugate gradients, opts->method).
 * Convergence is always decided on a freshly computed residual of the final X.
 * Y, X: n x nrhs FP64 column-major on the device.  opts/info may be NULL.
 * Returns KRR_ERROR_NOT_CONVERGED if the tolerance is not met within
 * max_iters (X holds the last iterate).  Blocks once per iteration.
 */
krr_status krr_solve(krr_context ctx, krr_factorization F, const double *Y, int64_t nrhs, int64_t ldy,
                     double *X, int64_t ldx, const krr_refine_opts *opts, krr_solve_info *info);

/*
 * Predict (Algorithm 4): P = K_test X with K_test[i, j] = exp(-gamma d(t_i, g_j))
 * built by the INT8 cross Gram between T (n_test x m, ldt) and the kernel's
 * G, exponentiated and multiplied in FP64.  X: n x nrhs (ldx), P: n_test x
 * nrhs (ldp), FP64 column-major.
 */
krr_status krr_predict(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test, int64_t ldt,
                       const double *X, int64_t nrhs, int64_t ldx, double *P, int64_t ldp);
/* Predict for any kernel of krr_build_kernel_ex: the IBS kernel compares the
 * encoded test rows; with confounders Ct (n_test x q FP64 row-major, ldct >=
 * q, device) holds the test rows' covariates (NULL otherwise).  krr_predict
 * returns KRR_ERROR_INVALID_VALUE for a kernel with confounders. */
krr_status krr_predict_ex(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test,
                          int64_t ldt, const double *Ct, int64_t ldct, const double *X,
                          int64_t nrhs, int64_t ldx, double *P, int64_t ldp);

/*
 * Predict without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as krr_predict (the same
 * kernels, so P is bit-identical), but the working buffers (genotype-check
 * flag, test-row norms, the row-major copy of X, the cross distances of a
 * chunk of test rows) live in a fixed device scratch of
 * KRR_NOALLOC_SCRATCH_BYTES that each device holds from krr_create until the
 * process ends.  Calls no hipMalloc/hipFree and no allocating library routine.
 * Gaussian kernels without confounders only (KRR_ERROR_NOT_SUPPORTED
 * otherwise).  Limit: 256 + 4*n_test + 8*np*nrhs + 4*64*np bytes (rounded up to 256 each;
 * np = n rounded up to the tile size) must fit, else
 * KRR_ERROR_SCRATCH_TOO_SMALL before any work (krr_noalloc_limits answers
 * the question in advance).  Every call on one device shares that device's
 * scratch and leaves its contents behind: calls that overlap on one device
 * (two host threads, or two streams in flight) race and must be serialised
 * by the caller.  Blocks for the genotype check and at the end, like
 * krr_predict.
 */
#define KRR_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
krr_status krr_predict_noalloc(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test,
                               int64_t ldt, const double *X, int64_t nrhs, int64_t ldx, double *P,
                               int64_t ldp);
/* Host-only check: *fits = 1 if krr_predict_noalloc accepts n training
 * patients (tile size `tile`, 0 = 512), n_test test patients and nrhs
 * columns; *scratch_bytes = KRR_NOALLOC_SCRATCH_BYTES.  No GPU work. */
krr_status krr_noalloc_limits(int64_t n, int64_t n_test, int64_t nrhs, int32_t tile,
                              int64_t *scratch_bytes, int32_t *fits);
/* Bytes of device memory the context currently holds for live buffers and
 * in its block cache (host values; no GPU work). */
krr_status krr_context_memory(krr_context ctx, int64_t *allocated, int64_t *cached);
/* HIP graphs of the batched calls: the number the context keeps instantiated
 * (one per launch shape; at most 64) and the number of graph launches so far.
 * The batched factorization's lockstep launches and the batched solve's sweeps
 * are captured on their first call with a shape and replayed afterwards
 * (KRR_NO_GRAPH=1 in the environment launches them directly). */
krr_status krr_context_graphs(krr_context ctx, int64_t *cached, int64_t *launches);

/* ---- batches of independent instances ---------------------------------
 * Many KRR problems at once, as in a cross-validation over (gamma, lambda)
 * pairs on one genotype panel (the Overview's hyperparameter search): each
 * call takes `batch` instances through the same phase.  Array arguments are
 * HOST arrays of length `batch` (the pointers they hold are device
 * pointers); outputs are written per instance and every instance behaves as
 * in the single-instance call.  On any error no handle is returned (out[]
 * all NULL) and the status is that of the first failure.
 */

/* Build of `batch` kernels sharing the SNP count m: instance b has G[b]
 * (n[b] x m, ldg[b]), gamma[b], lambda[b].  Row norms, exp tables, the INT8
 * Gram with its epilogue and the tile norms each run as ONE launch over all
 * instances (larger instances first).  KRR_ERROR_BAD_GENOTYPE if any G[b]
 * holds a value > 2.  Blocks until the build is done. */
krr_status krr_build_kernel_batched(krr_context ctx, int32_t batch, const int8_t *const *G,
                                    const int64_t *n, int64_t m, const int64_t *ldg,
                                    const double *gamma, const double *lambda, krr_kernel *out);
/* Factorization of `batch` distinct kernels under one policy (NULL =
 * ADAPTIVE defaults), in lockstep on the context stream: every POTRF step,
 * tile-inverse level, TRSM, operand conversion and trailing update is one
 * launch for all instances that have it (instances differ in tile count; the
 * schedule is the single-stream one of krr_factor, with the panel solved as
 * a product with the tile inverse).  Each instance gets its own workspace.
 * An instance that breaks down is then factored again on its own with
 * promotion, exactly as krr_factor does.  Blocks until all are done. */
krr_status krr_factor_batched(krr_context ctx, int32_t batch, const krr_kernel *K,
                              const krr_precision_policy *policy, krr_factorization *out);
/* Solve of `batch` factorizations with nrhs right-hand sides each: Y[b],
 * X[b] are n_b x nrhs FP64 column-major (ldy[b], ldx[b] >= n_b).  In
 * lockstep on the context stream: each sweep step is one launch for all
 * instances, each refinement pass one FP64 residual launch for the
 * instances not yet converged, and one host wait per pass for the whole
 * batch.  info (NULL or `batch` entries) reports
 * each instance; KRR_ERROR_NOT_CONVERGED if any instance missed the
 * tolerance (its X holds the last iterate). */
krr_status krr_solve_batched(krr_context ctx, int32_t batch, const krr_factorization *F,
                             const double *const *Y, int64_t nrhs, const int64_t *ldy,
                             double *const *X, const int64_t *ldx, const krr_refine_opts *opts,
                             krr_solve_info *info);

/* Predict (Algorithm 4) for `batch` kernels: P[b] = K_test,b X[b] with
 * K_test,b built from T[b] (n_test[b] x m_b, ldt[b]) and kernel K[b]'s G.
 * X[b]: n_b x nrhs (ldx[b]), P[b]: n_test[b] x nrhs (ldp[b]), FP64
 * column-major device arrays.  Every instance's genotype check runs first
 * (one wait; KRR_ERROR_BAD_GENOTYPE and no output if any fails), then the
 * instances' cross Grams and products in order on the context stream, in
 * one cross-distance buffer sized for the largest.  Blocks until done. */
krr_status krr_predict_batched(krr_context ctx, int32_t batch, const krr_kernel *K,
                               const int8_t *const *T, const int64_t *n_test, const int64_t *ldt,
                               const double *const *X, int64_t nrhs, const int64_t *ldx,
                               double *const *P, const int64_t *ldp);

/* ---- Ridge Regression ---------------------------------------------------
 * The RR subsection (Eq. 1-2): beta = (X^T X + lambda I)^-1 X^T Y minimises
 * ||Y - X beta||^2 + lambda ||beta||^2, X = G the n x m genotype matrix
 * (int8 {0,1,2}, row-major, ldg as for krr_build_kernel).  X^T X (m x m) is
 * the linear kernel of the SNP columns, formed by the INT8 Gram on X^T
 * (exact int32, n <= 2^22 so that its entries stay exact in FP32); X^T Y in
 * FP64; then krr_factor under `policy` and krr_solve with `refine` (FP64
 * refinement against the exact X^T X).  Y: n x nrhs, beta: m x nrhs, FP64
 * column-major device arrays.  Errors as krr_build_kernel / krr_factor /
 * krr_solve (KRR_ERROR_NOT_CONVERGED with beta written).  Blocks. */
krr_status krr_rr_fit(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                      const double *Y, int64_t nrhs, int64_t ldy, double lambda,
                      const krr_precision_policy *policy, const krr_refine_opts *refine,
                      double *beta, int64_t ldb, krr_solve_info *info);
/* Predictions of the fitted model, P = T beta (n_test x nrhs, FP64
 * column-major; T int8 n_test x m row-major, ldt >= m).  Blocks. */
krr_status krr_rr_predict(krr_context ctx, const int8_t *T, int64_t n_test, int64_t m,
                          int64_t ldt, const double *beta, int64_t nrhs, int64_t ldb, double *P,
                          int64_t ldp);

/* ---- diagnostics (tests and reports) ---------------------------------- */

/* Copy the rows x cols block at (i0, j0) of the exact int32 distance
 * matrix (either triangle; the matrix is symmetric) into dst (row-major,
 * leading dimension ld, device memory). */
krr_status krr_kernel_copy_distances(krr_kernel K, int64_t i0, int64_t j0, int64_t rows,
                                     int64_t cols, int32_t *dst, int64_t ld);
/* Same for the FP32 matrix K + lambda*I (valid until the first krr_factor
 * consumes it; KRR_ERROR_INVALID_VALUE afterwards). */
krr_status krr_kernel_copy_matrix(krr_kernel K, int64_t i0, int64_t j0, int64_t rows,
                                  int64_t cols, float *dst, int64_t ld);
/* Copy the FP32 Cholesky factor's rows x cols block at (i0, j0) (zeros
 * above the diagonal) into dst (row-major, device memory). */
krr_status krr_factor_copy_l(krr_factorization F, int64_t i0, int64_t j0, int64_t rows, int64_t cols,
                             float *dst, int64_t ld);
/* Test hook: encode n FP32 values (device) to OCP FP8 E4M3FN bytes (device)
 * with the factorization's round-to-nearest-even, saturating encoder. */
krr_status krr_debug_encode_fp8(krr_context ctx, const float *x, int64_t n, uint8_t *out);
/* Per-tile FP64 Frobenius norms of K + lambda*I, NT(NT+1)/2 values in
 * packed lower-triangle tile order, copied to HOST memory. */
krr_status krr_kernel_tile_norms(krr_kernel K, double *host_dst, int64_t count);
/* Precision chosen for each update: host array of NT * NT(NT+1)/2 bytes,
 * entry [k * NT(NT+1)/2 + I(I+1)/2 + J] for the update of tile (I, J) by
 * panel k (255 where no update happens), recorded at every NT. */
krr_status krr_factor_precision_map(krr_factorization F, uint8_t *host_dst, int64_t count);

/* ---- schedule tuning and the autotuner ---------------------------------- */

/* Schedule choices of a context (0 or -1: the library's default). */
typedef struct krr_tuning {
  int32_t tile;           /* Cholesky tile nb: 256 or 512 */
  int32_t panel_group;    /* panels per grouped trailing update, 1 .. 8 (0: 8 for FP16/FP8
                             updates, 4 for FP32) */
  int32_t residual_split; /* column ranges of the FP64 residual, 1 .. 16, each stored tile
                             read twice (0: min(8, NT)); -1: each stored tile read once, its
                             two products in slots of their own (NT np nrhs doubles of
                             workspace, used up to 1 GiB, else the default) */
  int32_t sweep_pairs;    /* 1: triangular sweeps over tile pairs, 0: one tile per step (-1: 1) */
  int32_t lookahead;      /* 1: three-stream factorization schedule, 0: one stream (-1: 1) */
  int32_t aux_cu_eighths; /* eighths of the compute units the stream of the wide trailing
                             updates may use, 1 .. 8 (0: all); the rest stay free for the
                             critical path (a CU mask over groups of eight CUs: a hardware
                             queue of its own; not searched by krr_autotune) */
} krr_tuning;

/* Set or read the context's tuning.  Changing the tile needs a context with
 * no live kernel or factor handles (KRR_ERROR_INVALID_VALUE otherwise). */
krr_status krr_set_tuning(krr_context ctx, const krr_tuning *t);
krr_status krr_get_tuning(krr_context ctx, krr_tuning *t);

/*
 * Autotuner: chooses the context's tuning for one problem shape by timing
 * whole build + factor + solve steps (HIP events on the context stream) on
 * the caller's data, searching one choice at a time: the tile (256, 512,
 * each after an untimed warm-up), then the panel group (4, 6, 8), the
 * residual form (8, 4 or 16 column ranges with each stored tile read twice,
 * or each read once) and the sweep pairing, each at the best choices so far.
 * The result is kept in the context (krr_get_tuning) and written to
 * *out and *best_ms.  With cache_path (a host path, may be NULL) the choice
 * is looked up first under the key of krr_tuning_key, and stored there after
 * a search; a cached choice is applied without running anything.  The
 * context must have no live handles (the tile may change).  Candidates that
 * fail (for instance NOT_CONVERGED) are skipped; KRR_ERROR_NOT_CONVERGED if
 * all do.  Arguments as krr_build_kernel / krr_factor / krr_solve.
 */
krr_status krr_autotune(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                        double gamma, double lambda, const double *Y, int64_t nrhs, int64_t ldy,
                        const krr_precision_policy *policy, const krr_refine_opts *refine,
                        const char *cache_path, krr_tuning *out, double *best_ms);

/* The autotuner's cache key for a problem on `device` (host only; no GPU
 * work beyond reading the device's properties): architecture, compute-unit
 * count, n, m, nrhs, the policy's mode and diagonal precision, the
 * refinement method.  Written NUL-terminated into key (cap bytes). */
krr_status krr_tuning_key(int device, int64_t n, int64_t m, int64_t nrhs,
                          const krr_precision_policy *policy, const krr_refine_opts *refine,
                          char *key, int32_t cap);
/* The cache file (host only, no GPU): a JSON object with one entry per key,
 * {"key": {"tile": .., "panel_group": .., "residual_split": .., "sweep_pairs": ..,
 * "lookahead": .., "aux_cu_eighths": .., "ms": ..}, ...}.  store adds or replaces one entry (the
 * file is rewritten whole, through a temporary file and a rename); load sets
 * *found to 0 when the file or the key is absent, KRR_ERROR_INVALID_VALUE on
 * a malformed entry for the key. */
krr_status krr_tuning_cache_store(const char *path, const char *key, const krr_tuning *t,
                                  double ms);
krr_status krr_tuning_cache_load(const char *path, const char *key, krr_tuning *t, double *ms,
                                 int32_t *found);

/* ---- per-stage timers (HIP events on the context stream) -------------- */

enum {
  KRR_STAGE_ROW_NORMS = 0, /* genotype squared norms + value check + the Gram's
                              slab-major copy of the genotypes */
  KRR_STAGE_GRAM = 1,      /* INT8 symmetric Gram + distance/exp epilogue */
  KRR_STAGE_POTRF = 2,     /* diagonal-tile Cholesky + inverse */
  KRR_STAGE_TRSM = 3,      /* panel triangular solve */
  KRR_STAGE_CONVERT = 4,   /* panel FP16/FP8 conversion */
  KRR_STAGE_UPDATE = 5,    /* trailing-matrix update */
  KRR_STAGE_FWD = 6,       /* forward substitution sweep */
  KRR_STAGE_BWD = 7,       /* back substitution sweep */
  KRR_STAGE_RESIDUAL = 8,  /* FP64 residual */
  KRR_STAGE_CROSS_GRAM = 9,/* INT8 cross Gram for predict */
  KRR_STAGE_PREDICT = 10,  /* FP64 exp + product for predict */
  KRR_STAGE_COUNT = 11
};

/* Enable (1) or disable (0) stage timing on ctx; either call clears the
 * accumulated totals.  While enabled, every stage launch is bracketed by a
 * pair of HIP events recorded on the context stream. */
krr_status krr_timers_enable(krr_context ctx, int32_t enable);
/* Time only the stages whose bit (1 << KRR_STAGE_*) is set in stage_mask (0:
 * none), clearing the totals.  Each timed stage launch records two events;
 * between dependent launches of the factorization they cost a few
 * microseconds each, so a timed run of every stage is slower than an
 * untimed one (about 2 ms per step at n = 32768). */
krr_status krr_timers_enable_stages(krr_context ctx, uint32_t stage_mask);
/* Wait for the stream, then return per-stage accumulated GPU time (ms) and
 * the number of timed intervals, for the first `count` stages (host arrays;
 * either may be NULL). */
krr_status krr_timers_read(krr_context ctx, double *total_ms, int64_t *intervals, int32_t count);
const char *krr_stage_name(int32_t stage);

const char *krr_status_string(krr_status s);

#ifdef __cplusplus
}
#endif

#endif /* KRR_H */
