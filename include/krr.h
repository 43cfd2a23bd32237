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

/* Context options. */
typedef struct krr_options {
  int32_t tile;             /* Cholesky tile size nb: 256 or 512 (0 = 512) */
  int32_t verbose;          /* 0 = silent; 1 = per-call summary on stderr */
  int64_t workspace_limit;  /* max bytes the library may allocate (0 = no cap) */
} krr_options;

/* Operand precisions of a trailing-matrix update. */
enum { KRR_PREC_FP32 = 0, KRR_PREC_FP16 = 1, KRR_PREC_FP8 = 2 };

/* Factorization precision policies. */
enum {
  KRR_POLICY_FP32 = 0,     /* every update in FP32 (the plain single-precision path) */
  KRR_POLICY_ADAPTIVE = 1, /* per-update precision from operand tile norms */
  KRR_POLICY_FIXED = 2     /* every off-diagonal update of panels >= high_panels in fixed_prec */
};

/*
 * Precision policy for krr_factor ("Deploying a Four-Precision
 * Cholesky-Based Solver"; the rule below is this library's reading of the
 * tile-centric adaptive precision the paper cites).
 *
 * ADAPTIVE: the update A_IJ -= L_IK L_JK^T (I > J > K) uses the lowest
 * allowed precision p with  u_p * ||L_IK||_F * ||L_JK||_F <= eps * ||A||_F / NT,
 * u_FP8 = 2^-4, u_FP16 = 2^-11; otherwise FP32.  Updates of diagonal tiles
 * and of panels K < high_panels are always FP32.  Low-precision operands
 * carry a per-tile power-of-two scale; accumulation is FP32.
 */
typedef struct krr_precision_policy {
  int32_t mode;            /* KRR_POLICY_* */
  int32_t allowed;         /* bit mask of (1 << KRR_PREC_FP16) | (1 << KRR_PREC_FP8) */
  double eps;              /* ADAPTIVE threshold (default 1.0) */
  int32_t high_panels;     /* panels K < high_panels update in FP32 (default 1) */
  int32_t fixed_prec;      /* FIXED mode: KRR_PREC_FP16 or KRR_PREC_FP8 */
  int32_t allow_promotion; /* on breakdown, drop the lowest precision and refactor */
  int32_t diag_fp64;       /* 1: diagonal-tile POTRF in FP64; 0: in FP32 */
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

/*
 * Predict without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as krr_predict (the same
 * kernels, so P is bit-identical), but the working buffers (genotype-check
 * flag, test-row norms, the row-major copy of X, the cross distances of a
 * chunk of test rows) live in a fixed device scratch of
 * KRR_NOALLOC_SCRATCH_BYTES that each device holds from krr_create until the
 * process ends.  Calls no hipMalloc/hipFree and no allocating library routine.
 * Limit: 256 + 4*n_test + 8*np*nrhs + 4*64*np bytes (rounded up to 256 each;
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

/* ---- per-stage timers (HIP events on the context stream) -------------- */

enum {
  KRR_STAGE_ROW_NORMS = 0, /* genotype squared norms + value check */
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
