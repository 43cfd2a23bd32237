/*
 * FP64 CPU oracle for Gaussian-kernel ridge regression on integer genotypes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the GPU path.
 *
 * Each routine is the plain definition of one step of the method, written for
 * a reader to check against the paper by eye: no blocking, fusion or
 * reordering of the arithmetic.  OpenMP only splits independent output rows
 * across threads; every individual sum runs in its natural index order.
 *
 *   Build     (Algorithm 2 + Gaussian case of Algorithm 5; distance
 *              definition of the "Engaging INT8 Tensor Cores" subsection):
 *             d_ij = sum_k (g_ik - g_jk)^2 exactly in integers,
 *             K_ij = exp(-gamma * d_ij) in FP64.
 *             IBS case of Algorithm 5 (identical-by-state, the SKAT kernel
 *             of the "Current State of the Art" section): s_ij = sum_k
 *             (alleles shared at SNP k) = sum_k (2 - |g_ik - g_jk|) exactly,
 *             K_ij = s_ij / (2 m), the count over the total number of alleles.
 *             Confounders (subsection "Engaging INT8 Tensor Cores": real
 *             covariates whose squared distances are added to the integer
 *             genotype distances before the exponential): with q real
 *             covariates c_i per patient, d_ij = sum_k (g_ik - g_jk)^2 +
 *             sum_l (c_il - c_jl)^2 and K_ij = exp(-gamma * d_ij).
 *   Associate (Algorithm 3): A = K + lambda*I, A = L L^T (Cholesky),
 *             then L Z = Y and L^T W = Z (forward / back substitution).
 *   Predict   (Algorithm 4): K_test = Build(gamma, T, G), P = K_test W.
 *   Ridge Regression (RR subsection, Eq. 1-2): beta = (X^T X + lambda I)^-1 X^T Y
 *             with X the n x m genotype matrix; X^T X and X^T Y by their
 *             definitions (sums over patients), then the same Cholesky and
 *             substitutions.  The linear kernel K_ij = sum_k g_ik g_jk.
 *
 * Matrices are row-major; Y, W, P are row-major n x r here (the Python
 * wrapper converts).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Squared Euclidean distances between genotype rows, by definition.
 * D[i*ldd + j] = sum_k (G1[i,k] - G2[j,k])^2 for i < n1, j < n2. */
void oracle_sqdist(const int8_t *G1, int64_t n1, int64_t ld1, const int8_t *G2,
                   int64_t n2, int64_t ld2, int64_t m, int64_t *D, int64_t ldd) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n1; ++i) {
    const int8_t *a = G1 + i * ld1;
    for (int64_t j = 0; j < n2; ++j) {
      const int8_t *b = G2 + j * ld2;
      int64_t s = 0;
      for (int64_t k = 0; k < m; ++k) {
        const int64_t t = (int64_t)a[k] - (int64_t)b[k];
        s += t * t;
      }
      D[i * ldd + j] = s;
    }
  }
}

/* Identical-by-state allele counts (Algorithm 5, IBS branch), by definition:
 * a genotype counts minor alleles, so two patients share 2 - |g1 - g2| alleles
 * at a SNP.  S[i*ldd + j] = sum_k (2 - |G1[i,k] - G2[j,k]|). */
void oracle_ibs_counts(const int8_t *G1, int64_t n1, int64_t ld1, const int8_t *G2,
                       int64_t n2, int64_t ld2, int64_t m, int64_t *S, int64_t ldd) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n1; ++i) {
    const int8_t *a = G1 + i * ld1;
    for (int64_t j = 0; j < n2; ++j) {
      const int8_t *b = G2 + j * ld2;
      int64_t s = 0;
      for (int64_t k = 0; k < m; ++k) {
        const int64_t t = (int64_t)a[k] - (int64_t)b[k];
        s += 2 - (t < 0 ? -t : t);
      }
      S[i * ldd + j] = s;
    }
  }
}

/* Squared distances between confounder rows, by definition, FP64:
 * Dc[i*ldd + j] = sum_l (C1[i,l] - C2[j,l])^2. */
void oracle_conf_sqdist(const double *C1, int64_t n1, int64_t ld1, const double *C2,
                        int64_t n2, int64_t ld2, int64_t q, double *Dc, int64_t ldd) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n1; ++i)
    for (int64_t j = 0; j < n2; ++j) {
      double s = 0.0;
      for (int64_t l = 0; l < q; ++l) {
        const double t = C1[i * ld1 + l] - C2[j * ld2 + l];
        s += t * t;
      }
      Dc[i * ldd + j] = s;
    }
}

/* Gaussian kernel (Algorithm 5): K_ij = exp(-gamma * d_ij), FP64. */
void oracle_gaussian(const int64_t *D, int64_t n1, int64_t n2, int64_t ldd,
                     double gamma, double *K, int64_t ldk) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n1; ++i)
    for (int64_t j = 0; j < n2; ++j)
      K[i * ldk + j] = exp(-gamma * (double)D[i * ldd + j]);
}

/* The Gaussian kernel on real squared distances (genotype plus confounder
 * distances): K_ij = exp(-gamma * d_ij), FP64. */
void oracle_gaussian_real(const double *D, int64_t n1, int64_t n2, int64_t ldd,
                          double gamma, double *K, int64_t ldk) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n1; ++i)
    for (int64_t j = 0; j < n2; ++j)
      K[i * ldk + j] = exp(-gamma * D[i * ldd + j]);
}

/* Cholesky A = L L^T of a symmetric positive definite matrix, in place on the
 * lower triangle (the strict upper triangle is set to zero).  Column by
 * column: L_jj = sqrt(A_jj - sum_{p<j} L_jp^2), then for every i > j
 * L_ij = (A_ij - sum_{p<j} L_ip L_jp) / L_jj.  Returns 0 on success, or
 * j+1 if the pivot of column j is not positive. */
int64_t oracle_cholesky(double *A, int64_t n, int64_t lda) {
  for (int64_t j = 0; j < n; ++j) {
    const double *Lj = A + j * lda;
    double s = A[j * lda + j];
    for (int64_t p = 0; p < j; ++p) s -= Lj[p] * Lj[p];
    if (!(s > 0.0)) return j + 1;
    const double ljj = sqrt(s);
    A[j * lda + j] = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      const double *Li = A + i * lda;
      double t = A[i * lda + j];
      for (int64_t p = 0; p < j; ++p) t -= Li[p] * Lj[p];
      A[i * lda + j] = t / ljj;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) A[i * lda + j] = 0.0;
  return 0;
}

/* Forward substitution L Z = B for r right-hand sides (B overwritten by Z).
 * Z_i = (B_i - sum_{p<i} L_ip Z_p) / L_ii, row by row. */
void oracle_forward(const double *L, int64_t n, int64_t ldl, double *B,
                    int64_t r, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < r; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      double s = B[i * ldb + c];
      for (int64_t p = 0; p < i; ++p) s -= L[i * ldl + p] * B[p * ldb + c];
      B[i * ldb + c] = s / L[i * ldl + i];
    }
  }
}

/* Back substitution L^T X = B (B overwritten by X).
 * X_i = (B_i - sum_{p>i} L_pi X_p) / L_ii, from the last row up. */
void oracle_backward(const double *L, int64_t n, int64_t ldl, double *B,
                     int64_t r, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < r; ++c) {
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = B[i * ldb + c];
      for (int64_t p = i + 1; p < n; ++p) s -= L[p * ldl + i] * B[p * ldb + c];
      B[i * ldb + c] = s / L[i * ldl + i];
    }
  }
}

/* Dense product C (n1 x r) = K (n1 x n2) * X (n2 x r), FP64, row-major. */
void oracle_matmul(const double *K, int64_t n1, int64_t n2, int64_t ldk,
                   const double *X, int64_t r, int64_t ldx, double *C,
                   int64_t ldc) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n1; ++i)
    for (int64_t c = 0; c < r; ++c) {
      double s = 0.0;
      for (int64_t j = 0; j < n2; ++j) s += K[i * ldk + j] * X[j * ldx + c];
      C[i * ldc + c] = s;
    }
}

/* Residual of the regularised system on selected rows, with the kernel
 * recomputed from the genotypes by definition (no stored matrix):
 *   R[t, c] = Y[rows[t], c] - sum_j (K_{rows[t], j} + lambda*[rows[t] == j]) X[j, c].
 * Used where the n x n matrix does not fit in host memory. */
/* kind 0: Gaussian exp(-gamma d); kind 1: IBS s / (2 m).  C (n x q, may be
 * NULL with q = 0): confounders, their squared distance added to d (Gaussian). */
void oracle_residual_rows(const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                          double gamma, double lambda, const int64_t *rows,
                          int64_t nrows, const double *X, int64_t ldx,
                          const double *Y, int64_t ldy, int64_t r, double *R,
                          int64_t ldr, int64_t kind, const double *C, int64_t q) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nrows; ++t) {
    const int64_t i = rows[t];
    const int8_t *a = G + i * ldg;
    double *acc = (double *)calloc((size_t)r, sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
      const int8_t *b = G + j * ldg;
      int64_t s = 0;
      for (int64_t k = 0; k < m; ++k) {
        const int64_t u = (int64_t)a[k] - (int64_t)b[k];
        s += kind == 1 ? 2 - (u < 0 ? -u : u) : u * u;
      }
      double dc = 0.0;
      for (int64_t l = 0; l < q; ++l) {
        const double t = C[i * q + l] - C[j * q + l];
        dc += t * t;
      }
      double kij = kind == 1 ? (double)s / (double)(2 * m) : exp(-gamma * ((double)s + dc));
      if (j == i) kij += lambda;
      for (int64_t c = 0; c < r; ++c) acc[c] += kij * X[j * ldx + c];
    }
    for (int64_t c = 0; c < r; ++c) R[t * ldr + c] = Y[i * ldy + c] - acc[c];
    free(acc);
  }
}

/* Linear kernel (inner products of genotype rows), by definition:
 * S[i*ldd + j] = sum_k G1[i,k] * G2[j,k]. */
void oracle_dot(const int8_t *G1, int64_t n1, int64_t ld1, const int8_t *G2, int64_t n2,
                int64_t ld2, int64_t m, int64_t *S, int64_t ldd) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n1; ++i) {
    const int8_t *a = G1 + i * ld1;
    for (int64_t j = 0; j < n2; ++j) {
      const int8_t *b = G2 + j * ld2;
      int64_t s = 0;
      for (int64_t k = 0; k < m; ++k) s += (int64_t)a[k] * (int64_t)b[k];
      S[i * ldd + j] = s;
    }
  }
}

/* X^T X of the n x m genotype matrix, by definition (a sum over patients):
 * S[a*m + b] = sum_i G[i,a] * G[i,b]  (RR subsection, Eq. 2). */
void oracle_xtx(const int8_t *G, int64_t n, int64_t m, int64_t ldg, int64_t *S) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < m; ++a)
    for (int64_t b = 0; b < m; ++b) {
      int64_t s = 0;
      for (int64_t i = 0; i < n; ++i) s += (int64_t)G[i * ldg + a] * (int64_t)G[i * ldg + b];
      S[a * m + b] = s;
    }
}

/* X^T Y, by definition: B[a*ldb + c] = sum_i G[i,a] * Y[i*ldy + c]  (Eq. 2). */
void oracle_xty(const int8_t *G, int64_t n, int64_t m, int64_t ldg, const double *Y, int64_t r,
                int64_t ldy, double *B, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a)
    for (int64_t c = 0; c < r; ++c) {
      double s = 0.0;
      for (int64_t i = 0; i < n; ++i) s += (double)G[i * ldg + a] * Y[i * ldy + c];
      B[a * ldb + c] = s;
    }
}
