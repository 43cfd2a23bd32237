"""FP64 CPU oracle for Gaussian-kernel ridge regression (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never links or calls it, and the two
share no code: the oracle is the plain definition of each step, in
``krr_oracle.c`` (FP64, no blocking, fusion or reordering) plus the Python
glue below.

Paper passages followed (arXiv 2409.01712):
  * Algorithm 1 (KRR driver): Build, then Associate, then Predict.
  * Algorithm 2 (Build) and Algorithm 5 (Gaussian kernel): K_ij = exp(-gamma ||g_i - g_j||^2).
  * Confounders ("Engaging INT8 Tensor Cores" subsection): real covariates
    whose squared distances are added to the integer genotype distances before
    the exponential of the Gaussian kernel.
  * Algorithm 5, IBS branch (the SKAT kernel described in "Current State of the
    Art"): the alleles two patients share identical by state, summed over SNPs,
    over the total number of alleles 2 m (the reading of the text; the
    algorithm's listing divides by m).
  * Subsection "Engaging INT8 Tensor Cores for Distance Calculations": the
    squared distance d_ij = sum_k (g_ik - g_jk)^2 between patient rows.
  * Algorithm 3 (Associate): factorize K + lambda I (the paper names the
    regularisation alpha), then solve for the weights W.
  * Algorithm 4 (Predict): K_test = Build(gamma, T, G), P = K_test W.
  * Ridge Regression subsection, Eq. 1-2: beta = (X^T X + lambda I)^-1 X^T Y, the
    minimiser of ||Y - X beta||^2 + lambda ||beta||^2, with X^T X and X^T Y by their
    definitions; predictions T beta.  The linear kernel K = G1 G2^T.

Every function here has a pin in tests/test_oracle.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "krr_oracle.c")
_SO = os.path.join(_HERE, "libkrr_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over independent rows)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P, I = ctypes.c_void_p, ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_sqdist.argtypes = [P, I, I, P, I, I, I, P, I]
        lib.oracle_ibs_counts.argtypes = [P, I, I, P, I, I, I, P, I]
        lib.oracle_conf_sqdist.argtypes = [P, I, I, P, I, I, I, P, I]
        lib.oracle_gaussian.argtypes = [P, I, I, I, D, P, I]
        lib.oracle_gaussian_real.argtypes = [P, I, I, I, D, P, I]
        lib.oracle_cholesky.argtypes = [P, I, I]
        lib.oracle_cholesky.restype = I
        lib.oracle_forward.argtypes = [P, I, I, P, I, I]
        lib.oracle_backward.argtypes = [P, I, I, P, I, I]
        lib.oracle_matmul.argtypes = [P, I, I, I, P, I, I, P, I]
        lib.oracle_residual_rows.argtypes = [P, I, I, I, D, D, P, I, P, I, P, I, I, P, I, I, P, I]
        lib.oracle_dot.argtypes = [P, I, I, P, I, I, I, P, I]
        lib.oracle_xtx.argtypes = [P, I, I, I, P]
        lib.oracle_xty.argtypes = [P, I, I, I, P, I, I, P, I]
        for f in ("oracle_sqdist", "oracle_ibs_counts", "oracle_conf_sqdist", "oracle_gaussian",
                  "oracle_gaussian_real", "oracle_forward", "oracle_backward",
                  "oracle_matmul", "oracle_residual_rows", "oracle_dot", "oracle_xtx",
                  "oracle_xty"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle runs with (OMP_NUM_THREADS, else all cores)."""
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)


def _rows(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def sqdist(G1: np.ndarray, G2: np.ndarray | None = None) -> np.ndarray:
    """Squared Euclidean distances between genotype rows, by definition (int64).

    d_ij = sum_k (G1[i,k] - G2[j,k])^2 -- the distance of the "Engaging INT8
    Tensor Cores" subsection, with patients as rows as in Algorithm 1.
    """
    G1 = _rows(G1, np.int8)
    G2 = G1 if G2 is None else _rows(G2, np.int8)
    assert G1.shape[1] == G2.shape[1]
    n1, m = G1.shape
    n2 = G2.shape[0]
    D = np.empty((n1, n2), np.int64)
    _load().oracle_sqdist(G1.ctypes.data, n1, m, G2.ctypes.data, n2, m, m, D.ctypes.data, n2)
    return D


def ibs_counts(G1: np.ndarray, G2: np.ndarray | None = None) -> np.ndarray:
    """Alleles shared identical by state, by definition (int64):
    s_ij = sum_k (2 - |G1[i,k] - G2[j,k]|) (Algorithm 5, IBS branch)."""
    G1 = _rows(G1, np.int8)
    G2 = G1 if G2 is None else _rows(G2, np.int8)
    assert G1.shape[1] == G2.shape[1]
    n1, m = G1.shape
    n2 = G2.shape[0]
    S = np.empty((n1, n2), np.int64)
    _load().oracle_ibs_counts(G1.ctypes.data, n1, m, G2.ctypes.data, n2, m, m, S.ctypes.data, n2)
    return S


def conf_sqdist(C1: np.ndarray, C2: np.ndarray | None = None) -> np.ndarray:
    """Squared Euclidean distances between confounder rows, by definition (FP64)."""
    C1 = _rows(C1, np.float64)
    C2 = C1 if C2 is None else _rows(C2, np.float64)
    if C1.ndim == 1:
        C1 = C1[:, None]
    if C2.ndim == 1:
        C2 = C2[:, None]
    n1, q = C1.shape
    n2 = C2.shape[0]
    Dc = np.empty((n1, n2), np.float64)
    _load().oracle_conf_sqdist(C1.ctypes.data, n1, q, C2.ctypes.data, n2, q, q, Dc.ctypes.data, n2)
    return Dc


def ibs(S: np.ndarray, m: int) -> np.ndarray:
    """IBS kernel: shared-allele counts over the total number of alleles, s / (2 m), FP64."""
    return np.asarray(S, np.int64).astype(np.float64) / float(2 * m)


def gaussian(D: np.ndarray, gamma: float) -> np.ndarray:
    """Gaussian kernel of Algorithm 5 on squared distances: exp(-gamma d), FP64."""
    D = _rows(D, np.int64)
    n1, n2 = D.shape
    K = np.empty((n1, n2), np.float64)
    _load().oracle_gaussian(D.ctypes.data, n1, n2, n2, float(gamma), K.ctypes.data, n2)
    return K


def build_kernel(G: np.ndarray, gamma: float, T: np.ndarray | None = None,
                 kind: str = "gaussian", C: np.ndarray | None = None,
                 Ct: np.ndarray | None = None) -> np.ndarray:
    """Algorithm 2 Build(gamma, G1, G2, K) with the Gaussian or the IBS kernel of
    Algorithm 5 (gamma unused by IBS).  C (n x q) / Ct (rows of T): confounders of the
    Gaussian kernel, exp(-gamma (d_genotypes + d_confounders))."""
    A = G if T is None else T
    if kind == "ibs":
        return ibs(ibs_counts(A, G), G.shape[1])
    assert kind == "gaussian", kind
    if C is None:
        return gaussian(sqdist(A, G), gamma)
    D = sqdist(A, G).astype(np.float64) + conf_sqdist(C if T is None else Ct, C)
    n1, n2 = D.shape
    K = np.empty((n1, n2), np.float64)
    _load().oracle_gaussian_real(D.ctypes.data, n1, n2, n2, float(gamma), K.ctypes.data, n2)
    return K


def cholesky(A: np.ndarray) -> np.ndarray:
    """A = L L^T (lower L), FP64; raises numpy.linalg.LinAlgError if not SPD."""
    L = np.array(A, dtype=np.float64, order="C", copy=True)
    n = L.shape[0]
    info = _load().oracle_cholesky(L.ctypes.data, n, n)
    if info:
        raise np.linalg.LinAlgError("oracle: non-positive pivot in column %d" % (info - 1))
    return L


def forward(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve L Z = B (L lower triangular)."""
    L = _rows(L, np.float64)
    Z = np.array(B, dtype=np.float64, order="C", copy=True)
    if Z.ndim == 1:
        Z = Z[:, None]
    n, r = Z.shape
    _load().oracle_forward(L.ctypes.data, n, n, Z.ctypes.data, r, r)
    return Z


def backward(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve L^T X = B (L lower triangular)."""
    L = _rows(L, np.float64)
    X = np.array(B, dtype=np.float64, order="C", copy=True)
    if X.ndim == 1:
        X = X[:, None]
    n, r = X.shape
    _load().oracle_backward(L.ctypes.data, n, n, X.ctypes.data, r, r)
    return X


def matmul(K: np.ndarray, X: np.ndarray) -> np.ndarray:
    K = _rows(K, np.float64)
    X = _rows(X, np.float64)
    if X.ndim == 1:
        X = X[:, None]
    n1, n2 = K.shape
    r = X.shape[1]
    C = np.empty((n1, r), np.float64)
    _load().oracle_matmul(K.ctypes.data, n1, n2, n2, X.ctypes.data, r, r, C.ctypes.data, r)
    return C


def associate(K: np.ndarray, Y: np.ndarray, lam: float) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 3: L = Factorize(K + lambda I), W = Solve(L, Y).  Returns (W, L)."""
    A = np.array(K, dtype=np.float64, copy=True)
    A[np.diag_indices_from(A)] += lam
    L = cholesky(A)
    W = backward(L, forward(L, Y))
    return W, L


def fit(G: np.ndarray, Y: np.ndarray, gamma: float, lam: float,
        kind: str = "gaussian", C: np.ndarray | None = None) -> np.ndarray:
    """Algorithm 1 phases 1-2: Build then Associate; returns the weights W (n x r)."""
    return associate(build_kernel(G, gamma, kind=kind, C=C), Y, lam)[0]


def predict(G: np.ndarray, T: np.ndarray, W: np.ndarray, gamma: float,
            kind: str = "gaussian", C: np.ndarray | None = None,
            Ct: np.ndarray | None = None) -> np.ndarray:
    """Algorithm 4: K_test = Build(gamma, T, G) (n_test x n), P = K_test W."""
    return matmul(build_kernel(G, gamma, T, kind=kind, C=C, Ct=Ct), W)


def residual_rows(G: np.ndarray, gamma: float, lam: float, X: np.ndarray, Y: np.ndarray,
                  rows, kind: str = "gaussian", C: np.ndarray | None = None) -> np.ndarray:
    """r = Y - (K + lambda I) X on the given rows, K recomputed from G by definition."""
    G = _rows(G, np.int8)
    X = _rows(X, np.float64)
    Y = _rows(Y, np.float64)
    if X.ndim == 1:
        X, Y = X[:, None], Y[:, None]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n, m = G.shape
    Cc, q = None, 0
    if C is not None:
        Cc = _rows(C, np.float64).reshape(n, -1)
        q = Cc.shape[1]
    r = X.shape[1]
    R = np.empty((len(rows), r), np.float64)
    _load().oracle_residual_rows(G.ctypes.data, n, m, m, float(gamma), float(lam),
                                 rows.ctypes.data, len(rows), X.ctypes.data, r,
                                 Y.ctypes.data, r, r, R.ctypes.data, r,
                                 1 if kind == "ibs" else 0,
                                 Cc.ctypes.data if Cc is not None else None, q)
    return R


def dot(G1: np.ndarray, G2: np.ndarray | None = None) -> np.ndarray:
    """Linear kernel between genotype rows, by definition: S_ij = sum_k G1[i,k] G2[j,k] (int64)."""
    G1 = _rows(G1, np.int8)
    G2 = G1 if G2 is None else _rows(G2, np.int8)
    assert G1.shape[1] == G2.shape[1]
    n1, m = G1.shape
    n2 = G2.shape[0]
    S = np.empty((n1, n2), np.int64)
    _load().oracle_dot(G1.ctypes.data, n1, m, G2.ctypes.data, n2, m, m, S.ctypes.data, n2)
    return S


def xtx(G: np.ndarray) -> np.ndarray:
    """X^T X of the genotype matrix (m x m, int64), a sum over patients (Eq. 2)."""
    G = _rows(G, np.int8)
    n, m = G.shape
    S = np.empty((m, m), np.int64)
    _load().oracle_xtx(G.ctypes.data, n, m, m, S.ctypes.data)
    return S


def xty(G: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """X^T Y (m x r, FP64), a sum over patients (Eq. 2)."""
    G = _rows(G, np.int8)
    Y = _rows(Y, np.float64)
    if Y.ndim == 1:
        Y = Y[:, None]
    n, m = G.shape
    r = Y.shape[1]
    B = np.empty((m, r), np.float64)
    _load().oracle_xty(G.ctypes.data, n, m, m, Y.ctypes.data, r, r, B.ctypes.data, r)
    return B


def rr_fit(G: np.ndarray, Y: np.ndarray, lam: float) -> np.ndarray:
    """Ridge Regression, Eq. 2: beta = (X^T X + lambda I)^-1 X^T Y through the Cholesky
    factor of X^T X + lambda I and two substitutions (m x r, FP64)."""
    A = xtx(G).astype(np.float64)
    A[np.diag_indices_from(A)] += lam
    L = cholesky(A)
    return backward(L, forward(L, xty(G, Y)))


def rr_predict(T: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Predictions of the linear model, T beta (FP64)."""
    return matmul(np.asarray(T, np.float64), beta)
