"""Pins for the FP64 CPU oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's own formula: each compares it with an
independent fact -- a hand-worked instance of the paper's distance example,
brute force on tiny inputs, the Gram identity the paper's INT8 trick rests on,
closed forms for A = b I + c 11^T, LAPACK through numpy, dense inverses, and
invariants of the regularised system.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def _tiny_genotypes(n, m, seed):
    return np.random.default_rng(seed).integers(0, 3, size=(n, m)).astype(np.int8)


# --- distances (Algorithm 5 / "Engaging INT8 Tensor Cores" subsection) ---------------

def test_three_patient_example(golden_dir):
    """The paper's 3-patient, 2-marker example: D~ = D + D^T - 2 G^T G."""
    spec = json.load(open(os.path.join(golden_dir, "three_patients.json")))
    for case in spec["cases"]:
        pts = case["patients"]
        G = np.array([pts["a"], pts["b"], pts["c"]], np.int8)  # patients as rows
        D = oracle.sqdist(G)
        assert D.tolist() == case["D_tilde"]
        assert (G.astype(np.int64) ** 2).sum(1).tolist() == case["norms"]


def test_sqdist_brute_force():
    G = _tiny_genotypes(6, 9, 1)
    T = _tiny_genotypes(4, 9, 2)
    D = oracle.sqdist(T, G)
    for i in range(4):
        for j in range(6):
            want = sum((int(T[i, k]) - int(G[j, k])) ** 2 for k in range(9))
            assert D[i, j] == want


def test_sqdist_gram_identity():
    """d_ij = n_i + n_j - 2 g_i . g_j (the identity behind the INT8 GEMM)."""
    G = _tiny_genotypes(37, 501, 3).astype(np.int64)
    nrm = (G * G).sum(1)
    want = nrm[:, None] + nrm[None, :] - 2 * (G @ G.T)
    assert np.array_equal(oracle.sqdist(G.astype(np.int8)), want)


def test_sqdist_special_cases():
    # identical rows are at distance 0
    G = _tiny_genotypes(5, 40, 4)
    G2 = np.vstack([G, G])
    D = oracle.sqdist(G2)
    assert all(D[i, i + 5] == 0 for i in range(5))
    # rows 2 * e_i (one-hot, M >= N): every off-diagonal distance is 2^2 + 2^2 = 8
    n, m = 7, 11
    H = np.zeros((n, m), np.int8)
    H[np.arange(n), np.arange(n)] = 2
    D = oracle.sqdist(H)
    assert np.array_equal(D, 8 * (1 - np.eye(n, dtype=np.int64)))
    # extreme values: all-2 row vs all-0 row over m SNPs -> 4 m
    E = np.array([[2] * 300, [0] * 300], np.int8)
    assert oracle.sqdist(E)[0, 1] == 1200


def test_sqdist_metric_properties():
    G = _tiny_genotypes(20, 64, 5)
    D = oracle.sqdist(G).astype(np.float64)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0) and np.all(D >= 0)
    R = np.sqrt(D)  # Euclidean distance obeys the triangle inequality
    for i in range(20):
        for j in range(20):
            assert np.all(R[i, j] <= R[i, :] + R[:, j] + 1e-12)


# --- kernel matrix -------------------------------------------------------------------

def test_gaussian_matches_library_exp():
    D = oracle.sqdist(_tiny_genotypes(30, 80, 6))
    g = 1.0 / 80
    K = oracle.gaussian(D, g)
    # libm exp vs numpy's vectorised exp: both faithfully rounded, so within 1 ulp
    assert np.max(np.abs(K / np.exp(-g * D.astype(np.float64)) - 1)) <= 2.3e-16
    assert np.allclose(np.diag(K), 1.0) and np.all(K > 0) and np.all(K <= 1.0)
    assert np.array_equal(K, K.T)


def _golden_gaussian_cases(golden_dir):
    spec = json.load(open(os.path.join(golden_dir, "gaussian_values.json")))
    for case in spec["cases"]:
        pts = case["patients"]
        G = np.array([pts["a"], pts["b"], pts["c"]], np.int8)
        g = np.log(2.0) if case["gamma"] == "ln2" else float(case["gamma"])
        want = np.array([[float(v) for v in row] for row in case["K"]])
        yield G, g, want


def _golden_ok(gauss, golden_dir):
    """Every hand-worked entry within 4 FP64 ulps (gamma = ln 2 carries one rounding)."""
    for G, g, want in _golden_gaussian_cases(golden_dir):
        K = gauss(oracle.sqdist(G), g)
        if not np.all(np.abs(K - want) <= 4 * np.spacing(want)):
            return False
    return True


def test_gaussian_golden_values(golden_dir):
    """Algorithm 5's Gaussian on the paper's three-patient example, against values worked
    out by hand: 2^-d at gamma = ln 2 and e^-(d/4) at gamma = 1/4."""
    assert _golden_ok(oracle.gaussian, golden_dir)
    for G, g, want in _golden_gaussian_cases(golden_dir):
        assert np.all(np.abs(oracle.build_kernel(G, g) - want) <= 4 * np.spacing(want))


def test_gaussian_planted_mistakes_are_caught(golden_dir):
    """Plausible slips in the kernel formula -- gamma halved, the distance square-rooted,
    the minus sign dropped, gamma doubled -- each fail the hand-worked values."""
    mutants = {
        "half_gamma": lambda D, g: oracle.gaussian(D, g / 2),
        "double_gamma": lambda D, g: oracle.gaussian(D, 2 * g),
        "sqrt_distance": lambda D, g: np.exp(-g * np.sqrt(D.astype(np.float64))),
        "no_minus": lambda D, g: np.exp(g * D.astype(np.float64)),
    }
    for name, f in mutants.items():
        assert not _golden_ok(f, golden_dir), name


# --- confounders ("Engaging INT8 Tensor Cores" subsection) ----------------------------

def _golden_conf(golden_dir):
    spec = json.load(open(os.path.join(golden_dir, "confounder_values.json")))
    G = np.array([spec["patients"][k] for k in "abc"], np.int8)
    C = np.array([spec["confounders"][k] for k in "abc"], np.float64)
    want = np.array([[float(v) for v in row] for row in spec["K_ln2"]])
    return spec, G, C, want


def test_confounder_golden_values(golden_dir):
    spec, G, C, want = _golden_conf(golden_dir)
    assert oracle.conf_sqdist(C).tolist() == spec["conf_sqdist"]
    K = oracle.build_kernel(G, np.log(2.0), C=C)
    assert np.all(np.abs(K - want) <= 4 * np.spacing(want))


def test_confounder_planted_mistakes_are_caught(golden_dir):
    """Leaving the confounder term out, or adding its distance unsquared, fails the
    hand-worked values."""
    spec, G, C, want = _golden_conf(golden_dir)
    g = np.log(2.0)
    without = oracle.build_kernel(G, g)
    unsquared = np.exp(-g * (oracle.sqdist(G) + np.sqrt(oracle.conf_sqdist(C))))
    for bad in (without, unsquared):
        assert not np.all(np.abs(bad - want) <= 4 * np.spacing(want))


def test_confounder_distances_brute_force_and_syrk_form():
    """By definition against a Python loop, and the SYRK form the GPU uses,
    ||c_i||^2 + ||c_j||^2 - 2 c_i . c_j, through numpy's product."""
    rng = np.random.default_rng(31)
    C1, C2 = rng.standard_normal((6, 5)), rng.standard_normal((4, 5))
    Dc = oracle.conf_sqdist(C2, C1)
    for i in range(4):
        for j in range(6):
            assert abs(Dc[i, j] - sum((C2[i, l] - C1[j, l]) ** 2 for l in range(5))) <= 1e-13
    C = rng.standard_normal((50, 12))
    nrm = (C * C).sum(1)
    syrk = nrm[:, None] + nrm[None, :] - 2 * (C @ C.T)
    assert np.max(np.abs(oracle.conf_sqdist(C) - syrk)) <= 1e-12 * np.max(syrk)


def test_confounder_kernel_reductions():
    """Zero confounders reduce to the genotype kernel; identical genotypes leave only the
    confounder kernel; the full kernel stays PSD; the fit with confounders matches a
    dense inverse and its residual rows vanish."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=200)
    Y = w.phenotypes(G)
    C = np.random.default_rng(32).standard_normal((200, 3)) * 10.0
    assert np.array_equal(oracle.build_kernel(G, w.gamma, C=np.zeros((200, 3))),
                          oracle.build_kernel(G, w.gamma))
    Gsame = np.repeat(G[:1], 200, axis=0)
    Kc = oracle.build_kernel(Gsame, 0.01, C=C)
    assert np.max(np.abs(Kc - np.exp(-0.01 * oracle.conf_sqdist(C)))) <= 1e-15
    K = oracle.build_kernel(G, w.gamma, C=C)
    assert np.linalg.eigvalsh(K).min() > -1e-12
    W = oracle.fit(G, Y, w.gamma, w.lam, C=C)
    want = np.linalg.inv(K + w.lam * np.eye(200)) @ Y
    assert np.max(np.abs(W - want)) <= 1e-10 * np.max(np.abs(want))
    R = oracle.residual_rows(G, w.gamma, w.lam, W, Y, [0, 77, 199], C=C)
    assert np.max(np.abs(R)) <= 1e-9


# --- IBS kernel (Algorithm 5, IBS branch) ------------------------------------------------

def _shared_alleles_brute(a, b):
    """Alleles shared identical by state at one SNP, from the allele multisets: genotype g
    carries g minor and 2 - g major alleles; the shared count is the multiset overlap."""
    return min(a, b) + min(2 - a, 2 - b)


def test_ibs_golden_values(golden_dir):
    spec = json.load(open(os.path.join(golden_dir, "ibs_values.json")))
    for case in spec["cases"]:
        pts = case["patients"]
        G = np.array([pts["a"], pts["b"], pts["c"]], np.int8)
        assert oracle.ibs_counts(G).tolist() == case["shared"]
        want = np.array([[float(v) for v in row] for row in case["K"]])
        assert np.array_equal(oracle.build_kernel(G, 0.0, kind="ibs"), want)


def test_ibs_planted_mistakes_are_caught(golden_dir):
    """Dividing by m (the listing's literal N_S) or counting squared differences
    instead of absolute ones fails the hand-worked values."""
    spec = json.load(open(os.path.join(golden_dir, "ibs_values.json")))
    G = np.array([spec["cases"][0]["patients"][k] for k in "abc"], np.int8)
    want = np.array([[float(v) for v in row] for row in spec["cases"][0]["K"]])
    m = G.shape[1]
    by_m = oracle.ibs_counts(G) / m
    sq = (2 * m - oracle.sqdist(G)) / (2 * m)
    assert not np.array_equal(by_m, want) and not np.array_equal(sq, want)


def test_ibs_brute_force_and_identity():
    """Counts against the allele-multiset overlap on tiny inputs, and the identity behind
    the GPU's INT8 form: s = 2m - d + 2 (C02 + C20), C02 counting SNPs with g_i = 0 and
    g_j = 2 (one-hot products)."""
    G = _tiny_genotypes(7, 11, 21)
    T = _tiny_genotypes(5, 11, 22)
    S = oracle.ibs_counts(T, G)
    for i in range(5):
        for j in range(7):
            assert S[i, j] == sum(_shared_alleles_brute(int(T[i, k]), int(G[j, k]))
                                  for k in range(11))
    G = _tiny_genotypes(40, 300, 23).astype(np.int64)
    z, t = (G == 0).astype(np.int64), (G == 2).astype(np.int64)
    want = 2 * 300 - oracle.sqdist(G.astype(np.int8)) + 2 * (z @ t.T + t @ z.T)
    assert np.array_equal(oracle.ibs_counts(G.astype(np.int8)), want)


def test_ibs_kernel_properties():
    """Unit diagonal, symmetric, entries in [0, 1], positive semi-definite (a sum over
    SNPs of inner products of allele indicators)."""
    G = synth.WORKLOADS["small"].genotypes(rows=300)
    K = oracle.build_kernel(G, 0.0, kind="ibs")
    assert np.all(np.diag(K) == 1.0) and np.array_equal(K, K.T)
    assert K.min() >= 0.0 and K.max() <= 1.0
    assert np.linalg.eigvalsh(K).min() > -1e-10


def test_ibs_fit_dense_inverse_and_residual():
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=200)
    Y = w.phenotypes(G)
    W = oracle.fit(G, Y, 0.0, w.lam, kind="ibs")
    A = oracle.build_kernel(G, 0.0, kind="ibs") + w.lam * np.eye(200)
    want = np.linalg.inv(A) @ Y
    assert np.max(np.abs(W - want)) <= 1e-10 * np.max(np.abs(want))
    R = oracle.residual_rows(G, 0.0, w.lam, W, Y, [0, 5, 199], kind="ibs")
    assert np.max(np.abs(R)) <= 1e-9


def test_kernel_is_psd():
    """The Gaussian kernel matrix is positive semi-definite (so lambda_min(K + lambda I) >= lambda)."""
    G = synth.WORKLOADS["small"].genotypes(rows=300)
    K = oracle.build_kernel(G, 1.0 / G.shape[1])
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-12


# --- Cholesky and solves (Algorithm 3) ----------------------------------------------------

def _bc_matrix(n, b, c):
    return b * np.eye(n) + c * np.ones((n, n))


def test_cholesky_closed_form():
    """A = b I + c 11^T: with s_j = b + j c,
    L_jj = sqrt(b s_{j+1} / s_j) and L_ij = c sqrt(b) / sqrt(s_j s_{j+1}) for i > j."""
    n, b, c = 300, 0.6, 0.45
    L = oracle.cholesky(_bc_matrix(n, b, c))
    s = b + c * np.arange(n + 1)
    for j in range(n):
        assert abs(L[j, j] - np.sqrt(b * s[j + 1] / s[j])) <= 1e-14 * L[j, j]
        col = c * np.sqrt(b) / np.sqrt(s[j] * s[j + 1])
        if j + 1 < n:
            assert np.max(np.abs(L[j + 1:, j] - col)) <= 1e-14 * abs(col)
    assert np.all(np.triu(L, 1) == 0)


def test_cholesky_vs_lapack_and_backward_error():
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=512)
    A = oracle.build_kernel(G, w.gamma)
    A[np.diag_indices_from(A)] += w.lam
    L = oracle.cholesky(A)
    assert np.linalg.norm(A - L @ L.T) / np.linalg.norm(A) <= 1e-13
    assert np.max(np.abs(L - np.linalg.cholesky(A))) <= 1e-12


def test_cholesky_detects_indefinite():
    A = _bc_matrix(10, 1.0, 0.5)
    A[4, 4] = -1.0
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky(A)
    # lambda = 0 with duplicated genotype rows: K is singular -> breakdown (or no positive pivot)
    G = _tiny_genotypes(8, 16, 7)
    K = oracle.build_kernel(np.vstack([G, G]), 1.0 / 16)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky(K - 1e-9 * np.eye(16))


def test_triangular_solves():
    rng = np.random.default_rng(8)
    n, r = 120, 5
    A = _bc_matrix(n, 0.7, 0.3) + 0.01 * np.diag(rng.random(n))
    L = oracle.cholesky(A)
    B = rng.standard_normal((n, r))
    Z = oracle.forward(L, B)
    assert np.allclose(L @ Z, B, rtol=0, atol=1e-12)
    X = oracle.backward(L, Z)
    assert np.allclose(L.T @ X, Z, rtol=0, atol=1e-12)


def test_sherman_morrison():
    """(b I + c 11^T) x = y has x = (y - c (1^T y) / (b + n c) 1) / b."""
    n, b, c = 257, 0.55, 0.48
    y = np.random.default_rng(9).standard_normal((n, 3))
    W, _ = oracle.associate(c * np.ones((n, n)), y, b)  # K = c 11^T, lambda = b
    want = (y - c * y.sum(0) / (b + n * c)) / b
    assert np.max(np.abs(W - want)) <= 1e-13 * np.max(np.abs(want))


def test_dense_inverse_small():
    """At N <= 256 the weights equal inv(K + lambda I) Y (numpy's LAPACK inverse)."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=200)
    Y = w.phenotypes(G)
    W = oracle.fit(G, Y, w.gamma, w.lam)
    A = oracle.build_kernel(G, w.gamma) + w.lam * np.eye(200)
    want = np.linalg.inv(A) @ Y
    assert np.max(np.abs(W - want)) <= 1e-10 * np.max(np.abs(want))


def test_large_gamma_limit():
    """Distinct rows and huge gamma: K -> I, so W = Y / (1 + lambda)."""
    G = _tiny_genotypes(50, 64, 10)
    assert len({g.tobytes() for g in G}) == 50
    Y = np.random.default_rng(11).standard_normal((50, 2))
    W = oracle.fit(G, Y, 50.0, 0.3)
    assert np.allclose(W, Y / 1.3, rtol=1e-14, atol=0)


# --- Predict (Algorithm 4) and residual ---------------------------------------------------

def test_predict_on_training_set():
    """Predicting the training patients gives K W = Y - lambda W."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=256)
    Y = w.phenotypes(G)
    W = oracle.fit(G, Y, w.gamma, w.lam)
    P = oracle.predict(G, G, W, w.gamma)
    assert np.max(np.abs(P - (Y - w.lam * W))) <= 1e-9 * np.max(np.abs(Y))


def test_predict_brute_force():
    G = _tiny_genotypes(9, 13, 12)
    T = _tiny_genotypes(4, 13, 13)
    W = np.random.default_rng(14).standard_normal((9, 2))
    g = 0.07
    P = oracle.predict(G, T, W, g)
    for i in range(4):
        for c in range(2):
            s = 0.0
            for j in range(9):
                d = sum((int(T[i, k]) - int(G[j, k])) ** 2 for k in range(13))
                s += np.exp(-g * d) * W[j, c]
            assert abs(P[i, c] - s) <= 1e-13 * (1 + abs(s))


def test_residual_rows():
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=300)
    Y = w.phenotypes(G)
    W = oracle.fit(G, Y, w.gamma, w.lam)
    rows = [0, 17, 299]
    R = oracle.residual_rows(G, w.gamma, w.lam, W, Y, rows)
    assert np.max(np.abs(R)) <= 1e-10
    R0 = oracle.residual_rows(G, w.gamma, w.lam, np.zeros_like(W), Y, rows)
    assert np.array_equal(R0, Y[rows])


def test_planted_mistake_is_caught():
    """A Cholesky with a dropped term (no subtraction for the first column) fails the pins."""
    n, b, c = 40, 0.6, 0.45
    A = _bc_matrix(n, b, c)
    good = oracle.cholesky(A)
    bad = good.copy()
    bad[1:, 1] += good[1:, 0] * good[1, 0] / good[1, 1]  # what skipping p=0 would leave
    s = b + c * np.arange(n + 1)
    col = c * np.sqrt(b) / np.sqrt(s[1] * s[2])
    assert np.max(np.abs(good[2:, 1] - col)) <= 1e-14
    assert np.max(np.abs(bad[2:, 1] - col)) > 1e-3


# --- input generator ----------------------------------------------------------------

def test_philox_known_answers():
    """Philox4x32-10 known-answer vectors from Salmon et al. (SC'11)."""
    assert synth.philox4x32_10([0, 0, 0, 0], [0, 0]).tolist() == \
        [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert synth.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2).tolist() == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert synth.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                               [0xa4093822, 0x299f31d0]).tolist() == \
        [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_generator_row_addressable_and_binomial():
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=64)
    G2 = w.genotypes(rows=16, row0=40)
    assert np.array_equal(G[40:56], G2)
    assert set(np.unique(G).tolist()) <= {0, 1, 2}
    Gb = w.genotypes(rows=2048)
    p = w.maf_vector()
    assert abs(Gb.mean() - 2 * p.mean()) < 0.01


def test_ld_blocks():
    w = synth.WORKLOADS["large"]
    spec = w.ld_spec()
    founders, length, prob = spec
    G = synth.genotypes(400, w.m, w.maf_vector(), w.seed, ld_blocks=spec)
    f = founders[0]
    same = (G[:, f + 1:f + length] == G[:, f:f + 1]).mean()
    assert 0.85 < same < 0.99  # ~10% resampled, some of those equal by chance


# --- Ridge Regression (RR subsection, Eq. 1-2) -----------------------------------------

def _rr_golden(golden_dir):
    spec = json.load(open(os.path.join(golden_dir, "ridge_regression.json")))
    X = np.array(spec["X"], np.int8)
    Y = np.array(spec["Y"], np.float64)[:, None]
    return spec, X, Y


def test_rr_golden_values(golden_dir):
    spec, X, Y = _rr_golden(golden_dir)
    assert oracle.xtx(X).tolist() == spec["XtX"]
    assert oracle.xty(X, Y)[:, 0].tolist() == spec["XtY"]
    beta = oracle.rr_fit(X, Y, spec["lambda"])[:, 0]
    want = np.array([float(v) for v in spec["beta"]])
    assert np.all(np.abs(beta - want) <= 4 * np.spacing(np.abs(want)))
    P = oracle.rr_predict(np.array(spec["T"], np.int8), beta[:, None])[:, 0]
    assert abs(P[0] - float(spec["P"][0])) <= 4 * np.spacing(0.625)


def test_rr_planted_mistakes_are_caught(golden_dir):
    """The regulariser subtracted instead of added, X X^T in place of X^T X, and a
    transposed X^T Y each fail the hand-worked solution or its dimensions."""
    spec, X, Y = _rr_golden(golden_dir)
    want = np.array([float(v) for v in spec["beta"]])[:, None]
    lam = spec["lambda"]
    A = oracle.xtx(X).astype(np.float64)
    minus = np.linalg.solve(A - lam * np.eye(2), oracle.xty(X, Y))
    assert not np.allclose(minus, want, rtol=1e-12, atol=0)
    wrong_gram = oracle.dot(X).astype(np.float64) + lam * np.eye(3)  # n x n, not m x m
    assert wrong_gram.shape != A.shape
    swapped = np.linalg.solve(A + lam * np.eye(2), oracle.xty(X[:, ::-1], Y))
    assert not np.allclose(swapped, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,m", [(60, 40), (30, 80)])
def test_rr_is_the_penalised_least_squares_minimiser(n, m):
    """Eq. 2's beta minimises Eq. 1: it equals the least-squares solution of the
    augmented system [X; sqrt(lambda) I] beta = [Y; 0] (LAPACK's SVD-based lstsq), and
    it satisfies the stationarity condition X^T (Y - X beta) = lambda beta -- with more
    patients than SNPs and with fewer (N_P << N_S, where the regulariser is needed)."""
    rng = np.random.default_rng(n * m)
    G = synth.genotypes(n, m, synth.maf_uniform(m, 0.05, 0.5, 7), 7)
    Y = rng.standard_normal((n, 3))
    lam = 0.7
    beta = oracle.rr_fit(G, Y, lam)
    X = G.astype(np.float64)
    aug = np.vstack([X, np.sqrt(lam) * np.eye(m)])
    ref = np.linalg.lstsq(aug, np.vstack([Y, np.zeros((m, 3))]), rcond=None)[0]
    assert np.max(np.abs(beta - ref)) <= 1e-10 * np.max(np.abs(ref))
    grad = X.T @ (Y - X @ beta) - lam * beta
    assert np.max(np.abs(grad)) <= 1e-9 * np.max(np.abs(X.T @ Y))


def test_rr_products_by_definition():
    """X^T X and X^T Y against brute force over patients; the linear kernel is the
    inner product of rows, and X^T X is the linear kernel of the SNP columns."""
    G = synth.genotypes(37, 23, synth.maf_uniform(23, 0.05, 0.5, 3), 3)
    Y = np.random.default_rng(1).standard_normal((37, 2))
    S = oracle.xtx(G)
    for a in range(23):
        for b in range(23):
            assert S[a, b] == sum(int(G[i, a]) * int(G[i, b]) for i in range(37))
    B = oracle.xty(G, Y)
    for a in (0, 11, 22):
        assert abs(B[a, 1] - sum(float(G[i, a]) * Y[i, 1] for i in range(37))) <= 1e-12
    assert np.array_equal(oracle.dot(np.ascontiguousarray(G.T)), S)
    assert np.array_equal(oracle.dot(G), G.astype(np.int64) @ G.T.astype(np.int64))
