"""GPU parity of the kernel types of Algorithm 5 beyond the plain Gaussian: the
IBS kernel (identical-by-state allele sharing) and the Gaussian kernel with
confounders (real covariates whose squared distances join the genotype
distances before the exponential), through krr_build_kernel_ex / krr_predict_ex,
against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2409_01712_amd as krr  # noqa: E402

DEV = "cuda:0"
TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _gen(n, m, seed):
    return synth.genotypes(n, m, synth.maf_uniform(m, 0.05, 0.5, seed), seed)


def _colrel(A, B):
    A = np.asarray(A).reshape(len(A), -1)
    B = np.asarray(B).reshape(len(B), -1)
    return max(np.max(np.abs(A[:, c] - B[:, c])) / np.max(np.abs(B[:, c])) for c in range(B.shape[1]))


def _ulps(A, want64):
    want = want64.astype(np.float32)
    return np.abs(A.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))


# --- IBS ------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,m", [(1, 1), (2, 17), (300, 63), (513, 1000), (700, 4096)])
def test_ibs_distances_bit_exact(n, m):
    """d = sum_k |g_ik - g_jk| of the encoded rows equals 2m minus the oracle's
    shared-allele count, bit for bit (ragged n and m, m not a multiple of 16)."""
    G = _gen(n, m, seed=n + 3 * m)
    ctx = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel_ex(ctx, _dev(G), 1.0, 0.1, kind=krr.KRR_KERNEL_IBS)
    D = krr.krr_kernel_copy_distances(K, 0, 0, n, n).cpu().numpy().astype(np.int64)
    assert np.array_equal(2 * m - D, oracle.ibs_counts(G))
    ctx.close()


def test_ibs_matrix_and_solve_and_predict():
    n, nt_, m, r = 1500, 200, 3000, 3
    Gall = _gen(n + nt_, m, seed=11)
    G, T = Gall[:n], Gall[n:]
    Y = synth.phenotypes(G, r, n_pairs=10, n_add=5, seed=12, h2=0.5)
    lam = 0.1
    ctx = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel_ex(ctx, _dev(G), 1.0, lam, kind=krr.KRR_KERNEL_IBS)
    A = krr.krr_kernel_copy_matrix(K, 0, 0, n, n).cpu().numpy()
    Ko = oracle.build_kernel(G, 1.0, kind="ibs")
    Ko[np.diag_indices_from(Ko)] += lam
    assert _ulps(A, Ko).max() <= 1
    Wo = oracle.fit(G, Y, 1.0, lam, kind="ibs")
    F = krr.krr_factor(ctx, K)
    X, info, _ = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), Wo) <= TOL
    # the certificate: the oracle's FP64 residual of the returned X
    Xh = X.cpu().numpy()
    R = oracle.residual_rows(G, 1.0, lam, Xh, Y, np.arange(0, n, 7), kind="ibs")
    assert np.all(np.linalg.norm(R, axis=0) <= lam * 1e-8 * np.linalg.norm(Xh, axis=0) * 1.01)
    # predict with the oracle's weights isolates the step
    P = krr.krr_predict_ex(ctx, K, _dev(T), _dev(Wo)).cpu().numpy()
    assert _colrel(P, oracle.predict(G, T, Wo, 1.0, kind="ibs")) <= 1e-12
    # a second factorization re-expands the IBS values from the stored distances
    X2, _, _ = krr.krr_solve(ctx, krr.krr_factor(ctx, K), _dev(Y), krr.Refine(tol=1e-8))
    assert torch.equal(X, X2)
    ctx.close()


# --- confounders -----------------------------------------------------------------------------

def _conf_case(n, nt_, m, q, seed):
    Gall = _gen(n + nt_, m, seed=seed)
    gamma = 1.0 / m
    # covariates whose squared distances are ~0.2 / gamma on average
    Call = synth.confounders(n + nt_, q, seed=seed, sd=np.sqrt(0.1 / (gamma * q)))
    return Gall[:n], Gall[n:], Call[:n], Call[n:], gamma


def test_confounder_matrix_and_solve():
    n, m, q, r = 1400, 2000, 6, 4
    G, _, C, _, gamma = _conf_case(n, 0, m, q, seed=21)
    Y = synth.phenotypes(G, r, n_pairs=10, n_add=5, seed=22, h2=0.5)
    lam = 0.05
    ctx = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel_ex(ctx, _dev(G), gamma, lam, C=_dev(C))
    A = krr.krr_kernel_copy_matrix(K, 0, 0, n, n).cpu().numpy()
    Ko = oracle.build_kernel(G, gamma, C=C)
    Ko[np.diag_indices_from(Ko)] += lam
    assert _ulps(A, Ko).max() <= 1
    # the confounders matter: the matrix differs from the genotype-only one
    assert np.max(np.abs(Ko - oracle.build_kernel(G, gamma))) > 0.05
    Wo = oracle.fit(G, Y, gamma, lam, C=C)
    for pol in (krr.Policy(), krr.plain_fp32_policy()):
        F = krr.krr_factor(ctx, K, pol)
        X, info, _ = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(tol=1e-8))
        assert info.converged == 1
        assert _colrel(X.cpu().numpy(), Wo) <= TOL
    Xh = X.cpu().numpy()
    R = oracle.residual_rows(G, gamma, lam, Xh, Y, np.arange(0, n, 5), C=C)
    assert np.all(np.linalg.norm(R, axis=0) <= lam * 1e-8 * np.linalg.norm(Xh, axis=0) * 1.01)
    ctx.close()


def test_confounder_predict_and_unsupported_paths():
    n, nt_, m, q = 1000, 150, 1500, 3
    G, T, C, Ct, gamma = _conf_case(n, nt_, m, q, seed=31)
    ctx = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel_ex(ctx, _dev(G), gamma, 0.1, C=_dev(C))
    W = np.random.default_rng(3).standard_normal((n, 2))
    P = krr.krr_predict_ex(ctx, K, _dev(T), _dev(W), Ct=_dev(Ct)).cpu().numpy()
    assert _colrel(P, oracle.predict(G, T, W, gamma, C=C, Ct=Ct)) <= 1e-12
    # plain krr_predict cannot serve a kernel with confounders; neither can the
    # batched solve and predict, nor the no-allocation Predict
    with pytest.raises(krr.KRRError) as e:
        krr.krr_predict(ctx, K, _dev(T), _dev(W))
    assert e.value.status == krr.KRR_ERROR_INVALID_VALUE
    with pytest.raises(krr.KRRError) as e:
        krr.krr_predict_noalloc(ctx, K, _dev(T), _dev(W))
    assert e.value.status == krr.KRR_ERROR_NOT_SUPPORTED
    F = krr.krr_factor(ctx, K)
    Y = np.random.default_rng(4).standard_normal((n, 1))
    with pytest.raises(krr.KRRError) as e:
        krr.krr_solve_batched(ctx, [F], [_dev(Y)])
    assert e.value.status == krr.KRR_ERROR_NOT_SUPPORTED
    # bad descriptions are rejected before any work
    with pytest.raises(krr.KRRError) as e:
        krr.krr_build_kernel_ex(ctx, _dev(G), gamma, 0.1, kind=krr.KRR_KERNEL_IBS, C=_dev(C))
    assert e.value.status == krr.KRR_ERROR_INVALID_VALUE
    with pytest.raises(krr.KRRError) as e:
        krr.krr_build_kernel_ex(ctx, _dev(G), gamma, 0.1, kind=7)
    assert e.value.status == krr.KRR_ERROR_INVALID_VALUE
    ctx.close()


# --- linear kernel and Ridge Regression (RR subsection, Eq. 1-2) ------------------------------

def test_linear_kernel_inner_products_bit_exact():
    """KRR_KERNEL_LINEAR keeps the exact inner products g_i . g_j (ragged n and m)."""
    for n, m in [(5, 3), (300, 129), (700, 2000)]:
        G = _gen(n, m, seed=n + m)
        ctx = krr.krr_create(0, tile=256)
        K = krr.krr_build_kernel_ex(ctx, _dev(G), 1.0, 0.5, kind=krr.KRR_KERNEL_LINEAR)
        S = krr.krr_kernel_copy_distances(K, 0, 0, n, n).cpu().numpy().astype(np.int64)
        assert np.array_equal(S, oracle.dot(G))
        A = krr.krr_kernel_copy_matrix(K, 0, 0, n, n).cpu().numpy()
        want = oracle.dot(G).astype(np.float64) + 0.5 * np.eye(n)
        assert np.array_equal(A.astype(np.float64), want)  # exact in FP32
        ctx.close()


@pytest.mark.parametrize("n,m", [(2000, 900), (600, 1500)])
def test_ridge_regression_parity(n, m):
    """beta and the predictions against the oracle's Eq. 2, with more patients than
    SNPs and with fewer (the regulariser then carries the system), under the plain
    FP32 factorization and the adaptive one restricted to FP16 (X^T X is far less
    well conditioned than the Gaussian kernel matrix), refined in FP64."""
    G = _gen(n + 50, m, seed=n)
    G, T = G[:n], G[n:]
    Y = synth.phenotypes(G, 3, n_pairs=5, n_add=20, seed=n + 1, h2=0.5)
    lam = 0.05 * float(np.mean(np.sum(G.astype(np.float64) ** 2, axis=0)))
    bo = oracle.rr_fit(G, Y, lam)
    ctx = krr.krr_create(0, tile=256)
    pols = [krr.plain_fp32_policy(),
            krr.Policy(allowed=1 << krr.KRR_PREC_FP16, eps=1e-3)]
    for pol in pols:
        beta, info, st = krr.krr_rr_fit(ctx, _dev(G), _dev(Y), lam, pol,
                                        krr.Refine(method=krr.KRR_REFINE_AUTO, tol=1e-10,
                                                   max_iters=100))
        assert st == krr.KRR_SUCCESS and info.converged == 1
        assert _colrel(beta.cpu().numpy(), bo) <= TOL
    P = krr.krr_rr_predict(ctx, _dev(T), _dev(bo)).cpu().numpy()
    assert _colrel(P, oracle.rr_predict(T, bo)) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("kind", ["gauss", "gauss_table", "linear", "confounders"])
@pytest.mark.parametrize("r", [3, 40])
def test_residual_read_once_matches_oracle(kind, r):
    """The residual with every stored distance tile read once (residual_split = -1: each
    tile's direct and transposed products into slots of their own, summed in fixed
    order) gives the oracle's FP64 residual for the unrefined X, as the two-read form
    does, for every way a stored integer becomes a kernel value (two-level exponential
    tables, the plain table at a large gamma, the linear kernel, confounder factors),
    with 1 and 3 blocks of 16 right-hand sides and a ragged n (3 tiles of 256)."""
    n, m, lam = 700, 500, 0.05
    G = _gen(n, m, seed=41 + r)
    Y = synth.phenotypes(G, r, n_pairs=8, n_add=4, seed=42, h2=0.5)
    C = None
    if kind == "linear":
        gamma = 0.0
    elif kind == "gauss_table":
        gamma = 2000.0 / m
    elif kind == "confounders":
        G, _, C, _, gamma = _conf_case(n, 0, m, 4, seed=43)
        Y = synth.phenotypes(G, r, n_pairs=8, n_add=4, seed=42, h2=0.5)
    else:
        gamma = 1.0 / m
    for split in (8, -1):
        c = krr.krr_create(0, tile=256)
        krr.krr_set_tuning(c, tile=256, residual_split=split)
        if kind == "linear":
            K = krr.krr_build_kernel_ex(c, _dev(G), 1.0, lam, kind=krr.KRR_KERNEL_LINEAR)
        elif C is not None:
            K = krr.krr_build_kernel_ex(c, _dev(G), gamma, lam, C=_dev(C))
        else:
            K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
        F = krr.krr_factor(c, K, krr.plain_fp32_policy())
        X, info, _ = krr.krr_solve(c, F, _dev(Y), krr.Refine(max_iters=0, tol=0.0), check=False)
        Xh = X.cpu().numpy()
        if kind == "linear":
            Kf = oracle.dot(G).astype(np.float64) + lam * np.eye(n)
            R = Y - Kf @ Xh
        else:
            R = oracle.residual_rows(G, gamma, lam, Xh, Y, np.arange(n), C=C)
        want = np.max(np.linalg.norm(R, axis=0) / (lam * np.linalg.norm(Xh, axis=0)))
        np.testing.assert_allclose(info.fwd_err_bound, want, rtol=1e-8)
        F.release()
        K.release()
        c.close()
