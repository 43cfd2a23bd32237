"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Integer work (squared distances) must match bit for bit.  Floating-point
results are held to the tolerances of the benchmark target: 1e-5 relative
error of the weights X and predictions P per phenotype column, after FP64
refinement; the FP32 kernel matrix within 1 FP32 ulp of the FP64 value; the
FP32 Cholesky factor within FP32 backward error.
"""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2409_01712_amd as krr  # noqa: E402

DEV = "cuda:0"
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = krr.krr_create(0)
    yield c
    c.close()


def _gen(n, m, seed=12345, lo=0.05, hi=0.5):
    p = synth.maf_uniform(m, lo, hi, seed)
    return synth.genotypes(n, m, p, seed)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _colrel(A, B):
    """max over columns of max|A - B| / max|B|."""
    A = np.asarray(A).reshape(len(A), -1)
    B = np.asarray(B).reshape(len(B), -1)
    return max(np.max(np.abs(A[:, c] - B[:, c])) / np.max(np.abs(B[:, c])) for c in range(B.shape[1]))


# --- Build: distances and kernel matrix ---------------------------------------------------

@pytest.mark.parametrize("n,m", [(1, 1), (2, 16), (255, 63), (257, 65), (513, 4097), (300, 16),
                                 (1100, 333)])
def test_distances_bit_exact_ragged(ctx, n, m):
    G = _gen(n, m, seed=n * 7 + m)
    K = krr.krr_build_kernel(ctx, _dev(G), 1.0 / m, 0.1)
    D = krr.krr_kernel_copy_distances(K, 0, 0, n, n).cpu().numpy()
    assert np.array_equal(D.astype(np.int64), oracle.sqdist(G))


def test_distances_bit_exact_small_config(ctx):
    w = synth.WORKLOADS["small"]
    G = w.genotypes()
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    D = krr.krr_kernel_copy_distances(K, 0, 0, w.n, w.n).cpu().numpy()
    assert np.array_equal(D.astype(np.int64), oracle.sqdist(G))


def test_distances_extreme_values(ctx):
    """All-2 versus all-0 rows give the largest distance 4m (int32 accumulator range)."""
    m = 70000
    G = np.zeros((6, m), np.int8)
    G[0] = 2
    G[2, ::2] = 2
    G[3] = 1
    G[4] = 2
    K = krr.krr_build_kernel(ctx, _dev(G), 1.0 / m, 0.1)
    D = krr.krr_kernel_copy_distances(K, 0, 0, 6, 6).cpu().numpy()
    want = oracle.sqdist(G)
    assert want[0, 1] == 4 * m
    assert np.array_equal(D.astype(np.int64), want)


def test_kernel_matrix_fp32_within_one_ulp(ctx):
    w = synth.WORKLOADS["small"]
    n = 1300
    G = w.genotypes(rows=n)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    A = krr.krr_kernel_copy_matrix(K, 0, 0, n, n).cpu().numpy()
    Ko = oracle.build_kernel(G, w.gamma)
    Ko[np.diag_indices_from(Ko)] += w.lam
    want = Ko.astype(np.float32)
    ulps = np.abs(A.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == np.float32(1.0 + w.lam))


def test_tile_norms(ctx):
    w = synth.WORKLOADS["small"]
    n = 1100
    G = w.genotypes(rows=n)
    c2 = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c2, _dev(G), w.gamma, w.lam)
    A = krr.krr_kernel_copy_matrix(K, 0, 0, n, n).cpu().numpy().astype(np.float64)
    nb, nt = 256, (n + 255) // 256
    norms = krr.krr_kernel_tile_norms(K, nt)
    for I in range(nt):
        for J in range(I + 1):
            blk = A[I * nb:(I + 1) * nb, J * nb:(J + 1) * nb]
            want = np.sqrt((blk ** 2).sum() + (nb - blk.shape[0] if I == J else 0))
            assert abs(norms[I * (I + 1) // 2 + J] - want) <= 1e-12 * want


def test_fp8_encoder_matches_torch(ctx):
    """The factorization's E4M3 encoder: RNE, saturating at 448, zeros and subnormals."""
    g = torch.Generator().manual_seed(5)
    vals = [0.0, -0.0, 1.0, -1.0, 448.0, 500.0, -1e9, 2 ** -6, 2 ** -9, 2 ** -10, 1.5 * 2 ** -10,
            2 ** -11, 1e-30, 0.0625 + 2 ** -8, 1.0625, 1.1875, 240.0, 464.0, 3.0e-3]
    x = torch.cat([torch.tensor(vals, dtype=torch.float32),
                   torch.randn(20000, generator=g) * torch.exp2(torch.randint(-14, 9, (20000,),
                                                                              generator=g).float())])
    got = krr.krr_debug_encode_fp8(ctx, x.to(DEV)).cpu()
    want = x.clamp(-448.0, 448.0).to(torch.float8_e4m3fn).view(torch.uint8)
    assert torch.equal(got, want), (x[got != want][:8], got[got != want][:8], want[got != want][:8])


# --- Factor -------------------------------------------------------------------------------

def test_factor_fp32_backward_error_and_oracle(ctx):
    w = synth.WORKLOADS["small"]
    n = 1000
    G = w.genotypes(rows=n)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    F = krr.krr_factor(ctx, K, krr.plain_fp32_policy())
    L = krr.krr_factor_copy_l(F, 0, 0, n, n).cpu().numpy().astype(np.float64)
    A = oracle.build_kernel(G, w.gamma)
    A[np.diag_indices_from(A)] += w.lam
    assert np.linalg.norm(A - L @ L.T) / np.linalg.norm(A) <= 1e-5
    Lo = oracle.cholesky(A)
    assert np.max(np.abs(L - Lo)) <= 1e-4
    assert np.all(np.triu(L, 1) == 0)


@pytest.mark.parametrize("diag64", [0, 1])
def test_factor_closed_form(ctx, diag64):
    """Rows 2 e_i give A = b I + c 11^T (c = exp(-8 gamma), b = 1 - c + lambda), whose
    Cholesky factor has a closed form (pinned in the oracle tests)."""
    n, m, lam = 1200, 1280, 0.1
    G = np.zeros((n, m), np.int8)
    G[np.arange(n), np.arange(n)] = 2
    gamma = 1.0 / 64
    K = krr.krr_build_kernel(ctx, _dev(G), gamma, lam)
    pol = krr.plain_fp32_policy()
    pol.diag_fp64 = diag64
    F = krr.krr_factor(ctx, K, pol)
    L = krr.krr_factor_copy_l(F, 0, 0, n, n).cpu().numpy().astype(np.float64)
    c = np.exp(-8 * gamma)
    b = 1 - c + lam
    s = b + c * np.arange(n + 1)
    d = np.sqrt(b * s[1:] / s[:-1])
    col = c * np.sqrt(b) / np.sqrt(s[:-1] * s[1:])
    assert np.max(np.abs(np.diag(L) - d) / d) <= 2e-5
    low = np.tril(L, -1)
    want = np.tril(np.ones((n, n)), -1) * col[None, :]
    assert np.max(np.abs(low - want)) <= 2e-5 * np.max(col)


def test_factor_deterministic_precision_map(ctx):
    w = synth.WORKLOADS["small"]
    G = w.genotypes()
    maps = []
    for _ in range(2):
        K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
        F = krr.krr_factor(ctx, K, krr.Policy(eps=1.0))
        maps.append(krr.krr_factor_precision_map(F))
    assert np.array_equal(maps[0], maps[1])
    nt = maps[0].shape[0]
    # panel 0 (high panel) and every diagonal update are FP32
    tri = lambda i, j: i * (i + 1) // 2 + j
    for i in range(1, nt):
        assert maps[0][0, tri(i, i)] == krr.KRR_PREC_FP32
        for j in range(1, i + 1):
            assert maps[0][0, tri(i, j)] == krr.KRR_PREC_FP32


# --- Solve --------------------------------------------------------------------------------

POLICIES = {
    "plain_fp32_refined": krr.plain_fp32_policy(),
    "adaptive": krr.Policy(),
    "fixed_fp16": krr.Policy(mode=krr.KRR_POLICY_FIXED, fixed_prec=krr.KRR_PREC_FP16),
    "fixed_fp8": krr.Policy(mode=krr.KRR_POLICY_FIXED, fixed_prec=krr.KRR_PREC_FP8),
}


@pytest.mark.parametrize("name", list(POLICIES))
def test_solve_parity_small_config(ctx, name):
    w = synth.WORKLOADS["small"]
    G = w.genotypes()
    Y = w.phenotypes(G)
    Wo = oracle.fit(G, Y, w.gamma, w.lam)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    F = krr.krr_factor(ctx, K, POLICIES[name])
    X, info, st = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), Wo) <= TOL


def test_solve_parity_ragged_many_rhs(ctx):
    n, m, r = 1500, 2000, 40
    G = _gen(n, m, seed=99)
    Y = synth.phenotypes(G, r, n_pairs=10, n_add=5, seed=3, h2=0.5)
    gamma, lam = 0.5 / m, 1e-2
    Wo = oracle.fit(G, Y, gamma, lam)
    c2 = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c2, _dev(G), gamma, lam)
    F = krr.krr_factor(c2, K)
    X, info, st = krr.krr_solve(c2, F, _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), Wo) <= TOL


@pytest.mark.parametrize("n", [200, 700, 1200, 1500])
def test_paired_sweeps_match_single_steps(monkeypatch, n):
    """Triangular sweeps that take the tiles in pairs (a coupling tile standing in
    for the step between the two) agree with one-tile-per-step sweeps to FP32
    rounding, at tile counts 1, 3, 5 and 6 (tile 256); the refined result matches
    the oracle."""
    m, r = 900, 5
    G = _gen(n, m, seed=n)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 1, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    F = krr.krr_factor(c, K, krr.plain_fp32_policy())
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    X2, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.setenv("KRR_SWEEP_PAIRS", "0")
    X1, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.delenv("KRR_SWEEP_PAIRS")
    # both carry the FP32 factor's error; a wrong coupling or a missed panel
    # term would move X by O(1)
    assert _colrel(X2.cpu().numpy(), X1.cpu().numpy()) <= 2e-3
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, gamma, lam)) <= TOL
    F.release()
    K.release()
    c.close()


@pytest.mark.parametrize("n,r", [(1000, 5), (1200, 17), (1700, 5), (2200, 40)])
def test_quad_sweeps_match_pairs(monkeypatch, n, r):
    """Sweeps that take four tiles a step (the quad's block inverse through its
    two pair couplings and a 2 x 2 coupling block, the panels over four tiles
    of k) agree with the paired sweeps and with one tile a step to FP32
    rounding: 4, 5, 7 and 9 tiles (a quad alone, quads with pair and single
    tails), 1-3 column blocks; the refined result matches the oracle."""
    m = 600
    G = _gen(n, m, seed=n + 31)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 32, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    F = krr.krr_factor(c, K, krr.plain_fp32_policy())
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    Xq, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.setenv("KRR_SWEEP_QUADS", "0")
    Xp, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.setenv("KRR_SWEEP_PAIRS", "0")
    X1, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.delenv("KRR_SWEEP_PAIRS")
    monkeypatch.delenv("KRR_SWEEP_QUADS")
    # the same solution through other products; a wrong coupling tile, sign
    # or panel term would move X by O(1)
    assert _colrel(Xq.cpu().numpy(), Xp.cpu().numpy()) <= 2e-3
    assert _colrel(Xq.cpu().numpy(), X1.cpu().numpy()) <= 2e-3
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, gamma, lam)) <= TOL
    F.release()
    K.release()
    c.close()


@pytest.mark.parametrize("n,r", [(3072, 16), (4500, 5), (6000, 33)])
def test_split_quad_sweeps_match_one_stream(monkeypatch, n, r):
    """Quad sweep steps whose panel is split in two launches (the next quad's
    tiles on the solve's stream, the rest on a second stream that overlaps the
    next diagonal step) give the bits of the one-launch panels: every tile is
    updated by the same workgroup code in the same order.  12, 18 and 24 tiles
    (quads only; quads with a pair tail; 1-3 column blocks), ragged n; and the
    refined result matches the oracle."""
    m = 500
    G = _gen(n, m, seed=n + 41)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 42, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    F = krr.krr_factor(c, K, krr.plain_fp32_policy())
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    monkeypatch.setenv("KRR_SWEEP_SPLIT", "0")
    X0, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.setenv("KRR_SWEEP_SPLIT", "1")
    for rep in range(2):
        Xs, _, _ = krr.krr_solve(c, F, _dev(Y), none)
        assert torch.equal(Xs, X0), rep
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
    monkeypatch.delenv("KRR_SWEEP_SPLIT")
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, gamma, lam)) <= TOL
    F.release()
    K.release()
    c.close()


@pytest.mark.parametrize("n,r,tile", [(700, 5, 256), (1500, 17, 256), (1300, 40, 512),
                                       (2600, 16, 512)])
def test_wide_panel_sweeps_match_narrow(monkeypatch, n, r, tile):
    """The paired sweeps' panel launches with 64-row workgroups (right-hand sides
    staged in LDS, each wave summing its rows over all k) agree with the 16-row
    form (k blocks dealt over the waves, summed across them) to FP32 rounding:
    several panel tiles, 1-3 column blocks of right-hand sides, ragged n; the
    refined result matches the oracle.  (Pairs throughout: the quads of tile
    256 are compared with pairs in their own test.)"""
    monkeypatch.setenv("KRR_SWEEP_QUADS", "0")
    m = 700
    G = _gen(n, m, seed=n + 11)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 12, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=tile)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    F = krr.krr_factor(c, K, krr.plain_fp32_policy())
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    Xw, _, _ = krr.krr_solve(c, F, _dev(Y), none)  # 4 waves a workgroup
    monkeypatch.setenv("KRR_SWEEP_WIDE", "8")
    X8, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.setenv("KRR_SWEEP_WIDE", "0")
    Xn, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.delenv("KRR_SWEEP_WIDE")
    # the same FP32 products summed in another order; a missed k block, a wrong
    # tile or right-hand-side column would move X by O(1)
    assert _colrel(Xw.cpu().numpy(), Xn.cpu().numpy()) <= 1e-4
    # 4 or 8 waves a workgroup: the same sums in the same order
    assert np.array_equal(Xw.cpu().numpy(), X8.cpu().numpy())
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, gamma, lam)) <= TOL
    F.release()
    K.release()
    c.close()


@pytest.mark.parametrize("n,tile", [(1500, 256), (2600, 512), (5000, 256)])
def test_split_load_matches_single_load(monkeypatch, n, tile):
    """The diagonal-tile load split over K (chunk products in slots, a second
    launch adding them in chunk order and factoring block (0, 0)) gives the
    factor of the one-workgroup-per-block load to FP32 rounding, the same bits
    on a second run (the reduction order is fixed), and refined solutions that
    match the oracle.  n = 5000 at tile 256 spans a panel group boundary (a
    load folding several panels)."""
    m, r = 800, 6
    G = _gen(n, m, seed=n + 21)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 22, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=tile)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    Wo = oracle.fit(G, Y, gamma, lam)
    for policy in (krr.plain_fp32_policy(), None):  # FP32 throughout; adaptive
        xs, refined = [], []
        for split in ("1", "1", "0"):
            monkeypatch.setenv("KRR_LOAD_SPLIT", split)
            F = krr.krr_factor(c, K, policy)
            X, _, _ = krr.krr_solve(c, F, _dev(Y), none)
            xs.append(X.cpu().numpy())
            X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
            assert info.converged == 1
            refined.append(X.cpu().numpy())
            F.release()
        monkeypatch.delenv("KRR_LOAD_SPLIT")
        assert np.array_equal(xs[0], xs[1])
        if policy is not None:
            # FP32 products summed in another order: differences at FP32
            # rounding, grown by the conditioning (a missed chunk or a wrong
            # block would be O(1)); under the adaptive policy the reordering
            # also moves FP8 rounding decisions downstream, so only the
            # refined solutions are compared there
            assert _colrel(xs[0], xs[2]) <= 1e-4
        for Xr in refined:
            assert _colrel(Xr, Wo) <= TOL
    K.release()
    c.close()


@pytest.mark.parametrize("n,tile", [(1500, 256), (2600, 512), (5000, 256)])
def test_row_in_steps_matches_substitution(monkeypatch, n, tile):
    """Row tile k+1 of each panel formed by extra workgroups of POTRF(k)'s
    64-column steps (right-looking, from the stored tile, in FP64) gives the
    panel of the separate substitution TRSM to FP32 rounding, the same bits on
    a second run, and refined solutions that match the oracle (FP32 and
    adaptive policies; n = 5000 at tile 256 crosses a panel group boundary)."""
    m, r = 800, 6
    G = _gen(n, m, seed=n + 41)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 42, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=tile)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    Wo = oracle.fit(G, Y, gamma, lam)
    for policy in (krr.plain_fp32_policy(), None):
        xs, refined = [], []
        for on in ("1", "1", "0"):
            monkeypatch.setenv("KRR_ROW_IN_STEPS", on)
            F = krr.krr_factor(c, K, policy)
            X, _, _ = krr.krr_solve(c, F, _dev(Y), none)
            xs.append(X.cpu().numpy())
            X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
            assert info.converged == 1
            refined.append(X.cpu().numpy())
            F.release()
        monkeypatch.delenv("KRR_ROW_IN_STEPS")
        assert np.array_equal(xs[0], xs[1])
        if policy is not None:
            # the same panel by another order of FP64 products, rounded to
            # FP32; a wrong block, sign or missed update would be O(1)
            assert _colrel(xs[0], xs[2]) <= 1e-4
        for Xr in refined:
            assert _colrel(Xr, Wo) <= TOL
    K.release()
    c.close()


@pytest.mark.skip(reason="persistent one-launch sweeps are switched off (KRR_SWEEP_PAIRS=2 "
                  "returns KRR_ERROR_NOT_SUPPORTED): the first GPU runs hung at n=200 (one "
                  "tile), also with time-bounded waits, and the cause is not known")
@pytest.mark.parametrize("n,r", [(200, 5), (700, 40), (1500, 5), (3000, 17)])
def test_persistent_sweeps_match_single_steps(monkeypatch, n, r):
    """Sweeps as one persistent launch each (work items from an atomic ticket, waits on
    per-tile counters) agree with one-tile-per-step sweeps to FP32 rounding, at tile
    counts 1, 3, 6 and 12 (tile 256) and 1 to 3 blocks of 16 right-hand sides; the
    refined result matches the oracle."""
    m = 900
    G = _gen(n, m, seed=n + r)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=3, seed=n + 2, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    F = krr.krr_factor(c, K, krr.plain_fp32_policy())
    none = krr.Refine(method=krr.KRR_REFINE_NONE)
    monkeypatch.setenv("KRR_SWEEP_PAIRS", "0")
    X1, _, _ = krr.krr_solve(c, F, _dev(Y), none)
    monkeypatch.setenv("KRR_SWEEP_PAIRS", "2")
    Xp, _, st = krr.krr_solve(c, F, _dev(Y), none)
    assert st == krr.KRR_SUCCESS
    assert _colrel(Xp.cpu().numpy(), X1.cpu().numpy()) <= 2e-3
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
    assert st == krr.KRR_SUCCESS and info.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, gamma, lam)) <= TOL
    # the adaptive factor through the same sweeps, refined to the oracle
    F2 = krr.krr_factor(c, K)
    X2, info2, _ = krr.krr_solve(c, F2, _dev(Y), krr.Refine(tol=1e-8))
    assert info2.converged == 1
    assert _colrel(X2.cpu().numpy(), oracle.fit(G, Y, gamma, lam)) <= TOL
    monkeypatch.delenv("KRR_SWEEP_PAIRS")
    c.close()


@pytest.mark.parametrize("method", ["pcg", "auto"])
@pytest.mark.parametrize("policy", ["adaptive", "fixed_fp8"])
def test_pcg_parity(method, policy):
    """Conjugate gradients preconditioned by the mixed-precision factor (and AUTO,
    which starts with refinement) reach the oracle's FP64 solution at lambda = 1e-3,
    where refinement contracts slowest, with a ragged n (1500 at tile 256) and one
    all-zero right-hand side, whose solution is exactly zero."""
    n, m, r = 1500, 2000, 6
    G = _gen(n, m, seed=41)
    Y = synth.phenotypes(G, r, n_pairs=10, n_add=5, seed=5, h2=0.5)
    Y[:, 2] = 0.0
    gamma, lam, tol = 0.5 / m, 1e-3, 1e-8
    Wo = oracle.fit(G, Y, gamma, lam)
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), gamma, lam)
    F = krr.krr_factor(c, K, POLICIES[policy])
    meth = {"pcg": krr.KRR_REFINE_PCG, "auto": krr.KRR_REFINE_AUTO}[method]
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(method=meth, max_iters=60, tol=tol))
    X_ir, info_ir, _ = krr.krr_solve(c, F, _dev(Y), krr.Refine(max_iters=60, tol=tol), check=False)
    print(f"{method}/{policy}: iters {info.iters} (IR {info_ir.iters}), "
          f"first bound {info.first_bound:.2e}, final {info.fwd_err_bound:.2e}")
    assert st == krr.KRR_SUCCESS and info.converged == 1 and info.fwd_err_bound <= tol
    assert info.first_bound > tol and info.iters >= 1
    Xh = X.cpu().numpy()
    assert np.all(Xh[:, 2] == 0.0)
    keep = [0, 1, 3, 4, 5]
    assert _colrel(Xh[:, keep], Wo[:, keep]) <= TOL
    # the stop rule is certified on the oracle's own FP64 residual of the returned X
    R = oracle.residual_rows(G, gamma, lam, Xh, Y, np.arange(n))
    xn = np.linalg.norm(Xh, axis=0)
    assert np.all(np.linalg.norm(R, axis=0) <= lam * tol * xn * 1.01 + 1e-300)
    F.release()
    K.release()
    c.close()


def test_pcg_budget_and_batched_rejection():
    """PCG with no iteration budget reports NOT_CONVERGED with the first solve in X;
    the batched solve implements refinement only and rejects PCG."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=600)
    Y = w.phenotypes(G)
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), w.gamma, w.lam)
    F = krr.krr_factor(c, K)
    X0, info0, st0 = krr.krr_solve(c, F, _dev(Y), krr.Refine(method=krr.KRR_REFINE_NONE))
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(method=krr.KRR_REFINE_PCG, max_iters=0,
                                                          tol=1e-300), check=False)
    assert st == krr.KRR_ERROR_NOT_CONVERGED and info.iters == 0 and info.converged == 0
    assert torch.equal(X, X0)
    Ks = krr.krr_build_kernel_batched(c, [_dev(G)], [w.gamma], [w.lam])
    Fs = krr.krr_factor_batched(c, Ks)
    _, _, stb = krr.krr_solve_batched(c, Fs, [_dev(Y)], krr.Refine(method=krr.KRR_REFINE_PCG),
                                      check=False)
    assert stb == krr.KRR_ERROR_NOT_SUPPORTED
    Xa, infa, sta = krr.krr_solve_batched(c, Fs, [_dev(Y)],
                                          krr.Refine(method=krr.KRR_REFINE_AUTO, tol=1e-8))
    assert sta == krr.KRR_SUCCESS and infa[0].converged == 1
    c.close()


def test_refactor_from_distances(ctx):
    """A second factorization of one kernel re-expands K from the stored distances."""
    w = synth.WORKLOADS["small"]
    n = 900
    G = w.genotypes(rows=n)
    Y = w.phenotypes(G)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    X1 = krr.krr_solve(ctx, krr.krr_factor(ctx, K, krr.plain_fp32_policy()), _dev(Y))[0]
    X2 = krr.krr_solve(ctx, krr.krr_factor(ctx, K, krr.plain_fp32_policy()), _dev(Y))[0]
    assert torch.equal(X1, X2)


# --- Predict ------------------------------------------------------------------------------

def test_predict_parity(ctx):
    n, nt_, m, r = 1500, 333, 3000, 3
    Gall = _gen(n + nt_, m, seed=7)
    G, T = Gall[:n], Gall[n:]
    Y = synth.phenotypes(G, r, n_pairs=10, n_add=5, seed=5, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    Wo = oracle.fit(G, Y, gamma, lam)
    Po = oracle.predict(G, T, Wo, gamma)
    K = krr.krr_build_kernel(ctx, _dev(G), gamma, lam)
    F = krr.krr_factor(ctx, K)
    X, info, st = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(tol=1e-8))
    P = krr.krr_predict(ctx, K, _dev(T), X).cpu().numpy()
    assert _colrel(P, Po) <= TOL
    # predicting with the oracle's weights isolates the predict step
    P2 = krr.krr_predict(ctx, K, _dev(T), _dev(Wo)).cpu().numpy()
    assert _colrel(P2, Po) <= 1e-12


# --- error paths ---------------------------------------------------------------------------

def test_bad_genotype(ctx):
    G = _gen(100, 64)
    G[37, 5] = 3
    with pytest.raises(krr.KRRError) as e:
        krr.krr_build_kernel(ctx, _dev(G), 0.01, 0.1)
    assert e.value.status == krr.KRR_ERROR_BAD_GENOTYPE
    G[37, 5] = 1
    K = krr.krr_build_kernel(ctx, _dev(G), 0.01, 0.1)
    F = krr.krr_factor(ctx, K)
    T = _gen(10, 64, seed=4)
    T[2, 63] = -1
    with pytest.raises(krr.KRRError) as e:
        krr.krr_predict(ctx, K, _dev(T), torch.zeros((100, 1), dtype=torch.float64, device=DEV))
    assert e.value.status == krr.KRR_ERROR_BAD_GENOTYPE


def test_breakdown_singular(ctx):
    """Identical genotype rows and lambda = 0: K = 11^T has a zero pivot."""
    G = np.ones((300, 48), np.int8)
    K = krr.krr_build_kernel(ctx, _dev(G), 0.01, 0.0)
    with pytest.raises(krr.KRRError) as e:
        krr.krr_factor(ctx, K, krr.plain_fp32_policy())
    assert e.value.status == krr.KRR_ERROR_NOT_POSITIVE_DEFINITE


def test_not_converged_reports(ctx):
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=600)
    Y = w.phenotypes(G)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    F = krr.krr_factor(ctx, K)
    X, info, st = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(max_iters=0, tol=1e-300), check=False)
    assert st == krr.KRR_ERROR_NOT_CONVERGED
    assert info.converged == 0 and info.fwd_err_bound > 0 and torch.isfinite(X).all()


def test_workspace_limit(ctx):
    c2 = krr.krr_create(0, workspace_limit=1 << 20)
    G = _gen(2048, 256)
    with pytest.raises(krr.KRRError) as e:
        krr.krr_build_kernel(c2, _dev(G), 0.01, 0.1)
    assert e.value.status == krr.KRR_ERROR_OUT_OF_MEMORY


# --- the benchmark's full size, in its launch configuration ---------------------------------

def test_full_size_single_workload_sampled():
    """n = 32768, m = 65536, r = 16, tile 512, adaptive policy with lookahead and the
    benchmark's refinement target.  The oracle cannot hold the 32768^2 matrix, so it
    checks sampled blocks of distances (by definition, bit for bit) and of K (one FP32
    ulp), and the FP64 residual r = Y - (K + lambda I) X on sampled rows: each column's
    sampled residual norm must stay below lambda * tol * ||x_j||, the stop rule whose
    PSD bound certifies the 1e-5 relative error."""
    w = synth.WORKLOADS["single"]
    n, m = w.n, w.m
    G = w.genotypes()
    Y = w.phenotypes(G)
    assert G.shape == (32768, 65536) and Y.shape[1] == 16
    c = krr.krr_create(0, tile=512)
    Gd = _dev(G)
    K = krr.krr_build_kernel(c, Gd, w.gamma, w.lam)
    blocks = [(0, 0), (n - 64, 0), (n - 64, n - 64), (16484, 7003), (511, 31000), (20000, 20000)]
    for i0, j0 in blocks:
        d = krr.krr_kernel_copy_distances(K, i0, j0, 64, 64).cpu().numpy()
        ref = oracle.sqdist(G[i0:i0 + 64], G[j0:j0 + 64])
        assert np.array_equal(d.astype(np.int64), ref), (i0, j0)
        a = krr.krr_kernel_copy_matrix(K, i0, j0, 64, 64).cpu().numpy().astype(np.float64)
        kref = oracle.gaussian(ref, w.gamma)
        gi = np.arange(i0, i0 + 64)[:, None]
        gj = np.arange(j0, j0 + 64)[None, :]
        kref = np.where(gi == gj, 1.0 + w.lam, kref)
        ulp = np.spacing(kref.astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(a - kref) <= ulp), (i0, j0)
    F = krr.krr_factor(c, K, krr.Policy())
    tol = 9.9e-6
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(method=krr.KRR_REFINE_IR,
                                                          max_iters=30, tol=tol))
    assert info.converged == 1 and info.fwd_err_bound <= 1e-5
    fi = krr.krr_factor_get_info(F)
    assert fi.updates[2] > 0  # the adaptive rule did use FP8
    Xh = X.cpu().numpy()
    rng = np.random.default_rng(7)
    rows = np.sort(np.concatenate([[0, n - 1], rng.choice(n, 30, replace=False)]))
    R = oracle.residual_rows(G, w.gamma, w.lam, Xh, Y, rows)
    xnorm = np.linalg.norm(Xh, axis=0)
    assert np.all(np.linalg.norm(R, axis=0) <= w.lam * tol * xnorm)
    F.release()
    K.release()
    c.close()


# --- batches of independent instances -------------------------------------------------------

def _batch_instances(seed=2024):
    """Five instances of uneven n on one genotype panel (rows of one stream), with the
    (gamma, lambda) grid of a cross-validation sweep."""
    ns = [300, 1024, 700, 1536, 257]
    m = 2000
    Gall = _gen(sum(ns), m, seed=seed)
    offs = np.cumsum([0] + ns)
    Gs = [np.ascontiguousarray(Gall[offs[b]:offs[b + 1]]) for b in range(len(ns))]
    gammas = [g / m for g in (0.5, 1.0, 2.0, 0.5, 1.0)]
    lams = [1e-2, 1e-1, 1.0, 1e-1, 1e-2]
    Ys = [synth.phenotypes(G, 3, n_pairs=10, n_add=5, seed=11 + b, h2=0.5)
          for b, G in enumerate(Gs)]
    return Gs, gammas, lams, Ys


def test_batched_build_bit_exact_and_matches_single():
    Gs, gammas, lams, _ = _batch_instances()
    c = krr.krr_create(0, tile=256)
    Ks = krr.krr_build_kernel_batched(c, [_dev(G) for G in Gs], gammas, lams)
    for G, g, lam, K in zip(Gs, gammas, lams, Ks):
        n = len(G)
        d = krr.krr_kernel_copy_distances(K, 0, 0, n, n).cpu().numpy().astype(np.int64)
        ref = oracle.sqdist(G)
        assert np.array_equal(d, ref)
        a = krr.krr_kernel_copy_matrix(K, 0, 0, n, n).cpu().numpy().astype(np.float64)
        kref = oracle.gaussian(ref, g) + lam * np.eye(n)
        ulp = np.spacing(kref.astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(a - kref) <= ulp)
        # the single-instance build gives the same bytes
        K1 = krr.krr_build_kernel(c, _dev(G), g, lam)
        a1 = krr.krr_kernel_copy_matrix(K1, 0, 0, n, n)
        assert torch.equal(a1.cpu(), torch.from_numpy(a.astype(np.float32)))
        nt = (n + 255) // 256
        assert np.array_equal(krr.krr_kernel_tile_norms(K, nt), krr.krr_kernel_tile_norms(K1, nt))
        # ||K + lambda I||_F of the stored FP32 matrix, which the precision rule uses
        np.testing.assert_allclose(krr.krr_factor_get_info(krr.krr_factor(c, K)).norm_a,
                                   np.linalg.norm(a), rtol=1e-12)


@pytest.mark.parametrize("policy", ["adaptive", "plain"])
def test_batched_fit_parity(policy):
    Gs, gammas, lams, Ys = _batch_instances()
    pol = krr.Policy() if policy == "adaptive" else krr.plain_fp32_policy()
    c = krr.krr_create(0, tile=256)
    Ks = krr.krr_build_kernel_batched(c, [_dev(G) for G in Gs], gammas, lams)
    Fs = krr.krr_factor_batched(c, Ks, pol)
    Xs, infos, st = krr.krr_solve_batched(c, Fs, [_dev(Y) for Y in Ys], krr.Refine(tol=1e-8))
    for b, (G, g, lam, Y) in enumerate(zip(Gs, gammas, lams, Ys)):
        assert infos[b].converged == 1, b
        Wo = oracle.fit(G, Y, g, lam)
        assert _colrel(Xs[b].cpu().numpy(), Wo) <= TOL, b
    # one instance through the single-instance calls agrees to the same bar
    K = krr.krr_build_kernel(c, _dev(Gs[3]), gammas[3], lams[3])
    X1, info1, _ = krr.krr_solve(c, krr.krr_factor(c, K, pol), _dev(Ys[3]), krr.Refine(tol=1e-8))
    assert _colrel(Xs[3].cpu().numpy(), X1.cpu().numpy()) <= TOL


def test_batched_bad_genotype_returns_nothing():
    Gs, gammas, lams, _ = _batch_instances()
    Gs[2] = Gs[2].copy()
    Gs[2][5, 7] = 3
    c = krr.krr_create(0, tile=256)
    with pytest.raises(krr.KRRError) as e:
        krr.krr_build_kernel_batched(c, [_dev(G) for G in Gs], gammas, lams)
    assert e.value.status == krr.KRR_ERROR_BAD_GENOTYPE


@pytest.mark.parametrize("gamma_scale", [1.0, 2000.0])
def test_residual_bound_matches_oracle(ctx, gamma_scale):
    """The FP64 residual behind the refinement's stop rule: the bound the library reports
    for the unrefined X equals max_j ||Y_j - (K + lambda I) X_j|| / (lambda ||X_j||) with the
    oracle's residual (exp by definition).  gamma_scale 2000 takes the kernel's table
    path instead of the factored exponential."""
    n, m, r = 1100, 300, 3
    G = _gen(n, m, seed=21)
    Y = synth.phenotypes(G, r, n_pairs=10, n_add=5, seed=8, h2=0.5)
    gamma, lam = gamma_scale / m, 0.05
    K = krr.krr_build_kernel(ctx, _dev(G), gamma, lam)
    F = krr.krr_factor(ctx, K)
    X, info, st = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(max_iters=0, tol=0.0), check=False)
    Xh = X.cpu().numpy()
    R = oracle.residual_rows(G, gamma, lam, Xh, Y, np.arange(n))
    bound = np.max(np.linalg.norm(R, axis=0) / (lam * np.linalg.norm(Xh, axis=0)))
    assert info.first_bound > 0
    np.testing.assert_allclose(info.fwd_err_bound, bound, rtol=1e-8)


def test_batched_edge_sizes():
    """A batch of one, a one-patient instance, and sizes either side of a tile."""
    m = 200
    ns = [1, 255, 256, 257, 513]
    Gall = _gen(sum(ns), m, seed=31)
    offs = np.cumsum([0] + ns)
    Gs = [np.ascontiguousarray(Gall[offs[b]:offs[b + 1]]) for b in range(len(ns))]
    gammas = [1.0 / m] * len(ns)
    lams = [0.1] * len(ns)
    Ys = [synth.phenotypes(G, 2, n_pairs=5, n_add=2, seed=40 + b, h2=0.5) if len(G) > 1
          else np.array([[0.7, -0.3]]) for b, G in enumerate(Gs)]
    c = krr.krr_create(0, tile=256)
    for sel in ([3], list(range(len(ns)))):
        Ks = krr.krr_build_kernel_batched(c, [_dev(Gs[b]) for b in sel], [gammas[b] for b in sel],
                                          [lams[b] for b in sel])
        Fs = krr.krr_factor_batched(c, Ks)
        Xs, infos, st = krr.krr_solve_batched(c, Fs, [_dev(Ys[b]) for b in sel],
                                              krr.Refine(tol=1e-8))
        for q, b in enumerate(sel):
            n = ns[b]
            d = krr.krr_kernel_copy_distances(Ks[q], 0, 0, n, n).cpu().numpy().astype(np.int64)
            assert np.array_equal(d, oracle.sqdist(Gs[b]))
            assert infos[q].converged == 1
            Wo = oracle.fit(Gs[b], Ys[b], gammas[b], lams[b])
            assert _colrel(Xs[q].cpu().numpy(), Wo) <= TOL, (b, n)


def test_batched_singular_instance_fails_the_batch():
    """Identical rows and lambda = 0 in one instance: the factorization breaks down, promotion
    cannot cure it, and the batched call returns no handles."""
    Gs, gammas, lams, _ = _batch_instances()
    Gs[1] = np.ones((300, Gs[0].shape[1]), np.int8)
    lams[1] = 0.0
    c = krr.krr_create(0, tile=256)
    Ks = krr.krr_build_kernel_batched(c, [_dev(G) for G in Gs], gammas, lams)
    with pytest.raises(krr.KRRError) as e:
        krr.krr_factor_batched(c, Ks)
    assert e.value.status == krr.KRR_ERROR_NOT_POSITIVE_DEFINITE


def test_single_stream_factorization(monkeypatch):
    """The factorization without lookahead (one stream, substitution TRSM, tile inverses at the
    end) reaches the same refined X."""
    monkeypatch.setenv("KRR_NO_LOOKAHEAD", "1")
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=1300)
    Y = w.phenotypes(G)
    Wo = oracle.fit(G, Y, w.gamma, w.lam)
    c = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(c, _dev(G), w.gamma, w.lam)
    X, info, st = krr.krr_solve(c, krr.krr_factor(c, K), _dev(Y), krr.Refine(tol=1e-8))
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), Wo) <= TOL


def test_full_size_batched_workload_sampled():
    """The 48-instance batch (n in [1536, 16384], m = 16384, r = 8, the (gamma, lambda)
    grid), as the batched benchmark runs it: every instance converges to the 1e-5 target;
    a 64 x 64 block of distances per instance is bit-exact against the oracle's per-pair
    definition; on four instances (the smallest and largest lambda, the largest n) the
    oracle's FP64 residual on sampled rows stays below lambda * tol * ||x_j||."""
    insts = synth.batched_workloads()
    assert len(insts) == 48
    Gs, Ys = [], []
    for w, row0 in insts:
        G = w.genotypes(rows=w.n, row0=row0)
        Gs.append(G)
        Ys.append(w.phenotypes(G))
    gammas = [w.gamma for w, _ in insts]
    lams = [w.lam for w, _ in insts]
    c = krr.krr_create(0, tile=512)
    Ks = krr.krr_build_kernel_batched(c, [_dev(G) for G in Gs], gammas, lams)
    rng = np.random.default_rng(11)
    for b, (G, K) in enumerate(zip(Gs, Ks)):
        n = len(G)
        i0, j0 = int(rng.integers(0, n - 64)), int(rng.integers(0, n - 64))
        d = krr.krr_kernel_copy_distances(K, i0, j0, 64, 64).cpu().numpy().astype(np.int64)
        assert np.array_equal(d, oracle.sqdist(G[i0:i0 + 64], G[j0:j0 + 64])), b
    Fs = krr.krr_factor_batched(c, Ks)
    tol = 9.9e-6
    Xs, infos, st = krr.krr_solve_batched(c, Fs, [_dev(Y) for Y in Ys],
                                          krr.Refine(max_iters=30, tol=tol))
    assert st == krr.KRR_SUCCESS
    assert all(i.converged == 1 and i.fwd_err_bound <= 1e-5 for i in infos)
    ns = [len(G) for G in Gs]
    pick = {int(np.argmin(lams)), int(np.argmax(lams)), int(np.argmax(ns)), 0}
    for b in sorted(pick):
        Xh = Xs[b].cpu().numpy()
        rows = np.sort(rng.choice(ns[b], 8, replace=False))
        R = oracle.residual_rows(Gs[b], gammas[b], lams[b], Xh, Ys[b], rows)
        assert np.all(np.linalg.norm(R, axis=0) <= lams[b] * tol * np.linalg.norm(Xh, axis=0)), b


# --- the two largest workloads (about a minute each, most of it host-side generation) ------

_LARGE = pytest.mark.skipif(os.environ.get("KRR_SKIP_LARGE") == "1",
                            reason="KRR_SKIP_LARGE=1: the two largest workloads are skipped")


def _large_check(name, predict=False):
    w = synth.WORKLOADS[name]
    G = w.genotypes()
    Y = w.phenotypes(G)
    n = w.n
    c = krr.krr_create(0, tile=512)
    K = krr.krr_build_kernel(c, _dev(G), w.gamma, w.lam)
    rng = np.random.default_rng(5)
    for _ in range(3):
        i0, j0 = int(rng.integers(0, n - 64)), int(rng.integers(0, n - 64))
        d = krr.krr_kernel_copy_distances(K, i0, j0, 64, 64).cpu().numpy().astype(np.int64)
        assert np.array_equal(d, oracle.sqdist(G[i0:i0 + 64], G[j0:j0 + 64]))
    F = krr.krr_factor(c, K)
    tol = 9.9e-6
    X, info, st = krr.krr_solve(c, F, _dev(Y), krr.Refine(max_iters=30, tol=tol))
    assert info.converged == 1 and info.fwd_err_bound <= 1e-5
    Xh = X.cpu().numpy()
    rows = np.sort(rng.choice(n, 8, replace=False))
    R = oracle.residual_rows(G, w.gamma, w.lam, Xh, Y, rows)
    assert np.all(np.linalg.norm(R, axis=0) <= w.lam * tol * np.linalg.norm(Xh, axis=0))
    if predict:
        T = w.test_genotypes()
        P = krr.krr_predict(c, K, _dev(T), X).cpu().numpy()
        trows = np.sort(rng.choice(len(T), 8, replace=False))
        Kt = oracle.build_kernel(G, w.gamma, T[trows])
        Po = oracle.matmul(Kt, Xh)
        # Both sides sum the same n FP64 products k_ij x_jc in different orders, from
        # kernel entries within one ulp of each other (table lookup against exp), so
        # |P - Po| <= (2 n + 4) u sum_j |k_ij x_jc| entry by entry (u = 2^-53; the
        # standard bound n u on a recursive sum, on each side, plus the entries' ulp).
        # The relative difference is that bound times the cancellation ratio
        # sum_j |k_ij x_jc| / |P_ic|.
        u = 2.0 ** -53
        mag = oracle.matmul(np.abs(Kt), np.abs(Xh))
        assert np.all(np.abs(P[trows] - Po) <= (2 * n + 4) * u * mag)
        # the weights' certified error carried to the predictions:
        # ||P - P*|| <= ||K_t||_F ||x - x*|| on the sampled rows (reported)
        xerr = info.fwd_err_bound / (1 - info.fwd_err_bound) * np.linalg.norm(Xh, axis=0)
        pbound = np.linalg.norm(Kt) * xerr / np.linalg.norm(Po, axis=0)
        print("predict: max rel diff %.2e, certified rel bound on the sampled rows %.2e"
              % (_colrel(P[trows], Po), pbound.max()))


@_LARGE
def test_large_workload_sampled():
    """n = 131072, m = 262144 (5% of SNPs in linkage blocks), r = 64, lambda = 0.05."""
    _large_check("large")


@_LARGE
def test_trainpredict_workload_sampled():
    """n = 200000, m = 100000 (MAF ~ Beta(0.5, 2)), r = 128, then Predict for 20000 test
    patients: sampled predictions with the library's weights against the oracle's."""
    _large_check("trainpredict", predict=True)
