"""GPU checks of the precision policy (the paper's four-precision Cholesky, with
this library's reading of its adaptive rule): the map is recomputed on the host
from the exported factor, a caller-supplied map replays a factorization bit for
bit, a forced FP8 breakdown is cured by panel promotion, the tile-norm rule, the
unscaled-FP8 switch, batched Predict and the release of every factor buffer."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2409_01712_amd as krr  # noqa: E402

DEV = "cuda:0"
TOL = 1e-5
U8, U16 = 2.0 ** -4, 2.0 ** -11


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _tri(i, j):
    return i * (i + 1) // 2 + j


def _colrel(A, B):
    A = np.asarray(A).reshape(len(A), -1)
    B = np.asarray(B).reshape(len(B), -1)
    return max(np.max(np.abs(A[:, c] - B[:, c])) / np.max(np.abs(B[:, c])) for c in range(B.shape[1]))


def _panel_norms(L, nb):
    """FP32 Frobenius norm of every tile (i, k), i > k, of the factor, as the
    library keeps them (FP64 sum of squares, rounded to FP32)."""
    nt = L.shape[0] // nb
    out = np.zeros((nt, nt), np.float64)
    for k in range(nt):
        for i in range(k + 1, nt):
            t = L[i * nb:(i + 1) * nb, k * nb:(k + 1) * nb].astype(np.float64)
            out[i, k] = float(np.float32(np.sqrt(np.sum(t * t))))
    return out


def _rule_map(norms, nt, thr, high_panels, allow8=True, allow16=True):
    """Expected precision of every update (panel k onto tile (i, j), i >= j > k) by
    the operand rule u_p ||L_ik|| ||L_jk|| <= thr; entries within 1e-6 of a
    threshold are marked -1 (either side is correct)."""
    want = np.full((nt, nt * (nt + 1) // 2), 255, np.int16)
    for k in range(nt):
        for j in range(k + 1, nt):
            for i in range(j, nt):
                if i == j or k < high_panels:
                    want[k, _tri(i, j)] = krr.KRR_PREC_FP32
                    continue
                prod = norms[i, k] * norms[j, k]
                p = krr.KRR_PREC_FP32
                near = False
                for u, q, ok in ((U8, krr.KRR_PREC_FP8, allow8), (U16, krr.KRR_PREC_FP16, allow16)):
                    if not ok:
                        continue
                    near = near or abs(u * prod - thr) <= 1e-6 * thr
                    if u * prod <= thr:
                        p = q
                        break
                want[k, _tri(i, j)] = -1 if near else p
    return want


def _check_map(got, want):
    sure = want >= 0
    assert np.array_equal(got[sure].astype(np.int16), want[sure])
    amb = ~sure
    assert np.all(np.isin(got[amb], (krr.KRR_PREC_FP32, krr.KRR_PREC_FP16, krr.KRR_PREC_FP8)))


@pytest.fixture(scope="module")
def mixed():
    """n = 4096 (16 tiles of 256), eps chosen from a first factorization so that
    later panels' updates split between FP8 and FP16."""
    w = synth.WORKLOADS["small"]
    n, nb = 4096, 256
    G = w.genotypes(rows=n)
    Y = w.phenotypes(G)
    ctx = krr.krr_create(0, tile=nb)
    K0 = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    F0 = krr.krr_factor(ctx, K0, krr.Policy(eps=1.0))
    info = krr.krr_factor_get_info(F0)
    L0 = krr.krr_factor_copy_l(F0, 0, 0, n, n).cpu().numpy()
    nrm = _panel_norms(L0, nb)
    nt = n // nb
    vals = [U8 * nrm[i, k] * nrm[j, k] * nt / info.norm_a
            for k in range(1, nt) for j in range(k + 1, nt) for i in range(j + 1, nt)]
    eps = float(np.median(vals))
    F0.release()
    K0.release()
    return dict(w=w, n=n, nb=nb, nt=nt, G=G, Y=Y, ctx=ctx, eps=eps)


def test_precision_map_recomputed_from_exported_factor(mixed):
    m = mixed
    K = krr.krr_build_kernel(m["ctx"], _dev(m["G"]), m["w"].gamma, m["w"].lam)
    F = krr.krr_factor(m["ctx"], K, krr.Policy(eps=m["eps"]))
    info = krr.krr_factor_get_info(F)
    got = krr.krr_factor_precision_map(F)
    assert info.updates[krr.KRR_PREC_FP16] > 0 and info.updates[krr.KRR_PREC_FP8] > 0, \
        list(info.updates)
    L = krr.krr_factor_copy_l(F, 0, 0, m["n"], m["n"]).cpu().numpy()
    thr = m["eps"] * info.norm_a / m["nt"]
    _check_map(got, _rule_map(_panel_norms(L, m["nb"]), m["nt"], thr, high_panels=1))
    for q in range(3):
        assert int(np.sum(got == q)) == info.updates[q]
    # the mixed factor still gives the FP64 solution after refinement
    X, sinfo, _ = krr.krr_solve(m["ctx"], F, _dev(m["Y"]), krr.Refine(tol=1e-8))
    assert sinfo.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(m["G"], m["Y"], m["w"].gamma, m["w"].lam)) <= TOL


def test_fixed_map_replays_factor_bit_for_bit(mixed):
    m = mixed
    K1 = krr.krr_build_kernel(m["ctx"], _dev(m["G"]), m["w"].gamma, m["w"].lam)
    F1 = krr.krr_factor(m["ctx"], K1, krr.Policy(eps=m["eps"]))
    pmap = krr.krr_factor_precision_map(F1)
    L1 = krr.krr_factor_copy_l(F1, 0, 0, m["n"], m["n"])
    K2 = krr.krr_build_kernel(m["ctx"], _dev(m["G"]), m["w"].gamma, m["w"].lam)
    F2 = krr.krr_factor(m["ctx"], K2, krr.Policy(mode=krr.KRR_POLICY_FIXED_MAP, fixed_map=pmap))
    assert np.array_equal(krr.krr_factor_precision_map(F2), pmap)
    assert torch.equal(krr.krr_factor_copy_l(F2, 0, 0, m["n"], m["n"]), L1)
    # a map of the wrong size is rejected; the batched factorization takes none
    with pytest.raises(krr.KRRError) as e:
        krr.krr_factor(m["ctx"], K2, krr.Policy(mode=krr.KRR_POLICY_FIXED_MAP,
                                                fixed_map=pmap.ravel()[:-1]))
    assert e.value.status == krr.KRR_ERROR_INVALID_VALUE
    with pytest.raises(krr.KRRError) as e:
        krr.krr_factor_batched(m["ctx"], [K2], krr.Policy(mode=krr.KRR_POLICY_FIXED_MAP,
                                                          fixed_map=pmap))
    assert e.value.status == krr.KRR_ERROR_NOT_SUPPORTED


def test_tile_rule_map_from_build_norms(mixed):
    """KRR_RULE_TILE: u_p ||A_IJ||_F <= eps ||A||_F / NT with the build's tile norms."""
    m = mixed
    K = krr.krr_build_kernel(m["ctx"], _dev(m["G"]), m["w"].gamma, m["w"].lam)
    tn = krr.krr_kernel_tile_norms(K, m["nt"])
    nt = m["nt"]
    # eps between the FP8 thresholds of the off-diagonal tiles
    off = np.array([tn[_tri(i, j)] for i in range(nt) for j in range(i)])
    eps = float(np.median(U16 * off * nt / np.sqrt(np.sum(_full_sq(tn, nt)))))
    F = krr.krr_factor(m["ctx"], K, krr.Policy(eps=eps, rule=krr.KRR_RULE_TILE))
    info = krr.krr_factor_get_info(F)
    got = krr.krr_factor_precision_map(F)
    thr = eps * info.norm_a / nt
    want = np.full(got.shape, 255, np.int16)
    for k in range(nt):
        for j in range(k + 1, nt):
            for i in range(j, nt):
                if i == j or k < 1:
                    want[k, _tri(i, j)] = 0
                    continue
                a = tn[_tri(i, j)]
                p = 0
                if abs(U8 * a - thr) <= 1e-9 * thr or abs(U16 * a - thr) <= 1e-9 * thr:
                    p = -1
                elif U8 * a <= thr:
                    p = 2
                elif U16 * a <= thr:
                    p = 1
                want[k, _tri(i, j)] = p
    _check_map(got, want)
    assert info.updates[krr.KRR_PREC_FP16] > 0 and info.updates[krr.KRR_PREC_FP32] > 0
    X, sinfo, _ = krr.krr_solve(m["ctx"], F, _dev(m["Y"]), krr.Refine(tol=1e-8))
    assert sinfo.converged == 1


def _full_sq(tn, nt):
    """Squared tile norms of the whole symmetric matrix (off-diagonal tiles twice)."""
    sq = []
    for i in range(nt):
        for j in range(i + 1):
            sq.append(tn[_tri(i, j)] ** 2 * (1 if i == j else 2))
    return np.array(sq)


def test_promotion_cures_forced_fp8_breakdown():
    """FP8 on every off-diagonal update from the first panel on (high_panels = 0),
    without the per-tile scale, breaks the factorization down; with promotion the
    panels before the failing tile row move to FP16 and the solve reaches the FP64
    solution."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes()
    Y = w.phenotypes(G)
    ctx = krr.krr_create(0, tile=256)
    forced = dict(mode=krr.KRR_POLICY_FIXED, fixed_prec=krr.KRR_PREC_FP8, high_panels=0,
                  no_fp8_scale=1)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    with pytest.raises(krr.KRRError) as e:
        krr.krr_factor(ctx, K, krr.Policy(allow_promotion=0, **forced))
    assert e.value.status == krr.KRR_ERROR_NOT_POSITIVE_DEFINITE
    F = krr.krr_factor(ctx, K, krr.Policy(allow_promotion=1, **forced))
    info = krr.krr_factor_get_info(F)
    assert info.promotions >= 1 and info.breakdown_col >= 0
    pmap = krr.krr_factor_precision_map(F)
    X, sinfo, _ = krr.krr_solve(ctx, F, _dev(Y), krr.Refine(tol=1e-8))
    assert sinfo.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, w.gamma, w.lam)) <= TOL
    # promoted panels are FP16 (or FP32 after repeated promotion), never FP8
    brow = info.breakdown_col // 256
    assert not np.any(pmap[:max(brow, 1)] == krr.KRR_PREC_FP8)
    ctx.close()


def test_scaled_fp8_needs_no_promotion_where_unscaled_does():
    """The per-tile power-of-two scale keeps small L entries out of FP8's subnormal
    range: the same forced-FP8 policy with the scale factors without promotion."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes()
    ctx = krr.krr_create(0, tile=256)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    F = krr.krr_factor(ctx, K, krr.Policy(mode=krr.KRR_POLICY_FIXED, fixed_prec=krr.KRR_PREC_FP8,
                                          high_panels=1, allow_promotion=1))
    assert krr.krr_factor_get_info(F).promotions == 0
    ctx.close()


def test_factor_release_returns_every_buffer():
    """factor + solve + release, repeated under a workspace cap, never runs out and
    leaves the context's live allocation where it started."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=1500)
    Y = w.phenotypes(G)
    ctx = krr.krr_create(0, tile=256, workspace_limit=3 << 30)
    K = krr.krr_build_kernel(ctx, _dev(G), w.gamma, w.lam)
    base = None  # after the first release: the first factor consumed the build's matrix
    for _ in range(6):
        F = krr.krr_factor(ctx, K)
        krr.krr_solve(ctx, F, _dev(Y), krr.Refine(tol=1e-8))
        F.release()
        live = krr.krr_context_memory(ctx)[0]
        base = live if base is None else base
        assert live == base
    K.release()
    ctx.close()


def test_predict_batched_matches_single():
    w = synth.WORKLOADS["small"]
    ctx = krr.krr_create(0, tile=256)
    Ks, Ts, Xs, Ps = [], [], [], []
    for b, (n, nt_) in enumerate([(700, 90), (1300, 257), (300, 33)]):
        Gall = w.genotypes(rows=n + nt_, row0=10000 * b)
        G, T = Gall[:n], Gall[n:]
        K = krr.krr_build_kernel(ctx, _dev(G), (b + 1) / w.m, 0.1)
        X = np.random.default_rng(b).standard_normal((n, 3))
        Ks.append(K)
        Ts.append(_dev(T))
        Xs.append(_dev(X))
        Ps.append(oracle.predict(G, T, X, (b + 1) / w.m))
    got = krr.krr_predict_batched(ctx, Ks, Ts, Xs)
    for b in range(3):
        single = krr.krr_predict(ctx, Ks[b], Ts[b], Xs[b])
        assert torch.equal(got[b], single)
        assert _colrel(got[b].cpu().numpy(), Ps[b]) <= 1e-12
    ctx.close()


def test_caller_allocator_serves_every_device_buffer():
    """With a caller-supplied allocator (torch's caching allocator here) every
    library buffer comes from it, all of it is handed back at krr_destroy, and
    the results are those of the default allocator."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=900)
    Y = w.phenotypes(G)
    live = {}
    calls = {"alloc": 0, "free": 0}

    def alloc(nbytes):
        calls["alloc"] += 1
        p = torch.cuda.caching_allocator_alloc(nbytes, 0)
        live[p] = nbytes
        return p

    def free(p, nbytes):
        calls["free"] += 1
        assert live.pop(p) == nbytes
        torch.cuda.caching_allocator_delete(p)

    def run(c):
        K = krr.krr_build_kernel(c, _dev(G), w.gamma, w.lam)
        F = krr.krr_factor(c, K)
        X, info, _ = krr.krr_solve(c, F, _dev(Y), krr.Refine(tol=1e-8))
        X = X.clone()
        F.release()
        K.release()
        return X

    c1 = krr.krr_create(0, tile=256, allocator=(alloc, free))
    X1 = run(c1)
    assert calls["alloc"] > 0 and len(live) > 0  # cached in the context until destroy
    c1.close()
    assert not live and calls["alloc"] == calls["free"]
    c0 = krr.krr_create(0, tile=256)
    X0 = run(c0)
    c0.close()
    assert torch.equal(X1, X0)


def test_autotuner_searches_caches_and_applies(tmp_path):
    """The autotuner times whole steps over its candidates, leaves the best in the
    context, stores it under the problem's key, and a second call with the cache
    applies it without a search; results under the tuned schedule match the oracle."""
    w = synth.WORKLOADS["small"]
    G = w.genotypes(rows=1800)
    Y = w.phenotypes(G)
    ctx = krr.krr_create(0)
    cache = str(tmp_path / "tune.json")
    ref = krr.Refine(tol=1e-8)
    t1, ms1 = krr.krr_autotune(ctx, _dev(G), _dev(Y), w.gamma, w.lam, krr.Policy(), ref, cache)
    assert t1["tile"] in (256, 512) and ms1 > 0
    assert krr.krr_get_tuning(ctx) == t1
    import json
    doc = json.load(open(cache))
    assert len(doc) == 1 and list(doc.values())[0]["ms"] == pytest.approx(ms1, rel=1e-6)
    # cached: the same choice and time, no search
    ctx2 = krr.krr_create(0, tile=256 if t1["tile"] == 512 else 512)
    t2, ms2 = krr.krr_autotune(ctx2, _dev(G), _dev(Y), w.gamma, w.lam, krr.Policy(), ref, cache)
    assert t2 == t1 and ms2 == pytest.approx(ms1, rel=1e-6)
    assert krr.krr_get_tuning(ctx2) == t1
    K = krr.krr_build_kernel(ctx2, _dev(G), w.gamma, w.lam)
    F = krr.krr_factor(ctx2, K)
    X, info, _ = krr.krr_solve(ctx2, F, _dev(Y), ref)
    assert info.converged == 1
    assert _colrel(X.cpu().numpy(), oracle.fit(G, Y, w.gamma, w.lam)) <= TOL
    # the tile cannot change under live handles
    with pytest.raises(krr.KRRError):
        krr.krr_set_tuning(ctx2, tile=256 if t1["tile"] == 512 else 512)
    F.release()
    K.release()
    ctx.close()
    ctx2.close()


def test_stage_timer_mask_times_only_the_chosen_stages():
    """krr_timers_enable_stages: with only the Gram selected, a build + factor +
    solve records one Gram interval and nothing for the other stages; enabling
    every stage records the factorization's stages too."""
    n, m = 1100, 700
    G = synth.genotypes(n, m, synth.maf_uniform(m, 0.05, 0.5, 3), 3)
    Y = synth.phenotypes(G, 2, n_pairs=5, n_add=3, seed=4, h2=0.5)
    c = krr.krr_create(0, tile=256)
    Gd, Yd = _dev(G), _dev(Y)

    def run():
        K = krr.krr_build_kernel(c, Gd, 1.0 / m, 0.1)
        F = krr.krr_factor(c, K)
        krr.krr_solve(c, F, Yd)
        F.release()
        K.release()

    krr.krr_timers_enable_stages(c, ["gram"])
    run()
    st = krr.krr_timers_read(c)
    assert st["gram"][1] == 1 and st["gram"][0] > 0
    assert all(v[1] == 0 for k, v in st.items() if k != "gram")
    krr.krr_timers_enable(c, True)
    run()
    st = krr.krr_timers_read(c)
    assert st["gram"][1] == 1 and st["potrf"][1] > 0 and st["fwd_sweep"][1] > 0
    krr.krr_timers_enable(c, False)
    c.close()
