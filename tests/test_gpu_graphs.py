"""HIP graphs of the batched calls: the batched factorization's lockstep launches
and the batched solve's sweeps are captured on the first call with a launch shape
and replayed afterwards.  Every replay, with other work and synchronizations of
the program between replays, must give exactly the result of direct launches."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2409_01712_amd as krr  # noqa: E402

DEV = "cuda:0"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_batched_graph_replays_match_direct_launches(monkeypatch):
    m, r = 700, 3
    ns = [1100, 700, 1500, 256, 900]
    w = synth.WORKLOADS["small"]
    p = synth.maf_uniform(m, 0.05, 0.5, 77)
    Gs = [synth.genotypes(n, m, p, 77, row0=5000 * b) for b, n in enumerate(ns)]
    Ys = [synth.phenotypes(G, r, n_pairs=5, n_add=5, seed=b, h2=0.5) for b, G in enumerate(Gs)]
    gammas = [(0.5, 1.0, 2.0)[b % 3] / m for b in range(len(ns))]
    lams = [(1e-2, 1e-1, 1.0)[b % 3] for b in range(len(ns))]
    ctx = krr.krr_create(0, tile=256)
    ref = krr.Refine(tol=1e-8)

    def run():
        Ks = krr.krr_build_kernel_batched(ctx, [_dev(G) for G in Gs], gammas, lams)
        Fs = krr.krr_factor_batched(ctx, Ks)
        Xs, infos, st = krr.krr_solve_batched(ctx, Fs, [_dev(Y) for Y in Ys], ref)
        assert st == krr.KRR_SUCCESS and all(i.converged == 1 for i in infos)
        out = [X.clone() for X in Xs]
        for F in Fs:
            F.release()
        for K in Ks:
            K.release()
        return out

    monkeypatch.setenv("KRR_NO_GRAPH", "1")
    X_direct = run()
    assert krr.krr_context_graphs(ctx) == (0, 0)
    monkeypatch.delenv("KRR_NO_GRAPH")
    for rep in range(3):
        X = run()
        cached, launches = krr.krr_context_graphs(ctx)
        assert cached >= 2 and launches >= 2 * (rep + 1)
        for b in range(len(ns)):
            assert torch.equal(X[b], X_direct[b]), (rep, b)
        # other work of the program between replays, then a synchronization
        K = krr.krr_build_kernel(ctx, _dev(Gs[0]), gammas[0], lams[0])
        F = krr.krr_factor(ctx, K)
        krr.krr_solve(ctx, F, _dev(Ys[0]), ref)
        F.release()
        K.release()
        torch.cuda.synchronize()
    # the replayed result is the FP64 solution
    for b in (0, 2):
        Wo = oracle.fit(Gs[b], Ys[b], gammas[b], lams[b])
        assert np.max(np.abs(X[b].cpu().numpy() - Wo)) <= 1e-5 * np.max(np.abs(Wo))
    ctx.close()


@pytest.mark.skip(reason="the single-instance factorization's HIP graph is switched off "
                  "(KRR_FACTOR_GRAPH=1 returns KRR_ERROR_NOT_SUPPORTED): its first GPU runs "
                  "ended with a host segmentation fault inside krr_factor during the first "
                  "capture, also after moving the kernel attributes and event creation out of "
                  "the capture, and the cause is not known")
@pytest.mark.parametrize("n,tile", [(2600, 256), (3000, 512)])
def test_factor_graph_replays_match_direct_launches(monkeypatch, n, tile):
    """The single-instance factorization's three-stream schedule runs as a HIP
    graph (captured on the first call with a key of every address and value its
    launches take, replayed after).  Every replay -- with other work of the
    program and synchronizations between replays -- gives the bits of direct
    launches: the factor's solve, the update counts and the precision map."""
    m, r = 700, 4
    G = synth.genotypes(n, m, synth.maf_uniform(m, 0.05, 0.5, 5), 5)
    Y = synth.phenotypes(G, r, n_pairs=5, n_add=5, seed=6, h2=0.5)
    gamma, lam = 1.0 / m, 0.1
    ctx = krr.krr_create(0, tile=tile)
    none = krr.Refine(method=krr.KRR_REFINE_NONE)

    def run():
        K = krr.krr_build_kernel(ctx, _dev(G), gamma, lam)
        F = krr.krr_factor(ctx, K)
        X, _, _ = krr.krr_solve(ctx, F, _dev(Y), none)
        info = krr.krr_factor_get_info(F)
        out = (X.clone(), tuple(info.updates), krr.krr_factor_precision_map(F))
        F.release()
        K.release()
        return out

    monkeypatch.setenv("KRR_NO_GRAPH", "1")
    X0, u0, m0 = run()
    assert krr.krr_context_graphs(ctx) == (0, 0)
    monkeypatch.delenv("KRR_NO_GRAPH")
    for rep in range(4):
        X, u, pm = run()
        assert torch.equal(X, X0), rep
        assert u == u0 and np.array_equal(pm, m0), rep
        # other work of the program between replays, then a synchronization
        Kb = krr.krr_build_kernel(ctx, _dev(G[: n // 2]), gamma, lam)
        Fb = krr.krr_factor(ctx, Kb, krr.plain_fp32_policy())
        krr.krr_solve(ctx, Fb, _dev(Y[: n // 2]), none)
        Fb.release()
        Kb.release()
        torch.cuda.synchronize()
    cached, launches = krr.krr_context_graphs(ctx)
    # eight graphed factorizations, most of them replays of a cached graph
    assert launches >= 8 and cached < launches
    ctx.close()
