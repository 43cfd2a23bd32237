"""The no-allocation Predict entry point (krr_predict_noalloc) through the C ABI.

It must return exactly what krr_predict returns (the same kernels on buffers
carved from a fixed device scratch), allocate nothing, start clean on every
call although the scratch keeps the previous call's contents, and reject
inputs larger than its scratch before doing any work.
"""
import ctypes
import gc

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


def _case(n, nt, m, seed):
    p = synth.maf_uniform(m, 0.05, 0.5, seed)
    Gall = synth.genotypes(n + nt, m, p, seed)
    return Gall[:n], Gall[n:]


def _weights(n, r, seed):
    return np.random.default_rng(seed).standard_normal((n, r))


def _noalloc(ctx, K, T, X):
    """krr_predict_noalloc into a caller-made P, checking that neither the library
    nor torch allocated device memory during the call."""
    P = torch.full((X.shape[1], T.shape[0]), np.nan, dtype=torch.float64, device=DEV).t()
    torch.cuda.synchronize()
    # no collection of earlier tests' garbage may free torch memory during the call
    gc.collect()
    gc.disable()
    try:
        before_lib = krr.krr_context_memory(ctx)
        before_torch = torch.cuda.memory_allocated()
        out = krr.krr_predict_noalloc(ctx, K, T, X, P)
        torch.cuda.synchronize()
        after_lib = krr.krr_context_memory(ctx)
        after_torch = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    assert out.data_ptr() == P.data_ptr()
    assert after_lib == before_lib
    assert after_torch == before_torch
    return out.cpu().numpy()


def test_noalloc_predict_matches_predict_twice_then_smaller():
    ctx = krr.krr_create(0)
    n, m, gamma = 1500, 3000, 1.0 / 3000
    G, T = _case(n, 700, m, seed=31)
    K = krr.krr_build_kernel(ctx, _dev(G), gamma, 0.1)
    # first call: 700 test rows, 3 columns
    X1 = _weights(n, 3, 1)
    Td1, Xd1 = krr.padded_genotypes(_dev(T)), _dev(X1)
    Xd1 = krr._colmajor(Xd1, n)
    P_ref1 = krr.krr_predict(ctx, K, Td1, Xd1).cpu().numpy()
    P_na1 = _noalloc(ctx, K, Td1, Xd1)
    assert np.array_equal(P_na1, P_ref1)
    Po1 = oracle.predict(G, T, X1, gamma)
    assert np.max(np.abs(P_na1 - Po1)) <= 1e-12 * np.max(np.abs(Po1))
    # second call, smaller: 130 test rows, 2 columns; the scratch still holds call 1
    T2 = T[:130]
    X2 = _weights(n, 2, 2)
    Td2, Xd2 = krr.padded_genotypes(_dev(T2)), krr._colmajor(_dev(X2), n)
    P_ref2 = krr.krr_predict(ctx, K, Td2, Xd2).cpu().numpy()
    P_na2 = _noalloc(ctx, K, Td2, Xd2)
    assert np.array_equal(P_na2, P_ref2)
    Po2 = oracle.predict(G, T2, X2, gamma)
    assert np.max(np.abs(P_na2 - Po2)) <= 1e-12 * np.max(np.abs(Po2))
    K.release()
    ctx.close()


def test_noalloc_predict_chunked_rows_match_predict():
    """A training set wide enough that the scratch takes the test rows in several chunks."""
    ctx = krr.krr_create(0)
    n, m, gamma = 20000, 256, 1.0 / 256
    G, T = _case(n, 1000, m, seed=32)
    K = krr.krr_build_kernel(ctx, _dev(G), gamma, 0.05)
    X = _weights(n, 4, 3)
    Td, Xd = krr.padded_genotypes(_dev(T)), krr._colmajor(_dev(X), n)
    P_ref = krr.krr_predict(ctx, K, Td, Xd).cpu().numpy()
    P_na = _noalloc(ctx, K, Td, Xd)
    assert np.array_equal(P_na, P_ref)
    rows = np.arange(0, 1000, 97)
    Po = oracle.predict(G, T[rows], X, gamma)
    assert np.max(np.abs(P_na[rows] - Po)) <= 1e-12 * np.max(np.abs(Po))
    K.release()
    ctx.close()


def test_noalloc_predict_rejects_oversized_input_before_any_work():
    ctx = krr.krr_create(0)
    n, m = 600, 64
    G, T = _case(n, 8, m, seed=33)
    K = krr.krr_build_kernel(ctx, _dev(G), 1.0 / m, 0.1)
    Td = krr.padded_genotypes(_dev(T))
    X = krr._colmajor(_dev(_weights(n, 1, 4)), n)
    P = torch.zeros((8, 1), dtype=torch.float64, device=DEV)
    big = 20_000_000  # test-row norms alone exceed the scratch
    _, fits = krr.krr_noalloc_limits(n, big, 1)
    assert not fits
    st = krr.load().krr_predict_noalloc(ctx.handle, K.handle, Td.data_ptr(), big, Td.stride(0),
                                        X.data_ptr(), 1, n, P.data_ptr(), big)
    assert st == krr.KRR_ERROR_SCRATCH_TOO_SMALL
    torch.cuda.synchronize()
    assert torch.count_nonzero(P).item() == 0  # nothing was written
    # a bad genotype is reported as by krr_predict
    Tb = T.copy()
    Tb[3, 7] = 3
    with pytest.raises(krr.KRRError) as e:
        krr.krr_predict_noalloc(ctx, K, _dev(Tb), X)
    assert e.value.status == krr.KRR_ERROR_BAD_GENOTYPE
    # and the next good call is unaffected by the flag the bad one left set
    P_ref = krr.krr_predict(ctx, K, Td, X).cpu().numpy()
    assert np.array_equal(krr.krr_predict_noalloc(ctx, K, Td, X).cpu().numpy(), P_ref)
    K.release()
    ctx.close()
