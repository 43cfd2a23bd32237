"""MI355X (gfx950) kernel ridge regression for multivariate GWAS.

Python binding over the C ABI in include/krr.h (libkrr.so, built in-tree by
``paper_2409_01712_amd.build``).  The functions carry the C names and only
marshal arguments: torch tensors provide device memory and the stream, every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkrr.so")

# status codes (krr_status)
KRR_SUCCESS = 0
KRR_ERROR_INVALID_VALUE = 1
KRR_ERROR_BAD_GENOTYPE = 2
KRR_ERROR_OUT_OF_MEMORY = 3
KRR_ERROR_NOT_POSITIVE_DEFINITE = 4
KRR_ERROR_NOT_CONVERGED = 5
KRR_ERROR_HIP = 6
KRR_ERROR_NOT_SUPPORTED = 7
KRR_ERROR_SCRATCH_TOO_SMALL = 8
KRR_NOALLOC_SCRATCH_BYTES = 64 << 20

KRR_PREC_FP32, KRR_PREC_FP16, KRR_PREC_FP8 = 0, 1, 2
KRR_POLICY_FP32, KRR_POLICY_ADAPTIVE, KRR_POLICY_FIXED, KRR_POLICY_FIXED_MAP = 0, 1, 2, 3
KRR_RULE_OPERAND, KRR_RULE_TILE, KRR_RULE_BOTH = 0, 1, 2
KRR_KERNEL_GAUSSIAN, KRR_KERNEL_IBS, KRR_KERNEL_LINEAR = 0, 1, 2
KRR_REFINE_NONE, KRR_REFINE_IR, KRR_REFINE_PCG, KRR_REFINE_AUTO = 0, 1, 2, 3


KRR_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)
KRR_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)


class krr_options(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("workspace_limit", ctypes.c_int64), ("device_alloc", KRR_ALLOC_FN),
                ("device_free", KRR_FREE_FN), ("alloc_user", ctypes.c_void_p)]


class krr_precision_policy(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("allowed", ctypes.c_int32), ("eps", ctypes.c_double),
                ("high_panels", ctypes.c_int32), ("fixed_prec", ctypes.c_int32),
                ("allow_promotion", ctypes.c_int32), ("diag_fp64", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("no_fp8_scale", ctypes.c_int32),
                ("fixed_map", ctypes.c_void_p), ("fixed_map_count", ctypes.c_int64)]


class krr_kernel_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("C", ctypes.c_void_p),
                ("q", ctypes.c_int64), ("ldc", ctypes.c_int64)]


class krr_tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("panel_group", ctypes.c_int32),
                ("residual_split", ctypes.c_int32), ("sweep_pairs", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("aux_cu_eighths", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class krr_refine_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double)]


class krr_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("fwd_err_bound", ctypes.c_double), ("backward_err", ctypes.c_double),
                ("first_bound", ctypes.c_double)]


class krr_factor_info(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_int64 * 3), ("promotions", ctypes.c_int32),
                ("breakdown_col", ctypes.c_int64), ("nt", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("norm_a", ctypes.c_double)]


_lib = None

# (name, restype, argtypes) for every entry point of include/krr.h
_P, _I64, _D, _I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
_SIGS = [
    ("krr_create", _I, [ctypes.POINTER(_P), _I, _P, ctypes.POINTER(krr_options)]),
    ("krr_destroy", _I, [_P]),
    ("krr_set_stream", _I, [_P, _P]),
    ("krr_build_kernel", _I, [_P, _P, _I64, _I64, _I64, _D, _D, ctypes.POINTER(_P)]),
    ("krr_build_kernel_ex", _I, [_P, _P, _I64, _I64, _I64, _D, _D,
                                 ctypes.POINTER(krr_kernel_desc), ctypes.POINTER(_P)]),
    ("krr_kernel_release", _I, [_P]),
    ("krr_factor", _I, [_P, _P, ctypes.POINTER(krr_precision_policy), ctypes.POINTER(_P)]),
    ("krr_factor_release", _I, [_P]),
    ("krr_factor_get_info", _I, [_P, ctypes.POINTER(krr_factor_info)]),
    ("krr_solve", _I, [_P, _P, _P, _I64, _I64, _P, _I64, ctypes.POINTER(krr_refine_opts),
                       ctypes.POINTER(krr_solve_info)]),
    ("krr_predict", _I, [_P, _P, _P, _I64, _I64, _P, _I64, _I64, _P, _I64]),
    ("krr_predict_ex", _I, [_P, _P, _P, _I64, _I64, _P, _I64, _P, _I64, _I64, _P, _I64]),
    ("krr_predict_batched", _I, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _I64, _P, _P, _P]),
    ("krr_predict_noalloc", _I, [_P, _P, _P, _I64, _I64, _P, _I64, _I64, _P, _I64]),
    ("krr_noalloc_limits", _I, [_I64, _I64, _I64, ctypes.c_int32, ctypes.POINTER(_I64),
                                ctypes.POINTER(ctypes.c_int32)]),
    ("krr_context_memory", _I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    ("krr_context_graphs", _I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    ("krr_build_kernel_batched", _I, [_P, ctypes.c_int32, _P, _P, _I64, _P, _P, _P, _P]),
    ("krr_factor_batched", _I, [_P, ctypes.c_int32, _P, ctypes.POINTER(krr_precision_policy),
                                _P]),
    ("krr_solve_batched", _I, [_P, ctypes.c_int32, _P, _P, _I64, _P, _P, _P,
                               ctypes.POINTER(krr_refine_opts), _P]),
    ("krr_rr_fit", _I, [_P, _P, _I64, _I64, _I64, _P, _I64, _I64, _D,
                        ctypes.POINTER(krr_precision_policy), ctypes.POINTER(krr_refine_opts), _P,
                        _I64, ctypes.POINTER(krr_solve_info)]),
    ("krr_rr_predict", _I, [_P, _P, _I64, _I64, _I64, _P, _I64, _I64, _P, _I64]),
    ("krr_kernel_copy_distances", _I, [_P, _I64, _I64, _I64, _I64, _P, _I64]),
    ("krr_kernel_copy_matrix", _I, [_P, _I64, _I64, _I64, _I64, _P, _I64]),
    ("krr_factor_copy_l", _I, [_P, _I64, _I64, _I64, _I64, _P, _I64]),
    ("krr_kernel_tile_norms", _I, [_P, _P, _I64]),
    ("krr_factor_precision_map", _I, [_P, _P, _I64]),
    ("krr_debug_encode_fp8", _I, [_P, _P, _I64, _P]),
    ("krr_set_tuning", _I, [_P, ctypes.POINTER(krr_tuning)]),
    ("krr_get_tuning", _I, [_P, ctypes.POINTER(krr_tuning)]),
    ("krr_autotune", _I, [_P, _P, _I64, _I64, _I64, _D, _D, _P, _I64, _I64,
                          ctypes.POINTER(krr_precision_policy), ctypes.POINTER(krr_refine_opts),
                          ctypes.c_char_p, ctypes.POINTER(krr_tuning), ctypes.POINTER(_D)]),
    ("krr_tuning_key", _I, [_I, _I64, _I64, _I64, ctypes.POINTER(krr_precision_policy),
                            ctypes.POINTER(krr_refine_opts), ctypes.c_char_p, ctypes.c_int32]),
    ("krr_tuning_cache_store", _I, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(krr_tuning),
                                    _D]),
    ("krr_tuning_cache_load", _I, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(krr_tuning),
                                   ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int32)]),
    ("krr_timers_enable", _I, [_P, ctypes.c_int32]),
    ("krr_timers_enable_stages", _I, [_P, ctypes.c_uint32]),
    ("krr_timers_read", _I, [_P, _P, _P, ctypes.c_int32]),
    ("krr_stage_name", ctypes.c_char_p, [ctypes.c_int32]),
    ("krr_status_string", ctypes.c_char_p, [_I]),
]

KRR_STAGE_COUNT = 11


def load():
    """Load libkrr.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("libkrr.so is not built: run paper_2409_01712_amd.build.build() "
                          "(hipcc --offload-arch=gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class KRRError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = load().krr_status_string(status).decode()
        super().__init__("%s: %s (status %d)" % (where, msg, status))


def _check(status: int, where: str):
    if status != KRR_SUCCESS:
        raise KRRError(status, where)


def _ptr(t) -> int:
    return t.data_ptr()


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# Live handles, released in dependency order (factors, kernels, contexts) at
# interpreter exit, before the HIP runtime is torn down.
_live = {"factor": weakref.WeakSet(), "kernel": weakref.WeakSet(), "context": weakref.WeakSet()}
_exiting = False


@atexit.register
def _release_all():
    global _exiting
    for kind in ("factor", "kernel", "context"):
        for h in list(_live[kind]):
            try:
                h._free()
            except Exception:
                pass
    _exiting = True


class _Handle:
    kind = ""

    def __init__(self, handle):
        self.handle = handle
        _live[self.kind].add(self)

    def _free(self):
        if self.handle and not _exiting:
            getattr(load(), self._release_fn)(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self._free()
        except Exception:
            pass


class Context(_Handle):
    kind, _release_fn = "context", "krr_destroy"

    def __init__(self, handle, device):
        super().__init__(handle)
        self.device = device

    def close(self):
        self._free()


class Kernel(_Handle):
    """Device-resident kernel matrix; keeps the genotype tensor and the context alive."""
    kind, _release_fn = "kernel", "krr_kernel_release"

    def __init__(self, handle, ctx, G, n, m, gamma, lam):
        super().__init__(handle)
        self.ctx, self.G = ctx, G
        self.n, self.m, self.gamma, self.lam = n, m, gamma, lam

    def release(self):
        self._free()


class Factor(_Handle):
    """Cholesky factor; keeps its kernel alive (solves read the kernel's distances)."""
    kind, _release_fn = "factor", "krr_factor_release"

    def __init__(self, handle, kernel):
        super().__init__(handle)
        self.kernel = kernel

    def release(self):
        self._free()


@dataclass
class Policy:
    mode: int = KRR_POLICY_ADAPTIVE
    allowed: int = (1 << KRR_PREC_FP16) | (1 << KRR_PREC_FP8)
    eps: float = 1.0
    high_panels: int = 1
    fixed_prec: int = KRR_PREC_FP16
    allow_promotion: int = 1
    diag_fp64: int = 1
    rule: int = KRR_RULE_OPERAND
    no_fp8_scale: int = 0
    fixed_map: object = None  # numpy uint8 array (FIXED_MAP)

    def c(self):
        pol = krr_precision_policy(self.mode, self.allowed, self.eps, self.high_panels,
                                   self.fixed_prec, self.allow_promotion, self.diag_fp64,
                                   self.rule, self.no_fp8_scale, None, 0)
        if self.fixed_map is not None:
            import numpy as np
            fm = np.ascontiguousarray(self.fixed_map, dtype=np.uint8)
            pol.fixed_map = fm.ctypes.data
            pol.fixed_map_count = fm.size
            pol._keep = fm  # the array outlives the call through the struct
        return pol


def plain_fp32_policy() -> Policy:
    """Every update and the diagonal POTRF in FP32: the plain single-precision path."""
    return Policy(mode=KRR_POLICY_FP32, allowed=0, diag_fp64=0, allow_promotion=0)


@dataclass
class Refine:
    method: int = KRR_REFINE_IR
    max_iters: int = 30
    tol: float = 1e-6

    def c(self):
        return krr_refine_opts(self.method, self.max_iters, self.tol)


def krr_create(device: int = 0, stream=None, tile: int = 512, verbose: int = 0,
               workspace_limit: int = 0, allocator=None) -> Context:
    """allocator: optional (alloc(bytes) -> int device pointer, free(ptr, bytes)) pair of
    Python callables the library uses instead of hipMalloc/hipFree."""
    lib = load()
    h = ctypes.c_void_p()
    opts = krr_options(tile, verbose, workspace_limit)
    keep = None
    if allocator is not None:
        alloc, free = allocator
        keep = (KRR_ALLOC_FN(lambda b, u: alloc(int(b)) or None),
                KRR_FREE_FN(lambda p, b, u: free(int(p), int(b))))
        opts.device_alloc, opts.device_free = keep
    _check(lib.krr_create(ctypes.byref(h), device, _stream_handle(stream), ctypes.byref(opts)),
           "krr_create")
    c = Context(h, device)
    c._alloc_fns = keep  # the callbacks live as long as the context
    return c


def krr_set_stream(ctx: Context, stream=None):
    _check(load().krr_set_stream(ctx.handle, _stream_handle(stream)), "krr_set_stream")


def padded_genotypes(G):
    """Return G (int8, n x m, on the GPU) with a row pitch that is a multiple of 16 bytes."""
    import torch
    assert G.dtype == torch.int8 and G.dim() == 2 and G.is_cuda
    n, m = G.shape
    if G.stride(1) == 1 and G.stride(0) % 16 == 0 and G.stride(0) >= m and G.data_ptr() % 16 == 0:
        return G
    pitch = (m + 15) // 16 * 16
    buf = torch.zeros((n, pitch), dtype=torch.int8, device=G.device)
    buf[:, :m] = G
    return buf[:, :m]


def krr_set_tuning(ctx: Context, tile=512, panel_group=0, residual_split=0, sweep_pairs=-1,
                   lookahead=-1, aux_cu_eighths=0):
    t = krr_tuning(tile, panel_group, residual_split, sweep_pairs, lookahead, aux_cu_eighths)
    _check(load().krr_set_tuning(ctx.handle, ctypes.byref(t)), "krr_set_tuning")


def krr_get_tuning(ctx: Context) -> dict:
    t = krr_tuning()
    _check(load().krr_get_tuning(ctx.handle, ctypes.byref(t)), "krr_get_tuning")
    return t.as_dict()


def krr_autotune(ctx: Context, G, Y, gamma: float, lam: float, policy: Policy | None = None,
                 refine: Refine | None = None, cache_path: str | None = None):
    """Search the context's schedule choices on this problem (see include/krr.h);
    returns (tuning dict, best step time in ms)."""
    G = padded_genotypes(G)
    n, m = G.shape
    Yc = _colmajor(Y, n)
    t = krr_tuning()
    ms = ctypes.c_double()
    pol = (policy or Policy()).c()
    ref = (refine or Refine()).c()
    _check(load().krr_autotune(ctx.handle, _ptr(G), n, m, G.stride(0), float(gamma), float(lam),
                               _ptr(Yc), Yc.shape[1], n, ctypes.byref(pol), ctypes.byref(ref),
                               cache_path.encode() if cache_path else None, ctypes.byref(t),
                               ctypes.byref(ms)), "krr_autotune")
    return t.as_dict(), float(ms.value)


def krr_tuning_cache_store(path: str, key: str, tuning: dict, ms: float):
    t = krr_tuning(*(int(tuning[f]) for f, _ in krr_tuning._fields_))
    _check(load().krr_tuning_cache_store(path.encode(), key.encode(), ctypes.byref(t), ms),
           "krr_tuning_cache_store")


def krr_tuning_cache_load(path: str, key: str):
    """(tuning dict, ms), or None when the key is not in the file."""
    t = krr_tuning()
    ms = ctypes.c_double()
    found = ctypes.c_int32()
    _check(load().krr_tuning_cache_load(path.encode(), key.encode(), ctypes.byref(t),
                                        ctypes.byref(ms), ctypes.byref(found)),
           "krr_tuning_cache_load")
    return (t.as_dict(), float(ms.value)) if found.value else None


def krr_timers_enable(ctx: Context, enable: bool = True):
    _check(load().krr_timers_enable(ctx.handle, 1 if enable else 0), "krr_timers_enable")


def krr_timers_enable_stages(ctx: Context, stages):
    """Time only the named stages (names as krr_timers_read returns them)."""
    lib = load()
    names = {lib.krr_stage_name(i).decode(): i for i in range(KRR_STAGE_COUNT)}
    mask = 0
    for s in stages:
        mask |= 1 << names[s]
    _check(lib.krr_timers_enable_stages(ctx.handle, mask), "krr_timers_enable_stages")


def krr_timers_read(ctx: Context) -> dict:
    """{stage name: (total GPU ms, number of timed intervals)} since the last enable."""
    import numpy as np
    ms = np.zeros(KRR_STAGE_COUNT, np.float64)
    cnt = np.zeros(KRR_STAGE_COUNT, np.int64)
    lib = load()
    _check(lib.krr_timers_read(ctx.handle, ms.ctypes.data, cnt.ctypes.data, KRR_STAGE_COUNT),
           "krr_timers_read")
    return {lib.krr_stage_name(i).decode(): (float(ms[i]), int(cnt[i]))
            for i in range(KRR_STAGE_COUNT)}


def krr_build_kernel(ctx: Context, G, gamma: float, lam: float) -> Kernel:
    G = padded_genotypes(G)
    n, m = G.shape
    h = ctypes.c_void_p()
    _check(load().krr_build_kernel(ctx.handle, _ptr(G), n, m, G.stride(0), float(gamma),
                                   float(lam), ctypes.byref(h)), "krr_build_kernel")
    return Kernel(h, ctx, G, n, m, gamma, lam)


def krr_build_kernel_ex(ctx: Context, G, gamma: float, lam: float, kind: int = KRR_KERNEL_GAUSSIAN,
                        C=None) -> Kernel:
    """Build with a kernel type of Algorithm 5 (KRR_KERNEL_GAUSSIAN / KRR_KERNEL_IBS) and,
    for the Gaussian kernel, optional confounders C (n x q float64 on the GPU)."""
    import torch
    G = padded_genotypes(G)
    n, m = G.shape
    desc = krr_kernel_desc(kind, 0, None, 0, 0)
    Cd = None
    if C is not None:
        Cd = C.to(torch.float64)
        if Cd.dim() == 1:
            Cd = Cd[:, None]
        Cd = Cd.contiguous()
        assert Cd.shape[0] == n
        desc.C, desc.q, desc.ldc = Cd.data_ptr(), Cd.shape[1], Cd.shape[1]
    h = ctypes.c_void_p()
    _check(load().krr_build_kernel_ex(ctx.handle, _ptr(G), n, m, G.stride(0), float(gamma),
                                      float(lam), ctypes.byref(desc), ctypes.byref(h)),
           "krr_build_kernel_ex")
    K = Kernel(h, ctx, G, n, m, gamma, lam)
    K.kind, K.q = kind, (0 if Cd is None else Cd.shape[1])
    return K


def krr_factor(ctx: Context, K: Kernel, policy: Policy | None = None) -> Factor:
    h = ctypes.c_void_p()
    pol = (policy or Policy()).c()
    _check(load().krr_factor(ctx.handle, K.handle, ctypes.byref(pol), ctypes.byref(h)),
           "krr_factor")
    return Factor(h, K)


def krr_factor_get_info(F: Factor) -> krr_factor_info:
    info = krr_factor_info()
    _check(load().krr_factor_get_info(F.handle, ctypes.byref(info)), "krr_factor_get_info")
    return info


def _colmajor(Y, n):
    import torch
    Y = Y.to(torch.float64)
    if Y.dim() == 1:
        Y = Y[:, None]
    assert Y.shape[0] == n
    return Y.t().contiguous().t()  # column-major, leading dimension n


def krr_solve(ctx: Context, F: Factor, Y, refine: Refine | None = None, check: bool = True):
    """Solve (K + lambda I) X = Y; returns (X, info).  Y: (n, r) float64 on the GPU."""
    import torch
    n = F.kernel.n
    Yc = _colmajor(Y, n)
    r = Yc.shape[1]
    X = torch.empty((r, n), dtype=torch.float64, device=Yc.device).t()
    info = krr_solve_info()
    opts = (refine or Refine()).c()
    st = load().krr_solve(ctx.handle, F.handle, _ptr(Yc), r, n, _ptr(X), n, ctypes.byref(opts),
                          ctypes.byref(info))
    if check:
        _check(st, "krr_solve")
    return X, info, st


def _host_array(ctype, values):
    return (ctype * len(values))(*values)


def krr_build_kernel_batched(ctx: Context, Gs, gammas, lams) -> list:
    """Kernels of len(Gs) instances sharing the SNP count (one launch per Build stage)."""
    Gs = [padded_genotypes(G) for G in Gs]
    B = len(Gs)
    m = Gs[0].shape[1]
    assert all(G.shape[1] == m for G in Gs) and len(gammas) == B and len(lams) == B
    out = (ctypes.c_void_p * B)()
    _check(load().krr_build_kernel_batched(
        ctx.handle, B, _host_array(ctypes.c_void_p, [_ptr(G) for G in Gs]),
        _host_array(ctypes.c_int64, [G.shape[0] for G in Gs]), m,
        _host_array(ctypes.c_int64, [G.stride(0) for G in Gs]),
        _host_array(ctypes.c_double, [float(g) for g in gammas]),
        _host_array(ctypes.c_double, [float(x) for x in lams]), out), "krr_build_kernel_batched")
    return [Kernel(ctypes.c_void_p(out[b]), ctx, Gs[b], Gs[b].shape[0], m, gammas[b], lams[b])
            for b in range(B)]


def krr_factor_batched(ctx: Context, Ks, policy: Policy | None = None) -> list:
    B = len(Ks)
    out = (ctypes.c_void_p * B)()
    pol = (policy or Policy()).c()
    _check(load().krr_factor_batched(ctx.handle, B,
                                     _host_array(ctypes.c_void_p, [K.handle.value for K in Ks]),
                                     ctypes.byref(pol), out), "krr_factor_batched")
    return [Factor(ctypes.c_void_p(out[b]), Ks[b]) for b in range(B)]


def krr_solve_batched(ctx: Context, Fs, Ys, refine: Refine | None = None, check: bool = True):
    """Solve every instance; returns ([X_b], [info_b], status).  Ys[b]: (n_b, r) float64."""
    import torch
    B = len(Fs)
    Yc = [_colmajor(Y, F.kernel.n) for Y, F in zip(Ys, Fs)]
    r = Yc[0].shape[1]
    assert all(Y.shape[1] == r for Y in Yc)
    Xs = [torch.empty((r, F.kernel.n), dtype=torch.float64, device=Y.device).t()
          for F, Y in zip(Fs, Yc)]
    infos = (krr_solve_info * B)()
    opts = (refine or Refine()).c()
    lds = _host_array(ctypes.c_int64, [F.kernel.n for F in Fs])
    st = load().krr_solve_batched(ctx.handle, B,
                                  _host_array(ctypes.c_void_p, [F.handle.value for F in Fs]),
                                  _host_array(ctypes.c_void_p, [_ptr(Y) for Y in Yc]), r, lds,
                                  _host_array(ctypes.c_void_p, [_ptr(X) for X in Xs]), lds,
                                  ctypes.byref(opts), infos)
    if check:
        _check(st, "krr_solve_batched")
    return Xs, [infos[b] for b in range(B)], st


def krr_predict(ctx: Context, K: Kernel, T, X):
    """P = K_test X with K_test built from test genotypes T (n_test x m, int8, GPU)."""
    import torch
    T = padded_genotypes(T)
    nt, m = T.shape
    assert m == K.m
    Xc = _colmajor(X, K.n)
    r = Xc.shape[1]
    P = torch.empty((r, nt), dtype=torch.float64, device=Xc.device).t()
    _check(load().krr_predict(ctx.handle, K.handle, _ptr(T), nt, T.stride(0), _ptr(Xc), r, K.n,
                              _ptr(P), nt), "krr_predict")
    return P


def krr_predict_ex(ctx: Context, K: Kernel, T, X, Ct=None):
    """P = K_test X for any kernel of krr_build_kernel_ex; Ct: the test rows' confounders."""
    import torch
    T = padded_genotypes(T)
    nt, m = T.shape
    assert m == K.m
    Xc = _colmajor(X, K.n)
    r = Xc.shape[1]
    P = torch.empty((r, nt), dtype=torch.float64, device=Xc.device).t()
    Ctd, ldct = None, 0
    if Ct is not None:
        Ctd = Ct.to(torch.float64)
        if Ctd.dim() == 1:
            Ctd = Ctd[:, None]
        Ctd = Ctd.contiguous()
        ldct = Ctd.shape[1]
    _check(load().krr_predict_ex(ctx.handle, K.handle, _ptr(T), nt, T.stride(0),
                                 _ptr(Ctd) if Ctd is not None else None, ldct, _ptr(Xc), r, K.n,
                                 _ptr(P), nt), "krr_predict_ex")
    return P


def krr_predict_batched(ctx: Context, Ks, Ts, Xs) -> list:
    """[P_b] = [K_test,b X_b] for every instance (test genotypes Ts[b], weights Xs[b])."""
    import torch
    B = len(Ks)
    Ts = [padded_genotypes(T) for T in Ts]
    Xc = [_colmajor(X, K.n) for X, K in zip(Xs, Ks)]
    r = Xc[0].shape[1]
    assert all(X.shape[1] == r for X in Xc) and len(Ts) == B
    Ps = [torch.empty((r, T.shape[0]), dtype=torch.float64, device=T.device).t() for T in Ts]
    _check(load().krr_predict_batched(
        ctx.handle, B, _host_array(ctypes.c_void_p, [K.handle.value for K in Ks]),
        _host_array(ctypes.c_void_p, [_ptr(T) for T in Ts]),
        _host_array(ctypes.c_int64, [T.shape[0] for T in Ts]),
        _host_array(ctypes.c_int64, [T.stride(0) for T in Ts]),
        _host_array(ctypes.c_void_p, [_ptr(X) for X in Xc]), r,
        _host_array(ctypes.c_int64, [K.n for K in Ks]),
        _host_array(ctypes.c_void_p, [_ptr(P) for P in Ps]),
        _host_array(ctypes.c_int64, [T.shape[0] for T in Ts])), "krr_predict_batched")
    return Ps


def krr_predict_noalloc(ctx: Context, K: Kernel, T, X, P=None):
    """krr_predict through the no-allocation entry point: the library allocates
    nothing; P (n_test x r, float64, column-major) may be passed in by the caller."""
    import torch
    T = padded_genotypes(T)
    nt, m = T.shape
    assert m == K.m
    Xc = _colmajor(X, K.n)
    r = Xc.shape[1]
    if P is None:
        P = torch.empty((r, nt), dtype=torch.float64, device=Xc.device).t()
    assert P.shape == (nt, r) and P.stride(0) == 1 and P.dtype == torch.float64
    _check(load().krr_predict_noalloc(ctx.handle, K.handle, _ptr(T), nt, T.stride(0), _ptr(Xc), r,
                                      K.n, _ptr(P), P.stride(1)), "krr_predict_noalloc")
    return P


def krr_noalloc_limits(n: int, n_test: int, nrhs: int, tile: int = 512):
    """(scratch bytes, whether krr_predict_noalloc accepts these sizes); host only."""
    b = ctypes.c_int64()
    f = ctypes.c_int32()
    _check(load().krr_noalloc_limits(n, n_test, nrhs, tile, ctypes.byref(b), ctypes.byref(f)),
           "krr_noalloc_limits")
    return int(b.value), bool(f.value)


def krr_context_memory(ctx: Context):
    """(bytes in live library buffers, bytes in the context's block cache)."""
    a, c = ctypes.c_int64(), ctypes.c_int64()
    _check(load().krr_context_memory(ctx.handle, ctypes.byref(a), ctypes.byref(c)),
           "krr_context_memory")
    return int(a.value), int(c.value)


def krr_rr_fit(ctx: Context, G, Y, lam: float, policy: Policy | None = None,
               refine: Refine | None = None, check: bool = True):
    """Ridge Regression (Eq. 2): beta = (X^T X + lambda I)^-1 X^T Y with X = G (n x m int8
    on the GPU); returns (beta (m x r float64), info, status)."""
    import torch
    G = padded_genotypes(G)
    n, m = G.shape
    Yc = _colmajor(Y, n)
    r = Yc.shape[1]
    beta = torch.empty((r, m), dtype=torch.float64, device=Yc.device).t()
    info = krr_solve_info()
    pol = (policy or Policy()).c()
    ref = (refine or Refine()).c()
    st = load().krr_rr_fit(ctx.handle, _ptr(G), n, m, G.stride(0), _ptr(Yc), r, n, float(lam),
                           ctypes.byref(pol), ctypes.byref(ref), _ptr(beta), m,
                           ctypes.byref(info))
    if check:
        _check(st, "krr_rr_fit")
    return beta, info, st


def krr_rr_predict(ctx: Context, T, beta):
    """P = T beta for test genotypes T (n_test x m int8 on the GPU)."""
    import torch
    T = padded_genotypes(T)
    nt, m = T.shape
    B = _colmajor(beta, m)
    r = B.shape[1]
    P = torch.empty((r, nt), dtype=torch.float64, device=B.device).t()
    _check(load().krr_rr_predict(ctx.handle, _ptr(T), nt, m, T.stride(0), _ptr(B), r, m, _ptr(P),
                                 nt), "krr_rr_predict")
    return P


def krr_context_graphs(ctx: Context):
    """(graphs the context keeps instantiated, graph launches so far)."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().krr_context_graphs(ctx.handle, ctypes.byref(a), ctypes.byref(b)),
           "krr_context_graphs")
    return int(a.value), int(b.value)


def krr_debug_encode_fp8(ctx: Context, x):
    """FP8 E4M3FN bytes of a float32 GPU tensor, from the library's encoder."""
    import torch
    x = x.to(torch.float32).contiguous()
    out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    _check(load().krr_debug_encode_fp8(ctx.handle, _ptr(x), x.numel(), _ptr(out)),
           "krr_debug_encode_fp8")
    return out


def krr_kernel_copy_distances(K: Kernel, i0: int, j0: int, rows: int, cols: int):
    import torch
    out = torch.empty((rows, cols), dtype=torch.int32, device=K.G.device)
    _check(load().krr_kernel_copy_distances(K.handle, i0, j0, rows, cols, _ptr(out), cols),
           "krr_kernel_copy_distances")
    return out


def krr_kernel_copy_matrix(K: Kernel, i0: int, j0: int, rows: int, cols: int):
    import torch
    out = torch.empty((rows, cols), dtype=torch.float32, device=K.G.device)
    _check(load().krr_kernel_copy_matrix(K.handle, i0, j0, rows, cols, _ptr(out), cols),
           "krr_kernel_copy_matrix")
    return out


def krr_factor_copy_l(F: Factor, i0: int, j0: int, rows: int, cols: int):
    import torch
    out = torch.empty((rows, cols), dtype=torch.float32, device=F.kernel.G.device)
    _check(load().krr_factor_copy_l(F.handle, i0, j0, rows, cols, _ptr(out), cols),
           "krr_factor_copy_l")
    return out


def krr_kernel_tile_norms(K: Kernel, nt: int):
    import numpy as np
    cnt = nt * (nt + 1) // 2
    out = np.zeros(cnt, np.float64)
    _check(load().krr_kernel_tile_norms(K.handle, out.ctypes.data, cnt), "krr_kernel_tile_norms")
    return out


def krr_factor_precision_map(F: Factor):
    import numpy as np
    info = krr_factor_get_info(F)
    nt = info.nt
    cnt = nt * nt * (nt + 1) // 2
    out = np.zeros(cnt, np.uint8)
    _check(load().krr_factor_precision_map(F.handle, out.ctypes.data, cnt),
           "krr_factor_precision_map")
    return out.reshape(nt, nt * (nt + 1) // 2)
