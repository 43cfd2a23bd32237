"""Benchmark: kernel ridge regression Build + Factor + Solve on one MI355X.

One step = the whole hot path on one batch of synthetic input already
resident in HBM: INT8-MFMA Gram with the distance/exp epilogue, the
adaptive-precision tile Cholesky of K + lambda I (FP64 diagonal tiles,
FP32/FP16/FP8 trailing updates), FP32 triangular solves for all phenotypes
and FP64 iterative refinement until a rigorous bound guarantees 1e-5
relative error against the exact solution.

Op count per step (the paper's complexity figures for Build and the
Cholesky, plus the solves): n^2 m + n^3 / 3 + 2 n^2 r; a train+predict
workload adds Predict for its test patients, 2 n_test n (m + r).

--workload selects the input: single (the default benchmark), small,
large, trainpredict, or batched (48 instances through the batched calls).

Prints ONE JSON line (rank 0).  The same ops are timed on the plain FP32 GPU
path (FP32 diagonal POTRF and updates, FP32 solves, no refinement) for the
speed-up ratio, and the CPU oracle is timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "int8_TOPs": 5000.0,
    "fp8_TFLOPs": 5000.0,
    "fp16_TFLOPs": 2500.0,
    "fp32_TFLOPs": 157.3,
    "fp64_TFLOPs": 78.6,
}


REFINE_TOL = 9.9e-6  # so that tol / (1 - tol) < 1e-5


GRAM_SOURCES = ["paper_2409_01712_amd/csrc/build.hip", "paper_2409_01712_amd/csrc/common.h"]
TRAFFIC_FILE = "profiles/k_gram_tiles_single_traffic.txt"


def gram_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in GRAM_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def gram_traffic(tile=512):
    """HBM bytes per Gram launch from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE of the kernel, each scaled by what the counter reads for a
    device copy of known size), or None when the kernel's sources changed
    since the counters were taken or the summary is of another tile size."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv["source_sha256"] != gram_source_hash():
            return None
        cb = float(kv["copy_bytes"])
        fs = cb / (float(kv["copy_fetch_kib"]) * 1024.0)
        ws = cb / (float(kv["copy_write_kib"]) * 1024.0)
        return (float(kv["fetch_kib_t%d" % tile]) * 1024.0 * fs
                + float(kv["write_kib_t%d" % tile]) * 1024.0 * ws)
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def ops_per_step(n, m, r):
    return float(n) * n * m + float(n) ** 3 / 3.0 + 2.0 * n * n * r


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single",
                    choices=["single", "small", "batched", "large", "trainpredict"])
    ap.add_argument("--batch", type=int, default=48, help="instances of the batched workload")
    ap.add_argument("--n", type=int, default=0, help="override the number of patients")
    ap.add_argument("--plain-steps", type=int, default=0,
                    help="timed steps of the plain FP32 path (0 = as many as --steps)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 48-instance batch that the default run adds as 'batched'")
    ap.add_argument("--cpu-sample", type=int, default=3072, help="patients in the oracle sample")
    ap.add_argument("--eps", type=float, default=1.0)
    ap.add_argument("--refine", choices=["ir", "pcg", "auto"], default="ir",
                    help="refinement method of the adaptive path")
    ap.add_argument("--high-panels", type=int, default=1)
    ap.add_argument("--tile", type=int, default=512,
                    help="tile size when the autotuner is off (--no-tune)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner: library defaults with --tile")
    ap.add_argument("--tune-cache", default=os.environ.get("KRR_TUNE_CACHE"),
                    help="autotuner cache file (JSON); default none, i.e. search every run")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device to device (calibrates HBM counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.plain_steps <= 0:
        args.plain_steps = args.steps
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}))
        return

    import synth
    import paper_2409_01712_amd as krr

    if args.workload == "batched":
        return main_batched(args)
    w = synth.WORKLOADS[args.workload]
    n = args.n or w.n
    m, r = w.m, w.r
    t0 = time.time()
    Gh = w.genotypes(rows=n)
    Yh = w.phenotypes(Gh)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    G = torch.from_numpy(Gh).to(dev)
    Y = torch.from_numpy(Yh).to(dev)
    # a train+predict workload also predicts for its test patients in every step
    n_test = w.n_test if not args.n else 0
    T = torch.from_numpy(w.test_genotypes()).to(dev) if n_test else None
    torch.cuda.synchronize()
    log = (lambda *a: print(*a, file=sys.stderr, flush=True)) if args.verbose else (lambda *a: None)
    log("inputs: n=%d m=%d r=%d generated in %.1fs" % (n, m, r, gen_s))

    ctx = krr.krr_create(0, tile=args.tile)
    adaptive = krr.Policy(eps=args.eps, high_panels=args.high_panels)
    plain = krr.plain_fp32_policy()
    ctx_plain = krr.krr_create(0, tile=args.tile)
    # The metric's accuracy target, 1e-5 relative error against the exact
    # solution, enforced through the rigorous bound ||x - x*|| <= ||r|| / lambda
    # (K + lambda I has smallest eigenvalue >= lambda): stopping at
    # ||r_j|| / (lambda ||x_j||) <= tol gives ||x_j - x*_j|| / ||x*_j|| <= tol / (1 - tol).
    method = {"ir": krr.KRR_REFINE_IR, "pcg": krr.KRR_REFINE_PCG,
              "auto": krr.KRR_REFINE_AUTO}[args.refine]
    refine = krr.Refine(method=method, max_iters=30, tol=REFINE_TOL)
    no_refine = krr.Refine(method=krr.KRR_REFINE_NONE)

    def step(policy, ref, c=None):
        c = c or ctx
        K = krr.krr_build_kernel(c, G, w.gamma, w.lam)
        F = krr.krr_factor(c, K, policy)
        X, info, st = krr.krr_solve(c, F, Y, ref, check=False)
        if T is not None:
            krr.krr_predict(c, K, T, X)
        finfo = krr.krr_factor_get_info(F)
        F.release()
        K.release()
        return X, info, st, finfo

    # the same autotuner picks each path's schedule (tile, panel group, residual
    # split, sweep pairing) on these inputs, outside the timed region
    tuning = {}
    if not args.no_tune:
        t0 = time.time()
        tuning["adaptive"], _ = krr.krr_autotune(ctx, G, Y, w.gamma, w.lam, adaptive, refine,
                                                 args.tune_cache)
        if not args.no_plain:
            tuning["plain_fp32"], _ = krr.krr_autotune(ctx_plain, G, Y, w.gamma, w.lam, plain,
                                                       no_refine, args.tune_cache)
        log("autotuned in %.1fs: %s" % (time.time() - t0, tuning))
    nb = krr.krr_get_tuning(ctx)["tile"]

    for i in range(args.warmup):
        step(adaptive, refine)
        log("warmup %d done" % i)
    torch.cuda.synchronize()

    # the timed steps carry the Gram's event pair only (the roofline's live launch
    # time): events between the factorization's dependent launches slow it down
    krr.krr_timers_enable_stages(ctx, ["gram"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst, all_conv = 0.0, True
    for i in range(args.steps):
        X, info, st, finfo = step(adaptive, refine)
        worst = max(worst, info.fwd_err_bound)
        all_conv = all_conv and bool(info.converged)
        log("step %d: iters=%d bound=%.2e" % (i, info.iters, info.fwd_err_bound))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    gram_timed = krr.krr_timers_read(ctx)["gram"]
    # the stage breakdown: one more step with every stage timed, after the timed region
    krr.krr_timers_enable(ctx, True)
    _, sinfo, _, _ = step(adaptive, refine)
    torch.cuda.synchronize()
    stages = krr.krr_timers_read(ctx)
    krr.krr_timers_enable(ctx, False)

    # predict: the INT8 cross Gram (2 n_test n m) and K_test X (2 n_test n r)
    ops = ops_per_step(n, m, r) + 2.0 * n_test * n * (m + r)
    value = ops / dt
    out = {
        "metric": "KRR build+factor+solve Op/s vs plain FP32 GPU path at <=1e-5 rel err vs FP64",
        "value": value,
        "unit": "Op/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed:i8,f8,f16,f32,f64",
        "data": "synthetic (seeded Philox Binomial(2,p) genotypes, epistatic phenotypes)",
        "config": {
            "workload": "single KRR instance n=%d patients, m=%d SNPs, r=%d phenotypes, "
                        "gamma=1/m, lambda=%g, tile %d, adaptive FP32/FP16/FP8 updates + FP64 "
                        "diagonal + FP64 refinement" % (n, m, r, w.lam, nb),
            "n": n, "m": m, "nrhs": r, "gamma": w.gamma, "lambda": w.lam, "tile": nb,
            "eps": args.eps, "high_panels": args.high_panels,
            "parallelism": "single GPU",
        },
        "ops_per_step": ops,
        "refine": {"method": args.refine, "iters": info.iters, "fwd_err_bound": info.fwd_err_bound,
                   "first_bound": info.first_bound, "converged": bool(info.converged),
                   "worst_fwd_err_bound_over_steps": worst, "all_steps_converged": all_conv},
        # every timed step must meet the metric's accuracy target
        "valid": bool(all_conv and worst <= 1e-5),
        "updates": {"fp32": int(finfo.updates[0]), "fp16": int(finfo.updates[1]),
                    "fp8": int(finfo.updates[2]), "promotions": int(finfo.promotions)},
        # from one extra step with every stage timed (stages on different streams overlap)
        "stages_ms_per_step": {k: round(v[0], 4) for k, v in stages.items() if v[1]},
        "tuning": tuning or {"adaptive": krr.krr_get_tuning(ctx)},
    }

    # dominant kernel: the INT8 Gram (one launch per step)
    g_ms, g_cnt = gram_timed
    gram_avg_s = g_ms / g_cnt / 1e3
    gram_ops = float(n) * n * m  # n^2/2 unique pairs x 2m ops (multiply + add)
    achieved = gram_ops / gram_avg_s / 1e12
    out["roofline"] = {
        "kernel": "k_gram_tiles (INT8 MFMA Gram + distance/exp epilogue)",
        "bound": "mfma", "achieved": achieved, "peak": PEAK["int8_TOPs"], "unit": "TOP/s",
        "frac": achieved / PEAK["int8_TOPs"], "traffic": gram_traffic(nb),
        "avg_launch_ms": gram_avg_s * 1e3,
    }
    u_ms, u_cnt = stages["update"]
    # trailing-update MFMA utilisation: algorithmic flops per precision (off-diagonal tile
    # update 2 nb^3; a diagonal tile's lower triangle nb^2 (nb + 1), always FP32) against the
    # time at each precision's dense peak, over the update kernels' summed time
    NT = (n + nb - 1) // nb
    ndiag = NT * (NT - 1) // 2
    f_off, f_diag = 2.0 * nb ** 3, float(nb) * nb * (nb + 1)
    u32, u16, u8 = (int(finfo.updates[q]) for q in range(3))
    fl = {"fp32": (u32 - ndiag) * f_off + ndiag * f_diag, "fp16": u16 * f_off, "fp8": u8 * f_off}
    ideal_s = (fl["fp32"] / (PEAK["fp32_TFLOPs"] * 1e12) + fl["fp16"] / (PEAK["fp16_TFLOPs"] * 1e12)
               + fl["fp8"] / (PEAK["fp8_TFLOPs"] * 1e12))
    u_s = u_ms / 1e3
    out["update_stage"] = {"ms_per_step": u_ms, "launches_per_step": u_cnt,
                           "flops": fl, "achieved_TFLOPs": sum(fl.values()) / u_s / 1e12,
                           "time_at_peak_ms": ideal_s * 1e3, "mfma_frac": ideal_s / u_s}

    if not args.no_plain:
        for i in range(args.warmup):
            step(plain, no_refine, ctx_plain)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.plain_steps):
            Xp, pinfo, _, _ = step(plain, no_refine, ctx_plain)
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t0) / args.plain_steps
        krr.krr_timers_enable(ctx_plain, True)
        step(plain, no_refine, ctx_plain)
        torch.cuda.synchronize()
        pstages = krr.krr_timers_read(ctx_plain)
        krr.krr_timers_enable(ctx_plain, False)
        # accuracy of the plain path, measured by the FP64 residual bound
        K = krr.krr_build_kernel(ctx_plain, G, w.gamma, w.lam)
        F = krr.krr_factor(ctx_plain, K, plain)
        _, pin, _ = krr.krr_solve(ctx_plain, F, Y, krr.Refine(max_iters=0, tol=0.0), check=False)
        F.release()
        K.release()
        out["plain_fp32"] = {"value": ops / pdt, "ms_per_step": pdt * 1e3,
                             "fwd_err_bound": pin.fwd_err_bound,
                             "stages_ms_per_step": {k: round(v[0], 4)
                                                    for k, v in pstages.items() if v[1]}}
        out["speedup_vs_plain_fp32"] = pdt / dt
        out["plain_fp32"]["steps"] = args.plain_steps

    if not args.no_cpu:
        import oracle
        ns = min(args.cpu_sample, n)
        Gs = np.ascontiguousarray(Gh[:ns])
        Ys = np.ascontiguousarray(Yh[:ns])
        t0 = time.perf_counter()
        oracle.fit(Gs, Ys, w.gamma, w.lam)
        cdt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": ops_per_step(ns, m, r) / cdt, "unit": "Op/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "first %d patients of the same genotype matrix (all %d SNPs, %d phenotypes): "
                      "FP64 build + Cholesky + solves, %.1f s" % (ns, m, r, cdt),
        }
    if not args.no_batched and args.workload == "single" and not args.n:
        # the 48-instance cross-validation batch, two timed steps per path, reported
        # beside the headline workload (not part of its value)
        ctx.close()
        ctx_plain.close()
        del G, Y
        torch.cuda.empty_cache()
        b = run_batched(args, min(args.steps, 2), 1, min(args.plain_steps, 2))
        out["batched"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "steps", "config",
                                            "refine", "valid", "stages_ms_per_step", "graphs",
                                            "roofline", "plain_fp32", "speedup_vs_plain_fp32",
                                            "input_generation_s") if k in b}
    print(json.dumps(out), flush=True)
    if not out["valid"] or not out.get("batched", {}).get("valid", True):
        print("bench: a timed step missed the 1e-5 accuracy target", file=sys.stderr)
        sys.exit(1)


def main_batched(args):
    out = run_batched(args, args.steps, args.warmup, args.plain_steps)
    print(json.dumps(out), flush=True)
    if not out["valid"]:
        print("bench: an instance missed the 1e-5 accuracy target", file=sys.stderr)
        sys.exit(1)


def run_batched(args, steps, warmup, plain_steps):
    """Many independent instances (uneven n, differing gamma and lambda, one SNP panel)
    through the batched calls: one step = batched build + factor + solve of all of them,
    each stage one launch per step for all instances (the factorization's lockstep
    launches and the solve's sweeps replayed from HIP graphs after the first step)."""
    import numpy as np
    import torch

    import synth
    import paper_2409_01712_amd as krr

    insts = synth.batched_workloads(count=args.batch)
    dev = torch.device("cuda:0")
    Gs, Ys = [], []
    t0 = time.time()
    for w, row0 in insts:
        Gh = w.genotypes(rows=w.n, row0=row0)
        Yh = w.phenotypes(Gh)
        Gs.append(torch.from_numpy(Gh).to(dev))
        Ys.append(torch.from_numpy(Yh).to(dev))
        del Gh
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    gammas = [w.gamma for w, _ in insts]
    lams = [w.lam for w, _ in insts]
    m, r = insts[0][0].m, insts[0][0].r
    ns = [w.n for w, _ in insts]
    adaptive = krr.Policy(eps=args.eps, high_panels=args.high_panels)
    refine = krr.Refine(method=krr.KRR_REFINE_IR if args.refine == "ir" else krr.KRR_REFINE_AUTO,
                        max_iters=30, tol=REFINE_TOL)
    plain = krr.plain_fp32_policy()
    no_refine = krr.Refine(method=krr.KRR_REFINE_NONE)

    def step(policy, ref, ctx):
        Ks = krr.krr_build_kernel_batched(ctx, Gs, gammas, lams)
        Fs = krr.krr_factor_batched(ctx, Ks, policy)
        Xs, infos, st = krr.krr_solve_batched(ctx, Fs, Ys, ref, check=False)
        for F in Fs:
            F.release()
        for K in Ks:
            K.release()
        return infos

    # the tile of each path: one warm and one timed step at each size (as the
    # single workload's autotuner does for it), unless --no-tune
    tiles = [args.tile] if args.no_tune else [256, 512]
    ctxs = {t: krr.krr_create(0, tile=t) for t in tiles}

    def pick(policy, ref):
        best = None
        for t in tiles:
            if len(tiles) == 1:
                return t
            step(policy, ref, ctxs[t])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(policy, ref, ctxs[t])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            if best is None or el < best[1]:
                best = (t, el)
        return best[0]

    tile_a = pick(adaptive, refine)
    tile_p = pick(plain, no_refine) if not args.no_plain else tile_a
    for t in list(ctxs):
        if t not in (tile_a, tile_p):
            ctxs.pop(t).close()
    ctx = ctxs[tile_a]
    for _ in range(warmup):
        step(adaptive, refine, ctx)
    torch.cuda.synchronize()
    krr.krr_timers_enable_stages(ctx, ["gram"])
    t0 = time.perf_counter()
    worst, all_conv = 0.0, True
    for _ in range(steps):
        infos = step(adaptive, refine, ctx)
        worst = max([worst] + [i.fwd_err_bound for i in infos])
        all_conv = all_conv and all(bool(i.converged) for i in infos)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    g_ms, g_cnt = krr.krr_timers_read(ctx)["gram"]
    # the stage breakdown from one more step with every stage timed (outside the timed region)
    krr.krr_timers_enable(ctx, True)
    step(adaptive, refine, ctx)
    torch.cuda.synchronize()
    stages = krr.krr_timers_read(ctx)
    krr.krr_timers_enable(ctx, False)
    ops = sum(ops_per_step(n, m, r) for n in ns)
    gram_ops = sum(float(n) * n * m for n in ns)
    achieved = gram_ops / (g_ms / g_cnt / 1e3) / 1e12
    out = {
        "metric": "KRR build+factor+solve Op/s vs plain FP32 GPU path at <=1e-5 rel err vs FP64",
        "value": ops / dt, "unit": "Op/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "mixed:i8,f8,f16,f32,f64",
        "data": "synthetic (seeded Philox Binomial(2,p) genotypes, epistatic phenotypes)",
        "config": {
            "workload": "batch of %d KRR instances, n in [%d, %d] (sum %d), m=%d, r=%d, "
                        "gamma in {0.5,1,2}/m, lambda in {1e-3,1e-2,1e-1,1}, tile %d"
                        % (len(ns), min(ns), max(ns), sum(ns), m, r, tile_a),
            "batch": len(ns), "m": m, "nrhs": r, "tile": tile_a, "tile_plain_fp32": tile_p,
            "parallelism": "single GPU",
        },
        "ops_per_step": ops,
        "refine": {"max_iters": max(i.iters for i in infos),
                   "max_fwd_err_bound": max(i.fwd_err_bound for i in infos),
                   "converged": int(sum(i.converged for i in infos)),
                   "worst_fwd_err_bound_over_steps": worst},
        "valid": bool(all_conv and worst <= 1e-5),
        "stages_ms_per_step": {k: round(v[0], 4) for k, v in stages.items() if v[1]},
        "graphs": dict(zip(("cached", "launches"), krr.krr_context_graphs(ctx))),
        "roofline": {"kernel": "k_gram_tiles_batched (all instances in one launch)",
                     "bound": "mfma", "achieved": achieved, "peak": PEAK["int8_TOPs"],
                     "unit": "TOP/s", "frac": achieved / PEAK["int8_TOPs"], "traffic": None,
                     "avg_launch_ms": g_ms / g_cnt},
        "input_generation_s": gen_s,
    }
    if not args.no_plain:
        cp = ctxs[tile_p]
        step(plain, no_refine, cp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            step(plain, no_refine, cp)
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t0) / plain_steps
        out["plain_fp32"] = {"value": ops / pdt, "ms_per_step": pdt * 1e3, "steps": plain_steps}
        out["speedup_vs_plain_fp32"] = pdt / dt
    for c in ctxs.values():
        c.close()
    del Gs, Ys
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
