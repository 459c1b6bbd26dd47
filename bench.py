"""Benchmark of the Pinv-Recon hot path on one MI355X.

Workload: 64x64 image (N=4096), 8 coils, variable-density spiral of 4096
samples per coil (M=32768), 1000 dynamic frames, shift 1e-3 * mean diag(E^H E).

One step = build R with the FP32 path (Gram, FP64 blocked Cholesky with L^-1,
W = L^-1 E^H, R = L^-H W) from the encoding alone, then reconstruct all 1000
frames (image = R data) with the refinement steps needed to reach 1e-5
relative error against the plain FP64 GPU path.  Inputs are resident in HBM
before the timed region; the plan is built fresh every step (uncached).

value = complex-equivalent algorithmic TFLOP/s of the whole step:
  (Gram 4MN^2 + Cholesky 4N^3/3 + two triangular solves 8MN^2 + apply 8NMF) / step time.
The JSON line also carries the build-only rate, apply frames/s, the same for
the plain FP64 GPU path, the error table, a roofline entry for the dominant
kernel and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "R-build TFLOP/s + apply frames/s vs plain FP64 GPU at stated error; p50/p99"
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w) -> dict:
    """Oracle Gram E^H E (FP64, numpy) over the first two coils' rows of the
    workload: a bounded sample of the build's dominant stage."""
    import oracle
    from paper_2410_06129_amd import synth
    enc = w.enc
    sub = synth.Encoding(enc.nx, enc.ny, enc.k, coil=enc.coil[:2])
    t0 = time.perf_counter()
    oracle.gram(sub)
    dt = time.perf_counter() - t0
    flops = 4.0 * sub.M * sub.N * sub.N
    threads = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        nums = [p.get("num_threads", 0) for p in threadpool_info() if p.get("user_api") == "blas"]
        if nums:
            threads = max(nums)
    except Exception:
        pass
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle Gram over coils 0-1 (M={sub.M} of {enc.M} rows, N={sub.N}), "
                      f"{flops:.3g} complex-equivalent flops in {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-reps", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_06129_amd import pinv as P
    from paper_2410_06129_amd import synth

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = synth.config2(F=args.frames)
    enc = w.enc
    N, M, F = enc.N, enc.M, w.images.shape[0]
    log(f"workload {w.name}: N={N} M={M} F={F}")
    ctx = P.pinv_context_create(0)

    # --- inputs resident in HBM: data = E x (FP64 GPU forward) + 30 dB noise ---
    p64 = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP64)
    P.pinv_plan_wait(p64)
    x_true = torch.from_numpy(w.images).to(dev)
    d64 = torch.empty((F, M), dtype=torch.complex128, device=dev)
    P.pinv_forward(ctx, p64, x_true, d64)
    noise = torch.from_numpy(w.noise).to(dev)
    sigma = torch.sqrt(torch.mean(torch.abs(d64) ** 2)) * 10 ** (-w.snr_db / 20)
    d64 += sigma * noise
    del noise
    d32 = d64.to(torch.complex64)
    x64 = torch.empty((F, N), dtype=torch.complex128, device=dev)
    P.pinv_apply(ctx, p64, d64, x64)
    torch.cuda.synchronize()
    ref_norm = torch.linalg.vector_norm(x64, dim=1)

    def rel_err(x):
        e = torch.linalg.vector_norm(x.to(torch.complex128) - x64, dim=1) / ref_norm
        return float(e.max()), float(e.median())

    flops_build = 12.0 * M * N * N + 4.0 * N ** 3 / 3.0
    flops_apply = 8.0 * N * M * F
    x32 = torch.empty((F, N), dtype=torch.complex64, device=dev)

    # --- choose refinement steps: the fewest that meet the tolerance ---
    p32 = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
    P.pinv_plan_wait(p32)
    err_table = {}
    refine = None
    for r in range(0, 3):
        P.pinv_apply(ctx, p32, d32, x32, refine_steps=r)
        torch.cuda.synchronize()
        err_table[r] = rel_err(x32)
        log(f"refine {r}: max rel err {err_table[r][0]:.3e} median {err_table[r][1]:.3e}")
        if refine is None and err_table[r][0] <= args.tol:
            refine = r
    if refine is None:
        refine = 2
    # apply-only and refinement timings (events on the launch stream)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    apply_ms, refine_ms = [], []
    for _ in range(3):
        e0.record(stream)
        P.pinv_apply(ctx, p32, d32, x32, refine_steps=0)
        e1.record(stream)
        P.pinv_apply(ctx, p32, d32, x32, refine_steps=refine)
        e2.record(stream)
        torch.cuda.synchronize()
        apply_ms.append(e0.elapsed_time(e1))
        refine_ms.append(e1.elapsed_time(e2) - e0.elapsed_time(e1))
    P.pinv_plan_release(p32)

    # --- timed steps ---
    def step():
        p = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
        P.pinv_apply(ctx, p, d32, x32, refine_steps=refine)
        return p

    for _ in range(args.warmup):
        p = step()
        P.pinv_plan_wait(p)
        P.pinv_plan_release(p)
    torch.cuda.synchronize()
    plans = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        plans.append(step())
        log(f"step {i} enqueued")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = []
    for p in plans:
        P.pinv_plan_wait(p)
        stages.append(P.pinv_plan_info_get(p)["stage_ms"])
        P.pinv_plan_release(p)
    stages = np.array(stages)
    st_mean = stages.mean(axis=0)
    err_final = rel_err(x32)
    ms_step = 1e3 * dt / args.steps
    value = (flops_build + flops_apply) / (ms_step * 1e-3) / 1e12
    build_ms = float(st_mean.sum())
    log(f"stage ms (gram, chol+inv, W, R): {np.round(st_mean, 3)}; step {ms_step:.2f} ms")

    # --- plain FP64 GPU comparator ---
    f64_build, f64_apply = [], []
    for _ in range(args.fp64_reps):
        q = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP64, P.FLAG_UNCACHED)
        P.pinv_plan_wait(q)
        f64_build.append(sum(P.pinv_plan_info_get(q)["stage_ms"]))
        e0.record(stream)
        P.pinv_apply(ctx, q, d64, x64)
        e1.record(stream)
        torch.cuda.synchronize()
        f64_apply.append(e0.elapsed_time(e1))
        P.pinv_plan_release(q)
    f64_build_ms, f64_apply_ms = float(np.median(f64_build)), float(np.median(f64_apply))

    # --- roofline of the dominant kernel (largest share of the step) ---
    kern = {
        "gram": (float(st_mean[0]), 4.0 * M * N * N),
        "trmm_w": (float(st_mean[2]), 4.0 * M * N * N),
        "trmm_r": (float(st_mean[3]), 4.0 * M * N * N),
        "apply": (float(np.median(apply_ms)), flops_apply),
    }
    name = max(kern, key=lambda k: kern[k][0])
    kms, kfl = kern[name]
    achieved = kfl / (kms * 1e-3) / 1e12
    roof = {"kernel": name, "bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA, "traffic": None,
            "per_kernel_tflops": {k: v[1] / (v[0] * 1e-3) / 1e12 for k, v in kern.items()}}

    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "N": N, "M": M, "F": F, "coils": enc.C,
                   "precision": "fp32 mfma, fp64 factorisation", "refine_steps": refine,
                   "lambda_rel": w.rel_lambda},
        "build_tflops": flops_build / (build_ms * 1e-3) / 1e12,
        "build_ms": build_ms,
        "stage_ms": {"gram": st_mean[0], "chol_inv": st_mean[1], "trmm_w": st_mean[2],
                     "trmm_r": st_mean[3]},
        "apply_frames_per_s": F / (np.median(apply_ms) * 1e-3),
        "apply_refined_frames_per_s": F / ((np.median(apply_ms) + np.median(refine_ms)) * 1e-3),
        "rel_err_vs_fp64_gpu": {"max": err_final[0], "median": err_final[1],
                                "by_refine_steps": {str(k): v[0] for k, v in err_table.items()}},
        "fp64_gpu": {"build_ms": f64_build_ms,
                     "build_tflops": flops_build / (f64_build_ms * 1e-3) / 1e12,
                     "apply_frames_per_s": F / (f64_apply_ms * 1e-3)},
        "roofline": roof,
    }
    out["speedup_vs_fp64_gpu"] = {"build": f64_build_ms / build_ms,
                                  "apply": f64_apply_ms / float(np.median(apply_ms))}
    P.pinv_plan_release(p64)
    P.pinv_context_destroy(ctx)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w)
    for k, v in list(out["stage_ms"].items()):
        out["stage_ms"][k] = float(v)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
