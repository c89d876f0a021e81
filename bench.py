#!/usr/bin/env python3
"""Throughput of the all-pairs Rotne-Prager mobility product on one MI355X.

Workload: one product v = M(x) F (Eq. 7a with the tensor of Eq. 7b) for
N = 65536 spheres of radius a = 1 at volume fraction 0.05 (random sequential
addition in a cube, minimum distance 2.2a, seed 1), forces i.i.d. N(0, 1)
(seed 2), FP32 pair evaluation with Kahan-compensated accumulation.  A step is
one call of mobility_apply (pair kernel + split merge); inputs are resident in
HBM before the timed region starts.

Printed: one JSON line with the metric (G pair-interactions/s = N^2 per step),
the FP64 path's rate and the speedup over it, the relative 2-norm error on
sampled rows against the FP64 oracle, the roofline of the pair kernel
(HIP-event timed inside the library on the launch stream) and the oracle's
own rate on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

FLOP_PER_PAIR = 35          # canonical useful flops per pair, see the design doc
PEAK_FP32_TFLOPS = 157.3    # MI355X published FP32 vector peak
PEAK_FP32_NONPACKED = 78.6  # the same without packed FP32 (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
METRIC = "G pair-interactions/s of RPY mobility product at N=65536 (FP32-comp vs FP64)"


def _to4(v, dtype, device):
    import torch
    out = np.zeros((v.shape[0], 4))
    out[:, :3] = v
    return torch.tensor(out, dtype=dtype, device=device)


def _time_path(sd, pos, frc, vel, prec, steps, warmup):
    """Warm up, then time `steps` products; returns (wall s, pair-kernel ms avg,
    event ms total)."""
    import torch
    for _ in range(warmup):
        sd.mobility_apply(pos, frc, vel, precision=prec)
    torch.cuda.synchronize()
    sd.sd_profile_reset()
    sd.sd_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        sd.mobility_apply(pos, frc, vel, precision=prec)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sd.sd_profile_enable(False)
    launches, kern_ms = sd.sd_profile_read()
    return t1 - t0, kern_ms / max(1, launches), ev0.elapsed_time(ev1)


def cpu_baseline(x32, f32, vgpu, n, target_s):
    """The FP64 oracle on a bounded sample of rows of the same product."""
    import oracle
    p = oracle.params()
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(n, size=min(n, 128), replace=False))
    t0 = time.perf_counter()
    ref = oracle.mobility_rows(p, x32, f32, rows)
    dt = time.perf_counter() - t0
    nrows = int(min(n, max(128, 128 * target_s / max(dt, 1e-3))))
    if nrows > 128:
        rows = np.sort(rng.choice(n, size=nrows, replace=False))
        t0 = time.perf_counter()
        ref = oracle.mobility_rows(p, x32, f32, rows)
        dt = time.perf_counter() - t0
    err = float(np.linalg.norm(vgpu[rows] - ref) / np.linalg.norm(ref))
    return {"value": len(rows) * n / dt / 1e9, "unit": "G pair-interactions/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d of %d rows of the N=%d product (%.2e pairs, %.1f s), FP64 oracle "
                      "(plain double loop, gcc -O2, OpenMP over rows)" % (len(rows), n, n,
                                                                          len(rows) * n, dt)}, err


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--tune", action="store_true", help="autotune the kernel shape first (untimed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the product is not sharded across GPUs in this "
              "build (see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1205_6333_amd as sd
    from paper_1205_6333_amd import workloads as W

    dev = torch.device("cuda", 0)
    n = args.n
    print("bench: generating inputs n=%d" % n, file=sys.stderr, flush=True)
    x = W.random_suspension(n, phi=0.05, seed=1)
    f = W.gaussian_forces(n, seed=2)
    pos32, frc32 = _to4(x, torch.float32, dev), _to4(f, torch.float32, dev)
    vel = torch.empty((n, 3), dtype=torch.float64, device=dev)
    tune_report = None
    if args.tune:
        tune_report = sd.sd_autotune(n, precision=sd.SD_FP32_KAHAN)
    cfg = sd.sd_get_kernel_config(sd.SD_FP32_KAHAN, n)
    print("bench: timing fp32-kahan %s" % cfg, file=sys.stderr, flush=True)
    wall, kern_ms, ev_ms = _time_path(sd, pos32, frc32, vel, sd.SD_FP32_KAHAN, args.steps,
                                      args.warmup)
    v32 = vel.cpu().numpy()
    pairs = float(n) * n
    value = pairs * args.steps / wall / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "G pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single RPY mobility product, N=%d spheres (a=1, mu0=1), random "
                               "suspension phi=0.05 (RSA, min distance 2.2a, seed 1), forces "
                               "N(0,1) (seed 2), FP32 evaluation + Kahan accumulation" % n,
                   "n": n, "precision": "fp32_kahan", "kernel": cfg},
        "event_ms_per_step": ev_ms / args.steps,
        "pair_kernel_ms": kern_ms,
    }
    achieved = FLOP_PER_PAIR * pairs / (kern_ms * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                       "flop_per_pair": FLOP_PER_PAIR,
                       "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
                       "kernel": "pair kernel (k_pair_f32_*)"}
    if not args.no_fp64:
        pos64, frc64 = _to4(x, torch.float64, dev), _to4(f, torch.float64, dev)
        vel64 = torch.empty((n, 3), dtype=torch.float64, device=dev)
        steps64 = max(3, args.steps // 4)
        print("bench: timing fp64", file=sys.stderr, flush=True)
        wall64, kern64, _ = _time_path(sd, pos64, frc64, vel64, sd.SD_FP64, steps64,
                                       min(args.warmup, 2))
        out["fp64_value"] = pairs * steps64 / wall64 / 1e9
        out["fp64_pair_kernel_ms"] = kern64
        out["speedup_vs_fp64"] = value / out["fp64_value"]
        v64 = vel64.cpu().numpy()
        out["fp32_vs_fp64_rel2"] = float(np.linalg.norm(v32 - v64) / np.linalg.norm(v64))
    if not args.no_cpu:
        print("bench: oracle cpu baseline", file=sys.stderr, flush=True)
        base, err = cpu_baseline(W.round_to_f32(x), W.round_to_f32(f), v32, n, args.cpu_seconds)
        out["cpu_baseline"] = base
        out["rel2_vs_oracle_sampled"] = err
    if tune_report:
        out["autotune"] = json.loads(tune_report)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
