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

Other rows of the hot path are measured with --workload (one JSON line each):
  timeloop  N = 65536 sedimentation, overlap-regularised RPY, AB2 dt = 0.005,
            FP32-compensated pair kernel with FP64 positions; FP64 path as the
            long reference (drift of the centre-of-mass velocity)
  batched   4096 independent clusters, N_c uniform on [4, 256], 100 Euler
            steps dt = 0.01 in one persistent graph-launched kernel
  adjoint   N = 8192, 200 Euler steps dt = 0.01, loss |x_N - x_target|^2,
            checkpoint every 20 steps: forward and backward times
  lubrication  N = 65536 suspension (gaps >= 0.6a), lubrication correction
            (Eq. 8) with the previous velocities, Euler dt = 0.001
            (--loop-steps steps)
  fcc       the benchmark of Sec. 3.3: sedimentation F = (0, 0, -1) from a
            perfect fcc lattice at n = 0.1/a^3 in a periodic cube (nearest
            image), Euler dt = 0.001, 100 steps, N = 4 m^3 from 256 to 202612:
            runtime per step, the lubrication step timed on the same
            configuration, and the FP64 path
  precision the numerical-stability study of Sec. 4: the four-sphere cluster
            integrated for --study-time tau_s with single / double-single
            (and Kahan, FP64) accumulation of the hydrodynamic interactions
            and positions, dt = 0.01 and 0.001, all runs in one launch per
            chunk; cycle duration and amplitude by parabolic fits of x_1(t)
  membench  the O(N^2) memory-access micro-benchmarks of App. A: naive,
            small-tiling and tiling kernels x linear / strided / unordered
            maps x float / float4, N = 4096 ... 65536, time per pair
  copy      a plain device copy of --copy-mib MiB (calibrates HBM counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# Useful flops of one ordered pair (FMA = 2, rsqrt = 1): d 3, r^2 5, rsqrt 1,
# r^-2 1, A 3, B 4, d.F 5, s = B (d.F) 1, A F + s d accumulated 12 (Eq. 7b).
FLOP_PER_PAIR = 35
PEAK_FP32_TFLOPS = 157.3    # MI355X published FP32 vector peak
METRIC = "G pair-interactions/s of RPY mobility product at N=65536 (FP32-comp vs FP64)"
SMALL_N = 16384             # the second size of the single-product benchmark

# HBM traffic of one product-kernel launch from two rocprofv3 counter passes
# (FETCH_SIZE, WRITE_SIZE; profiles/pair_kernel_f32_n65536_hbm_counters.md), each
# scaled by what the counter reads for a plain 256 MiB copy (fetch x 2.00,
# write x 1.00).  Valid only for the kernel sources (SHA-1 of mobility.hip
# followed by sym_chunk_asm.h) and launch configuration the counters were taken
# with; otherwise reported as null.
KERNEL_SOURCES = ("mobility.hip", "sym_chunk_asm.h")
PMC_TRAFFIC = {"source_sha1": "19e495dbf922c878aad9291638d7607c53cf5d45",
               "n": 65536,
               "config": {"variant": 2, "block": 256, "splits": 32, "ilp": 2, "kahan_block": 32},
               "fetch_kib": 16173.9, "write_kib": 121567.4, "fetch_scale": 2.0, "write_scale": 1.0}


def _measured_traffic(n, cfg):
    """HBM bytes per product-kernel launch, or None if the counters are stale."""
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1205_6333_amd", "csrc")
    h = hashlib.sha1()
    try:
        for name in KERNEL_SOURCES:
            h.update(open(os.path.join(csrc, name), "rb").read())
    except OSError:
        return None
    sha = h.hexdigest()
    m = PMC_TRAFFIC
    if sha != m["source_sha1"] or n != m["n"] or dict(cfg) != m["config"]:
        return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


# VALU wave instructions of one product-kernel launch (rocprofv3 SQ_INSTS_VALU,
# profiles/pair_kernel_f32_n65536_valu_counters.md), same validity rule.
PMC_VALU = {"source_sha1": PMC_TRAFFIC["source_sha1"], "n": 65536,
            "config": PMC_TRAFFIC["config"], "valu_wave_instr": 1189680640,
            # SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32 per dispatch (wave instructions)
            "add_f32": 158810112, "mul_f32": 319508480, "fma_f32": 622198784,
            "trans_f32": 33902592}


def _measured_valu(n, cfg):
    """(VALU lane-instructions, issued FP32 flops) per launch, or None if the
    counters are stale.  Issued flops: add, mul and transcendental count one,
    FMA two, per lane."""
    if _measured_traffic(n, cfg) is None or PMC_VALU["n"] != n or dict(cfg) != PMC_VALU["config"]:
        return None
    v = PMC_VALU
    flops = 64.0 * (v["add_f32"] + v["mul_f32"] + 2 * v["fma_f32"] + v["trans_f32"])
    return 64.0 * v["valu_wave_instr"], flops


def _to4(v, dtype, device):
    import torch
    out = np.zeros((v.shape[0], 4))
    out[:, :3] = v
    return torch.tensor(out, dtype=dtype, device=device)


def _prewarm(sd, pos, frc, vel, prec, warmup, seconds):
    """`warmup` untimed products, then more until `seconds` of wall time have
    passed: the clock of an idle GPU ramps up over its first few hundred ms of
    load, and the timed region should see the clock of a loaded GPU.  Returns
    the number of untimed products run."""
    import torch
    done = 0
    t0 = time.perf_counter()
    while done < warmup or time.perf_counter() - t0 < seconds:
        for _ in range(5):
            sd.mobility_apply(pos, frc, vel, precision=prec)
        done += 5
        torch.cuda.synchronize()
    return done


def _time_path(sd, pos, frc, vel, prec, steps, warmup, prewarm_s=0.0):
    """Warm up, then time `steps` products; returns (wall s, pair-kernel ms avg,
    event ms total, pair-kernel ms per launch, untimed products)."""
    import torch
    untimed = _prewarm(sd, pos, frc, vel, prec, warmup, prewarm_s)
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
    per = sd.sd_profile_times()
    return t1 - t0, kern_ms / max(1, launches), ev0.elapsed_time(ev1), per, untimed


def _kernel_name(cfg):
    if cfg.get("variant") == 2:
        return "k_pair_f32_sym_asm" if cfg.get("kahan_block") in (16, 32) else "k_pair_f32_sym"
    return "k_pair_f32_lds" if cfg.get("variant") == 0 else "k_pair_f32_smem"


def _small_product(sd, W, dev, args):
    """The product at N = SMALL_N (same recipe, seeds 1 and 2): wall-clock
    rate, median pair-kernel launch and its fraction of the FP32 peak."""
    import torch
    n = SMALL_N
    x = W.random_suspension(n, phi=0.05, seed=1)
    f = W.gaussian_forces(n, seed=2)
    pos, frc = _to4(x, torch.float32, dev), _to4(f, torch.float32, dev)
    vel = torch.empty((n, 3), dtype=torch.float64, device=dev)
    cfg = sd.sd_get_kernel_config(sd.SD_FP32_KAHAN, n)
    steps = max(20, args.steps)
    print("bench: timing fp32-kahan n=%d %s" % (n, cfg), file=sys.stderr, flush=True)
    wall, kern_ms, _, per, _ = _time_path(sd, pos, frc, vel, sd.SD_FP32_KAHAN, steps, 20,
                                          min(args.prewarm_s, 0.5))
    pairs = float(n) * n
    med = float(np.median(per)) if per else kern_ms
    return {"value": pairs * steps / wall / 1e9, "unit": "G pair-interactions/s",
            "steps": steps, "ms_per_step": wall * 1e3 / steps, "pair_kernel_ms": kern_ms,
            "pair_kernel_ms_median": med, "kernel": cfg, "kernel_name": _kernel_name(cfg),
            "frac_median": FLOP_PER_PAIR * pairs / (med * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}


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
    cores = oracle.threads()
    # the same loop on one thread, over a smaller sample (about 2 s)
    rows1 = np.sort(rng.choice(n, size=max(16, min(n, int(len(rows) * 2.0 / max(dt, 1e-3)
                                                          / max(cores, 1)))), replace=False))
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.mobility_rows(p, x32, f32, rows1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    return {"value": len(rows) * n / dt / 1e9, "unit": "G pair-interactions/s",
            "cores": cores, "kind": "oracle",
            "sample": "%d of %d rows of the N=%d product (%.2e pairs, %.1f s), FP64 oracle "
                      "(plain double loop, gcc -O2, OpenMP over rows)" % (len(rows), n, n,
                                                                          len(rows) * n, dt),
            "single_thread_value": len(rows1) * n / dt1 / 1e9,
            "single_thread_sample": "%d rows (%.2e pairs, %.1f s) on one thread"
                                    % (len(rows1), len(rows1) * n, dt1)}, err


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_timeloop(args, sd, W, dev):
    import torch
    n = args.n
    steps = args.loop_steps
    x0 = W.random_suspension(n, phi=0.05, seed=1)
    f = W.gravity_forces(n)
    p = sd.params(overlap=True)
    out = {"metric": "AB2 sedimentation steps/s at N=%d (FP32-comp pair kernel, FP64 positions)" % n,
           "unit": "steps/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "sedimentation, N=%d, random suspension phi=0.05, F=(0,0,-1), "
                                  "overlap-regularised RPY, AB2 dt=0.005, %d steps" % (n, steps)}}
    res = {}
    for prec in (sd.SD_FP32_KAHAN, sd.SD_FP64):
        dt4 = torch.float64 if prec == sd.SD_FP64 else torch.float32
        frc = _to4(f, dt4, dev)
        x = torch.tensor(x0, device=dev)
        vp = torch.zeros_like(x)
        sd.sd_run(x, frc, 0.005, 3, v_prev=vp, integrator=sd.SD_AB2, params=p, precision=prec)
        x = torch.tensor(x0, device=dev)
        vcm = []
        chunk = max(1, steps // 20)
        sd.sd_premise_counts(reset=True)

        def go():
            done = 0
            while done < steps:
                k = min(chunk, steps - done)
                sd.sd_run(x, frc, 0.005, k, step0=done, v_prev=vp, integrator=sd.SD_AB2,
                          params=p, precision=prec)
                done += k
                vcm.append(sd.sd_mean_vector(vp))
        t = _sync_time(go)
        res[prec] = (t, x.cpu().numpy(), torch.stack(vcm).cpu().numpy(),
                     sd.sd_premise_counts(reset=True))
    t32, x32, v32, pc32 = res[sd.SD_FP32_KAHAN]
    t64, x64, v64, _ = res[sd.SD_FP64]
    out.update({"value": steps / t32, "steps": steps, "ms_per_step": t32 * 1e3 / steps,
                "g_pairs_per_s": float(n) * n * steps / t32 / 1e9,
                "fp64_steps_per_s": steps / t64, "speedup_vs_fp64": t64 / t32,
                "vcm_z_final": float(v32[-1, 2]), "vcm_z_final_fp64": float(v64[-1, 2]),
                "vcm_drift_vs_fp64_max": float(np.abs(v32 - v64).max()),
                "x_final_vs_fp64_max_abs": float(np.abs(x32 - x64).max()),
                # overlapping pairs (r < 2a) met per step, on average over the run
                "overlapping_pairs_per_step": pc32[0] / steps,
                # v_cm after every chunk of steps: FP32-comp z, FP64 z, largest
                # component difference
                "vcm_series": [[min(steps, (k + 1) * chunk), float(v32[k, 2]), float(v64[k, 2]),
                                float(np.abs(v32[k] - v64[k]).max())] for k in range(len(v32))]})
    return out


def run_batched(args, sd, W, dev):
    import torch
    offsets, x0 = W.clusters(4096, nmin=4, nmax=256, sigma=4.0, seed=3)
    sizes = np.diff(offsets)
    pairs = float((sizes.astype(np.float64) ** 2).sum())
    f = W.gravity_forces(len(x0))
    frc = _to4(f, torch.float32, dev)
    b = sd.Batch(offsets)
    x = torch.tensor(x0, device=dev)
    steps = 100
    tune = b.autotune(x, frc, 0.01, steps)                      # untimed; x is not changed
    sd.sd_run_batched(b, x, frc, 0.01, steps, use_graph=True)  # capture + warm-up
    times = []
    for _ in range(max(1, args.steps // 4)):
        x.copy_(torch.tensor(x0, device=dev))
        times.append(_sync_time(lambda: sd.sd_run_batched(b, x, frc, 0.01, steps,
                                                          use_graph=True)))
    t = float(np.median(times))
    return {"metric": "G pair-interactions/s of batched clusters (4096 clusters, 100 Euler steps)",
            "value": pairs * steps / t / 1e9, "unit": "G pair-interactions/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "ms_per_launch": t * 1e3, "launches_timed": len(times),
            "kernel_shape": b.get_config(), "autotune": tune,
            "config": {"workload": "4096 free-space clusters, N_c~U{4..256} (seed 3), Gaussian "
                                   "sigma=4a with rejection < 2.2a, F=(0,0,-1), Euler dt=0.01, "
                                   "100 steps in one persistent HIP-graph launch, kernel shape "
                                   "chosen by sd_batch_autotune",
                       "particles": int(offsets[-1]), "sum_nc2": pairs}}


def run_adjoint(args, sd, W, dev):
    import torch
    from paper_1205_6333_amd import autograd as AG
    n, steps = 8192, 200
    x0 = W.random_suspension(n, phi=0.05, seed=1)
    F0 = W.gravity_forces(n)
    Fp = F0 + 0.1 * W.gaussian_forces(n, seed=4)
    out = {"metric": "backward/forward time ratio of the checkpointed Euler adjoint at N=8192",
           "unit": "ratio", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "N=8192 random suspension phi=0.05, 200 Euler steps dt=0.01, "
                                  "loss |x_N - x_target|^2, x_target from forces F0 + 0.1 N(0,1), "
                                  "checkpoint every 20 steps"}}
    xt = torch.tensor(x0, device=dev)
    sd.sd_run(xt, _to4(Fp, torch.float32, dev), 0.01, steps)
    x0t = torch.tensor(x0, device=dev, requires_grad=True)
    F0t = torch.tensor(F0, device=dev, requires_grad=True)
    xe = AG.run(x0t, F0t, 0.01, steps, checkpoint_every=20)  # warm-up
    ((xe - xt) ** 2).sum().backward()
    holder = {}

    def fwd():
        holder["xe"] = AG.run(x0t, F0t, 0.01, steps, checkpoint_every=20)

    def bwd():
        ((holder["xe"] - xt) ** 2).sum().backward()
    tf = _sync_time(fwd)
    tb = _sync_time(bwd)
    out.update({"value": tb / tf, "forward_s": tf, "backward_s": tb,
                "forward_g_pairs_per_s": float(n) * n * steps / tf / 1e9})
    return out


def _pair_roofline(sd, n, fn):
    """Run fn with the library's pair-kernel timing on; the roofline of the
    pair kernel (35 flop per pair, HIP events on the launch stream)."""
    import torch
    torch.cuda.synchronize()
    sd.sd_profile_reset()
    sd.sd_profile_enable(True)
    fn()
    torch.cuda.synchronize()
    sd.sd_profile_enable(False)
    launches, ms = sd.sd_profile_read()
    kern_ms = ms / max(1, launches)
    achieved = FLOP_PER_PAIR * float(n) * n / (kern_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
            "kernel": "pair kernel", "pair_kernel_ms": kern_ms, "launches": launches}


def run_lubrication(args, sd, W, dev):
    import torch
    n, steps = args.n, args.loop_steps
    # gaps >= 0.6a: the lagged correction is stable there (it diverges for
    # pairs closer than s = 0.28)
    x0 = W.random_suspension(n, phi=0.05, min_dist=2.6, seed=1)
    f = W.gravity_forces(n) + 0.1 * W.gaussian_forces(n, seed=2)
    fd = torch.tensor(f, device=dev)
    f4 = _to4(f, torch.float32, dev)
    x = torch.tensor(x0, device=dev)
    vp = torch.zeros_like(x)
    sd.sd_run_lub(x, fd, vp, 0.001, 3)  # warm-up
    vr = torch.tensor(W.gaussian_forces(n, seed=5), device=dev)   # any non-rigid motion
    n_close = int(sd.lubrication_forces(torch.tensor(x0, device=dev), vr).ne(0).any(1).sum())
    x = torch.tensor(x0, device=dev)
    vp.zero_()
    t_lub = _sync_time(lambda: sd.sd_run_lub(x, fd, vp, 0.001, steps))
    x2 = torch.tensor(x0, device=dev)
    t_plain = _sync_time(lambda: sd.sd_run(x2, f4, 0.001, steps))
    fo = torch.empty_like(x)
    t_forces = _sync_time(lambda: [sd.lubrication_forces(x, vp, fd, fo) for _ in range(steps)])
    roof = _pair_roofline(sd, n, lambda: sd.sd_run_lub(x, fd, vp, 0.001, 20))
    return {"metric": "Euler steps/s with lubrication at N=%d (FP32-comp pair kernel)" % n,
            "roofline": roof,
            "value": steps / t_lub, "unit": "steps/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic", "steps": steps,
            "ms_per_step": t_lub * 1e3 / steps, "ms_per_step_without_lubrication": t_plain * 1e3 / steps,
            "lubrication_forces_ms": t_forces * 1e3 / steps,
            "g_pairs_per_s": float(n) * n * steps / t_lub / 1e9,
            "particles_with_close_pairs_at_start": n_close,
            "config": {"workload": "N=%d random suspension phi=0.05 (RSA 2.6a), F=(0,0,-1) + 0.1 N(0,1), "
                                   "lubrication s<1 (s_min 1e-3) with the previous velocities, Euler "
                                   "dt=0.001, %d steps" % (n, steps)}}


FCC_M = (4, 6, 8, 11, 16, 20, 25, 32, 37)   # N = 4 m^3 = 256 ... 202612


def run_fcc(args, sd, W, dev):
    """Sec. 3.3: runtime per step from the perfect fcc lattice.  The lagged
    lubrication correction diverges on this dense lattice (phi ~ 0.42: a
    lattice mode grows by a factor of several per step, in the oracle as on
    the GPU), after which the particle cloud is meaningless; the loop is
    therefore timed without the correction (steps 1 and 3 of Sec. 3.1), and
    step 2 (cell list + Eq. 8 forces) is timed on the same configuration."""
    import torch
    steps, dt = 100, 0.001
    rows = []
    roof = None
    for m in FCC_M:
        x0, L = W.fcc_lattice(m, density=0.1)
        n = len(x0)
        f = W.gravity_forces(n)
        p = sd.params(box=L)
        fd = torch.tensor(f, device=dev)
        f4 = _to4(f, torch.float32, dev)
        f4d = _to4(f, torch.float64, dev)
        x = torch.tensor(x0, device=dev)
        sd.sd_run(x, f4, dt, steps, params=p)             # warm-up (captures the step graph)
        x.copy_(torch.tensor(x0, device=dev))
        t_plain = _sync_time(lambda: sd.sd_run(x, f4, dt, steps, params=p))
        v = sd.mobility_apply(_to4(x.cpu().numpy(), torch.float32, dev), f4, params=p)
        fo = torch.empty_like(x)
        sd.lubrication_forces(x, v, fd, fo, params=p)
        t_lub = _sync_time(lambda: [sd.lubrication_forces(x, v, fd, fo, params=p)
                                    for _ in range(steps)])
        s64 = steps if n <= 65536 else 10
        x.copy_(torch.tensor(x0, device=dev))
        sd.sd_run(x, f4d, dt, s64, params=p, precision=sd.SD_FP64)
        x.copy_(torch.tensor(x0, device=dev))
        t64 = _sync_time(lambda: sd.sd_run(x, f4d, dt, s64, params=p, precision=sd.SD_FP64))
        x.copy_(torch.tensor(x0, device=dev))
        roof = _pair_roofline(sd, n, lambda: sd.sd_run(x, f4, dt, 20, params=p))
        row = {"m": m, "n": n, "box": L, "ms_per_step": t_plain * 1e3 / steps,
               "lubrication_step_ms": t_lub * 1e3 / steps,
               "ms_per_step_with_lubrication_step": (t_plain + t_lub) * 1e3 / steps,
               "ms_per_step_fp64": t64 * 1e3 / s64,
               "speedup_vs_fp64": (t64 / s64) / (t_plain / steps),
               "pair_kernel_ms": roof["pair_kernel_ms"], "pair_kernel_frac": roof["frac"],
               "g_pairs_per_s": float(n) * n * steps / t_plain / 1e9,
               "sedimentation_velocity": float(v[:, 2].mean())}
        print("bench fcc: %s" % json.dumps(row), file=sys.stderr, flush=True)
        rows.append(row)
    big = rows[-1]
    return {"metric": "ms per Euler step of the fcc sedimentation benchmark at N=%d "
                      "(periodic box, FP32-comp pair kernel)" % big["n"],
            "value": big["ms_per_step"], "unit": "ms/step", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic", "steps": steps,
            "ms_per_step": big["ms_per_step"], "table": rows, "roofline": roof,
            "config": {"workload": "Sec. 3.3 benchmark: perfect fcc lattice, n=0.1/a^3, periodic "
                                   "cube with nearest-image interactions, F=(0,0,-1), RPY, Euler "
                                   "dt=0.001, 100 steps, N=4m^3 for m in %s; the lubrication step "
                                   "(cell list + Eq. 8 forces, s<1) timed separately on the same "
                                   "configuration, since the lagged correction diverges on this "
                                   "dense lattice" % (FCC_M,)}}


ACC_NAMES = {0: "single", 1: "kahan", 2: "double-single", 3: "fp64"}
POS_NAMES = {0: "single", 1: "double-single", 2: "fp64"}


def run_precision(args, sd, W, dev):
    import torch
    from paper_1205_6333_amd import observables as OB
    x0, f = W.four_sphere_tetrahedron()
    grid = [(a, p) for a in (0, 2) for p in (0, 1)] + [(1, 2), (3, 2)]
    runs = [(a, p, dt) for dt in (0.01, 0.001) for (a, p) in grid]
    t_total = float(args.study_time)
    chunk_t = min(2000.0, t_total)            # tau_s per call
    sample_t = 0.5                             # frame spacing in tau_s
    specs = []
    for a, p, dt in runs:
        steps = int(round(chunk_t / dt))
        specs.append(dict(acc=a, pos=p, dt=dt, steps=steps, stride=int(round(sample_t / dt))))
    state = torch.zeros((len(runs), 2, 4, 3), dtype=torch.float64, device=dev)
    state[:, 0] = torch.tensor(x0, device=dev)
    fd = torch.tensor(f, device=dev)
    nf = [s["steps"] // s["stride"] for s in specs]
    series = [[] for _ in runs]                # (x1, y1) frames per run
    n_calls = int(np.ceil(t_total / chunk_t))
    t_gpu = 0.0
    for c in range(n_calls):
        out = {}
        t_gpu += _sync_time(lambda: out.update(traj=sd.sd_cluster_run(state, fd, specs)))
        traj = out["traj"].cpu().numpy()
        off = 0
        for r, k in enumerate(nf):
            series[r].append(traj[off:off + k, 0, :2].copy())
            off += k
        if c % 10 == 0 or c == n_calls - 1:
            print("bench precision: %.0f of %.0f tau_s, %.1f s on the GPU" %
                  ((c + 1) * chunk_t, n_calls * chunk_t, t_gpu), file=sys.stderr, flush=True)
    rows = []
    window = 1.0e4
    for r, (a, p, dt) in enumerate(runs):
        xy = np.concatenate(series[r])
        t = sample_t * np.arange(1, len(xy) + 1)
        tc, dur, ta, amp = OB.cycles(t, xy[:, 0])
        row = {"hi_accumulation": ACC_NAMES[a], "positions": POS_NAMES[p], "dt": dt,
               "cycles": int(len(dur)), "max_abs_y1": float(np.abs(xy[:, 1]).max())}
        if len(dur):
            # Fig. 5: cycle duration and amplitude averaged over windows of 1e4 tau_s;
            # the motion has broken down once a cycle deviates by more than 5 % from
            # the first window's period
            edges = np.arange(0.0, t[-1] + window, window)
            wins = []
            for lo_t in edges[:-1]:
                sel = (tc >= lo_t) & (tc < lo_t + window)
                sa = (ta >= lo_t) & (ta < lo_t + window)
                if sel.any():
                    wins.append([float(lo_t + window / 2), float(dur[sel].mean()),
                                 float(amp[sa].mean()) if sa.any() else None])
            row["windows_t_period_amplitude"] = wins
        if len(dur):
            first = dur[tc < tc[0] + window]
            last = dur[tc > tc[-1] - window]
            row.update({"period_first_window": float(first.mean()),
                        "period_last_window": float(last.mean()),
                        "period_min": float(dur.min()), "period_max": float(dur.max()),
                        "amplitude_first": float(amp[0]) if len(amp) else None,
                        "amplitude_last": float(amp[-1]) if len(amp) else None,
                        "last_cycle_end": float(tc[-1] + 0.5 * dur[-1])})
        rows.append(row)
    # breakdown: the first window whose mean period differs by more than 2 % from
    # that of the FP64 run with the same dt (the Euler drift itself is common to
    # all precisions), or that has no cycle left while the FP64 run has one
    for row in rows:
        ref = [r for r in rows if r["hi_accumulation"] == "fp64" and r["dt"] == row["dt"]]
        rw = {round(w[0]): w[1] for w in ref[0].get("windows_t_period_amplitude", [])}
        mine = {round(w[0]): w[1] for w in row.get("windows_t_period_amplitude", [])}
        row["departs_from_fp64_t"] = None
        for t_w in sorted(rw):
            if t_w not in mine or abs(mine[t_w] / rw[t_w] - 1.0) > 0.02:
                row["departs_from_fp64_t"] = float(t_w)
                break
    steps_fine = int(round(n_calls * chunk_t / 0.001))
    return {"metric": "Euler steps/s of one four-sphere run (precision study of Sec. 4, "
                      "%d runs per launch)" % len(runs),
            "value": steps_fine / t_gpu, "unit": "steps/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "gpu_seconds": t_gpu, "simulated_tau_s": n_calls * chunk_t, "runs": rows,
            "config": {"workload": "four sedimenting spheres (tetrahedron of Fig. 4), F=(0,0,-1), "
                                   "RPY, mu0=a=1, Euler; HI accumulation x positions in "
                                   "{single, double-single} plus (kahan, fp64) and (fp64, fp64); "
                                   "dt in {0.01, 0.001}; x_1 sampled every 0.5 tau_s; periods "
                                   "averaged over windows of 1e4 tau_s"}}


def run_membench(args, sd, W, dev):
    import torch
    kinds = {0: "naive", 1: "smalltiling", 2: "tiling"}
    maps = {0: "linear", 1: "strided", 2: "unordered"}
    rows = []
    for n in (4096, 16384, 65536):
        reps = 100 if n <= 16384 else 20
        for width in (1, 4):
            x = torch.randint(0, 7, (n,) if width == 1 else (n, 4), device=dev).float()
            out = torch.empty_like(x)
            for kind in kinds:
                for m in maps:
                    sd.sd_membench(kind, m, x, out)
                    ev0 = torch.cuda.Event(enable_timing=True)
                    ev1 = torch.cuda.Event(enable_timing=True)
                    ev0.record()
                    for _ in range(reps):
                        sd.sd_membench(kind, m, x, out)
                    ev1.record()
                    torch.cuda.synchronize()
                    t = ev0.elapsed_time(ev1) / 1e3 / reps
                    rows.append({"n": n, "type": "float" if width == 1 else "float4",
                                 "kernel": kinds[kind], "map": maps[m], "ms": t * 1e3,
                                 "ps_per_pair": t / (float(n) * n) * 1e12,
                                 "gb_per_s": float(n) * n * 4 * width / t / 1e9})
        print("bench membench: n=%d done" % n, file=sys.stderr, flush=True)
    big = [r for r in rows if r["n"] == 65536]
    best = min(big, key=lambda r: r["ps_per_pair"] / (4 if r["type"] == "float4" else 1))
    return {"metric": "ps per pair of the App. A memory-access micro-benchmarks at N=65536",
            "value": best["ps_per_pair"], "unit": "ps/pair", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic", "rows": rows,
            "best": best,
            "config": {"workload": "App. A: N threads in work-groups of 128 each read N "
                                   "elements (float or float4) through linear k, strided "
                                   "131k mod N or unordered (131k + 64j) mod N maps; naive, "
                                   "small tiling (one wave fills a 64-element LDS tile), "
                                   "tiling (128-element tile); 100 repetitions (20 at N=65536)"}}


def run_copy(args, dev):
    import torch
    m = int(args.copy_mib * 2 ** 20 // 4)
    src = torch.ones(m, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"metric": "device copy", "bytes_per_copy": 4 * m, "copies": 3}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed products first (the clock ramps up over the first launches)")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the N = %d product timed beside the headline size" % SMALL_N)
    ap.add_argument("--prewarm-s", type=float, default=1.0,
                    help="untimed products continue until this many seconds have passed")
    ap.add_argument("--tune", action="store_true", help="autotune the kernel shape first (untimed)")
    ap.add_argument("--workload", default="product",
                    choices=["product", "timeloop", "batched", "adjoint", "lubrication", "fcc",
                             "precision", "membench", "copy"])
    ap.add_argument("--study-time", type=float, default=2.0e4,
                    help="simulated tau_s of --workload precision (the paper: 5e5)")
    ap.add_argument("--loop-steps", type=int, default=1000, help="steps of --workload timeloop")
    ap.add_argument("--copy-mib", type=float, default=256.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the product is not sharded across GPUs in this "
              "build; use --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1205_6333_amd as sd
    from paper_1205_6333_amd import workloads as W

    dev = torch.device("cuda", 0)
    n = args.n
    if args.workload != "product":
        fn = {"timeloop": lambda: run_timeloop(args, sd, W, dev),
              "batched": lambda: run_batched(args, sd, W, dev),
              "adjoint": lambda: run_adjoint(args, sd, W, dev),
              "lubrication": lambda: run_lubrication(args, sd, W, dev),
              "fcc": lambda: run_fcc(args, sd, W, dev),
              "precision": lambda: run_precision(args, sd, W, dev),
              "membench": lambda: run_membench(args, sd, W, dev),
              "copy": lambda: run_copy(args, dev)}[args.workload]
        print(json.dumps(fn()))
        return 0
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
    wall, kern_ms, ev_ms, per, untimed = _time_path(sd, pos32, frc32, vel, sd.SD_FP32_KAHAN,
                                                    args.steps, args.warmup, args.prewarm_s)
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
        "untimed_products": untimed,
        "pair_kernel_ms": kern_ms,
        "pair_kernel_ms_median": float(np.median(per)) if per else None,
        "pair_kernel_launches": len(per),
        "value_kernel_median": pairs / (float(np.median(per)) * 1e-3) / 1e9 if per else None,
    }
    achieved = FLOP_PER_PAIR * pairs / (kern_ms * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                       "traffic": _measured_traffic(n, cfg),
                       "flop_per_pair": FLOP_PER_PAIR,
                       "kernel": "pair kernel (%s)" % _kernel_name(cfg)}
    valu = _measured_valu(n, cfg)
    if valu is not None:
        instr, flops = valu
        out["roofline"]["valu_lane_instr_per_pair"] = instr / pairs
        out["roofline"]["valu_t_lane_instr_per_s"] = instr / (kern_ms * 1e-3) / 1e12
        out["roofline"]["issued_flop_per_pair"] = flops / pairs
        out["roofline"]["issued_tflops"] = flops / (kern_ms * 1e-3) / 1e12
    if not args.no_fp64:
        pos64, frc64 = _to4(x, torch.float64, dev), _to4(f, torch.float64, dev)
        vel64 = torch.empty((n, 3), dtype=torch.float64, device=dev)
        steps64 = max(3, args.steps // 4)
        print("bench: timing fp64", file=sys.stderr, flush=True)
        wall64, kern64, _, _, _ = _time_path(sd, pos64, frc64, vel64, sd.SD_FP64, steps64,
                                       min(args.warmup, 2))
        out["fp64_value"] = pairs * steps64 / wall64 / 1e9
        out["fp64_pair_kernel_ms"] = kern64
        out["speedup_vs_fp64"] = value / out["fp64_value"]
        v64 = vel64.cpu().numpy()
        out["fp32_vs_fp64_rel2"] = float(np.linalg.norm(v32 - v64) / np.linalg.norm(v64))
    if not args.no_small and n != SMALL_N:
        out["n%d" % SMALL_N] = _small_product(sd, W, dev, args)
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
