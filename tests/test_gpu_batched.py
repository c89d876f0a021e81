"""Batched independent clusters: one persistent kernel (optionally launched
through a captured HIP graph) against per-cluster oracle runs."""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import rel2, rowerr, to_dev3, to_dev4

pytestmark = pytest.mark.gpu


def _check(v, ref, tol, *what):
    """Relative 2-norm within tol and every particle (rowerr) within 10 tol."""
    err, row = rel2(v, ref), rowerr(v, ref)
    print(what, "rel2=%.3e row=%.3e" % (err, row))
    assert err <= tol, (what, err)
    assert row <= 10 * tol, (what, row)


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available()
    import paper_1205_6333_amd as sd
    sd.lib()
    return sd


def _dt(sd, prec):
    import torch
    return torch.float64 if prec == sd.SD_FP64 else torch.float32


def _per_cluster(offsets, fn):
    out = []
    for c in range(len(offsets) - 1):
        out.append(fn(offsets[c], offsets[c + 1]))
    return np.concatenate(out, 0)


@pytest.fixture(scope="module")
def clusters():
    offsets, x = W.clusters(96, nmin=4, nmax=256, seed=5)
    return offsets, x, W.gravity_forces(len(x)) + 0.2 * W.gaussian_forces(len(x), seed=6)


@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-12), (2, 1e-5)])
def test_apply_batched(sd, orc, clusters, prec, tol):
    import torch
    offsets, x, f = clusters
    b = sd.Batch(offsets)
    xo, fo = (x, f) if prec == 1 else (W.round_to_f32(x), W.round_to_f32(f))
    v = sd.mobility_apply_batched(b, to_dev4(xo, _dt(sd, prec)), to_dev4(fo, _dt(sd, prec)),
                                  precision=prec)
    torch.cuda.synchronize()
    p = orc.params()
    ref = _per_cluster(offsets, lambda a, e: orc.mobility(p, xo[a:e], fo[a:e]))
    _check(v.cpu().numpy(), ref, tol)
    b.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-12)])
@pytest.mark.parametrize("integ", [0, 1])
def test_run_batched_vs_oracle(sd, orc, clusters, prec, tol, integ):
    import torch
    offsets, x, f = clusters
    fo = f if prec == 1 else W.round_to_f32(f)
    b = sd.Batch(offsets)
    xd = to_dev3(x)
    sd.sd_run_batched(b, xd, to_dev4(fo, _dt(sd, prec)), 0.01, 30, integrator=integ,
                      precision=prec, use_graph=False)
    torch.cuda.synchronize()
    p = orc.params()
    ref = _per_cluster(offsets, lambda a, e: orc.run(p, x[a:e], fo[a:e], 0.01, 30, integ)[0])
    err = np.abs(xd.cpu().numpy() - ref).max() / np.abs(ref - x).max()
    print("prec=%d integ=%d err/disp=%.3e" % (prec, integ, err))
    assert err <= tol
    b.close()


def test_graph_replays_match_eager(sd, clusters):
    """Graph launch == eager launch bitwise, over several replays with eager
    work and synchronisations between them."""
    import torch
    offsets, x, f = clusters
    b = sd.Batch(offsets)
    frc = to_dev4(W.round_to_f32(f), torch.float32)
    eager = to_dev3(x)
    sd.sd_run_batched(b, eager, frc, 0.01, 10, use_graph=False)
    xg = to_dev3(x)
    for rep in range(4):
        xg.copy_(to_dev3(x))
        torch.cuda.synchronize()
        sd.sd_run_batched(b, xg, frc, 0.01, 10, use_graph=True)
        scratch = torch.randn(1000, device=xg.device).sum()  # unrelated eager work
        torch.cuda.synchronize()
        assert torch.equal(xg, eager), rep
        assert torch.isfinite(scratch)
    b.close()


def test_cluster_size_edges(sd, orc):
    """Clusters of 1, 2 and 3 particles, an empty cluster, and clusters above
    256 (several particles per lane) up to the maximum size."""
    import torch
    sizes = [1, 2, 0, 3, 257, 600, 1024, 5]
    rng = np.random.default_rng(9)
    xs = [W._sequential_reject(lambda k: rng.normal(0, 6.0, size=(k, 3)), s, 2.2, batch=64)
          if s else np.zeros((0, 3)) for s in sizes]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.concatenate(xs, 0)
    f = W.gravity_forces(len(x))
    b = sd.Batch(offsets)
    p = orc.params()
    for prec, tol in ((0, 1e-6), (1, 1e-12)):
        fo = f if prec == 1 else W.round_to_f32(f)
        xo = x if prec == 1 else W.round_to_f32(x)
        v = sd.mobility_apply_batched(b, to_dev4(xo, _dt(sd, prec)), to_dev4(fo, _dt(sd, prec)),
                                      precision=prec)
        xd = to_dev3(x)
        sd.sd_run_batched(b, xd, to_dev4(fo, _dt(sd, prec)), 0.02, 12, precision=prec)
        torch.cuda.synchronize()
        ref_v = np.concatenate([orc.mobility(p, xo[a:e], fo[a:e]) for a, e in
                                zip(offsets[:-1], offsets[1:]) if e > a], 0)
        _check(v.cpu().numpy(), ref_v, tol)
        ref_x = np.concatenate([orc.run(p, x[a:e], fo[a:e], 0.02, 12)[0] for a, e in
                                zip(offsets[:-1], offsets[1:]) if e > a], 0)
        assert np.abs(xd.cpu().numpy() - ref_x).max() <= tol * 100 * np.abs(ref_x - x).max()
    b.close()


def test_overlapping_clusters(sd, orc):
    import torch
    sizes = [40, 120, 7]
    rng = np.random.default_rng(10)
    x = rng.normal(0, 1.5, size=(sum(sizes), 3))
    x[5] = x[6]  # coincident pair
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    f = W.gaussian_forces(len(x), seed=11)
    pb = sd.params(overlap=True)
    b = sd.Batch(offsets, params=pb)
    p = orc.params(overlap=True)
    for prec, tol in ((0, 1e-6), (1, 1e-12)):
        xo = x if prec == 1 else W.round_to_f32(x)
        fo = f if prec == 1 else W.round_to_f32(f)
        v = sd.mobility_apply_batched(b, to_dev4(xo, _dt(sd, prec)), to_dev4(fo, _dt(sd, prec)),
                                      precision=prec)
        torch.cuda.synchronize()
        ref = np.concatenate([orc.mobility(p, xo[a:e], fo[a:e]) for a, e in
                              zip(offsets[:-1], offsets[1:])], 0)
        _check(v.cpu().numpy(), ref, tol)
    b.close()


def test_autotune_installs_a_valid_config(sd, orc):
    import torch
    n = 3000
    report = sd.sd_autotune(n, precision=sd.SD_FP32_KAHAN)
    assert '"ranked"' in report
    cfg = sd.sd_get_kernel_config(sd.SD_FP32_KAHAN, n)
    x = W.random_suspension(n, seed=12)
    f = W.gaussian_forces(n, seed=13)
    xo, fo = W.round_to_f32(x), W.round_to_f32(f)
    v = sd.mobility_apply(to_dev4(xo, torch.float32), to_dev4(fo, torch.float32))
    torch.cuda.synchronize()
    sd.sd_autotune_clear(sd.SD_FP32_KAHAN)
    _check(v.cpu().numpy(), orc.mobility(orc.params(), xo, fo), 1e-6, cfg)


def test_autotune_times_the_automatic_choice_and_the_assembly_shapes(sd, orc):
    """From N = 16384 on the automatic choice is the pair-symmetric kernel with
    its chunk loop in assembly (256 lanes, two particles per lane, Kahan block
    32): the tuner times it beside the other shapes, installs nothing slower,
    and the installed shape keeps parity.  Clearing restores the automatic
    choice."""
    import json
    import torch
    n = 16384
    auto = sd.sd_get_kernel_config(sd.SD_FP32_KAHAN, n)
    assert (auto["variant"], auto["block"], auto["ilp"], auto["kahan_block"]) == (2, 256, 2, 32)
    rep = json.loads(sd.sd_autotune(n, precision=sd.SD_FP32_KAHAN))
    try:
        assert rep["default_ms"] > 0
        ranked = rep["ranked"]
        assert ranked[0]["ms"] <= rep["default_ms"]
        cfg = sd.sd_get_kernel_config(sd.SD_FP32_KAHAN, n)
        assert {k: cfg[k] for k in ("variant", "block", "splits", "ilp", "kahan_block")} == \
            {k: ranked[0][k] for k in ("variant", "block", "splits", "ilp", "kahan_block")}
        x = W.random_suspension(n, seed=12)
        f = W.gaussian_forces(n, seed=13)
        xo, fo = W.round_to_f32(x), W.round_to_f32(f)
        v = sd.mobility_apply(to_dev4(xo, torch.float32), to_dev4(fo, torch.float32))
        torch.cuda.synchronize()
        rows = np.random.default_rng(5).choice(n, 512, replace=False)
        ref = orc.mobility_rows(orc.params(), xo, fo, rows)
        _check(v.cpu().numpy()[rows], ref, 1e-6, cfg)
    finally:
        sd.sd_autotune_clear(sd.SD_FP32_KAHAN)
    assert sd.sd_get_kernel_config(sd.SD_FP32_KAHAN, n) == auto


@pytest.mark.parametrize("prec,tol", [("SD_FP64", 1e-12), ("SD_FP32_PLAIN", 1e-5)])
def test_autotune_other_precisions(sd, orc, prec, tol):
    """The tuner for the FP64 path and for plain FP32 accumulation: it times the
    automatic choice, installs a valid shape no slower than it, the installed
    shape keeps parity, and clearing restores the automatic choice."""
    import json
    import torch
    P = getattr(sd, prec)
    n = 16384
    auto = sd.sd_get_kernel_config(P, n)
    rep = json.loads(sd.sd_autotune(n, precision=P))
    try:
        assert rep["default_ms"] > 0 and rep["ranked"][0]["ms"] <= rep["default_ms"]
        cfg = sd.sd_get_kernel_config(P, n)
        x = W.random_suspension(n, seed=14)
        f = W.gaussian_forces(n, seed=15)
        if P == sd.SD_FP64:
            xo, fo = x, f
            v = sd.mobility_apply(to_dev4(xo, torch.float64), to_dev4(fo, torch.float64),
                                  precision=P)
        else:
            xo, fo = W.round_to_f32(x), W.round_to_f32(f)
            v = sd.mobility_apply(to_dev4(xo, torch.float32), to_dev4(fo, torch.float32),
                                  precision=P)
        torch.cuda.synchronize()
        rows = np.random.default_rng(6).choice(n, 256, replace=False)
        _check(v.cpu().numpy()[rows], orc.mobility_rows(orc.params(), xo, fo, rows), tol, cfg)
    finally:
        sd.sd_autotune_clear(P)
    assert sd.sd_get_kernel_config(P, n) == auto


def test_batched_full_workload_sampled_clusters(sd, orc):
    """The 4096-cluster workload (N_c ~ U{4..256}, 100 Euler steps, dt = 0.01,
    graph launch) in its launch configuration; 48 sampled clusters (plus the
    largest and the smallest) against independent oracle runs."""
    import torch
    offsets, x = W.clusters(4096, nmin=4, nmax=256, sigma=4.0, seed=3)
    f = W.gravity_forces(len(x))
    b = sd.Batch(offsets)
    xd = to_dev3(x)
    sd.sd_run_batched(b, xd, to_dev4(f, torch.float32), 0.01, 100, use_graph=True)
    torch.cuda.synchronize()
    xg = xd.cpu().numpy()
    sizes = np.diff(offsets)
    pick = np.unique(np.concatenate([[int(np.argmax(sizes)), int(np.argmin(sizes))],
                                     np.random.default_rng(8).choice(4096, 48, replace=False)]))
    p = orc.params()
    worst = 0.0
    for c in pick:
        a, e = offsets[c], offsets[c + 1]
        ref, _, _ = orc.run(p, x[a:e], f[a:e], 0.01, 100)
        worst = max(worst, np.abs(xg[a:e] - ref).max() / np.abs(ref - x[a:e]).max())
    print("worst err/disp over %d clusters: %.3e" % (len(pick), worst))
    assert worst <= 1e-6
    b.close()


@pytest.mark.parametrize("workgroup,per_cu", [(128, 0), (128, 16), (256, 2), (512, 0), (512, 1)])
def test_kernel_shapes_vs_oracle(sd, orc, workgroup, per_cu):
    """Every work-group size and residency of the persistent kernel, on
    clusters that use both the several-lanes-per-particle and the
    rows-of-particles mappings (sizes 1 ... 1024), FP32-comp and FP64."""
    import torch
    sizes = [1, 3, 7, 60, 64, 65, 127, 128, 129, 200, 256, 300, 511, 512, 513, 1024, 2]
    rng = np.random.default_rng(21)
    xs = [W._sequential_reject(lambda k: rng.normal(0, 6.0, size=(k, 3)), s, 2.2, batch=64)
          for s in sizes]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.concatenate(xs, 0)
    f = W.gravity_forces(len(x)) + 0.2 * W.gaussian_forces(len(x), seed=22)
    b = sd.Batch(offsets)
    b.set_config(workgroup, per_cu)
    assert b.get_config() == {"workgroup": workgroup, "per_cu": per_cu}
    p = orc.params()
    for prec, tol in ((0, 1e-6), (1, 1e-12)):
        fo = f if prec == 1 else W.round_to_f32(f)
        xo = x if prec == 1 else W.round_to_f32(x)
        v = sd.mobility_apply_batched(b, to_dev4(xo, _dt(sd, prec)), to_dev4(fo, _dt(sd, prec)),
                                      precision=prec)
        xd = to_dev3(x)
        sd.sd_run_batched(b, xd, to_dev4(fo, _dt(sd, prec)), 0.02, 8, precision=prec,
                          integrator=1, use_graph=True)
        torch.cuda.synchronize()
        ref_v = _per_cluster(offsets, lambda a, e: orc.mobility(p, xo[a:e], fo[a:e]))
        _check(v.cpu().numpy(), ref_v, tol)
        ref_x = _per_cluster(offsets, lambda a, e: orc.run(p, x[a:e], fo[a:e], 0.02, 8, 1)[0])
        assert np.abs(xd.cpu().numpy() - ref_x).max() <= tol * 100 * np.abs(ref_x - x).max()
    b.close()


def test_batched_autotune_keeps_the_fastest_shape(sd, orc, clusters):
    import torch
    offsets, x, f = clusters
    b = sd.Batch(offsets)
    xd = to_dev3(x)
    frc = to_dev4(W.round_to_f32(f), torch.float32)
    rep = b.autotune(xd, frc, 0.01, 20)
    assert torch.equal(xd, to_dev3(x))                 # x is not changed
    cands = rep["candidates"]
    assert len(cands) >= 7
    best = min(cands, key=lambda c: c["ms"])
    assert b.get_config() == {"workgroup": best["workgroup"], "per_cu": best["per_cu"]}
    sd.sd_run_batched(b, xd, frc, 0.01, 20)
    torch.cuda.synchronize()
    p = orc.params()
    fo = W.round_to_f32(f)
    ref = _per_cluster(offsets, lambda a, e: orc.run(p, x[a:e], fo[a:e], 0.01, 20)[0])
    assert np.abs(xd.cpu().numpy() - ref).max() <= 1e-6 * np.abs(ref - x).max()
    b.close()
