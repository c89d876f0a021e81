"""GPU parity of mobility_apply against the FP64 oracle.

Tolerances, against the oracle fed the same FP32-rounded inputs: relative
2-norm over all 3n components, and per particle (rowerr: the worst
particle's error relative to the larger of its reference norm and the
median reference norm, so that no single row can hide in the aggregate):
                 2-norm   per particle
  SD_FP32_KAHAN  1e-6     1e-5   (the accuracy target of the FP32-compensated path)
  SD_FP32_PLAIN  1e-5     1e-4   (uncompensated; reported, not a target)
  SD_FP64        1e-12    1e-11
"""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import rel2, rowerr, to_dev3, to_dev4  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {0: 1e-6, 2: 1e-5, 1: 1e-12}
ROW_TOL = {0: 1e-5, 2: 1e-4, 1: 1e-11}


def _check(v, ref, prec, *what):
    err, row = rel2(v, ref), rowerr(v, ref)
    print(what, "prec=%d rel2=%.3e row=%.3e" % (prec, err, row))
    assert err <= TOL[prec], (what, err)
    assert row <= ROW_TOL[prec], (what, row)


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1205_6333_amd as sd
    sd.lib()
    yield sd
    sd.sd_set_kernel_config(0, None)
    sd.sd_set_kernel_config(1, None)
    sd.sd_set_kernel_config(2, None)


def _run(sd, x, f, prec, p):
    import torch
    dt = torch.float64 if prec == sd.SD_FP64 else torch.float32
    v = sd.mobility_apply(to_dev4(x, dt), to_dev4(f, dt), params=p, precision=prec)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def _oracle_inputs(x, f, prec):
    if prec == 1:
        return x, f
    return W.round_to_f32(x), W.round_to_f32(f)


def _params(sd, orc, a=1.0, eta=1 / (6 * np.pi), tensor=0, overlap=False):
    return sd.params(a, eta, tensor, overlap), orc.params(a, eta, tensor, overlap)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 255, 257, 1000, 4097])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_parity_sizes(sd, orc, n, prec):
    x = W.random_suspension(n, seed=100 + n)
    f = W.gaussian_forces(n, seed=200 + n)
    ps, po = _params(sd, orc)
    v = _run(sd, x, f, prec, ps)
    xo, fo = _oracle_inputs(x, f, prec)
    ref = orc.mobility(po, xo, fo)
    _check(v, ref, prec, n)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("block", [64, 128, 256])
@pytest.mark.parametrize("ilp", [1, 2])
@pytest.mark.parametrize("kb", [1, 2, 4, 8])
def test_parity_kernel_configs(sd, orc, variant, block, ilp, kb):
    if kb == 8 and block < 128:
        pytest.skip("kahan_block 8 needs block >= 128 (rejected by the library)")
    n = 1337
    x = W.random_suspension(n, seed=7)
    f = W.gaussian_forces(n, seed=8)
    ps, po = _params(sd, orc)
    xo, fo = _oracle_inputs(x, f, 0)
    ref = orc.mobility(po, xo, fo)
    for splits in (1, 3, 7):
        sd.sd_set_kernel_config(0, dict(variant=variant, block=block, splits=splits, ilp=ilp,
                                        kahan_block=kb))
        v = _run(sd, x, f, 0, ps)
        _check(v, ref, 0, variant, block, ilp, kb, splits)
    sd.sd_set_kernel_config(0, None)


@pytest.mark.parametrize("block,splits", [(64, 1), (128, 5), (256, 2)])
def test_parity_fp64_configs(sd, orc, block, splits):
    n = 777
    x = W.random_suspension(n, seed=17)
    f = W.gaussian_forces(n, seed=18)
    ps, po = _params(sd, orc)
    ref = orc.mobility(po, x, f)
    sd.sd_set_kernel_config(1, dict(variant=0, block=block, splits=splits, ilp=1, kahan_block=0))
    v = _run(sd, x, f, 1, ps)
    sd.sd_set_kernel_config(1, None)
    _check(v, ref, 1, block, splits)


@pytest.mark.parametrize("tensor,overlap", [(0, True), (1, False), (0, False)])
@pytest.mark.parametrize("prec", [0, 1])
def test_parity_overlapping_and_oseen(sd, orc, tensor, overlap, prec):
    """Dense Gaussian blob: many pairs with r < 2a, some below r < a."""
    n = 700
    x = np.random.default_rng(31).normal(0.0, 3.0, size=(n, 3))
    f = W.gaussian_forces(n, seed=32)
    ps, po = _params(sd, orc, a=1.3, eta=0.21, tensor=tensor, overlap=overlap)
    v = _run(sd, x, f, prec, ps)
    xo, fo = _oracle_inputs(x, f, prec)
    ref = orc.mobility(po, xo, fo)
    _check(v, ref, prec, tensor, overlap)


@pytest.mark.parametrize("prec", [0, 1])
def test_coincident_spheres(sd, orc, prec):
    """Distinct spheres at the same point: mu0 F_j with the overlap form, 0 otherwise."""
    x = W.random_suspension(300, seed=41)
    x[10] = x[20]
    x[100] = x[101] = x[102]
    f = W.gaussian_forces(300, seed=42)
    for overlap in (False, True):
        ps, po = _params(sd, orc, overlap=overlap)
        v = _run(sd, x, f, prec, ps)
        xo, fo = _oracle_inputs(x, f, prec)
        ref = orc.mobility(po, xo, fo)
        assert np.all(np.isfinite(v))
        _check(v, ref, prec, overlap)


@pytest.mark.parametrize("prec", [0, 1])
def test_single_particle_and_pair(sd, orc, prec):
    ps, po = _params(sd, orc, a=0.8, eta=0.3)
    x = np.array([[1.0, -2.0, 0.5]])
    f = np.array([[0.3, 0.2, -1.0]])
    v = _run(sd, x, f, prec, ps)
    np.testing.assert_allclose(v, f / (6 * np.pi * 0.3 * 0.8), rtol=1e-7 if prec == 0 else 1e-15)
    x = np.array([[0.0, 0.0, 0.0], [1.6, 0.0, 0.0]])  # touching, r = 2a
    f = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    v = _run(sd, x, f, prec, ps)
    np.testing.assert_allclose(v, orc.mobility(po, x, f), rtol=1e-7 if prec == 0 else 1e-14)


def test_deterministic(sd):
    import torch
    n = 3000
    x = W.random_suspension(n, seed=51)
    f = W.gaussian_forces(n, seed=52)
    ps = sd.params()
    pos, frc = to_dev4(x, torch.float32), to_dev4(f, torch.float32)
    ref = sd.mobility_apply(pos, frc, params=ps).clone()
    for _ in range(10):
        v = sd.mobility_apply(pos, frc, params=ps)
        assert torch.equal(v, ref)


@pytest.mark.parametrize("n", [16384])
def test_parity_full_16384(sd, orc, n):
    """Random suspension workload at n = 16384, full product."""
    x = W.random_suspension(n, phi=0.05, seed=1)
    f = W.gaussian_forces(n, seed=2)
    ps, po = _params(sd, orc)
    ref = orc.mobility(po, W.round_to_f32(x), W.round_to_f32(f))
    for prec in (0, 1):
        v = _run(sd, x, f, prec, ps)
        xo, fo = _oracle_inputs(x, f, prec)
        r = ref if prec == 0 else orc.mobility(po, xo, fo)
        _check(v, r, prec, n)


def test_parity_sampled_65536(sd, orc):
    """n = 65536 in the automatic launch configuration: 1024 sampled rows
    (including the first and last) against the oracle: the 2-norm over the
    sampled rows and the worst sampled row."""
    n = 65536
    x = W.random_suspension(n, phi=0.05, seed=1)
    f = W.gaussian_forces(n, seed=2)
    ps, po = _params(sd, orc)
    rows = np.unique(np.concatenate([[0, n - 1],
                                     np.random.default_rng(3).choice(n, 1022, replace=False)]))
    xo, fo = W.round_to_f32(x), W.round_to_f32(f)
    ref = orc.mobility_rows(po, xo, fo, rows)
    v = _run(sd, x, f, 0, ps)
    _check(v[rows], ref, 0, "n=65536 sampled")
    v64 = _run(sd, x, f, 1, ps)
    ref64 = orc.mobility_rows(po, x, f, rows)
    _check(v64[rows], ref64, 1, "n=65536 sampled")


def test_parity_full_65536(sd, orc):
    """n = 65536 (the benchmark product) in the automatic launch
    configuration against the full oracle product, every row (FP32 +
    Kahan; the oracle runs on all host cores)."""
    n = 65536
    x = W.random_suspension(n, phi=0.05, seed=1)
    f = W.gaussian_forces(n, seed=2)
    ps, po = _params(sd, orc)
    xo, fo = W.round_to_f32(x), W.round_to_f32(f)
    ref = orc.mobility(po, xo, fo)
    v = _run(sd, x, f, 0, ps)
    _check(v, ref, 0, "n=65536 full")


def test_parity_sampled_2_20(sd, orc):
    """n = 2^20 (a jittered fcc lattice at 0.1 / a^3, nearest pairs 2.3a apart),
    in the automatic launch configuration: sampled rows against the oracle in
    free space and in the periodic cube of the lattice, FP32 + Kahan and FP64."""
    n = 1 << 20
    x, L = W.jittered_fcc(64)
    assert x.shape[0] == n
    f = W.gaussian_forces(n, seed=7)
    rows = np.unique(np.concatenate([[0, n - 1],
                                     np.random.default_rng(8).choice(n, 254, replace=False)]))
    xo, fo = W.round_to_f32(x), W.round_to_f32(f)
    for box in (None, L):
        ps = sd.params(box=box) if box else sd.params()
        po = orc.params(box=box) if box else orc.params()
        v = _run(sd, x, f, 0, ps)
        _check(v[rows], orc.mobility_rows(po, xo, fo, rows), 0, "n=2^20", box)
        v64 = _run(sd, x, f, 1, ps)
        _check(v64[rows], orc.mobility_rows(po, x, f, rows), 1, "n=2^20", box)
