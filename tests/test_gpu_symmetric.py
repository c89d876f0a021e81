"""GPU parity of the pair-symmetric product kernel (kernel variant 2) against
the FP64 oracle.

Variant 2 evaluates every pair of particles in different blocks once and
hands T(r_ij) F_i to particle j through DPP rotations within 16-lane rows
(block symmetry of M, Sec. 3.3).  The cases cover every shape of its block
schedule: one block (no off-diagonal work), two blocks (only the antipode),
odd and even block counts, ragged last blocks, splits from one to more than
there are tiles, near and overlapping pairs on both sides of a pair,
coincident spheres, the Oseen tensor, the periodic cube and the time loop.
Tolerances as in test_gpu_mobility.py (relative 2-norm): 1e-6 for FP32 +
Kahan, 1e-5 for plain FP32.
"""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import rel2, to_dev4  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {0: 1e-6, 2: 1e-5}


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1205_6333_amd as sd
    sd.lib()
    yield sd
    for prec in (0, 1, 2):
        sd.sd_set_kernel_config(prec, None)


def _apply(sd, x, f, prec, p, cfg):
    import torch
    sd.sd_set_kernel_config(prec, cfg)
    try:
        v = sd.mobility_apply(to_dev4(x, torch.float32), to_dev4(f, torch.float32), params=p,
                              precision=prec)
        torch.cuda.synchronize()
    finally:
        sd.sd_set_kernel_config(prec, None)
    return v.cpu().numpy()


def _cfg(block, splits, kb, ilp=1):
    return dict(variant=2, block=block, splits=splits, ilp=ilp, kahan_block=kb)


# (work-group size, particles per lane): blocks of 128 to 512 particles
SHAPES = [(128, 1), (256, 1), (512, 1), (128, 2), (256, 2)]


@pytest.mark.parametrize("n", [1, 2, 17, 128, 129, 255, 256, 257, 511, 512, 513, 769, 1000,
                               1337, 2049])
@pytest.mark.parametrize("block,ilp", SHAPES)
def test_sym_sizes(sd, orc, n, block, ilp):
    x = W.random_suspension(n, seed=400 + n)
    f = W.gaussian_forces(n, seed=500 + n)
    ref = orc.mobility(orc.params(), W.round_to_f32(x), W.round_to_f32(f))
    for splits in (1, 3, 1000):
        v = _apply(sd, x, f, 0, sd.params(), _cfg(block, splits, 8, ilp))
        err = rel2(v, ref)
        print("n=%d block=%d ilp=%d splits=%d rel2=%.3e" % (n, block, ilp, splits, err))
        assert err <= TOL[0], (n, block, ilp, splits, err)


@pytest.mark.parametrize("kb,prec", [(0, 2), (4, 0), (8, 0)])
@pytest.mark.parametrize("tensor", [0, 1])
@pytest.mark.parametrize("ilp", [1, 2])
def test_sym_accumulation_and_tensor(sd, orc, kb, prec, tensor, ilp):
    n = 3001
    x = W.random_suspension(n, seed=410)
    f = W.gaussian_forces(n, seed=411)
    po = orc.params(tensor=tensor)
    ref = orc.mobility(po, W.round_to_f32(x), W.round_to_f32(f))
    v = _apply(sd, x, f, prec, sd.params(tensor=tensor), _cfg(256, 4, kb, ilp))
    assert rel2(v, ref) <= TOL[prec]


@pytest.mark.parametrize("tensor,overlap", [(0, True), (1, False), (0, False)])
def test_sym_overlapping_pairs(sd, orc, tensor, overlap):
    """Dense Gaussian blob: many near pairs (r < 2a, some r < a) between
    blocks, evaluated in FP64 on both sides."""
    n = 1500
    x = np.random.default_rng(431).normal(0.0, 4.0, size=(n, 3))
    f = W.gaussian_forces(n, seed=432)
    po = orc.params(a=1.3, eta=0.21, tensor=tensor, overlap=overlap)
    ps = sd.params(1.3, 0.21, tensor, overlap)
    ref = orc.mobility(po, W.round_to_f32(x), W.round_to_f32(f))
    for block, ilp in SHAPES:
        v = _apply(sd, x, f, 0, ps, _cfg(block, 2, 8, ilp))
        assert rel2(v, ref) <= TOL[0], (block, ilp)


def test_sym_coincident_spheres(sd, orc):
    n = 700
    x = W.random_suspension(n, seed=441)
    x[10] = x[300]          # different blocks of 128 and of 256
    x[5] = x[6] = x[600]
    f = W.gaussian_forces(n, seed=442)
    for overlap in (False, True):
        ref = orc.mobility(orc.params(overlap=overlap), W.round_to_f32(x), W.round_to_f32(f))
        for block, ilp in SHAPES:
            v = _apply(sd, x, f, 0, sd.params(overlap=overlap), _cfg(block, 3, 8, ilp))
            assert np.all(np.isfinite(v))
            assert rel2(v, ref) <= TOL[0], (overlap, block, ilp)


@pytest.mark.parametrize("n", [700, 3001])
def test_sym_periodic(sd, orc, n):
    """Nearest image in a periodic cube (fixed-point records), with pairs
    close to contact (min distance 2.02a) across the faces."""
    x, L = W.periodic_suspension(n, phi=0.2, min_dist=2.02, seed=450 + n)
    f = W.gaussian_forces(n, seed=451)
    ref = orc.mobility(orc.params(box=L), W.round_to_f32(x), W.round_to_f32(f))
    for block, ilp in SHAPES:
        v = _apply(sd, x, f, 0, sd.params(box=L), _cfg(block, 5, 8, ilp))
        assert rel2(v, ref) <= TOL[0], (block, ilp)


def test_sym_matches_variant0_and_is_deterministic(sd):
    import torch
    n = 5000
    x = W.random_suspension(n, seed=461)
    f = W.gaussian_forces(n, seed=462)
    p = sd.params()
    a = _apply(sd, x, f, 0, p, _cfg(256, 8, 8))
    b = _apply(sd, x, f, 0, p, dict(variant=0, block=256, splits=8, ilp=1, kahan_block=8))
    assert rel2(a, b) <= 1e-6
    sd.sd_set_kernel_config(0, _cfg(256, 8, 8))
    try:
        pos, frc = to_dev4(x, torch.float32), to_dev4(f, torch.float32)
        ref = sd.mobility_apply(pos, frc, params=p).clone()
        for _ in range(5):
            assert torch.equal(sd.mobility_apply(pos, frc, params=p), ref)
    finally:
        sd.sd_set_kernel_config(0, None)


def test_sym_time_loop(sd, orc):
    """AB2 time loop with the overlap form through the symmetric kernel
    against the oracle's run (FP64 positions, near pairs in FP64): 40 steps
    of a dense suspension (phi = 0.2, contacts at 2a)."""
    import torch
    n = 1200
    x0 = W.random_suspension(n, phi=0.2, min_dist=2.0, seed=471)
    f = W.gravity_forces(n) + 0.3 * W.gaussian_forces(n, seed=472)
    xr, vr, _ = orc.run(orc.params(overlap=True), x0, W.round_to_f32(f), 0.005, 40, orc.AB2)
    for block, ilp in SHAPES:
        sd.sd_set_kernel_config(0, _cfg(block, 3, 8, ilp))
        try:
            xd = torch.tensor(x0, dtype=torch.float64, device="cuda")
            vp = torch.zeros_like(xd)
            sd.sd_run(xd, to_dev4(f, torch.float32), 0.005, 40, v_prev=vp,
                      params=sd.params(overlap=True), integrator=sd.SD_AB2,
                      precision=sd.SD_FP32_KAHAN)
            torch.cuda.synchronize()
        finally:
            sd.sd_set_kernel_config(0, None)
        err = np.abs(xd.cpu().numpy() - xr).max() / np.abs(xr - x0).max()
        print("block=%d ilp=%d time loop err/disp = %.3e" % (block, ilp, err))
        assert err <= 1e-6
