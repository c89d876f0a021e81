"""GPU parity in a periodic cubic box (nearest image, footnote of Sec. 3.1)
against the FP64 oracle: the mobility product, the time loop and the
lubrication correction, on tie-free configurations (random periodic
suspensions, a jittered fcc lattice); on the perfect fcc lattice of the
Sec. 3.3 benchmark only what is unique is compared (see
test_perfect_fcc_is_translation_invariant).

Tolerances as in free space: relative 2-norm 1e-6 (FP32-compensated),
1e-5 (plain FP32), 1e-12 (FP64), and per particle (rowerr) 1e-5, 1e-4 and
1e-11; the oracle is fed the FP32-rounded inputs of the FP32 paths."""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import rel2, rowerr, to_dev3, to_dev4

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
    assert torch.cuda.is_available()
    import paper_1205_6333_amd as sd
    sd.lib()
    yield sd
    for prec in (0, 1, 2):
        sd.sd_set_kernel_config(prec, None)


def _apply(sd, x, f, prec, p):
    import torch
    dt = torch.float64 if prec == sd.SD_FP64 else torch.float32
    v = sd.mobility_apply(to_dev4(x, dt), to_dev4(f, dt), params=p, precision=prec)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def _in(x, prec):
    return x if prec == 1 else W.round_to_f32(x)


@pytest.mark.parametrize("n", [1, 2, 65, 257, 1000, 4099])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("tensor", [0, 1])
def test_periodic_product_parity(sd, orc, n, prec, tensor):
    if n == 1:
        x, L = np.array([[1.0, 2.0, 3.0]]), 10.0
    elif n == 2:  # a near-contact pair across the boundary (FP64 branch)
        L = 12.0
        x = np.array([[0.4, 6.0, 6.0], [L - 1.6008, 6.0, 6.0]])
    else:
        x, L = W.periodic_suspension(n, phi=0.1, min_dist=2.05, seed=300 + n)
    f = W.gaussian_forces(n, seed=301 + n)
    ps = sd.params(tensor=tensor, box=L)
    po = orc.params(tensor=tensor, box=L)
    v = _apply(sd, x, f, prec, ps)
    ref = orc.mobility(po, _in(x, prec), _in(f, prec))
    _check(v, ref, prec, n, tensor, L)


@pytest.mark.parametrize("variant,block,ilp,kb", [(0, 64, 1, 1), (0, 128, 2, 4), (1, 256, 1, 8),
                                                  (1, 64, 2, 2), (0, 256, 1, 0)])
def test_periodic_kernel_shapes(sd, orc, variant, block, ilp, kb):
    n = 3001
    x, L = W.periodic_suspension(n, phi=0.2, min_dist=2.02, seed=310)
    f = W.gaussian_forces(n, seed=311)
    prec = 0 if kb else 2
    sd.sd_set_kernel_config(prec, dict(variant=variant, block=block, splits=5, ilp=ilp,
                                       kahan_block=kb))
    try:
        v = _apply(sd, x, f, prec, sd.params(box=L))
    finally:
        sd.sd_set_kernel_config(prec, None)
    ref = orc.mobility(orc.params(box=L), _in(x, prec), _in(f, prec))
    _check(v, ref, prec, variant, block, ilp, kb)


def test_periodic_wrapping_invariance(sd, orc):
    """Positions given outside the box (shifted by whole box sides) give the
    velocities of the wrapped positions."""
    n = 777
    x, L = W.periodic_suspension(n, phi=0.1, seed=320)
    f = W.gaussian_forces(n, seed=321)
    shift = np.random.default_rng(322).integers(-3, 4, size=x.shape) * L
    xs = W.round_to_f32(x + shift)
    for prec in (0, 1):
        v = _apply(sd, xs, f, prec, sd.params(box=L))
        ref = orc.mobility(orc.params(box=L), _in(xs, prec), _in(f, prec))
        _check(v, ref, prec, "wrapped")


@pytest.mark.parametrize("m", [4, 5])
def test_jittered_fcc_parity(sd, orc, m):
    x, L = W.jittered_fcc(m, jitter=0.05, seed=330 + m)
    f = W.gravity_forces(len(x)) + 0.1 * W.gaussian_forces(len(x), seed=331)
    for prec in (0, 1):
        v = _apply(sd, x, f, prec, sd.params(box=L))
        ref = orc.mobility(orc.params(box=L), _in(x, prec), _in(f, prec))
        _check(v, ref, prec, "jittered fcc", m)


def test_perfect_fcc_is_translation_invariant(sd, orc):
    """On the perfect fcc lattice pairs half a box apart have two nearest
    images, and which one a path takes follows from the rounding of its
    coordinates.  Under a force along z both images give the same z-velocity
    term, so v_z is unique: it is the same for every particle (each sees the
    same surroundings) and is compared with the oracle."""
    x, L = W.fcc_lattice(4)
    f = W.gravity_forces(len(x))
    for prec in (0, 1):
        v = _apply(sd, x, f, prec, sd.params(box=L))
        vz = v[:, 2]
        assert np.abs(vz - vz.mean()).max() / np.abs(vz).max() <= (1e-6 if prec == 0 else 1e-12)
        ref = orc.mobility(orc.params(box=L), _in(x, prec), _in(f, prec))
        assert rel2(vz, ref[:, 2]) <= TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("integ", [0, 1])
def test_periodic_run_parity(sd, orc, prec, integ):
    """Sedimentation in a box: particles leave through the bottom and enter
    through the top (the master positions stay unwrapped on both sides)."""
    import torch
    n = 500
    x0, L = W.periodic_suspension(n, phi=0.1, min_dist=2.2, seed=340)
    f = W.gravity_forces(n) + 0.3 * W.gaussian_forces(n, seed=341)
    fo = _in(f, prec)
    po = orc.params(box=L)
    steps, dt = 40, 0.05
    xr, _, _ = orc.run(po, x0, fo, dt, steps, integ)
    assert np.abs(xr - x0).max() > 1.0
    xd = to_dev3(x0)
    f4 = to_dev4(f, torch.float64 if prec == 1 else torch.float32)
    vp = torch.zeros_like(xd)
    sd.sd_run(xd, f4, dt, steps, params=sd.params(box=L), integrator=integ, precision=prec,
              v_prev=vp)
    torch.cuda.synchronize()
    err = np.abs(xd.cpu().numpy() - xr).max() / np.abs(xr - x0).max()
    print("prec=%d integ=%d err/disp=%.3e" % (prec, integ, err))
    assert err <= (1e-11 if prec == 1 else 1e-6)


def test_periodic_lubrication_parity(sd, orc):
    """Cell list in a box: close pairs across the faces, a grid of three cells
    per side (the smallest with distinct neighbours) and of one cell."""
    import torch
    rng = np.random.default_rng(350)
    lb_s, lb_o = sd.lub(), orc.lub()
    cases = []
    x, L = W.periodic_suspension(3000, phi=0.3, min_dist=2.02, seed=351)
    cases.append((x, L))
    x, L = W.periodic_suspension(60, phi=0.15, min_dist=2.02, seed=352)  # L ~ 11.5: 3 cells
    cases.append((x, L))
    L = 5.0                                                               # 1 cell
    cases.append((np.array([[0.2, 0.2, 0.2], [4.1, 0.3, 0.1], [2.5, 2.6, 4.8]]), L))
    for x, L in cases:
        v = rng.standard_normal(x.shape)
        ref = orc.lubrication_force(orc.params(box=L), lb_o, x, v)
        got = sd.lubrication_forces(to_dev3(x), to_dev3(v), params=sd.params(box=L),
                                    lub_params=lb_s)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert np.abs(ref).max() > 0.1
        assert rel2(got, ref) <= 1e-12


@pytest.mark.parametrize("prec", [1, 0])
def test_periodic_run_lub_parity(sd, orc, prec):
    import torch
    # phi = 0.1 with gaps >= 0.4a: the lagged correction stays bounded (denser
    # periodic packings amplify close-pair velocities step by step and blow up
    # in the oracle as well)
    n = 400
    x0, L = W.periodic_suspension(n, phi=0.1, min_dist=2.4, seed=360)
    f = W.gravity_forces(n) + 0.5 * W.gaussian_forces(n, seed=361)
    po, lo = orc.params(box=L), orc.lub()
    xr, vr, _ = orc.run_lub(po, lo, x0, f, 0.01, 30, 0)
    assert np.abs(orc.lubrication_force(po, lo, x0, vr)).max() > 0.1  # active correction
    xd = to_dev3(x0)
    vp = torch.zeros_like(xd)
    sd.sd_run_lub(xd, to_dev3(f), vp, 0.01, 30, params=sd.params(box=L), precision=prec)
    torch.cuda.synchronize()
    err = np.abs(xd.cpu().numpy() - xr).max() / np.abs(xr - x0).max()
    print("prec=%d err/disp=%.3e" % (prec, err))
    assert err <= (1e-11 if prec == 1 else 1e-6)


def test_fcc_full_size_sampled(sd, orc):
    """The largest size of the fcc benchmark (m = 37, N = 202612) in its launch
    configuration, jittered so that every nearest image is unique: 48 sampled
    rows of the FP32-compensated product against the oracle."""
    import torch
    x, L = W.jittered_fcc(37, jitter=0.05, seed=370)
    n = len(x)
    f = W.gravity_forces(n) + 0.1 * W.gaussian_forces(n, seed=371)
    x32, f32 = W.round_to_f32(x), W.round_to_f32(f)
    v = _apply(sd, x32, f32, 0, sd.params(box=L))
    rows = np.random.default_rng(372).choice(n, 48, replace=False)
    ref = orc.mobility_rows(orc.params(box=L), x32, f32, rows)
    _check(v[rows], ref, 0, "fcc sampled", n)


@pytest.mark.parametrize("prec", [0, 1])
def test_small_and_large_boxes(sd, orc, prec):
    """A box just larger than a sphere diameter (every pair near contact or
    overlapping through some image; overlap-regularised RPY) and a box far
    larger than the suspension (the nearest image is the free-space pair)."""
    rng = np.random.default_rng(380)
    L = 3.0
    x = rng.uniform(0.0, L, size=(7, 3))
    f = rng.standard_normal((7, 3))
    ps = sd.params(overlap=True, box=L)
    po = orc.params(overlap=True, box=L)
    v = _apply(sd, x, f, prec, ps)
    ref = orc.mobility(po, _in(x, prec), _in(f, prec))
    _check(v, ref, prec, "small box")
    x = W.random_suspension(500, phi=0.05, seed=381) + 100.0
    f = W.gaussian_forces(500, seed=382)
    v = _apply(sd, x, f, prec, sd.params(box=2000.0))
    ref = orc.mobility(orc.params(), _in(x, prec), _in(f, prec))   # free space
    _check(v, ref, prec, "large box")
