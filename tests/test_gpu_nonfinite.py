"""Non-finite inputs (NaN / Inf) are not checked by the library and propagate
into the results: a product whose inputs hold one NaN position or one Inf
force returns without error, and since every row sums a term of every other
particle (Eq. 7a), every output row is non-finite.  The next product on clean
inputs is unaffected (no workspace, flag or counter state survives), and no
pair is counted as breaking the r >= 2a premise.  In a periodic box positions
enter as fixed-point records, so a non-finite position becomes some point of
the box: the call still succeeds and leaves no state behind."""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import rel2, to_dev3, to_dev4  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    (0, dict(variant=0, block=256, splits=3, ilp=1, kahan_block=8)),
    (0, dict(variant=0, block=64, splits=2, ilp=2, kahan_block=2)),
    (2, dict(variant=1, block=128, splits=2, ilp=1, kahan_block=0)),
    (0, dict(variant=2, block=256, splits=4, ilp=1, kahan_block=8)),
    (0, dict(variant=2, block=256, splits=4, ilp=2, kahan_block=32)),
    (2, dict(variant=2, block=512, splits=2, ilp=1, kahan_block=0)),
    (1, None),
]


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1205_6333_amd as sd
    sd.lib()
    yield sd
    for prec in (0, 1, 2):
        sd.sd_set_kernel_config(prec, None)


def _apply(sd, x, f, prec, p):
    import torch
    dt = torch.float64 if prec == 1 else torch.float32
    v = sd.mobility_apply(to_dev4(x, dt), to_dev4(f, dt), params=p, precision=prec)
    torch.cuda.synchronize()
    return v.cpu().numpy()


@pytest.mark.parametrize("prec,cfg", CASES)
def test_nan_position_and_inf_force_propagate(sd, orc, prec, cfg):
    n = 1500
    x = W.random_suspension(n, phi=0.05, seed=61)
    f = W.gaussian_forces(n, seed=62)
    xr = x if prec == 1 else W.round_to_f32(x)
    fr = f if prec == 1 else W.round_to_f32(f)
    ref = orc.mobility(orc.params(overlap=True), xr, fr)
    p = sd.params(overlap=True)
    sd.sd_set_kernel_config(prec, cfg)
    try:
        sd.sd_premise_counts(reset=True)
        xb = x.copy()
        xb[700, 1] = np.nan
        v = _apply(sd, xb, f, prec, p)
        assert not np.isfinite(v).any()
        fb = f.copy()
        fb[3, 2] = np.inf
        v = _apply(sd, x, fb, prec, p)
        assert not np.isfinite(v).any()
        xb = x.copy()
        xb[n - 1] = [np.inf, -np.inf, np.nan]
        v = _apply(sd, xb, f, prec, p)
        assert not np.isfinite(v).any()
        assert sd.sd_premise_counts(reset=True) == (0, 0)
        v = _apply(sd, x, f, prec, p)
        assert rel2(v, ref) <= (1e-12 if prec == 1 else 1e-5)
    finally:
        sd.sd_set_kernel_config(prec, None)


@pytest.mark.parametrize("prec", [0, 1])
def test_periodic_box_non_finite_inputs(sd, orc, prec):
    L = 40.0
    n = 1200
    rng = np.random.default_rng(63)
    x = rng.uniform(0.0, L, size=(n, 3))
    f = W.gaussian_forces(n, seed=64)
    xr = x if prec == 1 else W.round_to_f32(x)
    fr = f if prec == 1 else W.round_to_f32(f)
    p = sd.params(overlap=True, box=L)
    ref = orc.mobility(orc.params(overlap=True, box=L), xr, fr)
    fb = f.copy()
    fb[10, 0] = np.nan
    assert not np.isfinite(_apply(sd, x, fb, prec, p)).any()
    xb = x.copy()
    xb[20] = [np.nan, np.inf, -np.inf]
    _apply(sd, xb, f, prec, p)                  # succeeds; the values are unspecified
    v = _apply(sd, x, f, prec, p)
    assert rel2(v, ref) <= (1e-12 if prec == 1 else 1e-5)


def test_time_step_with_a_nan_position(sd):
    """One Euler step from FP64 positions holding a NaN: every particle's new
    position is non-finite (every velocity is)."""
    import torch
    n = 900
    x = W.random_suspension(n, phi=0.05, seed=65)
    x[450, 0] = np.nan
    f = W.gravity_forces(n)
    for prec in (0, 1):
        dt = torch.float64 if prec == 1 else torch.float32
        xd = to_dev3(x)
        sd.sd_step(xd, to_dev4(f, dt), 1e-3, precision=prec)
        torch.cuda.synchronize()
        assert not np.isfinite(xd.cpu().numpy()).any()
