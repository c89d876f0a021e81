"""mobility_apply_noalloc (the product with its scratch in a static device
array, for callers that cannot allocate) against mobility_apply, through the
C ABI: two calls in a row on the same device, the second with a smaller
input, for every precision, in free space and in a periodic cube.  Bar: the
parity tolerances of the product (relative 2-norm 1e-6 and worst particle
1e-5 for FP32 + Kahan; 1e-12 / 1e-11 for FP64).  Sizes beyond the array are
rejected with SD_EINVAL before anything is enqueued."""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import rel2, rowerr, to_dev4  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {0: (1e-6, 1e-5), 2: (1e-5, 1e-4), 1: (1e-12, 1e-11)}


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1205_6333_amd as sd
    sd.lib()
    return sd


def _pair(sd, n, prec, box, seed):
    import torch
    if box:
        x, L = W.periodic_suspension(n, phi=0.1, seed=seed)
        p = sd.params(box=L)
    else:
        x = W.random_suspension(n, phi=0.05, seed=seed)
        p = sd.params()
    f = W.gaussian_forces(n, seed=seed + 1)
    dt = torch.float64 if prec == sd.SD_FP64 else torch.float32
    return to_dev4(x, dt), to_dev4(f, dt), p


@pytest.mark.parametrize("prec", [0, 2, 1])
@pytest.mark.parametrize("box", [False, True])
def test_noalloc_matches_mobility_apply(sd, prec, box):
    import torch
    if box and prec == 1:
        sizes = (3001, 700)
    else:
        sizes = (40000, 1337) if prec != 1 else (9000, 1337)
    for k, n in enumerate(sizes):
        pos, frc, p = _pair(sd, n, prec, box, seed=700 + 10 * k + prec)
        ref = sd.mobility_apply(pos, frc, params=p, precision=prec)
        out = torch.full((n, 3), float("nan"), dtype=torch.float64, device=pos.device)
        sd.mobility_apply_noalloc(pos, frc, out, params=p, precision=prec)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        err, row = rel2(a, b), rowerr(a, b)
        print("prec=%d box=%s n=%d rel2=%.3e row=%.3e" % (prec, box, n, err, row))
        assert np.all(np.isfinite(a))
        assert err <= TOL[prec][0], (n, err)
        assert row <= TOL[prec][1], (n, row)


def test_noalloc_rejects_sizes_beyond_its_scratch(sd):
    import torch
    n = (32 << 20) // 24 + 1
    pos = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    vel = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(sd.SdError) as e:
        sd.mobility_apply_noalloc(pos, pos, vel, precision=sd.SD_FP32_KAHAN)
    assert e.value.status == 1
    torch.cuda.synchronize()
    assert float(vel.abs().max()) == 0.0
