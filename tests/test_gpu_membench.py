"""GPU App. A micro-benchmarks (sd_membench) against the oracle, bit-exact:
inputs are small integers, so every float sum is exact whatever its order."""
import numpy as np
import pytest

from oracle import membench as MB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available()
    import paper_1205_6333_amd as sd
    sd.lib()
    return sd


def _x(n, width, seed):
    shape = (n,) if width == 1 else (n, 4)
    return np.random.default_rng(seed).integers(0, 7, size=shape).astype(np.float32)


@pytest.mark.parametrize("n", [1, 63, 128, 1000, 1048, 4099])
@pytest.mark.parametrize("width", [1, 4])
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("kind_map", [0, 1, 2])
def test_membench_parity(sd, n, width, kind, kind_map):
    import torch
    x = _x(n, width, seed=n + width)
    got = sd.sd_membench(kind, kind_map, torch.tensor(x, device="cuda"))
    torch.cuda.synchronize()
    want = MB.membench(kind, kind_map, x.astype(np.float64))
    assert np.array_equal(got.cpu().numpy().astype(np.float64), want)


@pytest.mark.parametrize("width", [1, 4])
def test_membench_full_size(sd, width):
    """N = 65536 (the size of the benchmark): gcd(131, N) = 1, so every
    thread of the naive kernel, and of the tiled kernels with linear or
    strided access, adds the total of the array (a property at any size)."""
    import torch
    n = 65536
    x = _x(n, width, seed=9)
    xd = torch.tensor(x, device="cuda")
    want = x.astype(np.float64) + x.astype(np.float64).sum(axis=0)
    for kind, kind_map in [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (2, 0), (2, 1)]:
        got = sd.sd_membench(kind, kind_map, xd)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().astype(np.float64), want), (kind, kind_map)
    # tiled unordered: one value per work-group, checked on sampled groups
    for kind in (1, 2):
        got = sd.sd_membench(kind, 2, xd).cpu().numpy().astype(np.float64) - x
        tile = MB.WAVE if kind == 1 else MB.BLOCK
        for base in (0, 128 * 17, n - 128):
            s = np.arange(tile)
            tot = 0.0
            for m in range(0, n, tile):
                tot = tot + x[MB.map_indices(2, m + s, base + s, n)].astype(np.float64).sum(axis=0)
            assert np.array_equal(got[base:base + 128], np.broadcast_to(tot, got[base:base + 128].shape))
