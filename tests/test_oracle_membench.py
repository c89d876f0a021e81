"""Pins of the App. A micro-benchmark oracle (oracle/membench.py): the maps
of App. A are permutations when gcd(p, N) = 1, so every thread of the naive
kernel (and of the tiled kernels with linear or strided access) adds the total
of the array; for N a multiple of p the strided map visits the multiples of p
only; the tiled kernels give one sum per work-group."""
import numpy as np
import pytest

from oracle import membench as MB


def _x(n, width, seed=0):
    shape = (n,) if width == 1 else (n, 4)
    return np.random.default_rng(seed).integers(0, 7, size=shape).astype(np.float64)


@pytest.mark.parametrize("n", [1, 100, 257, 1000])
@pytest.mark.parametrize("width", [1, 4])
def test_coprime_maps_sum_the_whole_array(n, width):
    x = _x(n, width)
    total = x.sum(axis=0)
    for kind_map in (0, 1, 2):
        np.testing.assert_array_equal(MB.membench(0, kind_map, x), x + total)
    for kind in (1, 2):
        for kind_map in (0, 1):
            np.testing.assert_array_equal(MB.membench(kind, kind_map, x), x + total)


def test_strided_map_with_common_factor():
    n = 3 * MB.P
    x = _x(n, 1, seed=1)
    want = x + MB.P * x[::MB.P].sum()  # k p mod 3p visits 0, p, 2p, each p times
    np.testing.assert_array_equal(MB.membench(0, 1, x), want)
    np.testing.assert_array_equal(MB.membench(2, 1, x), want)


def test_unordered_map_is_a_shifted_permutation():
    """Thread j of the naive kernel visits (k p + j M) mod N: a permutation for
    gcd(p, N) = 1, whose first index is j M mod N."""
    n = 1000
    k = np.arange(n)
    for j in (0, 1, 17, 999):
        idx = MB.map_indices(2, k, j, n)
        assert sorted(idx) == list(range(n))
        assert idx[0] == (j * MB.M) % n


@pytest.mark.parametrize("kind", [1, 2])
def test_tiled_unordered_is_uniform_per_work_group(kind):
    n = 700
    x = _x(n, 1, seed=2)
    out = MB.membench(kind, 2, x) - x
    for base in range(0, n, MB.BLOCK):
        blk = out[base:base + MB.BLOCK]
        assert np.all(blk == blk[0])
    # each tile slot reads one element: the per-group sum counts n elements
    brute = 0.0
    tile = MB.WAVE if kind == 1 else MB.BLOCK
    for m in range(0, n, tile):
        for s in range(min(tile, n - m)):
            brute += x[((m + s) * MB.P + s * MB.M) % n]
    assert out[0] == brute
