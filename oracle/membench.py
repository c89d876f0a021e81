"""Oracle of the App. A memory-access micro-benchmarks (test infrastructure
only: used by tests/, never by the library).

Plain numpy, written from the definitions of App. A: N threads, thread j sums
its own element and the N elements its access map visits.  Maps: linear
k -> k, strided k -> k p mod N, unordered k -> (k p + j M) mod N, with p = 131
and M = 64 (the wavefront of the GPU the kernels run on; the paper's M = 32 is
its warp size).  In the tiled kernels thread n of a work-group of B threads
loads tile slot n (n < TILE) for every tile m = 0, TILE, ..., i.e. element
m + n through the map evaluated with j = (work-group base) + n; every thread of
the work-group adds the whole tile.  The sums are exact when the inputs are
small integers (as in the tests), so the comparison is bit-exact.
"""
from __future__ import annotations

import numpy as np

P, M, BLOCK, WAVE = 131, 64, 128, 64


def map_indices(kind_map: int, k: np.ndarray, j, n: int) -> np.ndarray:
    """Element index of access k for thread(s) j (broadcasting)."""
    k = np.asarray(k, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    if kind_map == 0:
        return k + 0 * j
    if kind_map == 1:
        return (k * P) % n + 0 * j
    return (k * P + j * M) % n


def naive(x: np.ndarray, kind_map: int) -> np.ndarray:
    """out[j] = x[j] + sum_k x[map(k, j)], k < N."""
    n = x.shape[0]
    out = np.empty_like(x, dtype=np.float64)
    k = np.arange(n)
    for j in range(n):
        out[j] = x[j] + x[map_indices(kind_map, k, j, n)].sum(axis=0)
    return out


def tiled(x: np.ndarray, kind_map: int, tile: int) -> np.ndarray:
    """The tiled kernels: for every tile m, slot s < min(tile, N - m) holds
    x[map(m + s, base + s)]; every thread of the work-group adds every slot."""
    n = x.shape[0]
    out = np.empty_like(x, dtype=np.float64)
    for base in range(0, n, BLOCK):
        tot = np.zeros(x.shape[1:])
        for m in range(0, n, tile):
            s = np.arange(min(tile, n - m))
            tot = tot + x[map_indices(kind_map, m + s, base + s, n)].sum(axis=0)
        hi = min(n, base + BLOCK)
        out[base:hi] = x[base:hi] + tot
    return out


def membench(kind: int, kind_map: int, x: np.ndarray) -> np.ndarray:
    """kind: 0 naive, 1 small tiling (tile = one wave), 2 tiling (tile = block)."""
    x = np.asarray(x, dtype=np.float64)
    if kind == 0:
        return naive(x, kind_map)
    return tiled(x, kind_map, WAVE if kind == 1 else BLOCK)
