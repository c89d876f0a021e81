"""Seeded synthetic inputs for the mobility product and the time loop.

This module only draws positions and forces; it holds none of the method's
arithmetic.  Both the GPU library's callers (tests, benchmark) and the FP64
oracle's tests take their inputs from here, so the two sides always see the
same numbers.

Recipes (the paper's own workloads are synthetic too: Sec. 3.3 uses particles
on an fcc lattice under a constant sedimentation force, Sec. 4 a four-sphere
cluster):

* ``random_suspension``: random sequential addition in a cube centred at the
  origin.  Candidates are drawn uniformly, one after another, from a seeded
  PCG64 stream; a candidate closer than ``min_dist`` to any accepted particle
  is rejected.  The cube side follows from the volume fraction,
  L = (n * 4 pi a^3 / 3 / phi)^(1/3).
* ``gaussian_forces``: i.i.d. N(0, 1) components.
* ``gravity_forces``: the constant sedimentation force (0, 0, -F) of Sec. 3.3.
* ``clusters``: independent clusters with sizes uniform on [nmin, nmax],
  Gaussian positions (standard deviation ``sigma``) with the same sequential
  rejection inside each cluster.
* ``four_sphere_tetrahedron`` and ``square_xz``: the small sedimenting clusters
  of Sec. 4 (see the docstrings for the reading of the printed coordinates).
"""
from __future__ import annotations

import numpy as np

try:  # scipy is used only to accelerate the rejection test
    from scipy.spatial import cKDTree
except Exception:  # pragma: no cover
    cKDTree = None


def box_side(n: int, phi: float, a: float = 1.0) -> float:
    """Side of the cube holding n spheres of radius a at volume fraction phi."""
    return float((n * 4.0 * np.pi * a ** 3 / 3.0 / phi) ** (1.0 / 3.0))


def _sequential_reject(draw, n: int, min_dist: float, batch: int = 8192,
                       boxsize: float | None = None) -> np.ndarray:
    """Accept candidates from ``draw(k) -> (k, 3)`` in stream order; a candidate
    is rejected when its distance to an already accepted one is < min_dist.
    Exactly the one-at-a-time procedure, evaluated batch-wise.  ``boxsize``:
    distances are nearest-image distances of that periodic cube (candidates
    must lie in [0, boxsize))."""
    acc = np.empty((n, 3))
    count = 0
    idle = 0
    while count < n:
        if idle > 100:  # jammed: no candidate accepted in 100 batches
            raise RuntimeError("cannot place %d spheres at minimum distance %g (placed %d)"
                               % (n, min_dist, count))
        cand = draw(batch)
        ok = np.ones(len(cand), dtype=bool)
        if count:
            if cKDTree is not None:
                d, _ = cKDTree(acc[:count], boxsize=boxsize).query(cand, k=1)
            else:
                d = np.sqrt((_img(cand[:, None, :] - acc[None, :count, :], boxsize) ** 2)
                            .sum(-1)).min(1)
            ok &= d >= min_dist
        idx = np.nonzero(ok)[0]
        c2 = cand[idx]
        keep = np.ones(len(c2), dtype=bool)
        if len(c2) > 1:
            if cKDTree is not None:
                pairs = cKDTree(c2, boxsize=boxsize).query_pairs(min_dist * (1 - 1e-15),
                                                                 output_type="ndarray")
            else:
                dd = np.sqrt((_img(c2[:, None, :] - c2[None, :, :], boxsize) ** 2).sum(-1))
                ii, jj = np.nonzero(np.triu(dd < min_dist, 1))
                pairs = np.stack([ii, jj], 1)
            if len(pairs):
                pairs = np.sort(pairs, axis=1)
                # exact check of the boundary (query_pairs uses <=)
                dd = np.sqrt((_img(c2[pairs[:, 0]] - c2[pairs[:, 1]], boxsize) ** 2).sum(-1))
                pairs = pairs[dd < min_dist]
                earlier = {}
                for i, j in pairs:
                    earlier.setdefault(int(j), []).append(int(i))
                for j in sorted(earlier):
                    if any(keep[i] for i in earlier[j]):
                        keep[j] = False
        c2 = c2[keep]
        take = min(n - count, len(c2))
        acc[count:count + take] = c2[:take]
        count += take
        idle = 0 if take else idle + 1
    return acc


def _img(d, boxsize):
    """Nearest-image difference in a periodic cube (identity without a box);
    used only to measure distances for the rejection test."""
    return d if boxsize is None else d - boxsize * np.rint(d / boxsize)


def random_suspension(n: int, phi: float = 0.05, a: float = 1.0, min_dist: float = 2.2,
                      seed: int = 1) -> np.ndarray:
    """(n, 3) float64 positions: random sequential addition in a centred cube."""
    L = box_side(n, phi, a)
    rng = np.random.default_rng(seed)
    return _sequential_reject(lambda k: rng.uniform(-L / 2, L / 2, size=(k, 3)), n,
                              min_dist * a)


def periodic_suspension(n: int, phi: float = 0.05, a: float = 1.0, min_dist: float = 2.2,
                        seed: int = 1):
    """Random sequential addition in a periodic cube [0, L)^3 (nearest-image
    distances in the rejection test).  Returns (positions (n, 3), L)."""
    L = box_side(n, phi, a)
    rng = np.random.default_rng(seed)
    x = _sequential_reject(lambda k: rng.uniform(0.0, L, size=(k, 3)), n, min_dist * a,
                           boxsize=L)
    return x, L


def gaussian_forces(n: int, seed: int = 2) -> np.ndarray:
    """(n, 3) float64 forces with i.i.d. N(0, 1) components."""
    return np.random.default_rng(seed).standard_normal((n, 3))


def gravity_forces(n: int, F: float = 1.0) -> np.ndarray:
    """(n, 3) float64 constant forces (0, 0, -F)."""
    f = np.zeros((n, 3))
    f[:, 2] = -F
    return f


def cluster_sizes(n_clusters: int, nmin: int = 4, nmax: int = 256, seed: int = 3) -> np.ndarray:
    """Cluster sizes, integer-uniform on [nmin, nmax]."""
    return np.random.default_rng(seed).integers(nmin, nmax + 1, size=n_clusters).astype(np.int64)


def clusters(n_clusters: int, nmin: int = 4, nmax: int = 256, sigma: float = 4.0,
             min_dist: float = 2.2, a: float = 1.0, seed: int = 3):
    """Independent free-space clusters.

    Returns (offsets[C+1] int64, positions (sum N_c, 3) float64).  Cluster c
    owns rows offsets[c]:offsets[c+1]; its positions are N(0, sigma^2 a^2) per
    component with sequential rejection at min_dist (within the cluster only;
    clusters do not interact, so no global placement is needed).
    """
    sizes = cluster_sizes(n_clusters, nmin, nmax, seed)
    rng = np.random.default_rng(seed + 1000)
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.empty((int(offsets[-1]), 3))
    for c, nc in enumerate(sizes):
        pos[offsets[c]:offsets[c + 1]] = _sequential_reject(
            lambda k: rng.normal(0.0, sigma * a, size=(k, 3)), int(nc), min_dist * a, batch=64)
    return offsets, pos


def four_sphere_tetrahedron(a: float = 1.0, d: float = 5.0):
    """The four-sphere sedimenting cluster of Sec. 4 (Fig. 4a).

    The printed initial coordinates are garbled: as printed, the four points
    are coplanar, which contradicts both the "stretched tetrahedron with two
    opposing edges perpendicular to the force" and the stated symmetry
    relations (x3 = -x1, z3 = z1, z4 = z2, y1 = y3 = x2 = x4 = 0).  The reading
    that satisfies all of them: two horizontal couples, one along x at height
    +d a, one along y at height -d a:
        r1 = ( d, 0,  d) a,  r3 = (-d, 0,  d) a,
        r2 = ( 0, d, -d) a,  r4 = ( 0,-d, -d) a,
    each dragged by F = (0, 0, -1).
    """
    x = np.array([[d, 0.0, d], [0.0, d, -d], [-d, 0.0, d], [0.0, -d, -d]]) * a
    return x, gravity_forces(4)


def square_xz(side: float = 5.0, a: float = 1.0):
    """Four spheres on a square of the given side (in units of a) in the x-z
    plane, centred at the origin, labelled 1 = (+,+), 2 = (-,+), 3 = (-,-),
    4 = (+,-) in (x, z); constant force (0, 0, -1) on each."""
    h = 0.5 * side * a
    x = np.array([[h, 0.0, h], [-h, 0.0, h], [-h, 0.0, -h], [h, 0.0, -h]])
    return x, gravity_forces(4)


def fcc_lattice(m: int, density: float = 0.1, a: float = 1.0):
    """Sec. 3.3 benchmark start: a perfect fcc lattice of m^3 cubic unit cells
    (N = 4 m^3 particles) at number density n = N / L^3 (0.1 / a^3 in the
    paper).  Returns (positions (N, 3) in [0, L)^3, box side L)."""
    c = (4.0 / density) ** (1.0 / 3.0) * a
    basis = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    g = np.arange(m, dtype=np.float64)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * c
    return x, m * c


def jittered_fcc(m: int, density: float = 0.1, a: float = 1.0, jitter: float = 0.05,
                 seed: int = 4):
    """The fcc start of ``fcc_lattice`` with every coordinate displaced by
    U(-jitter, jitter) a and wrapped into [0, L): no pair is exactly half a box
    apart, so the nearest image of every pair is unique.  Returns (x, L)."""
    x, L = fcc_lattice(m, density, a)
    x = x + np.random.default_rng(seed).uniform(-jitter * a, jitter * a, size=x.shape)
    return x - L * np.floor(x / L), L


def to_float4(v: np.ndarray, dtype=np.float32) -> np.ndarray:
    """(n, 3) -> (n, 4) with w = 0, in the given dtype (the device layout)."""
    out = np.zeros((v.shape[0], 4), dtype=dtype)
    out[:, :3] = v
    return out


def round_to_f32(v: np.ndarray) -> np.ndarray:
    """Round to float32 and back: the values an FP32 input actually holds."""
    return np.asarray(v, dtype=np.float32).astype(np.float64)
