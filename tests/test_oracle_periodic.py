"""Pins of the oracle's periodic box with nearest-image interactions (footnote
of Sec. 3.1) and of the fcc benchmark workload of Sec. 3.3."""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W


@pytest.mark.parametrize("tensor", [0, 1])
def test_two_particles_nearest_image(orc, tensor):
    """In a box of side L a pair at separation d interacts as in free space at
    d if |d| < L/2 and at d - L otherwise (the nearest image)."""
    L = 20.0
    pb = orc.params(tensor=tensor, box=L)
    pf = orc.params(tensor=tensor)
    F = np.array([[0.3, -0.2, 1.0], [-0.5, 0.4, 0.1]])
    for d in (3.0, 7.5, 12.5, 16.9):
        dv = np.array([d, 0.4, -0.3])
        xb = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0] + dv])
        near = dv.copy()
        near[0] = d if d < L / 2 else d - L
        xf = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0] + near])
        np.testing.assert_allclose(orc.mobility(pb, xb, F), orc.mobility(pf, xf, F),
                                   rtol=1e-13, atol=1e-15)


def test_periodic_translation_invariance(orc):
    x, L = W.fcc_lattice(3)
    x = x + np.random.default_rng(1).normal(0, 0.3, size=x.shape)
    f = W.gaussian_forces(len(x), seed=2)
    p = orc.params(box=[L, L, L])
    v = orc.mobility(p, x, f)
    y = x.copy()
    y[5] += np.array([L, -2 * L, 0.0])       # a lattice translation of one particle
    y[17] -= np.array([0.0, 0.0, 3 * L])
    np.testing.assert_allclose(orc.mobility(p, y, f), v, rtol=1e-12, atol=1e-13)
    s = np.array([0.37 * L, -1.9 * L, 2.2])   # global shift, then wrap into the box
    np.testing.assert_allclose(orc.mobility(p, np.mod(x + s, L), f), v, rtol=1e-12, atol=1e-13)


def test_large_box_is_free_space(orc):
    x = W.random_suspension(60, phi=0.05, seed=3)
    f = W.gaussian_forces(60, seed=4)
    np.testing.assert_allclose(orc.mobility(orc.params(box=1e7), x, f),
                               orc.mobility(orc.params(), x, f), rtol=1e-13, atol=1e-15)


def test_lubrication_across_the_boundary(orc):
    L = 30.0
    pb, lb = orc.params(box=L), orc.lub()
    x = np.array([[0.5, 10.0, 10.0], [L - 2.0, 10.2, 9.9]])   # 2.5 apart through x = 0
    v = np.array([[0.1, -0.2, 0.3], [-0.4, 0.0, 0.2]])
    xf = x.copy()
    xf[1, 0] -= L
    np.testing.assert_allclose(orc.lubrication_force(pb, lb, x, v),
                               orc.lubrication_force(orc.params(), lb, xf, v), rtol=1e-13)


def test_fcc_lattice_generator():
    x, L = W.fcc_lattice(4)
    assert x.shape == (256, 3)
    np.testing.assert_allclose(len(x) / L ** 3, 0.1, rtol=1e-14)
    c = L / 4
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(len(x)) * 1e9
    np.testing.assert_allclose(r.min(1), c / np.sqrt(2), rtol=1e-12)
    assert np.all((np.abs(r - c / np.sqrt(2)) < 1e-9).sum(1) == 12)


def test_tie_free_lattice_sediments_uniformly(orc):
    """A simple cubic lattice with an odd number of sites per side has no pair
    exactly half a box apart, so every particle sees the same set of nearest
    images: under a uniform force all velocities are equal and, by the cubic
    symmetry, parallel to the force.  (The fcc start of Sec. 3.3 does have
    pairs at exactly L/2, where the nearest image is not unique.)"""
    m, c = 5, 3.1
    g = np.arange(m) * c
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = orc.params(box=m * c)
    v = orc.mobility(p, x, W.gravity_forces(len(x)))
    np.testing.assert_allclose(v[:, :2], 0.0, atol=1e-12)
    np.testing.assert_allclose(v[:, 2], v[0, 2], rtol=1e-12)
    assert v[0, 2] < -1.0  # hydrodynamic coupling speeds the lattice up


def test_periodic_adjoint_and_symmetry(orc):
    """In the box the matrix stays symmetric (nearest images are mutual) and
    the vector-Jacobian product matches central differences across the
    boundary."""
    L = 14.0
    rng = np.random.default_rng(21)
    x = rng.uniform(0, L, size=(12, 3))
    x[0] = [0.3, 7.0, 7.0]
    x[1] = [L - 1.9, 7.4, 6.8]   # close to x[0] through the x = 0 face
    p = orc.params(box=L, overlap=True)
    M = orc.dense_mobility(p, x)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-15)
    f, lam = W.gaussian_forces(12, seed=22), W.gaussian_forces(12, seed=23)
    np.testing.assert_allclose(orc.mobility_transpose(p, x, lam).reshape(-1),
                               M.T @ lam.reshape(-1), rtol=1e-13, atol=1e-15)
    g = orc.mobility_vjp_x(p, x, f, lam)
    fd = np.zeros_like(x)
    h = 1e-6
    for i in range(12):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd[i, k] = (np.sum(lam * orc.mobility(p, xp, f)) -
                        np.sum(lam * orc.mobility(p, xm, f))) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8 * np.abs(g).max())


def test_periodic_input_generators():
    """Inputs of the periodic tests: the periodic RSA keeps the nearest-image
    distance, the jittered lattice lies in [0, L) and has no pair exactly half
    a box apart along any axis (its nearest images are unique)."""
    x, L = W.periodic_suspension(400, phi=0.2, min_dist=2.1, seed=5)
    d = x[:, None] - x[None]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    assert r.min() >= 2.1 and x.min() >= 0 and x.max() < L
    xj, Lj = W.jittered_fcc(4, jitter=0.05, seed=6)
    assert xj.min() >= 0 and xj.max() < Lj
    dj = np.abs(xj[:, None] - xj[None])
    assert np.abs(dj - Lj / 2).min() > 1e-6
