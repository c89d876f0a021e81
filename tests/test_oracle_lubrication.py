"""Pins of the oracle's lubrication correction (Eq. 8, Sec. 2.3; step 2 of the
algorithm of Sec. 3.1) against lubrication theory and invariants."""
import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_reynolds_squeeze_film_limit(orc):
    """Two equal spheres approaching along their line of centres: the leading
    lubrication resistance is Reynolds' squeeze film between spheres of reduced
    radius a/2, F = 6 pi eta (a/2)^2 U / h, h = r - 2a."""
    a, eta = 1.7, 0.35
    p = orc.params(a=a, eta=eta)
    lb = orc.lub(s_min=1e-15)
    for s in (1e-9, 1e-10):
        h = s * a
        Z = orc.lub_tensor(p, lb, [0.0, 0.0, 2 * a + h])
        reynolds = 6 * np.pi * eta * (a / 2) ** 2 / h
        assert abs(Z[2, 2] / reynolds - 1) < 1e-6


def test_jeffrey_onishi_coefficients(orc):
    """The coefficients of Eq. 8 are the equal-size (lambda = 1) values of
    Jeffrey & Onishi's near-contact resistance functions,
    X^A_11 ~ g1/xi + g2 log(1/xi),  Y^A_11 ~ g3 log(1/xi) (units 6 pi eta a),
    g1 = 2 l^2/(1+l)^3, g2 = l (1 + 7 l + l^2) / (5 (1+l)^3),
    g3 = 4 l (2 + l + 2 l^2) / (15 (1+l)^3).
    Both coefficients are recovered from the oracle's tensor at two
    separations by solving the 2x2 linear system."""
    lam = 1.0
    g1 = 2 * lam ** 2 / (1 + lam) ** 3
    g2 = lam * (1 + 7 * lam + lam ** 2) / (5 * (1 + lam) ** 3)
    g3 = 4 * lam * (2 + lam + 2 * lam ** 2) / (15 * (1 + lam) ** 3)
    a, eta = 1.0, 0.2
    mu0 = 1 / (6 * np.pi * eta * a)
    p = orc.params(a=a, eta=eta)
    lb = orc.lub()
    s1, s2 = 0.01, 0.3
    Zs = [orc.lub_tensor(p, lb, [0.0, 0.0, (2 + s) * a]) * mu0 for s in (s1, s2)]
    A = np.array([[1 / s1, np.log(1 / s1)], [1 / s2, np.log(1 / s2)]])
    c = np.linalg.solve(A, [Zs[0][2, 2], Zs[1][2, 2]])
    np.testing.assert_allclose(c, [g1, g2], rtol=1e-12)
    for Z, s in zip(Zs, (s1, s2)):
        np.testing.assert_allclose(Z[0, 0], g3 * np.log(1 / s), rtol=1e-12)
        np.testing.assert_allclose(Z[1, 1], Z[0, 0], rtol=1e-14)


def test_truncation_and_clamp(orc):
    p = orc.params()
    lb = orc.lub(s_cut=1.0, s_min=1e-3)
    assert np.all(orc.lub_tensor(p, lb, [3.0, 0, 0]) == 0)          # s = 1: cut
    assert np.all(orc.lub_tensor(p, lb, [0, 3.5, 0]) == 0)
    assert orc.lub_tensor(p, lb, [2.999, 0, 0])[0, 0] > 0             # s < 1: active
    np.testing.assert_array_equal(orc.lub_tensor(p, lb, [2.0 + 1e-6, 0, 0]),
                                  orc.lub_tensor(p, lb, [2.0 + 1e-3, 0, 0]))  # clamp
    np.testing.assert_array_equal(orc.lub_tensor(p, lb, [1.5, 0, 0]),
                                  orc.lub_tensor(p, lb, [2.0 + 1e-3, 0, 0]))  # overlap


@pytest.fixture(scope="module")
def dense():
    x = W.random_suspension(200, phi=0.3, min_dist=2.02, seed=91)
    v = W.gaussian_forces(200, seed=92)
    return x, v


def test_lubrication_conserves_momentum_and_dissipates(orc, dense):
    """Pairwise forces are equal and opposite (sum f = 0), vanish for rigid
    translation, and dissipate: sum f_i . v_i < 0 (the friction is positive
    definite for s < 1)."""
    x, v = dense
    p, lb = orc.params(), orc.lub()
    f = orc.lubrication_force(p, lb, x, v)
    assert np.abs(f).max() > 0.1  # the configuration has close pairs
    np.testing.assert_allclose(f.sum(0), 0, atol=1e-10 * np.abs(f).max())
    np.testing.assert_allclose(orc.lubrication_force(p, lb, x, v + np.array([3.0, -1.0, 2.0])), f,
                               rtol=1e-12, atol=1e-12)
    assert np.sum(f * v) < 0
    rng = np.random.default_rng(93)
    for _ in range(5):
        w = rng.standard_normal(v.shape)
        assert np.sum(orc.lubrication_force(p, lb, x, w) * w) < 0


def test_lubrication_linear_and_equivariant(orc, dense):
    x, v = dense
    p, lb = orc.params(), orc.lub()
    w = W.gaussian_forces(len(x), seed=94)
    f = orc.lubrication_force(p, lb, x, v)
    np.testing.assert_allclose(orc.lubrication_force(p, lb, x, 2 * v - w),
                               2 * f - orc.lubrication_force(p, lb, x, w), rtol=1e-11, atol=1e-11)
    Q = _rot(95)
    np.testing.assert_allclose(orc.lubrication_force(p, lb, x @ Q.T, v @ Q.T), f @ Q.T,
                               rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(orc.lubrication_force(p, lb, x + 7.0, v), f, rtol=1e-10, atol=1e-10)


def test_run_lub_reduces_to_plain_run_without_close_pairs(orc):
    """Without pairs closer than 3a the loop is the plain mobility loop."""
    x0 = W.random_suspension(50, phi=0.01, min_dist=3.5, seed=96)
    f = W.gravity_forces(50)
    p = orc.params()
    xa, _, _ = orc.run(p, x0, f, 0.01, 20)
    xb, _, _ = orc.run_lub(p, orc.lub(), x0, f, 0.01, 20)
    np.testing.assert_allclose(xb, xa, rtol=1e-14, atol=1e-14)


def test_lubrication_is_a_hard_core(orc):
    """Two spheres pushed into each other by opposite forces: without the
    correction they overlap, with it the gap stays open (the paper's reason for
    including lubrication, Sec. 3.1)."""
    p = orc.params(overlap=True)
    x0 = np.array([[-1.15, 0.0, 0.0], [1.15, 0.0, 0.0]])
    f = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    x_plain, _, _ = orc.run(p, x0, f, 0.01, 400)
    x_lub, _, traj = orc.run_lub(p, orc.lub(s_min=1e-6), x0, f, 0.01, 400, stride=1)
    assert np.linalg.norm(x_plain[0] - x_plain[1]) < 2.0
    gaps = np.linalg.norm(traj[:, 0] - traj[:, 1], axis=1)
    assert gaps.min() > 2.0


@pytest.mark.parametrize("s_gap", [0.05, 0.2, 0.3, 0.6])
def test_lagged_correction_multiplies_relative_velocity(orc, s_gap):
    """Step 2 of Sec. 3.1 with the previous velocities: two spheres without
    external force whose previous velocities are +-u along their line of
    centres move next with relative velocity -mu_rel zeta_P times the previous
    one, where mu_rel = 2 mu0 (1 - 3a/2r + a^3/r^3) (RPY, Eq. 7b, along the
    line) and mu0 zeta_P = 1/(4s) - 9/40 log s (Eq. 8).  The factor exceeds 1
    below s = 0.28: the explicit lagged loop is only stable for wider gaps."""
    a = 1.0
    r = (2.0 + s_gap) * a
    p = orc.params()
    x0 = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    u = 1e-3
    vp = np.array([[u, 0.0, 0.0], [-u, 0.0, 0.0]])
    _, v, _ = orc.run_lub(p, orc.lub(), x0, np.zeros((2, 3)), 1e-12, 1, v_prev=vp)
    mu_rel = 2.0 * (1.0 - 3.0 * a / (2.0 * r) + a ** 3 / r ** 3)
    zeta = 1.0 / (4.0 * s_gap) - 9.0 / 40.0 * np.log(s_gap)
    ratio = (v[0, 0] - v[1, 0]) / (2 * u)
    np.testing.assert_allclose(ratio, -mu_rel * zeta, rtol=1e-12)
    assert (abs(ratio) > 1.0) == (s_gap < 0.28)


def test_lagged_correction_diverges_on_the_dense_fcc_start(orc):
    """The fcc start of the Sec. 3.3 benchmark (n = 0.1/a^3, phi ~ 0.42,
    twelve neighbours at s = 0.42) is far inside the unstable range of the
    lagged correction: a lattice mode grows by a large factor each step, so
    the loop with lubrication blows up within tens of steps, while the loop
    without it sediments uniformly.  (Hence the benchmark times the
    lubrication step on its own.)"""
    x0, L = W.fcc_lattice(6)
    f = W.gravity_forces(len(x0))
    p = orc.params(box=L)
    _, v_plain, _ = orc.run(p, x0, f, 0.001, 25)
    assert np.abs(v_plain).max() < 200.0
    _, v_lub, _ = orc.run_lub(p, orc.lub(), x0, f, 0.001, 25)
    assert np.abs(v_lub).max() > 1e6
