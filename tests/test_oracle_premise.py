"""Pins of the oracle's count of pairs that break the premise r >= 2a of the
far-field tensor (Eq. 4 is positive definite only for r >= 2a, Sec. 2.2):
hand-built configurations, the nearest image of a periodic box, and an
independent pairwise-distance routine on dense random configurations."""
import numpy as np
import pytest
from scipy.spatial.distance import pdist


def test_hand_built_configuration(orc):
    """Two coincident spheres, one at 1.5a from both, one at exactly 2a from
    both (not below 2a) and one far away: 2 pairs below 2a, 1 coincident."""
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [0.0, 2.0, 0.0],
                  [10.0, 10.0, 10.0]])
    assert orc.premise_counts(orc.params(), x) == (2, 1)
    # the same with a = 0.5: only the coincident pair is closer than 2a = 1
    assert orc.premise_counts(orc.params(a=0.5), x) == (0, 1)
    # a = 2: every pair among the first four is closer than 4 (the farthest is
    # 2.5 apart); the far sphere is 17.3 away
    assert orc.premise_counts(orc.params(a=2.0), x) == (5, 1)


def test_single_sphere_and_empty(orc):
    assert orc.premise_counts(orc.params(), np.zeros((1, 3))) == (0, 0)
    assert orc.premise_counts(orc.params(), np.zeros((0, 3))) == (0, 0)


def test_nearest_image_in_a_box(orc):
    """8.5 apart along x in a box of side 10: the nearest image is 1.5 away."""
    x = np.array([[0.5, 5.0, 5.0], [9.0, 5.0, 5.0]])
    assert orc.premise_counts(orc.params(), x) == (0, 0)
    assert orc.premise_counts(orc.params(box=10.0), x) == (1, 0)
    # a lattice translation of one sphere changes nothing in the box
    y = x + np.array([[0.0, 0.0, 0.0], [-20.0, 10.0, 30.0]])
    assert orc.premise_counts(orc.params(box=10.0), y) == (1, 0)


def _by_pdist(x, a):
    d = pdist(x)
    return int(np.count_nonzero((d > 0) & (d * d < 4 * a * a))), int(np.count_nonzero(d == 0))


@pytest.mark.parametrize("a", [1.0, 0.7])
def test_dense_random_against_pdist(orc, a):
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 25.0, size=(800, 3))
    x[700:720] = x[:20]                      # 20 coincident pairs
    sub, co = orc.premise_counts(orc.params(a=a), x)
    assert (sub, co) == _by_pdist(x, a)
    assert co == 20 and sub > 100
    # invariant under a permutation of the particles
    perm = rng.permutation(len(x))
    assert orc.premise_counts(orc.params(a=a), x[perm]) == (sub, co)


def test_periodic_against_images(orc):
    """In a periodic cube the count equals the free-space count over the 27
    nearest lattice images of the other sphere when the box is wider than 4a."""
    rng = np.random.default_rng(12)
    L = 12.0
    x = rng.uniform(0.0, L, size=(300, 3))
    want = 0
    for i in range(len(x)):
        for j in range(i + 1, len(x)):
            d = x[i] - x[j]
            best = min(np.linalg.norm(d + L * np.array([u, v, w]))
                       for u in (-1, 0, 1) for v in (-1, 0, 1) for w in (-1, 0, 1))
            want += best < 2.0
    assert orc.premise_counts(orc.params(box=L), x) == (want, 0)
    assert want > orc.premise_counts(orc.params(), x)[0]
