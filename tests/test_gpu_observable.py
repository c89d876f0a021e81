"""The observable of the sedimentation runs (Secs. 3.3 and 4): the mean vector
(1/n) sum_i v_i of sd_mean_vector, against an exactly rounded sum on the host,
for sizes from one particle to more than one full grouping (ragged ranges
included), and bitwise repeatable."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available()
    import paper_1205_6333_amd as sd
    sd.lib()
    return sd


@pytest.mark.parametrize("n", [1, 7, 255, 256, 1023, 1024, 1025, 65536, 300001, 1048576 + 3])
def test_mean_vector_matches_exact_mean(sd, n):
    import torch
    rng = np.random.default_rng(n)
    v = rng.normal(size=(n, 3)) + np.array([0.0, 0.0, -1.0])
    vd = torch.from_numpy(v).cuda()
    m1 = sd.sd_mean_vector(vd).cpu().numpy()
    m2 = sd.sd_mean_vector(vd).cpu().numpy()
    exact = np.array([math.fsum(v[:, c]) / n for c in range(3)])
    # a sum whose terms pass through at most k roundings is within k eps sum|v_i|
    # of the exact one; here k < log2(n) + 24 (per-lane runs, two 256-lane
    # trees, the division).  A dropped or repeated term is off by about 1/n.
    bound = (math.log2(n) + 24) * np.finfo(np.float64).eps * np.abs(v).sum(0) / n
    print("n=%d err=%s bound=%s" % (n, np.abs(m1 - exact), bound))
    assert np.all(np.abs(m1 - exact) <= bound)
    assert np.array_equal(m1, m2)
