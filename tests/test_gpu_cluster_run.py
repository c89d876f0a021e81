"""GPU runs of the precision study of Sec. 4 (sd_cluster_run) against the FP64
oracle's Euler loop on the four-sphere cluster of Fig. 4.

Bars: FP64 accumulation with FP64 positions 1e-12 of the displacement (the
same Euler loop in the same precision, summation order aside); compensated
FP32 accumulation (Kahan or double-single) with double-single or FP64
positions 1e-5; plain FP32 accumulation and positions 1e-3 (the FP32 rounding
of every step accumulates).  The period of the motion is the paper's
517 tau_s (tests/golden/four_sphere_period.json)."""
import json
import os

import numpy as np
import pytest

from paper_1205_6333_amd import workloads as W

from gpu_util import to_dev3

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "four_sphere_period.json")


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available()
    import paper_1205_6333_amd as sd
    sd.lib()
    return sd


def _state(x0, runs):
    import torch
    st = torch.zeros((runs, 2) + x0.shape, dtype=torch.float64, device="cuda")
    st[:, 0] = torch.tensor(x0, device="cuda")
    return st


def _run(sd, x0, f, specs, params=None):
    import torch
    st = _state(x0, len(specs))
    traj = sd.sd_cluster_run(st, to_dev3(f), specs, params=params or sd.params())
    torch.cuda.synchronize()
    return st.cpu().numpy(), None if traj is None else traj.cpu().numpy()


MODES = [(3, 2, 1e-12), (1, 2, 1e-5), (2, 2, 1e-5), (1, 1, 1e-5), (2, 1, 1e-5), (0, 0, 1e-3),
         (0, 2, 1e-3), (2, 0, 1e-3)]


@pytest.mark.parametrize("acc,pos,tol", MODES)
def test_cluster_run_vs_oracle(sd, orc, acc, pos, tol):
    x0, f = W.four_sphere_tetrahedron()
    steps, stride, dt = 2000, 100, 0.01
    po = orc.params()
    xr, _, tr = orc.run(po, x0, f, dt, steps, 0, stride=stride)
    st, traj = _run(sd, x0, f, [dict(acc=acc, pos=pos, dt=dt, steps=steps, stride=stride)])
    disp = np.abs(xr - x0).max()
    x_end = st[0, 0] + st[0, 1]
    err = np.abs(x_end - xr).max() / disp
    frames_err = np.abs(traj - tr[1:]).max() / disp
    print("acc=%d pos=%d err/disp=%.3e frames=%.3e" % (acc, pos, err, frames_err))
    assert err <= tol and frames_err <= tol
    assert np.array_equal(traj[-1], x_end)


def test_cluster_run_continues_exactly(sd):
    """Two calls of k steps continue one trajectory: bitwise the result of one
    call of 2k steps, in every precision (the state round trip is exact)."""
    import torch
    x0, f = W.four_sphere_tetrahedron()
    specs = [dict(acc=a, pos=p, dt=0.01, steps=1500) for a in range(4) for p in range(3)]
    one, _ = _run(sd, x0, f, specs)
    st = _state(x0, len(specs))
    half = [dict(s, steps=750) for s in specs]
    fd = to_dev3(f)
    sd.sd_cluster_run(st, fd, half)
    sd.sd_cluster_run(st, fd, half)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), one)


def test_cluster_runs_are_independent(sd):
    """A launch of many runs gives each run's result of a launch of its own,
    with per-run step counts and strides."""
    x0, f = W.four_sphere_tetrahedron()
    specs = [dict(acc=a, pos=p, dt=dt, steps=s, stride=k)
             for (a, p, dt, s, k) in [(3, 2, 0.01, 900, 100), (0, 0, 0.001, 1200, 0),
                                      (2, 1, 0.01, 700, 7), (1, 2, 0.02, 1000, 250)]]
    st_all, tr_all = _run(sd, x0, f, specs)
    off = 0
    for r, s in enumerate(specs):
        st1, tr1 = _run(sd, x0, f, [s])
        assert np.array_equal(st_all[r], st1[0])
        nf = s["steps"] // s["stride"] if s["stride"] else 0
        if nf:
            assert np.array_equal(tr_all[off:off + nf], tr1)
        off += nf
    assert off == len(tr_all)


def test_four_sphere_symmetry_fp64(sd):
    """The symmetry relations of Sec. 4 hold to FP64 rounding along the run:
    y_1 = y_3 = x_2 = x_4 = 0, x_3 = -x_1, z_3 = z_1, z_4 = z_2, y_4 = -y_2."""
    x0, f = W.four_sphere_tetrahedron()
    _, tr = _run(sd, x0, f, [dict(acc=3, pos=2, dt=0.01, steps=20000, stride=500)])
    scale = np.abs(tr).max()
    for fr in tr:
        (x1, y1, z1), (x2, y2, z2), (x3, y3, z3), (x4, y4, z4) = fr
        dev = max(abs(y1), abs(y3), abs(x2), abs(x4), abs(x3 + x1), abs(z3 - z1), abs(z4 - z2),
                  abs(y4 + y2))
        assert dev <= 1e-12 * scale


def test_four_sphere_period_on_gpu(sd):
    """Two cycles of the FP64 run: the x_1 max-to-max time is the paper's
    period, and the compensated FP32 accumulation gives the same period."""
    from paper_1205_6333_amd import observables as OB
    g = json.load(open(GOLDEN))
    x0, f = W.four_sphere_tetrahedron()
    dt, stride, steps = 0.01, 10, 130000
    specs = [dict(acc=3, pos=2, dt=dt, steps=steps, stride=stride),
             dict(acc=1, pos=1, dt=dt, steps=steps, stride=stride)]
    _, tr = _run(sd, x0, f, specs)
    nf = steps // stride
    t = dt * stride * np.arange(1, nf + 1)
    periods = []
    for r in range(2):
        x1 = tr[r * nf:(r + 1) * nf, 0, 0]
        _, dur, _, amp = OB.cycles(t, x1)
        assert len(dur) >= 1
        periods.append(dur[0])
        assert abs(dur[0] - g["value"]) <= g["tolerance_abs"]
    assert abs(periods[0] - periods[1]) <= 1e-3


def test_cluster_run_random_cluster_64(sd, orc):
    """The largest cluster (64 spheres, a wave of lanes), overlap-regularised
    RPY with near pairs, against the oracle."""
    offs, x = W.clusters(1, nmin=64, nmax=64, sigma=2.5, min_dist=1.8, seed=44)
    x0 = x[:64]
    f = W.gravity_forces(64) + 0.2 * W.gaussian_forces(64, seed=45)
    po = orc.params(overlap=True)
    xr, _, _ = orc.run(po, x0, f, 0.01, 300)
    for acc, pos, tol in [(3, 2, 1e-12), (1, 2, 1e-5), (2, 1, 1e-5)]:
        st, _ = _run(sd, x0, f, [dict(acc=acc, pos=pos, dt=0.01, steps=300)],
                     params=sd.params(overlap=True))
        err = np.abs(st[0, 0] + st[0, 1] - xr).max() / np.abs(xr - x0).max()
        print("n=64 acc=%d pos=%d err=%.3e" % (acc, pos, err))
        assert err <= tol


def test_four_sphere_plane_symmetry_by_accumulation_precision(sd):
    """Sec. 4 (the figure of particle 1's deviation from the xz-plane, dt =
    0.001 tau_s): with the hydrodynamic interactions accumulated in
    double-single (or FP64), particle 1 stays in the plane exactly, y_1 = 0 in
    every frame bit for bit, whatever the precision of the positions; with
    single-precision accumulation and double-single positions y_1 leaves 0
    and its deviation grows over the run."""
    x0, f = W.four_sphere_tetrahedron()
    steps, stride, dt = 300000, 1000, 0.001
    specs = [dict(acc=2, pos=1, dt=dt, steps=steps, stride=stride),   # DS HI, DS positions
             dict(acc=2, pos=2, dt=dt, steps=steps, stride=stride),   # DS HI, FP64 positions
             dict(acc=3, pos=1, dt=dt, steps=steps, stride=stride),   # FP64 HI, DS positions
             dict(acc=0, pos=1, dt=dt, steps=steps, stride=stride)]   # single HI, DS positions
    st, tr = _run(sd, x0, f, specs)
    nf = steps // stride
    y1 = tr[:, 0, 1].reshape(len(specs), nf)
    for r in range(3):
        assert np.all(y1[r] == 0.0), (specs[r], np.abs(y1[r]).max())
        assert st[r, :, 0, 1].tolist() == [0.0, 0.0]       # hi and lo parts of y_1
    dev = np.abs(y1[3])
    print("single-HI |y1|: first nonzero frame %d, max %.3e, last %.3e"
          % (int(np.argmax(dev > 0)), dev.max(), dev[-1]))
    assert dev.max() > 0.0
    # the deviation grows: the last tenth of the run is above the first tenth
    k = nf // 10
    assert dev[-k:].max() > dev[:k].max()
