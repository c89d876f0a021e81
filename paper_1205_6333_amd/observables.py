"""Host-side observables of recorded trajectories (post-processing of the
frames the library writes; nothing here is on the device path).

Sec. 4 measures the periodic sedimentation of four spheres by the extrema of
x_1(t): each maximum and minimum is located by a parabola through the sample
at the discrete extremum and its two neighbours; successive maxima give the
cycle duration, a maximum and the following minimum the amplitude.
"""
from __future__ import annotations

import numpy as np


def parabolic_extrema(t: np.ndarray, y: np.ndarray):
    """Extrema of a uniformly sampled signal by parabolic interpolation.

    t, y: 1-D arrays of equal length, t uniformly spaced.  Returns
    (t_max, y_max, t_min, y_min): for every interior sample that is a strict
    local maximum (minimum) of y, the vertex of the parabola through it and its
    two neighbours."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if len(y) < 3:
        e = np.empty(0)
        return e, e, e, e
    h = t[1] - t[0]
    ym, y0, yp = y[:-2], y[1:-1], y[2:]
    out = []
    for sel in ((y0 > ym) & (y0 > yp), (y0 < ym) & (y0 < yp)):
        k = np.nonzero(sel)[0]
        a, b, c = ym[k], y0[k], yp[k]
        den = a - 2.0 * b + c
        off = 0.5 * (a - c) / den                  # vertex offset in samples, |off| <= 1/2
        out.append(t[k + 1] + off * h)
        out.append(b - 0.25 * (a - c) * off)
    return out[0], out[1], out[2], out[3]


def cycles(t: np.ndarray, y: np.ndarray):
    """Cycle durations (differences of successive maxima times) and amplitudes
    (half the difference of each maximum and the next minimum) of y(t).
    Returns (t_cycle, duration, t_amp, amplitude)."""
    tmax, ymax, tmin, ymin = parabolic_extrema(t, y)
    dur = np.diff(tmax)
    tc = 0.5 * (tmax[1:] + tmax[:-1])
    amps, ta = [], []
    for tm, ym in zip(tmax, ymax):
        k = np.searchsorted(tmin, tm)
        if k < len(tmin):
            amps.append(0.5 * (ym - ymin[k]))
            ta.append(tm)
    return tc, dur, np.array(ta), np.array(amps)
