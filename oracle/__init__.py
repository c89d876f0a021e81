"""FP64 CPU oracle for the all-pairs Stokesian-dynamics mobility product.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
does, and this package never imports the GPU library: the two share no code.

The arithmetic lives in ``sd_oracle.c`` (plain double loops, see the comments
there for the equation each function follows).  This module compiles it with
gcc and wraps it for numpy arrays of shape (n, 3), float64.  ``membench.py``
holds the (numpy) oracle of the App. A memory-access benchmarks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RPY, OSEEN = 0, 1
EULER, AB2 = 0, 1


class OracleParams(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("eta", ctypes.c_double),
                ("tensor", ctypes.c_int), ("overlap", ctypes.c_int),
                ("box", ctypes.c_double * 3)]


class OracleLub(ctypes.Structure):
    _fields_ = [("s_cut", ctypes.c_double), ("s_min", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile sd_oracle.c into liboracle.so (gcc -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(OracleParams)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_pair_tensor.argtypes = [P, d, d]
        lib.oracle_mobility.argtypes = [P, i64, d, d, d]
        lib.oracle_mobility_rows.argtypes = [P, i64, d, d, i64, ctypes.POINTER(i64), d]
        lib.oracle_dense_mobility.argtypes = [P, i64, d, d]
        lib.oracle_premise_counts.argtypes = [P, i64, d, ctypes.POINTER(i64)]
        lib.oracle_premise_counts.restype = None
        lib.oracle_run.argtypes = [P, i64, d, d, ctypes.c_double, i64, i64, ctypes.c_int, d, d, i64]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_pair_grad.argtypes = [P, d, d, d, d]
        lib.oracle_mobility_transpose.argtypes = [P, i64, d, d, d]
        lib.oracle_mobility_vjp_x.argtypes = [P, i64, d, d, d, d]
        lib.oracle_run_adjoint_euler.argtypes = [P, i64, d, d, ctypes.c_double, i64, d, d, d]
        lib.oracle_run_adjoint_euler.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        LP = ctypes.POINTER(OracleLub)
        lib.oracle_lub_tensor.argtypes = [P, LP, d, d]
        lib.oracle_lubrication_force.argtypes = [P, LP, i64, d, d, d]
        lib.oracle_run_lub.argtypes = [P, LP, i64, d, d, ctypes.c_double, i64, i64, ctypes.c_int,
                                       d, d, i64]
        lib.oracle_run_lub.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def set_threads(k: int) -> None:
    """Run the oracle's parallel loops on k threads (for timing)."""
    _load().oracle_set_threads(int(k))


def params(a: float = 1.0, eta: float = 1.0 / (6.0 * np.pi), tensor: int = RPY,
           overlap: bool = False, box=None) -> OracleParams:
    """Sphere radius a, viscosity eta; the defaults give mu0 = 1/(6 pi eta a) = 1.
    box: periodic box sides (nearest image), None / 0 = free space."""
    b = (0.0, 0.0, 0.0) if box is None else tuple(float(v) for v in np.broadcast_to(box, (3,)))
    return OracleParams(float(a), float(eta), int(tensor), int(bool(overlap)),
                        (ctypes.c_double * 3)(*b))


def _ptr(arr):
    if arr is None:
        return None
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x, n=None):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))
    if n is not None and x.shape[0] != n:
        raise ValueError("expected %d rows, got %d" % (n, x.shape[0]))
    return x


def pair_tensor(p: OracleParams, r) -> np.ndarray:
    """3x3 block T(r) for r = r_i - r_j (Eq. 4 / Eq. 7b / overlap reading)."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(3))
    T = np.empty(9)
    _load().oracle_pair_tensor(ctypes.byref(p), _ptr(r), _ptr(T))
    return T.reshape(3, 3)


def mobility(p: OracleParams, x, f) -> np.ndarray:
    """v_i = mu0 F_i + sum_{j != i} T(x_i - x_j) F_j for all i (Eq. 7a)."""
    x = _vec(x)
    f = _vec(f, x.shape[0])
    v = np.empty_like(x)
    _load().oracle_mobility(ctypes.byref(p), x.shape[0], _ptr(x), _ptr(f), _ptr(v))
    return v


def premise_counts(p: OracleParams, x):
    """(pairs i < j with 0 < r < 2a, pairs with r = 0): the pairs that break
    the premise r >= 2a of Eq. 4 (Sec. 2.2), nearest image in a box."""
    x = _vec(x)
    out = (ctypes.c_int64 * 2)()
    _load().oracle_premise_counts(ctypes.byref(p), x.shape[0], _ptr(x), out)
    return int(out[0]), int(out[1])


def mobility_rows(p: OracleParams, x, f, rows) -> np.ndarray:
    """The product restricted to the particle indices in `rows`."""
    x = _vec(x)
    f = _vec(f, x.shape[0])
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
    if rows.size and (rows.min() < 0 or rows.max() >= x.shape[0]):
        raise IndexError("row index out of range")
    v = np.empty((rows.size, 3))
    _load().oracle_mobility_rows(ctypes.byref(p), x.shape[0], _ptr(x), _ptr(f), rows.size,
                                 rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(v))
    return v


def mobility_transpose(p: OracleParams, x, y) -> np.ndarray:
    """(M^T y) from the transposed blocks."""
    x = _vec(x)
    y = _vec(y, x.shape[0])
    out = np.empty_like(x)
    _load().oracle_mobility_transpose(ctypes.byref(p), x.shape[0], _ptr(x), _ptr(y), _ptr(out))
    return out


def dense_mobility(p: OracleParams, x) -> np.ndarray:
    """The 3n x 3n mobility matrix (tiny n)."""
    x = _vec(x)
    n = x.shape[0]
    M = np.empty((3 * n, 3 * n))
    _load().oracle_dense_mobility(ctypes.byref(p), n, _ptr(x), _ptr(M))
    return M


def run(p: OracleParams, x0, f, dt: float, steps: int, integrator: int = EULER,
        step0: int = 0, v_prev=None, stride: int = 0):
    """Integrate dx/dt = M(x) F.  Returns (x_final, v_last, traj or None)."""
    x = _vec(x0).copy()
    n = x.shape[0]
    f = _vec(f, n)
    vp = np.zeros_like(x) if v_prev is None else _vec(v_prev, n).copy()
    traj = None
    if stride > 0:
        traj = np.empty((steps // stride + 1, n, 3))
    rc = _load().oracle_run(ctypes.byref(p), n, _ptr(x), _ptr(f), float(dt), int(steps),
                            int(step0), int(integrator), _ptr(vp), _ptr(traj), int(stride))
    if rc != 0:
        raise MemoryError("oracle_run failed")
    return x, vp, traj


def pair_grad(p: OracleParams, r, u, w) -> np.ndarray:
    """grad_r of u . T(r) w."""
    arrs = [np.ascontiguousarray(np.asarray(z, dtype=np.float64).reshape(3)) for z in (r, u, w)]
    g = np.empty(3)
    _load().oracle_pair_grad(ctypes.byref(p), _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), _ptr(g))
    return g


def mobility_vjp_x(p: OracleParams, x, f, lam) -> np.ndarray:
    """d/dx [lam . M(x) F]."""
    x = _vec(x)
    n = x.shape[0]
    f = _vec(f, n)
    lam = _vec(lam, n)
    g = np.empty_like(x)
    _load().oracle_mobility_vjp_x(ctypes.byref(p), n, _ptr(x), _ptr(f), _ptr(lam), _ptr(g))
    return g


def run_adjoint_euler(p: OracleParams, x0, f, dt: float, steps: int, lam_final):
    """Gradients (dL/dx0, dL/dF) of a loss of x_steps with dL/dx_steps = lam_final."""
    x0 = _vec(x0)
    n = x0.shape[0]
    f = _vec(f, n)
    lam = _vec(lam_final, n)
    gx = np.empty_like(x0)
    gf = np.empty_like(x0)
    rc = _load().oracle_run_adjoint_euler(ctypes.byref(p), n, _ptr(x0), _ptr(f), float(dt),
                                          int(steps), _ptr(lam), _ptr(gx), _ptr(gf))
    if rc != 0:
        raise MemoryError("oracle_run_adjoint_euler failed")
    return gx, gf


def lub(s_cut: float = 1.0, s_min: float = 1e-3) -> OracleLub:
    """Lubrication truncation (Sec. 2.3: s < 1) and the contact clamp s >= s_min."""
    return OracleLub(float(s_cut), float(s_min))


def lub_tensor(p: OracleParams, lb: OracleLub, r) -> np.ndarray:
    """3x3 singular friction zeta(r) of Eq. 8 (physical units)."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(3))
    Z = np.empty(9)
    _load().oracle_lub_tensor(ctypes.byref(p), ctypes.byref(lb), _ptr(r), _ptr(Z))
    return Z.reshape(3, 3)


def lubrication_force(p: OracleParams, lb: OracleLub, x, v) -> np.ndarray:
    """f_i = - sum_j zeta(r_i - r_j) (v_i - v_j)."""
    x = _vec(x)
    v = _vec(v, x.shape[0])
    f = np.empty_like(x)
    _load().oracle_lubrication_force(ctypes.byref(p), ctypes.byref(lb), x.shape[0], _ptr(x),
                                     _ptr(v), _ptr(f))
    return f


def run_lub(p: OracleParams, lb: OracleLub, x0, f_ext, dt: float, steps: int,
            integrator: int = EULER, step0: int = 0, v_prev=None, stride: int = 0):
    """The loop of Sec. 3.1 with lubrication; returns (x, v_last, traj or None)."""
    x = _vec(x0).copy()
    n = x.shape[0]
    f = _vec(f_ext, n)
    vp = np.zeros_like(x) if v_prev is None else _vec(v_prev, n).copy()
    traj = np.empty((steps // stride + 1, n, 3)) if stride > 0 else None
    rc = _load().oracle_run_lub(ctypes.byref(p), ctypes.byref(lb), n, _ptr(x), _ptr(f), float(dt),
                                int(steps), int(step0), int(integrator), _ptr(vp), _ptr(traj),
                                int(stride))
    if rc != 0:
        raise MemoryError("oracle_run_lub failed")
    return x, vp, traj
