"""ctypes binding of libsd.so (the C ABI in include/sd.h).

Argument marshalling only: tensors are checked for device, dtype, shape and
contiguity, their data pointers and the current HIP stream are passed to the
library, and a non-zero sd_status raises SdError.  Every step of the
computation runs in the library's HIP kernels.  There is no fallback: if
libsd.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
# SD_LIBRARY: another build of the library (e.g. the host-sanitized one of
# build.build_host_sanitized); the in-tree libsd.so otherwise
LIB_PATH = os.environ.get("SD_LIBRARY") or os.path.join(HERE, "libsd.so")

# enums of sd.h
SD_OK, SD_EINVAL, SD_EALIGN, SD_ENOMEM, SD_EDEVICE, SD_EUNSUPPORTED = range(6)
SD_RPY, SD_OSEEN = 0, 1
SD_OVERLAP_NONE, SD_OVERLAP_RPY = 0, 1
SD_FP32_KAHAN, SD_FP64, SD_FP32_PLAIN = 0, 1, 2
SD_EULER, SD_AB2 = 0, 1
SD_BATCH_MAX_CLUSTER = 1024
SD_ACC_FP32, SD_ACC_KAHAN, SD_ACC_DS, SD_ACC_FP64 = 0, 1, 2, 3
SD_POS_FP32, SD_POS_DS, SD_POS_FP64 = 0, 1, 2
SD_CLUSTER_MAX_N, SD_CLUSTER_MAX_RUNS = 64, 4096
SD_MB_NAIVE, SD_MB_SMALLTILING, SD_MB_TILING = 0, 1, 2
SD_MB_LINEAR, SD_MB_STRIDED, SD_MB_UNORDERED = 0, 1, 2
SD_MB_FLOAT, SD_MB_FLOAT4 = 0, 1


class SdParams(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("eta", ctypes.c_double),
                ("tensor", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("box", ctypes.c_double * 3)]


class SdLub(ctypes.Structure):
    _fields_ = [("s_cut", ctypes.c_double), ("s_min", ctypes.c_double)]


class SdClusterSpec(ctypes.Structure):
    _fields_ = [("acc", ctypes.c_int32), ("pos", ctypes.c_int32), ("dt", ctypes.c_double),
                ("steps", ctypes.c_int64), ("stride", ctypes.c_int64)]


def lub(s_cut: float = 1.0, s_min: float = 1e-3) -> SdLub:
    """Lubrication truncation (paper: s < 1) and contact clamp."""
    return SdLub(float(s_cut), float(s_min))


class SdKernelConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block", ctypes.c_int32),
                ("splits", ctypes.c_int32), ("ilp", ctypes.c_int32),
                ("kahan_block", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsd.so (after torch, whose HIP runtime it shares)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library links against)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsd.so is not built: run `python -m paper_1205_6333_amd.build` "
                               "(the library has no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(SdParams)
        vp, dp, i64, i32, d = (ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_double)
        sig = {
            "mobility_apply": [P, i64, vp, vp, dp, i32, vp],
            "mobility_apply_noalloc": [P, i64, vp, vp, dp, i32, vp],
            "mobility_adjoint": [P, i64, vp, vp, vp, dp, dp, i32, vp],
            "sd_step": [P, i64, dp, vp, dp, dp, d, i64, i32, i32, vp],
            "sd_run": [P, i64, dp, vp, dp, d, i64, i64, i32, i32, dp, i64, vp],
            "sd_run_adjoint": [P, i64, dp, vp, d, i64, i32, dp, i64, dp, dp, dp, vp],
            "sd_batch_create": [P, i64, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_void_p)],
            "sd_batch_destroy": [vp],
            "mobility_apply_batched": [vp, vp, vp, dp, i32, vp],
            "sd_run_batched": [vp, dp, vp, d, i64, i32, i32, i32, vp],
            "sd_batch_set_config": [vp, i32, i32],
            "sd_batch_get_config": [vp, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)],
            "sd_batch_autotune": [vp, dp, vp, d, i64, i32, i32, ctypes.c_char_p, i64, vp],
            "sd_set_kernel_config": [i32, ctypes.POINTER(SdKernelConfig)],
            "sd_get_kernel_config": [i32, i64, ctypes.POINTER(SdKernelConfig)],
            "sd_autotune": [P, i64, i32, vp, ctypes.c_char_p, i64],
            "sd_autotune_clear": [i32],
            "sd_pack": [i64, dp, vp, i32, vp],
            "lubrication_forces": [P, ctypes.POINTER(SdLub), i64, dp, dp, dp, dp, vp],
            "sd_run_lub": [P, ctypes.POINTER(SdLub), i64, dp, dp, dp, d, i64, i64, i32, i32, vp],
            "sd_mean_vector": [i64, dp, dp, vp],
            "sd_premise_counts": [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  i32, vp],
            "sd_set_graph_mode": [i32],
            "sd_cluster_run": [P, i64, i32, ctypes.POINTER(SdClusterSpec), dp, dp, dp, vp],
            "sd_membench": [i32, i32, i32, i64, vp, vp, vp],
            "sd_profile_enable": [i32],
            "sd_profile_read": [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
            "sd_profile_reset": [],
            "sd_profile_times": [ctypes.POINTER(ctypes.c_float), i64, ctypes.POINTER(ctypes.c_int64)],
            "sd_release": [],
            "sd_status_string": [i32],
            "sd_last_error": [],
            "sd_version": [],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.sd_status_string.restype = ctypes.c_char_p
        L.sd_last_error.restype = ctypes.c_char_p
        L.sd_batch_particles.argtypes = [vp]
        L.sd_batch_particles.restype = ctypes.c_int64
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != SD_OK:
        L = lib()
        raise SdError(status, "%s: %s" % (L.sd_status_string(status).decode(),
                                          L.sd_last_error().decode()))


def params(a: float = 1.0, eta: float = 1.0 / (6.0 * math.pi), tensor: int = SD_RPY,
           overlap: bool = False, box=None) -> SdParams:
    """Sphere radius, viscosity, pair tensor and overlap mode (defaults: mu0 = 1).
    ``box``: side of a periodic cubic box (a number or three equal sides;
    nearest-image interactions), None for free space."""
    if box is None:
        sides = (0.0, 0.0, 0.0)
    elif isinstance(box, (int, float)):
        sides = (float(box),) * 3
    else:
        sides = tuple(float(b) for b in box)
    return SdParams(float(a), float(eta), int(tensor), int(bool(overlap)),
                    (ctypes.c_double * 3)(*sides))


def _stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _vec4(t, precision: int, name: str):
    import torch
    want = torch.float64 if precision == SD_FP64 else torch.float32
    if not (t.is_cuda and t.dtype == want and t.dim() == 2 and t.shape[1] == 4
            and t.is_contiguous()):
        raise ValueError("%s must be a contiguous (n, 4) %s CUDA tensor" % (name, want))
    return t


def _vec3(t, n: int, name: str):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == 3 * n):
        raise ValueError("%s must be a contiguous float64 CUDA tensor with 3n elements" % name)
    return t


def _ptr(t) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _default_precision(t) -> int:
    import torch
    return SD_FP64 if t.dtype == torch.float64 else SD_FP32_KAHAN


def mobility_apply(pos, force, vel=None, *, params: SdParams = None, precision: int = None,
                   stream=None):
    """v = M(x) F.  pos/force: (n, 4) float32 (FP32 precisions) or float64
    (SD_FP64) CUDA tensors; returns vel (n, 3) float64."""
    import torch
    prec = _default_precision(pos) if precision is None else int(precision)
    _vec4(pos, prec, "pos")
    _vec4(force, prec, "force")
    n = pos.shape[0]
    if force.shape[0] != n:
        raise ValueError("pos and force differ in length")
    if vel is None:
        vel = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    _vec3(vel, n, "vel")
    p = params if params is not None else globals()["params"]()
    check(lib().mobility_apply(ctypes.byref(p), n, _ptr(pos), _ptr(force), _ptr(vel), prec,
                               _stream(stream)))
    return vel


def mobility_apply_noalloc(pos, force, vel, *, params: SdParams = None, precision: int = None,
                           stream=None):
    """v = M(x) F into the caller's vel (n, 3) float64, through the entry point
    that allocates no device memory (its scratch is a static device array)."""
    prec = _default_precision(pos) if precision is None else int(precision)
    _vec4(pos, prec, "pos")
    _vec4(force, prec, "force")
    n = pos.shape[0]
    if force.shape[0] != n:
        raise ValueError("pos and force differ in length")
    _vec3(vel, n, "vel")
    p = params if params is not None else globals()["params"]()
    check(lib().mobility_apply_noalloc(ctypes.byref(p), n, _ptr(pos), _ptr(force), _ptr(vel),
                                       prec, _stream(stream)))
    return vel


def mobility_adjoint(pos, force, lam, grad_pos=None, grad_force=None, *, want_force: bool = True,
                     params: SdParams = None, precision: int = None, stream=None):
    """Returns (d/dx[lam . M(x) F], M(x) lam) as (n, 3) float64 tensors."""
    import torch
    prec = _default_precision(pos) if precision is None else int(precision)
    for t, nm in ((pos, "pos"), (force, "force"), (lam, "lam")):
        _vec4(t, prec, nm)
    n = pos.shape[0]
    if grad_pos is None:
        grad_pos = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    if want_force and grad_force is None:
        grad_force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    _vec3(grad_pos, n, "grad_pos")
    if grad_force is not None:
        _vec3(grad_force, n, "grad_force")
    p = params if params is not None else globals()["params"]()
    check(lib().mobility_adjoint(ctypes.byref(p), n, _ptr(pos), _ptr(force), _ptr(lam),
                                 _ptr(grad_pos), _ptr(grad_force), prec, _stream(stream)))
    return grad_pos, grad_force


def sd_step(x, force, dt: float, step_index: int = 0, *, v_prev=None, v_out=None,
            integrator: int = SD_EULER, params: SdParams = None, precision: int = None,
            stream=None):
    """One step in place on x ((n, 3) float64).  Returns x."""
    prec = _default_precision(force) if precision is None else int(precision)
    n = x.shape[0]
    _vec3(x, n, "x")
    _vec4(force, prec, "force")
    if v_prev is not None:
        _vec3(v_prev, n, "v_prev")
    if v_out is not None:
        _vec3(v_out, n, "v_out")
    p = params if params is not None else globals()["params"]()
    check(lib().sd_step(ctypes.byref(p), n, _ptr(x), _ptr(force), _ptr(v_prev), _ptr(v_out),
                        float(dt), int(step_index), int(integrator), prec, _stream(stream)))
    return x


def sd_run(x, force, dt: float, steps: int, *, step0: int = 0, v_prev=None,
           integrator: int = SD_EULER, checkpoints=None, checkpoint_every: int = 0,
           params: SdParams = None, precision: int = None, stream=None):
    """`steps` steps in place on x.  checkpoints: float64 tensor with
    (steps // checkpoint_every + 1) * 3n elements, or None.  Returns x."""
    prec = _default_precision(force) if precision is None else int(precision)
    n = x.shape[0]
    _vec3(x, n, "x")
    _vec4(force, prec, "force")
    if v_prev is not None:
        _vec3(v_prev, n, "v_prev")
    if checkpoints is not None and int(checkpoint_every) >= 1:   # else the library says why
        _vec3(checkpoints, n * (steps // checkpoint_every + 1), "checkpoints")
    p = params if params is not None else globals()["params"]()
    check(lib().sd_run(ctypes.byref(p), n, _ptr(x), _ptr(force), _ptr(v_prev), float(dt),
                       int(steps), int(step0), int(integrator), prec, _ptr(checkpoints),
                       int(checkpoint_every), _stream(stream)))
    return x


def sd_run_adjoint(x0, force, dt: float, steps: int, grad_xN, *, checkpoints=None,
                   checkpoint_every: int = 20, grad_x0=None, grad_force=None,
                   params: SdParams = None, precision: int = None, stream=None):
    """Gradients (dL/dx0, dL/dF) of a loss of x_steps through Euler steps."""
    import torch
    prec = _default_precision(force) if precision is None else int(precision)
    n = x0.shape[0]
    _vec3(x0, n, "x0")
    _vec4(force, prec, "force")
    _vec3(grad_xN, n, "grad_xN")
    if grad_x0 is None:
        grad_x0 = torch.empty((n, 3), dtype=torch.float64, device=x0.device)
    if grad_force is None:
        grad_force = torch.empty((n, 3), dtype=torch.float64, device=x0.device)
    if checkpoints is not None and int(checkpoint_every) >= 1:   # else the library says why
        _vec3(checkpoints, n * (steps // checkpoint_every + 1), "checkpoints")
    p = params if params is not None else globals()["params"]()
    check(lib().sd_run_adjoint(ctypes.byref(p), n, _ptr(x0), _ptr(force), float(dt), int(steps),
                               prec, _ptr(checkpoints), int(checkpoint_every), _ptr(grad_xN),
                               _ptr(grad_x0), _ptr(grad_force), _stream(stream)))
    return grad_x0, grad_force


def lubrication_forces(x, v, f_ext=None, f_out=None, *, params: SdParams = None,
                       lub_params: SdLub = None, stream=None):
    """f_ext - sum' zeta (v_i - v_j) for (n, 3) float64 CUDA tensors."""
    import torch
    n = x.shape[0]
    _vec3(x, n, "x")
    _vec3(v, n, "v")
    if f_ext is not None:
        _vec3(f_ext, n, "f_ext")
    if f_out is None:
        f_out = torch.empty((n, 3), dtype=torch.float64, device=x.device)
    _vec3(f_out, n, "f_out")
    p = params if params is not None else globals()["params"]()
    lb = lub_params if lub_params is not None else lub()
    check(lib().lubrication_forces(ctypes.byref(p), ctypes.byref(lb), n, _ptr(x), _ptr(v),
                                   _ptr(f_ext), _ptr(f_out), _stream(stream)))
    return f_out


def sd_run_lub(x, f_ext, v_prev, dt: float, steps: int, *, step0: int = 0,
               integrator: int = SD_EULER, params: SdParams = None, lub_params: SdLub = None,
               precision: int = SD_FP32_KAHAN, stream=None):
    """`steps` steps with the lubrication correction, in place on x and v_prev."""
    n = x.shape[0]
    for t, nm in ((x, "x"), (f_ext, "f_ext"), (v_prev, "v_prev")):
        _vec3(t, n, nm)
    p = params if params is not None else globals()["params"]()
    lb = lub_params if lub_params is not None else lub()
    check(lib().sd_run_lub(ctypes.byref(p), ctypes.byref(lb), n, _ptr(x), _ptr(f_ext),
                           _ptr(v_prev), float(dt), int(steps), int(step0), int(integrator),
                           int(precision), _stream(stream)))
    return x


class Batch:
    """A plan for many independent clusters (sd_batch_create)."""

    def __init__(self, offsets, *, params: SdParams = None):
        self._h = None
        offs = [int(v) for v in offsets]
        arr = (ctypes.c_int64 * len(offs))(*offs)
        h = ctypes.c_void_p()
        self.params = params if params is not None else globals()["params"]()
        self.n_clusters = len(offs) - 1
        check(lib().sd_batch_create(ctypes.byref(self.params), self.n_clusters, arr,
                                    ctypes.byref(h)))
        self._h = h
        self.n = int(lib().sd_batch_particles(h))

    def set_config(self, workgroup: int = 0, per_cu: int = 0) -> None:
        """Persistent-kernel shape (sd_batch_set_config): lanes per
        work-group 128 / 256 / 512 (0 = 256), work-groups per CU (0 = auto)."""
        check(lib().sd_batch_set_config(self._h, int(workgroup), int(per_cu)))

    def get_config(self) -> dict:
        wg, pc = ctypes.c_int32(), ctypes.c_int32()
        check(lib().sd_batch_get_config(self._h, ctypes.byref(wg), ctypes.byref(pc)))
        return {"workgroup": wg.value, "per_cu": pc.value}

    def autotune(self, x, force, dt: float, steps: int, *, integrator: int = SD_EULER,
                 precision: int = None, stream=None) -> dict:
        """Time every kernel shape on a copy of x and keep the fastest
        (sd_batch_autotune); returns the JSON report as a dict."""
        import json
        prec = _default_precision(force) if precision is None else int(precision)
        _vec3(x, self.n, "x")
        _vec4(force, prec, "force")
        buf = ctypes.create_string_buffer(8192)
        check(lib().sd_batch_autotune(self._h, _ptr(x), _ptr(force), float(dt), int(steps),
                                      int(integrator), prec, buf, len(buf), _stream(stream)))
        return json.loads(buf.value.decode())

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.sd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mobility_apply_batched(batch: Batch, pos, force, vel=None, *, precision: int = None,
                           stream=None):
    import torch
    prec = _default_precision(pos) if precision is None else int(precision)
    _vec4(pos, prec, "pos")
    _vec4(force, prec, "force")
    if pos.shape[0] != batch.n or force.shape[0] != batch.n:
        raise ValueError("pos/force must hold the batch's %d particles" % batch.n)
    if vel is None:
        vel = torch.empty((batch.n, 3), dtype=torch.float64, device=pos.device)
    _vec3(vel, batch.n, "vel")
    check(lib().mobility_apply_batched(batch._h, _ptr(pos), _ptr(force), _ptr(vel), prec,
                                       _stream(stream)))
    return vel


def sd_run_batched(batch: Batch, x, force, dt: float, steps: int, *, integrator: int = SD_EULER,
                   precision: int = None, use_graph: bool = True, stream=None):
    prec = _default_precision(force) if precision is None else int(precision)
    _vec3(x, batch.n, "x")
    _vec4(force, prec, "force")
    if force.shape[0] != batch.n:
        raise ValueError("force must hold the batch's %d particles" % batch.n)
    check(lib().sd_run_batched(batch._h, _ptr(x), _ptr(force), float(dt), int(steps),
                               int(integrator), prec, int(bool(use_graph)), _stream(stream)))
    return x


def cluster_frames(specs) -> int:
    """Frames sd_cluster_run writes for these specs (all runs)."""
    return sum(int(s["steps"]) // int(s["stride"]) for s in specs if int(s.get("stride", 0)) > 0)


def sd_cluster_run(state, force, specs, traj=None, *, params: SdParams = None, stream=None):
    """Runs of the precision study of Sec. 4 (see sd.h).  state: (runs, 2, n, 3)
    float64 CUDA tensor (hi, lo) in/out; force: (n, 3) float64; specs: list of
    dicts with keys acc, pos, dt, steps, stride (default 0).  Returns traj, a
    (frames, n, 3) float64 tensor holding the frames of run 0, then run 1, ...
    (allocated when not given), or None when no run records frames."""
    import torch
    runs = len(specs)
    n = force.shape[0]
    if tuple(state.shape) != (runs, 2, n, 3) or state.dtype != torch.float64 or \
            not state.is_cuda or not state.is_contiguous():
        raise ValueError("state must be a contiguous CUDA float64 tensor of shape (runs, 2, n, 3)")
    _vec3(force, n, "force")
    arr = (SdClusterSpec * runs)()
    for k, sp in enumerate(specs):
        arr[k] = SdClusterSpec(int(sp["acc"]), int(sp["pos"]), float(sp["dt"]), int(sp["steps"]),
                               int(sp.get("stride", 0)))
    frames = cluster_frames(specs)
    if frames and traj is None:
        traj = torch.empty((frames, n, 3), dtype=torch.float64, device=force.device)
    if traj is not None:
        _vec3(traj, frames * n, "traj")
    p = params if params is not None else globals()["params"]()
    check(lib().sd_cluster_run(ctypes.byref(p), n, runs, arr, _ptr(state), _ptr(force),
                               _ptr(traj), _stream(stream)))
    return traj if frames else None


def sd_membench(kind: int, access: int, inp, out=None, stream=None):
    """One App. A micro-benchmark launch.  inp: contiguous CUDA float32 tensor
    of shape (n,) (float) or (n, 4) (float4).  Returns out (same shape)."""
    import torch
    if not (inp.is_cuda and inp.dtype == torch.float32 and inp.is_contiguous()
            and (inp.dim() == 1 or (inp.dim() == 2 and inp.shape[1] == 4))):
        raise ValueError("inp must be a contiguous float32 CUDA tensor of shape (n,) or (n, 4)")
    elem = SD_MB_FLOAT if inp.dim() == 1 else SD_MB_FLOAT4
    if out is None:
        out = torch.empty_like(inp)
    elif out.shape != inp.shape or out.dtype != inp.dtype or not out.is_contiguous():
        raise ValueError("out must match inp")
    check(lib().sd_membench(int(kind), int(access), elem, inp.shape[0], _ptr(inp), _ptr(out),
                            _stream(stream)))
    return out


def sd_set_graph_mode(mode: int) -> None:
    """sd_run launch mode: 0 eager, 1 graphs for small n (default), 2 graphs always."""
    check(lib().sd_set_graph_mode(int(mode)))


def sd_pack(v, precision: int = SD_FP32_KAHAN, out=None, stream=None):
    """(n, 3) float64 CUDA tensor -> (n, 4) float32 (FP32 precisions) or
    float64 (SD_FP64) record tensor with w = 0, staged by the library's kernel."""
    import torch
    n = v.shape[0]
    _vec3(v, n, "v")
    prec = int(precision)
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float64 if prec == SD_FP64 else torch.float32,
                          device=v.device)
    _vec4(out, prec, "out")
    check(lib().sd_pack(n, _ptr(v), _ptr(out), prec, _stream(stream)))
    return out


def sd_mean_vector(v, out=None, stream=None):
    """(1/n) sum_i v_i of an (n, 3) float64 CUDA tensor, as a (3,) tensor."""
    import torch
    n = v.shape[0]
    _vec3(v, n, "v")
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=v.device)
    _vec3(out, 1, "out")
    check(lib().sd_mean_vector(n, _ptr(v), _ptr(out), _stream(stream)))
    return out


def sd_premise_counts(reset: bool = False, stream=None):
    """(pairs with 0 < r < 2a, coincident pairs) met by the product kernels on
    the current device since the last reset (the premise r >= 2a of Eq. 4)."""
    sub = ctypes.c_int64()
    co = ctypes.c_int64()
    check(lib().sd_premise_counts(ctypes.byref(sub), ctypes.byref(co), int(bool(reset)),
                                  _stream(stream)))
    return int(sub.value), int(co.value)


def sd_set_kernel_config(precision: int, cfg: Optional[dict]) -> None:
    if cfg is None:
        check(lib().sd_set_kernel_config(int(precision), None))
        return
    c = SdKernelConfig(**{k: int(v) for k, v in cfg.items()})
    check(lib().sd_set_kernel_config(int(precision), ctypes.byref(c)))


def sd_get_kernel_config(precision: int, n: int) -> dict:
    c = SdKernelConfig()
    check(lib().sd_get_kernel_config(int(precision), int(n), ctypes.byref(c)))
    return c.as_dict()


def sd_autotune(n: int, *, params: SdParams = None, precision: int = SD_FP32_KAHAN,
                stream=None) -> str:
    buf = ctypes.create_string_buffer(16384)
    p = params if params is not None else globals()["params"]()
    check(lib().sd_autotune(ctypes.byref(p), int(n), int(precision), _stream(stream), buf,
                            len(buf)))
    return buf.value.decode()


def sd_autotune_clear(precision: int = SD_FP32_KAHAN) -> None:
    check(lib().sd_autotune_clear(int(precision)))


def sd_profile_enable(on: bool = True) -> None:
    check(lib().sd_profile_enable(int(bool(on))))


def sd_profile_read():
    cnt = ctypes.c_int64()
    ms = ctypes.c_double()
    check(lib().sd_profile_read(ctypes.byref(cnt), ctypes.byref(ms)))
    return int(cnt.value), float(ms.value)


def sd_profile_reset() -> None:
    check(lib().sd_profile_reset())


def sd_profile_times():
    """Per-launch pair-kernel times (ms) since the last reset, in launch order."""
    cnt = ctypes.c_int64()
    check(lib().sd_profile_times(None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_float * max(1, cnt.value))()
    check(lib().sd_profile_times(buf, cnt.value, ctypes.byref(cnt)))
    return [float(buf[i]) for i in range(min(cnt.value, len(buf)))]


def sd_release() -> None:
    check(lib().sd_release())


def sd_version() -> int:
    return int(lib().sd_version())
