"""Helpers shared by the GPU tests (marshalling only; no method arithmetic)."""
import numpy as np


def dev():
    import torch
    return torch.device("cuda", 0)


def to_dev4(v, dtype):
    """(n, 3) float64 numpy -> (n, 4) CUDA tensor of the given torch dtype, w = 0."""
    import torch
    out = np.zeros((v.shape[0], 4))
    out[:, :3] = v
    return torch.tensor(out, dtype=dtype, device=dev())


def to_dev3(v):
    import torch
    return torch.tensor(np.ascontiguousarray(v, dtype=np.float64), device=dev())


def rel2(a, b):
    """Relative 2-norm error over all components: |a - b| / |b|."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rowerr(a, b):
    """Largest error of one particle's vector, relative to the larger of that
    particle's reference norm and the median reference norm over the rows
    (rows whose velocity nearly cancels are measured on the typical scale):
    max_i |a_i - b_i| / max(|b_i|, median_k |b_k|), rows of 3 components."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    nb = np.linalg.norm(b, axis=1)
    floor = np.median(nb)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(nb, floor)))
