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
