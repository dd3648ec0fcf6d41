"""Helpers shared by the GPU parity tests (device transfer of complex arrays)."""
import numpy as np


def to_dev(a):
    import torch
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return torch.from_numpy(a.view(np.float64).reshape(*a.shape, 2)).cuda()


def from_dev(t):
    a = t.detach().to("cpu").numpy()
    if a.dtype != np.float64:
        a = a.astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))
