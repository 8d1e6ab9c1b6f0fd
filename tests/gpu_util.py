"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch.device("cuda:0")


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def to_dev(A, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(A))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel_fro(A, B):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / (nb if nb > 0 else 1.0))
