"""Helpers shared by the GPU parity tests (inputs only; no method arithmetic)."""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def say(*a):
    print(*a, flush=True)


def to_dev(arrs, dev):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
