"""Helpers shared by the GPU parity tests."""

import math
import sys

import numpy as np
import torch

DEV = "cuda"


def rel_l2(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV).to(dtype).contiguous()


def say(*args):
    """Name the case before a GPU step, flushed, so a failing run shows it."""
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def sample_pixels(rng, n_slices, ny, nx, n):
    return np.stack([rng.integers(0, n_slices, n), rng.integers(0, ny, n),
                     rng.integers(0, nx, n)], 1).astype(np.int64)


def fp32_angles(n):
    return np.arange(n, dtype=np.float64) * (math.pi / n)
