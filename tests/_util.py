"""Shared helpers for the test-suite (no method arithmetic)."""
import sys

import numpy as np


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def crandn(rng, *shape, dtype=np.complex128):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def announce(msg: str) -> None:
    """Print and flush the case about to run on the GPU."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_gpu(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()
