"""Shared test helpers (no arithmetic of the method here)."""
import numpy as np


def rel_fro(x, ref):
    """Relative Frobenius error ||x - ref|| / ||ref|| (0/0 -> 0)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(x - ref)
    n = np.linalg.norm(ref)
    if n == 0.0:
        return float(d)
    return float(d / n)


def say(*args):
    print(*args, flush=True)
