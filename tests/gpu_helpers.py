"""Shared helpers of the GPU tests: data layout conversions and error measures."""
import numpy as np

import synth


def flat(x):
    """(rows, n, n) -> (rows * n * n,) C-contiguous float64 (the C-ABI layout)."""
    return np.ascontiguousarray(x, dtype=np.float64).reshape(-1)


def grid(v, J, K):
    n = 2 ** K - 1
    return v.reshape(2 ** J + 1, n, n)


def rel_err(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    s = np.linalg.norm(np.asarray(b).ravel())
    return d / s if s > 0 else d


def max_rel(a, b):
    """max |a - b| / max |b| (elementwise comparison scaled by the data)."""
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def sin_u0(K):
    return synth.sine_product(K, 1, 1)
