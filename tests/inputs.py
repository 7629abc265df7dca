"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds random-number plumbing only (no step of the method): real fields with
unit Gaussian values, as the white noise of the paper's workloads has, and
index samples.  Values the method itself draws (the white noise) come from
each side's own Philox implementation, never from here.
"""
import numpy as np


def real_field(n, seed, dtype=np.float64):
    """An (n, n, n) field of i.i.d. N(0,1) values from numpy's PCG64."""
    return np.random.default_rng(seed).standard_normal((n, n, n)).astype(dtype)


def cell_sample(n, count, seed):
    """``count`` distinct linear cell indices of an n^3 lattice, sorted."""
    rng = np.random.default_rng(seed)
    total = n * n * n
    if count >= total:
        return np.arange(total, dtype=np.int64)
    return np.sort(rng.choice(total, size=count, replace=False)).astype(np.int64)


def subbox_origin(n, seed=42):
    """Origin of a periodic sub-box, as (i0, i1, i2)."""
    return tuple(int(v) for v in np.random.default_rng(seed).integers(0, n, 3))
