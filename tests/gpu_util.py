"""Helpers shared by the GPU parity tests: error metrics and cached oracle runs."""
import functools
import sys

import numpy as np

from oracle import cosmology as ocosmo
from oracle import noise as onoise
from oracle import pipeline as opipe


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


# measured figures that the session summary prints (tests/conftest.py), so
# they show in a quiet run's output as well
REPORT = []


def report(line):
    REPORT.append(line)
    say(line)


def rel_rms(got, want):
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    want = np.asarray(want, dtype=got.dtype)
    den = np.linalg.norm(want.ravel())
    return float(np.linalg.norm((got - want).ravel()) / (den if den > 0 else 1.0))


def max_rel(got, want):
    """max |got - want| / rms(want)."""
    got = np.asarray(got)
    want = np.asarray(want)
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    return float(np.abs(got - want).max() / (rms if rms > 0 else 1.0))


def ulp_diff_f32(a, b):
    """Per-element distance in float32 units in the last place."""
    ia = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    # map sign-magnitude to a monotone integer line
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


def periodic_abs_diff(a, b, box):
    """|a - b| on the periodic interval [0, box)."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    return np.minimum(d, box - d)


def oracle_cosmo(c):
    return ocosmo.Cosmology(c.omega_m, c.h, c.n_s, c.sigma8, c.z_init, amp=(c.amp if c.amp > 0 else None))


@functools.lru_cache(maxsize=4)
def oracle_noise(n, seed, dtype_name, stream=0):
    return onoise.noise_grid(n, seed, stream, dtype=np.float32 if dtype_name == "f32" else np.float64)


@functools.lru_cache(maxsize=3)
def oracle_ic(n, box, seed, dtype_name, offset=0.5):
    """(pos, vel, psi) of the oracle from the noise realisation the path of
    ``dtype_name`` consumes (float32-rounded deviates for f32)."""
    from paper_2511_10353_amd import Cosmo
    c = oracle_cosmo(Cosmo())
    w = oracle_noise(n, seed, dtype_name)
    psi = np.stack(opipe.displacement_fields(w, n, box, c, workers=8))
    pos = np.stack([opipe.positions(psi[j], n, box, offset, j) for j in range(3)])
    vel = np.stack([opipe.velocities(psi[j], c) for j in range(3)])
    return pos, vel, psi
