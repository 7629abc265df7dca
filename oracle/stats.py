"""Diagnostics of a field on the N^3 lattice, in float64 (test infrastructure).

The paper's pipeline can write the density field delta and its power
spectrum next to the velocity fields (Sec. 2.1, the list of outputs).  This
module defines both measurements plainly.

Binned power spectrum of a real field f of N^3 cells in a box of side L:
    F = forward transform of f (unnormalised, oracle.pipeline.forward);
    every mode n = (s0, s1, s2) of the full spectrum other than n = 0 with
    b = floor(|n|) < nbins falls in bin b (|n| in units of the fundamental
    mode k_f = 2 pi / L; s_j the signed index of oracle.pipeline, Nyquist
    taken as +N/2);
    P_b = (L^3 / N^6) <|F(n)|^2>_b,  kmean_b = k_f <|n|>_b,  count_b = modes in b.
With the normalisation of Eq. (1), delta~ = sqrt(P N^3 / L^3) W~, the
expectation of P_b for the density field is the input spectrum averaged over
the bin.  The half spectrum stores each pair n, -n once for 0 < s2 < N/2
(weight 2) and the planes s2 = 0 and s2 = N/2 in full (weight 1).

Field statistics: mean, standard deviation (population), minimum, maximum.

Pins (tests/test_oracle_stats.py): a single plane wave puts all its power in
one bin with the closed-form amplitude; the counts equal a brute-force count
of lattice vectors; sum_b count_b P_b is Parseval's sum; white noise has a
flat expectation L^3 / N^3; statistics against numpy's own reductions.
"""
import math

import numpy as np

from .pipeline import forward, signed_index


def mode_bins(n):
    """Bin index floor(|n|) and |n| of every stored mode of the half spectrum
    (shape (n, n, n/2+1)), and the weights 1 or 2."""
    s0 = signed_index(n).reshape(n, 1, 1)
    s1 = signed_index(n).reshape(1, n, 1)
    s2 = np.arange(n // 2 + 1).reshape(1, 1, n // 2 + 1)
    n2 = (s0 * s0 + s1 * s1 + s2 * s2).astype(np.int64)
    b = np.floor(np.sqrt(n2.astype(np.float64))).astype(np.int64)
    # exact integer square root (guards the float square root)
    b = np.where((b + 1) * (b + 1) <= n2, b + 1, b)
    b = np.where(b * b > n2, b - 1, b)
    w = np.where((s2 == 0) | (s2 == n // 2), 1.0, 2.0) * np.ones_like(n2, dtype=np.float64)
    return b, np.sqrt(n2.astype(np.float64)), w, n2


def power_spectrum(field, box, nbins, workers=None):
    """(pk, kmean, counts), each of length nbins, of the real field."""
    f = np.asarray(field, dtype=np.float64)
    n = f.shape[0]
    spec = forward(f, workers=workers)
    b, kn, w, n2 = mode_bins(n)
    keep = (n2 > 0) & (b < nbins)
    p = (np.abs(spec) ** 2)[keep]
    idx = b[keep]
    ww = w[keep]
    counts = np.bincount(idx, weights=ww, minlength=nbins)
    psum = np.bincount(idx, weights=ww * p, minlength=nbins)
    ksum = np.bincount(idx, weights=ww * kn[keep], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = np.where(counts > 0, psum / counts, 0.0) * (box ** 3 / float(n) ** 6)
        kmean = np.where(counts > 0, ksum / counts, 0.0) * (2.0 * math.pi / box)
    return pk, kmean, counts


def field_stats(field):
    """(mean, standard deviation, minimum, maximum) of all values."""
    f = np.asarray(field, dtype=np.float64).ravel()
    mean = float(f.mean())
    return mean, float(np.sqrt(np.mean((f - mean) ** 2))), float(f.min()), float(f.max())
