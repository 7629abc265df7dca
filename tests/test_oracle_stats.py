"""Pins for the oracle's diagnostics: binned power spectrum and field statistics."""
import math

import numpy as np
import pytest

from oracle import cosmology, pipeline, stats
from tests import inputs


def _plane_wave(n, n0, amp):
    m = np.indices((n, n, n)).reshape(3, -1).T
    return (amp * np.cos(2 * np.pi * (m @ np.asarray(n0)) / n)).reshape(n, n, n)


@pytest.mark.parametrize("n0,b", [((3, 4, 0), 5), ((1, 2, 2), 3), ((0, 0, 6), 6), ((8, 0, 0), 8)])
def test_plane_wave_power_in_one_bin(n0, b):
    n, box, amp = 16, 70.0, 1.7
    pk, kmean, counts = stats.power_spectrum(_plane_wave(n, n0, amp), box, 20)
    # two spikes of |F| = amp N^3 / 2 (one spike of amp N^3 at Nyquist, where cos is real and +-n0 coincide)
    nyq = any(abs(c) == n // 2 for c in n0)
    total = (amp * n ** 3) ** 2 if nyq else 2 * (amp * n ** 3 / 2) ** 2
    want = box ** 3 / n ** 6 * total / counts[b]
    assert abs(pk[b] - want) < 1e-12 * want
    others = np.delete(pk, b)
    assert np.abs(others).max() < 1e-20 * want
    assert abs(kmean[b] / (2 * math.pi / box) - np.mean([b])) < 1.0  # |n| inside the bin


def test_counts_equal_brute_force_lattice_count():
    n, nbins = 12, 12
    _, _, counts = stats.power_spectrum(np.zeros((n, n, n)), 10.0, nbins)
    s = pipeline.signed_index(n)
    want = np.zeros(nbins)
    for a in s:
        for b in s:
            for c in s:
                r2 = a * a + b * b + c * c
                if r2 == 0:
                    continue
                k = math.isqrt(int(r2))
                if k < nbins:
                    want[k] += 1
    assert np.array_equal(counts, want)


def test_parseval_over_all_bins():
    n, box = 16, 33.0
    f = inputs.real_field(n, 4)
    pk, _, counts = stats.power_spectrum(f, box, n)  # n > sqrt(3) n / 2 covers every mode
    lhs = float(np.sum(counts * pk))
    rhs = box ** 3 / n ** 3 * (np.sum(f * f) - n ** 3 * f.mean() ** 2)
    assert abs(lhs - rhs) < 1e-12 * rhs


def test_white_noise_is_flat():
    n, box = 32, 50.0
    acc = np.zeros(16)
    seeds = range(6)
    for sd in seeds:
        pk, _, counts = stats.power_spectrum(inputs.real_field(n, 100 + sd), box, 16)
        acc += pk
    acc /= len(seeds)
    expect = box ** 3 / n ** 3
    for b in range(4, 16):
        sigma = expect / math.sqrt(counts[b] * len(seeds) / 2)  # +-n pairs are one complex mode
        assert abs(acc[b] - expect) < 5 * sigma


def test_density_field_recovers_input_spectrum():
    # Eq. (1): <P_b> of delta is the bin average of P(k)
    n, box = 32, 200.0
    c = cosmology.Cosmology()
    acc = np.zeros(12)
    for sd in range(8):
        from oracle import noise
        d = pipeline.density_field(noise.noise_grid(n, sd), n, box, c)
        pk, kmean, counts = stats.power_spectrum(d, box, 12)
        acc += pk
    acc /= 8
    b, kn, w, n2 = stats.mode_bins(n)
    for bb in range(3, 12):
        sel = (b == bb) & (n2 > 0)
        p = cosmology.power(kn[sel] * 2 * math.pi / box, c)
        expect = float(np.sum(w[sel] * p) / np.sum(w[sel]))
        sigma = expect / math.sqrt(counts[bb] * 8 / 2)
        assert abs(acc[bb] - expect) < 5 * sigma


def test_field_stats_closed_forms():
    n = 8
    assert stats.field_stats(np.full((n, n, n), 2.5)) == (2.5, 0.0, 2.5, 2.5)
    f = np.arange(n ** 3, dtype=np.float64).reshape(n, n, n)
    mean, sd, lo, hi = stats.field_stats(f)
    m = n ** 3
    assert mean == (m - 1) / 2
    assert abs(sd - math.sqrt((m * m - 1) / 12)) < 1e-12 * sd
    assert (lo, hi) == (0.0, m - 1.0)
