"""Pins for the oracle's resolution degrade (NGP decimation + Fourier
translation, Sec. 2.3)."""
import numpy as np
import pytest

from oracle import degrade
from tests import inputs


def _grid(n):
    return np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")


def test_zero_shift_is_decimation():
    f = inputs.real_field(24, 3)
    out = degrade.degrade(f, 3, (0.0, 0.0, 0.0))
    assert out.shape == (8, 8, 8)
    assert np.abs(out - f[::3, ::3, ::3]).max() < 1e-14 * np.abs(f).max()


def test_integer_shift_is_a_roll():
    d = inputs.real_field(16, 4)
    out = degrade.translate(d, (1.0, -2.0, 3.0))
    assert np.abs(out - np.roll(d, (1, -2, 3), axis=(0, 1, 2))).max() < 1e-14 * np.abs(d).max()


@pytest.mark.parametrize("shift", [(0.5, 0.5, 0.5), (0.5, 0.25, -0.75), (1.3, -0.1, 2.6)])
def test_band_limited_plane_wave_moves_exactly(shift):
    # fine wave with |n_j| below the coarse Nyquist: its decimation is the same
    # wave on the coarse lattice, and the translation evaluates it at m - s
    n_hi, factor = 32, 2
    n_lo = n_hi // factor
    nv, phase = (3, -5, 2), 0.7
    m = _grid(n_hi)
    f = np.cos(2 * np.pi * sum(k * x for k, x in zip(nv, m)) / n_hi + phase)
    ml = _grid(n_lo)
    want = np.cos(2 * np.pi * sum(k * (x - s) for k, x, s in zip(nv, ml, shift)) / n_lo + phase)
    assert np.abs(degrade.degrade(f, factor, shift) - want).max() < 1e-13


def test_nyquist_pattern_scales_by_cos_pi_s():
    n = 8
    m = _grid(n)
    s = (0.5, 0.3, -1.0)
    one = (-1.0) ** m[0]
    assert np.abs(degrade.translate(one, s) - np.cos(np.pi * s[0]) * one).max() < 1e-14
    corner = (-1.0) ** (m[0] + m[1] + m[2])
    want = np.cos(np.pi * s[0]) * np.cos(np.pi * s[1]) * np.cos(np.pi * s[2]) * corner
    assert np.abs(degrade.translate(corner, s) - want).max() < 1e-14


def test_translations_compose_without_nyquist_content():
    n = 16
    d = inputs.real_field(n, 5)
    spec = np.fft.rfftn(d)
    spec[n // 2, :, :] = 0
    spec[:, n // 2, :] = 0
    spec[:, :, n // 2] = 0
    d = np.fft.irfftn(spec, s=d.shape, axes=(0, 1, 2))
    a, b = (0.3, -0.45, 0.8), (0.25, 0.5, -1.1)
    ab = tuple(x + y for x, y in zip(a, b))
    two = degrade.translate(degrade.translate(d, a), b)
    assert np.abs(two - degrade.translate(d, ab)).max() < 1e-14 * np.abs(d).max()
    # the mean is untouched
    assert abs(degrade.translate(d, a).mean() - d.mean()) < 1e-15


def test_rejects_bad_factor():
    with pytest.raises(ValueError):
        degrade.decimate(np.zeros((10, 10, 10)), 3)
