"""Pins for the oracle's transforms, Eq. (1)-(2) filter and Eq. (3) particles."""
import math

import numpy as np
import pytest

from oracle import cosmology, noise, pipeline
from tests import inputs

COSMO = cosmology.Cosmology()


def _direct_forward(f):
    n = f.shape[0]
    m = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    k = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n // 2 + 1), indexing="ij"), -1).reshape(-1, 3)
    e = np.exp(-2j * np.pi * (k @ m.T) / n)
    return (e @ f.reshape(-1)).reshape(n, n, n // 2 + 1)


def _direct_inverse_full(spec_full):
    n = spec_full.shape[0]
    m = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    e = np.exp(2j * np.pi * (m @ m.T) / n)
    return (e @ spec_full.reshape(-1)).reshape(n, n, n) / n ** 3


def _hermitian_full(half, n):
    full = np.zeros((n, n, n), dtype=complex)
    full[:, :, : n // 2 + 1] = half
    for kz in range(n // 2 + 1, n):
        full[:, :, kz] = np.conj(half[(-np.arange(n)) % n][:, (-np.arange(n)) % n][:, :, n - kz])
    return full


def test_forward_is_direct_dft():
    f = inputs.real_field(8, 1)
    assert np.abs(pipeline.forward(f) - _direct_forward(f)).max() < 1e-12


def test_inverse_is_direct_inverse_dft():
    f = inputs.real_field(8, 2)
    half = _direct_forward(f)
    back = pipeline.inverse(half, 8)
    direct = _direct_inverse_full(_hermitian_full(half, 8))
    assert np.abs(direct.imag).max() < 1e-12
    assert np.abs(back - direct.real).max() < 1e-12
    assert np.abs(back - f).max() < 1e-12


def test_parseval():
    n = 16
    f = inputs.real_field(n, 3)
    h = pipeline.forward(f)
    w = np.full(n // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    assert abs(np.sum(f * f) - np.sum(w * np.abs(h) ** 2) / n ** 3) < 1e-10 * np.sum(f * f)


def _real_space_gradient(field, box, axis):
    n = field.shape[0]
    s = pipeline.signed_index(n).astype(float)
    s[n // 2] = 0.0
    shape = [1, 1, 1]
    shape[axis] = n
    k = (2 * math.pi / box) * s.reshape(shape)
    spec = np.fft.fftn(field)
    return np.fft.ifftn(1j * k * spec).real


def test_plane_wave_closed_form():
    n, box, amp = 16, 100.0, 0.3
    a = np.array([2, -1, 3])
    m = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), 0)
    phase = 2 * math.pi * np.tensordot(a, m, axes=1) / n
    delta = amp * np.cos(phase)
    dhat = pipeline.forward(delta)
    k0 = 2 * math.pi * a / box
    for j in range(3):
        psi = pipeline.inverse(pipeline.displacement_spectrum(dhat, n, box, j), n)
        want = -amp * k0[j] / np.dot(k0, k0) * np.sin(phase)
        assert np.abs(psi - want).max() < 1e-14


def test_divergence_and_curl():
    n, box = 16, 100.0
    w = noise.noise_grid(n, 11)
    psi = pipeline.displacement_fields(w, n, box, COSMO)
    delta = pipeline.density_field(w, n, box, COSMO)
    div = sum(_real_space_gradient(psi[j], box, j) for j in range(3))
    scale = np.abs(delta).max()
    assert np.abs(div + delta).max() < 1e-13 * scale
    for a, b in ((0, 1), (1, 2), (0, 2)):
        curl = _real_space_gradient(psi[b], box, a) - _real_space_gradient(psi[a], box, b)
        assert np.abs(curl).max() < 1e-13 * scale


def test_filtered_spectrum_hermitian_and_zeroed():
    n, box = 16, 100.0
    w_hat = pipeline.forward(noise.noise_grid(n, 12))
    d = pipeline.density_spectrum(w_hat, n, box, COSMO)
    for spec in [d] + [pipeline.displacement_spectrum(d, n, box, j) for j in range(3)]:
        assert spec[0, 0, 0] == 0
        assert np.all(spec[n // 2] == 0) and np.all(spec[:, n // 2] == 0) and np.all(spec[:, :, n // 2] == 0)
        plane = spec[:, :, 0]
        neg = plane[(-np.arange(n)) % n][:, (-np.arange(n)) % n]
        assert np.abs(plane - np.conj(neg)).max() <= 1e-12 * np.abs(plane).max()


def test_power_spectrum_recovery():
    # <L^3 |N^-3 delta~|^2> over seeds equals the mode-averaged input P(k)
    n, box, seeds = 16, 100.0, 24
    (s0, s1, s2), n2, keep = pipeline._mode_geometry(n)
    kmag = (2 * math.pi / box) * np.sqrt(n2)
    p_in = cosmology.power(np.where(keep, kmag, 1.0), COSMO)
    acc = np.zeros(n2.shape)
    for seed in range(seeds):
        d = pipeline.density_spectrum(pipeline.forward(noise.noise_grid(n, seed)), n, box, COSMO)
        acc += box ** 3 * np.abs(d / n ** 3) ** 2
    acc /= seeds
    edges = np.arange(1, n // 2) * (2 * math.pi / box)
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = keep & (kmag >= lo) & (kmag < hi)
        modes = int(sel.sum())
        ratio = acc[sel].sum() / p_in[sel].sum()
        # each mode's |W~|^2/N^3 is exponential (mean 1); the kz = 0 plane holds
        # conjugate pairs, so count modes conservatively
        assert abs(ratio - 1.0) < 5.0 / math.sqrt(modes * seeds / 2.0)


def test_zero_displacement_gives_lattice():
    n, box = 8, 100.0
    z = np.zeros((n, n, n))
    for j in range(3):
        pos = pipeline.positions(z, n, box, 0.5, j)
        idx = np.arange(n).reshape([n if a == j else 1 for a in range(3)])
        want = np.broadcast_to(((idx + 0.5) * (box / n)).astype(np.float32), pos.shape)
        assert np.array_equal(pos, want)
    assert np.all(pipeline.velocities(z, COSMO) == 0)


def test_positions_wrap_into_box():
    n, box = 8, 100.0
    psi = np.full((n, n, n), -20.0)
    pos = pipeline.positions(psi, n, box, 0.5, 0)
    assert pos.min() >= 0 and pos.max() < box
    assert pos[0, 0, 0] == np.float32(0.5 * box / n - 20.0 + box)
    psi = np.full((n, n, n), 95.0)
    pos = pipeline.positions(psi, n, box, 0.5, 2)
    assert pos[0, 0, 7] == np.float32((7.5 * box / n + 95.0) - box)
    # a value just below L that rounds to L in float32 maps to 0
    psi = np.zeros((n, n, n))
    psi[-1, 0, 0] = box - 7.5 * box / n - 1e-9
    assert pipeline.positions(psi, n, box, 0.5, 0)[-1, 0, 0] == 0.0


@pytest.mark.parametrize("periods", [-3, -2, 2, 5])
def test_positions_wrap_several_periods(periods):
    # displacements of several box lengths land on the same periodic image:
    # exact multiples of L (L a power of two and psi of 26 bits, so every sum is exact) move
    # nothing, and the image lies in [0, L)
    n, box = 8, 64.0
    rng = np.random.default_rng(periods + 10)
    psi = np.round(rng.uniform(-0.9, 0.9, (n, n, n)) * 2.0 ** 20) * 2.0 ** -20 * box  # 26-bit values
    base = pipeline.positions(psi, n, box, 0.5, 1)
    moved = pipeline.positions(psi + periods * box, n, box, 0.5, 1)
    assert np.array_equal(base, moved)
    assert moved.min() >= 0 and moved.max() < box
    # the image is q + psi - L floor((q + psi)/L) evaluated exactly
    q = (np.arange(n).reshape(1, n, 1) + 0.5) * (box / n)
    x = q + psi + periods * box
    want = np.array([float(v) % box for v in x.ravel()]).reshape(x.shape).astype(np.float32)
    want = np.where(want >= np.float32(box), np.float32(0.0), want)
    assert np.array_equal(moved, want)


def test_linearity_translation_reflection():
    n, box = 16, 100.0
    w = noise.noise_grid(n, 21)
    psi = np.stack(pipeline.displacement_fields(w, n, box, COSMO))
    scale = np.abs(psi).max()
    psi2 = np.stack(pipeline.displacement_fields(2.5 * w, n, box, COSMO))
    assert np.abs(psi2 - 2.5 * psi).max() < 1e-13 * scale
    r = (3, -5, 7)
    psi_r = np.stack(pipeline.displacement_fields(np.roll(w, r, (0, 1, 2)), n, box, COSMO))
    assert np.abs(psi_r - np.roll(psi, r, (1, 2, 3))).max() < 1e-13 * scale
    idx = (-np.arange(n)) % n
    w_ref = w[idx][:, idx][:, :, idx]
    psi_ref = np.stack(pipeline.displacement_fields(w_ref, n, box, COSMO))
    assert np.abs(psi_ref + psi[:, idx][:, :, idx][:, :, :, idx]).max() < 1e-13 * scale


def test_amplitude_scaling():
    n, box = 8, 100.0
    w = noise.noise_grid(n, 5)
    a = cosmology.amplitude(COSMO)
    p1 = np.stack(pipeline.displacement_fields(w, n, box, COSMO))
    p4 = np.stack(pipeline.displacement_fields(w, n, box, COSMO, amp=4 * a))
    assert np.abs(p4 - 2 * p1).max() < 1e-13 * np.abs(p1).max()


def test_end_to_end_direct_sums_n8():
    # whole path with every transform replaced by its direct O(N^6) sum
    n, box = 8, 100.0
    w = noise.noise_grid(n, 42)
    pos, vel, psi = pipeline.make_ic(n, box, COSMO, 42)
    d = pipeline.density_spectrum(_direct_forward(w), n, box, COSMO)
    for j in range(3):
        spec = pipeline.displacement_spectrum(d, n, box, j)
        direct = _direct_inverse_full(_hermitian_full(spec, n)).real
        assert np.abs(psi[j] - direct).max() < 1e-12 * np.abs(direct).max()
    assert pos.dtype == np.float32 and vel.dtype == np.float32
    vf = cosmology.velocity_factor(COSMO)
    assert np.abs(vel - vf * psi).max() <= 1e-6 * np.abs(vf * psi).max()
