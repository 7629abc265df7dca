"""Noise -> density/displacement fields -> Zel'dovich particles, in float64.

Conventions (the paper gives no sign or normalisation for its transforms):

* Forward transform, unnormalised:  W~[n] = sum_m W[m] exp(-2 pi i n.m / N).
* Inverse transform, normalised:     f[m] = N^-3 sum_n f~[n] exp(+2 pi i n.m / N).
* Signed index s(n) = n for n < N/2, n - N for n > N/2; n = N/2 is Nyquist.
  k_j = 2 pi s_j / L (h/Mpc), n^2 = s_0^2 + s_1^2 + s_2^2.

Eq. (1) of Sec. 2.1: delta~ = sqrt(P(k) N^3 / L^3) W~, the volume factor making
<L^3 |N^-3 delta~|^2> = P(k).  Eq. (2): psi~_j = i k_j / k^2 delta~, so that
div psi = -delta.  The mode k = 0 is set to zero (mean removal) and so is every
mode with |s_j| = N/2 on any axis (keeps the field exactly real, and
div psi = -delta, curl psi = 0 mode by mode).

Sec. 2.2, Eq. (3): particle at lattice point q_j = (m_j + offset) Delta with
Delta = L/N moves to x_j = q_j + psi_j (sum in float64, wrapped periodically
into [0, L) as x - L floor(x/L), rounded to float32, a rounded value equal to L
mapped to 0), with
velocity v_j = a H f psi_j.  The paper's minus sign in Eq. (3) belongs to its
opposite Fourier sign convention; with the convention above the growing mode
moves particles along +psi.

Pins (tests/test_oracle_pipeline.py): the forward transform equals a direct
O(N^6) sum on 8^3 grids; Parseval; Hermitian symmetry of the filtered spectra;
a plane-wave density gives the closed-form displacement -A k0/k0^2 sin(k0.x);
div psi = -delta and curl psi = 0 spectrally; the binned power of delta over
many seeds recovers P(k); psi = 0 gives the exact lattice; linearity, lattice
translation and point reflection of the whole pipeline.
"""
import math

import numpy as np
import scipy.fft

from . import cosmology
from .noise import noise_grid


def signed_index(n):
    """s(i) for i in [0, n): i below n/2, i - n above; n/2 kept as +n/2."""
    i = np.arange(n)
    return np.where(i <= n // 2, i, i - n)


def forward(field, workers=None):
    """Unnormalised real-to-complex 3D transform, shape (n, n, n/2 + 1)."""
    return scipy.fft.rfftn(field, norm="backward", workers=workers)


def inverse(spec, n, workers=None):
    """Normalised complex-to-real 3D transform back to (n, n, n)."""
    return scipy.fft.irfftn(spec, s=(n, n, n), norm="backward", workers=workers)


def _mode_geometry(n):
    s0 = signed_index(n).reshape(n, 1, 1).astype(np.float64)
    s1 = signed_index(n).reshape(1, n, 1).astype(np.float64)
    s2 = np.arange(n // 2 + 1).reshape(1, 1, n // 2 + 1).astype(np.float64)
    n2 = s0 * s0 + s1 * s1 + s2 * s2
    half = n // 2
    keep = (n2 > 0) & (np.abs(s0) != half) & (np.abs(s1) != half) & (s2 != half)
    return (s0, s1, s2), n2, keep


def density_spectrum(w_hat, n, box, cosmo, amp=None):
    """Eq. (1): delta~ = sqrt(P(k) N^3/L^3) W~ (zero at k=0 and Nyquist)."""
    _, n2, keep = _mode_geometry(n)
    k = (2.0 * math.pi / box) * np.sqrt(np.where(keep, n2, 1.0))
    p = cosmology.power(k, cosmo, amp)
    scale = np.where(keep, np.sqrt(p * (n ** 3) / box ** 3), 0.0)
    return scale * w_hat


def displacement_spectrum(delta_hat, n, box, j):
    """Eq. (2): psi~_j = i k_j / k^2 delta~ for component j in {0, 1, 2}."""
    s, n2, keep = _mode_geometry(n)
    kj = (2.0 * math.pi / box) * s[j]
    k2 = (2.0 * math.pi / box) ** 2 * np.where(keep, n2, 1.0)
    ratio = np.where(keep, kj / k2, 0.0)
    return 1j * ratio * delta_hat


def lattice(n, box, offset, axis):
    """Lagrangian coordinate q along ``axis`` as a broadcastable array."""
    delta = box / n
    shape = [1, 1, 1]
    shape[axis] = n
    m = np.arange(n, dtype=np.float64).reshape(shape)
    return (m + offset) * delta


def periodic_wrap(x, box):
    """x - L floor(x/L) in float64: the periodic image of x in [0, L).  The
    quotient is rounded, so a result that lands on L or just below 0 is moved
    by one more period."""
    x = np.asarray(x, dtype=np.float64)
    x = x - box * np.floor(x / box)
    return np.where(x < 0.0, x + box, np.where(x >= box, x - box, x))


def positions(psi_j, n, box, offset, axis):
    """Eq. (3) for one component: float32 positions in [0, L)."""
    x = periodic_wrap(lattice(n, box, offset, axis) + np.asarray(psi_j, dtype=np.float64), box)
    out = x.astype(np.float32)
    return np.where(out >= np.float32(box), np.float32(0.0), out)


def velocities(psi_j, cosmo):
    """v_j = a H f psi_j, rounded to float32."""
    return (cosmology.velocity_factor(cosmo) * np.asarray(psi_j, dtype=np.float64)).astype(np.float32)


def displacement_fields(w, n, box, cosmo, amp=None, components=(0, 1, 2), workers=None):
    """psi_j (float64, shape (n,n,n)) for the requested components."""
    w_hat = forward(np.asarray(w, dtype=np.float64), workers=workers)
    delta_hat = density_spectrum(w_hat, n, box, cosmo, amp)
    del w_hat
    out = []
    for j in components:
        out.append(inverse(displacement_spectrum(delta_hat, n, box, j), n, workers=workers))
    return out


def density_field(w, n, box, cosmo, amp=None, workers=None):
    """delta(x) (float64), the inverse transform of Eq. (1)."""
    w_hat = forward(np.asarray(w, dtype=np.float64), workers=workers)
    return inverse(density_spectrum(w_hat, n, box, cosmo, amp), n, workers=workers)


def make_ic(n, box, cosmo, seed, noise_dtype=np.float64, stream=0, offset=0.5, workers=None):
    """Whole path from a seed: returns (pos, vel, psi) with shapes (3, n, n, n).

    ``noise_dtype`` selects which realisation is filtered: float64 noise, or the
    same deviates rounded to float32 (the single precision path's input).
    """
    w = noise_grid(n, seed, stream, dtype=noise_dtype)
    psi = np.stack(displacement_fields(w, n, box, cosmo, workers=workers))
    pos = np.stack([positions(psi[j], n, box, offset, j) for j in range(3)])
    vel = np.stack([velocities(psi[j], cosmo) for j in range(3)])
    return pos, vel, psi
