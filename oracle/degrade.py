"""Resolution degrade of a displacement field (Sec. 2.3, last paragraph), in
float64 (test infrastructure: only tests/, the smoke check and the benchmark's
CPU baseline use this package).

The paper lowers the resolution of an existing field in two steps: a
nearest-grid-point interpolation of the fine field onto the coarse lattice,
then a translation by half a coarse cell done in Fourier space.  It gives no
formulas; the reading used here:

  NGP        fine field f on N_H^3 points m Delta_H, coarse lattice of
             N_L = N_H / F points m Delta_L = (F m) Delta_H: each coarse point
             coincides with the fine point F m, whose value it takes,
             D[m] = f[F m];
  translate  out = D moved by s coarse cells along every axis (s = 1/2 in the
             paper): the band-limited interpolant of D evaluated at m - s.
             Mode n_j (signed, |n_j| < N_L / 2) of axis j is multiplied by
             exp(-2 pi i s n_j / N_L); on the Nyquist plane n_j = N_L / 2 the
             real interpolant cos(pi x) gives the factor cos(pi s), which keeps
             the field real (zero for s = 1/2).

Pins (tests/test_oracle_degrade.py): s = 0 is plain decimation; an integer s
is a periodic roll by s cells; a band-limited plane wave is moved exactly;
the pure Nyquist pattern is scaled by cos(pi s); translations compose.
"""
import numpy as np


def decimate(f, factor):
    """NGP onto the coarse lattice: D[m] = f[factor m] (periodic fine field)."""
    f = np.asarray(f, dtype=np.float64)
    n_hi = f.shape[0]
    if f.shape != (n_hi,) * 3 or factor < 1 or n_hi % factor:
        raise ValueError("fine field must be cubic with a side divisible by the factor")
    return f[::factor, ::factor, ::factor].copy()


def axis_factor(n, s, half=False):
    """Translation factor of each mode index along one axis of length n
    (indices 0..n-1 in FFT order, or 0..n/2 for the halved last axis)."""
    k = np.arange(n // 2 + 1) if half else np.arange(n)
    signed = np.where(k <= n // 2, k, k - n)
    fac = np.exp(-2j * np.pi * s * signed / n)
    if n % 2 == 0:
        fac[n // 2] = np.cos(np.pi * s)
    return fac


def translate(d, shift):
    """Move the periodic field d by shift = (s0, s1, s2) cells (band-limited)."""
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    spec = np.fft.rfftn(d)
    f0 = axis_factor(n, shift[0])[:, None, None]
    f1 = axis_factor(n, shift[1])[None, :, None]
    f2 = axis_factor(n, shift[2], half=True)[None, None, :]
    return np.fft.irfftn(spec * f0 * f1 * f2, s=d.shape, axes=(0, 1, 2))


def degrade(f, factor, shift=(0.5, 0.5, 0.5)):
    """Sec. 2.3 degrade: NGP decimation by `factor`, then the Fourier
    translation by `shift` coarse cells."""
    return translate(decimate(f, factor), shift)
