"""Power spectrum, its sigma_8 normalisation, growth and velocity factor.

The paper takes P(k) as a tabulated input and normalises it by sigma_8, the
r.m.s. density contrast in spheres of radius 8 Mpc/h (Sec. 2.1 and its
footnote).  The workloads here replace the table by an analytic spectrum:

    P(k, z) = D(z)^2 A k^n_s T(k)^2,     k in h/Mpc, P in (Mpc/h)^3

* T is the BBKS fit (Bardeen, Bond, Kaiser & Szalay 1986, ApJ 304, 15,
  eq. G3) with q = k / Gamma and shape parameter Gamma = Omega_m h:
  T = ln(1 + 2.34 q)/(2.34 q) [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3 + (6.71 q)^4]^(-1/4).
* A fixes sigma_8 at z = 0:
  sigma_8^2 = (1/2 pi^2) int k^2 P(k, 0) W(8 k)^2 dk,
  W(x) = 3 (sin x - x cos x)/x^3 (top hat), with W = 1 - x^2/10 + x^4/280
  for x < 1e-2.  The integral is taken over ln k in [ln 1e-5, ln 1e3] by
  composite Simpson with 2^16 intervals.
* D(z) = 1/(1+z): Einstein-de Sitter growth normalised to D(0) = 1.
* Velocities: v = a H(a) f psi with H(a) = 100 sqrt(Omega_m a^-3 + 1 - Omega_m)
  km/s per Mpc/h and growth rate f = 1 (Sec. 2.2 names D, its derivative and
  a; the EdS growth fixes f).

Pins (tests/test_oracle_cosmology.py): the sigma routine returns the closed
form A / V_sphere for a constant spectrum; the Simpson integral agrees with an
independent adaptive quadrature (scipy.integrate.quad) of the BBKS integrand;
T -> 1 as k -> 0; the velocity factor reduces to 100 sqrt(1+z) for Omega_m = 1.
"""
import math

import numpy as np

LN_K_MIN = math.log(1e-5)
LN_K_MAX = math.log(1e3)
SIMPSON_INTERVALS = 1 << 16
R8 = 8.0


class Cosmology:
    """Parameters of the analytic spectrum (defaults: the workloads' values)."""

    def __init__(self, omega_m=0.3, h=0.7, n_s=0.96, sigma8=0.8, z_init=100.0, amp=None):
        self.omega_m = float(omega_m)
        self.h = float(h)
        self.n_s = float(n_s)
        self.sigma8 = float(sigma8)
        self.z_init = float(z_init)
        # amp: if given, the z=0 amplitude A used instead of the sigma_8 value
        self.amp = None if amp is None else float(amp)

    @property
    def gamma(self):
        return self.omega_m * self.h


def bbks_transfer(k, gamma):
    """BBKS transfer function T(k) (k in h/Mpc, gamma = Omega_m h)."""
    k = np.asarray(k, dtype=np.float64)
    q = k / gamma
    aq = 2.34 * q
    lead = np.where(aq < 1e-8, 1.0 - 0.5 * aq, np.log1p(aq) / np.where(aq == 0.0, 1.0, aq))
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return lead * poly ** -0.25


def tophat_window(x):
    """Fourier transform of the unit top-hat sphere, W(x) = 3 j_1(x)/x."""
    x = np.asarray(x, dtype=np.float64)
    small = x < 1e-2
    xs = np.where(small, 1.0, x)
    full = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    series = 1.0 - x * x / 10.0 + x ** 4 / 280.0
    return np.where(small, series, full)


def sigma_r_squared(pk, radius=R8, n_intervals=SIMPSON_INTERVALS):
    """sigma^2(R) = (1/2 pi^2) int k^3 P(k) W(kR)^2 d ln k, composite Simpson."""
    lnk = np.linspace(LN_K_MIN, LN_K_MAX, n_intervals + 1)
    k = np.exp(lnk)
    f = k ** 3 * pk(k) * tophat_window(k * radius) ** 2
    w = np.ones(n_intervals + 1)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    step = (LN_K_MAX - LN_K_MIN) / n_intervals
    return float(np.sum(w * f) * step / 3.0) / (2.0 * math.pi ** 2)


def shape_spectrum(cosmo):
    """k^n_s T(k)^2 (the spectrum up to its amplitude), as a callable."""
    return lambda k: k ** cosmo.n_s * bbks_transfer(k, cosmo.gamma) ** 2


def amplitude(cosmo):
    """A such that sigma_8 at z=0 equals cosmo.sigma8 (or cosmo.amp if set)."""
    if cosmo.amp is not None:
        return cosmo.amp
    return cosmo.sigma8 ** 2 / sigma_r_squared(shape_spectrum(cosmo))


def growth(z):
    """Einstein-de Sitter linear growth, D(0) = 1."""
    return 1.0 / (1.0 + z)


def power(k, cosmo, amp=None):
    """P(k, z_init) in (Mpc/h)^3."""
    a_amp = amplitude(cosmo) if amp is None else amp
    d = growth(cosmo.z_init)
    return d * d * a_amp * shape_spectrum(cosmo)(np.asarray(k, dtype=np.float64))


def hubble(a, omega_m):
    """H(a) in km/s per Mpc/h for flat Lambda-CDM."""
    return 100.0 * math.sqrt(omega_m / a ** 3 + 1.0 - omega_m)


def velocity_factor(cosmo):
    """a H(a) f, with f = 1, at z_init: v = a H f psi in km/s."""
    a = 1.0 / (1.0 + cosmo.z_init)
    return a * hubble(a, cosmo.omega_m) * 1.0
