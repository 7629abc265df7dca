"""Pins for the oracle's spectrum, sigma_8 normalisation and velocity factor."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import cosmology


def test_sigma_closed_form_power_law():
    # P(k) = A/k: int_0^inf x W(x)^2 dx = 9/4 (Bessel-integral closed form),
    # so sigma^2(R) = 9 A / (8 pi^2 R^2); the integration limits cut < 2e-8
    amp = 3.7
    got = cosmology.sigma_r_squared(lambda k: amp / k, radius=8.0)
    want = 9.0 * amp / (8.0 * math.pi ** 2 * 64.0)
    assert abs(got / want - 1.0) < 1e-7


def test_sigma_closed_form_white_spectrum_other_radius():
    # P(k) = A: sigma^2(R) = A / (4/3 pi R^3) (variance of white noise in a
    # sphere).  Cutting the integral at K = 1e3 h/Mpc drops the tail
    # int_K^inf k^2 W(kR)^2 dk ~ 9/(2 R^4 K), a relative 3/(pi R K).
    amp = 2.0
    radius = 50.0
    got = cosmology.sigma_r_squared(lambda k: amp + 0 * k, radius=radius)
    want = amp / (4.0 / 3.0 * math.pi * radius ** 3)
    tail = 3.0 / (math.pi * radius * math.exp(cosmology.LN_K_MAX))
    assert abs(got / want - 1.0 + tail) < 1e-6


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_simpson_matches_adaptive_quadrature_bbks():
    c = cosmology.Cosmology()
    shape = cosmology.shape_spectrum(c)

    def integrand(lnk):
        k = math.exp(lnk)
        return float(k ** 3 * shape(np.array([k]))[0] * cosmology.tophat_window(np.array([8.0 * k]))[0] ** 2)

    pts = np.linspace(cosmology.LN_K_MIN, cosmology.LN_K_MAX, 40)
    total = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        total += integrate.quad(integrand, a, b, epsabs=0, epsrel=1e-13, limit=400)[0]
    want = total / (2 * math.pi ** 2)
    got = cosmology.sigma_r_squared(shape)
    assert abs(got / want - 1.0) < 1e-9


def test_amplitude_normalises_sigma8():
    c = cosmology.Cosmology()
    a = cosmology.amplitude(c)
    s2 = cosmology.sigma_r_squared(lambda k: a * cosmology.shape_spectrum(c)(k))
    assert abs(math.sqrt(s2) - 0.8) < 1e-12
    assert 1.4e6 < a < 1.55e6
    assert cosmology.amplitude(cosmology.Cosmology(amp=5.0)) == 5.0


def test_transfer_limits():
    g = 0.21
    assert abs(cosmology.bbks_transfer(np.array([1e-9]), g)[0] - 1.0) < 1e-7
    k = np.logspace(-4, 2, 200)
    t = cosmology.bbks_transfer(k, g)
    assert np.all(np.diff(t) < 0) and np.all(t > 0)


def test_window_series_joins_closed_form():
    x = np.array([0.00999999, 0.01000001])
    w = cosmology.tophat_window(x)
    assert abs(w[0] - w[1]) < 1e-9
    assert cosmology.tophat_window(np.array([0.0]))[0] == 1.0


def test_velocity_factor():
    # Einstein-de Sitter: a H(a) = 100 a^(-1/2) = 100 sqrt(1+z)
    eds = cosmology.Cosmology(omega_m=1.0, z_init=99.0)
    assert abs(cosmology.velocity_factor(eds) - 1000.0) < 1e-10
    lcdm = cosmology.Cosmology()
    assert abs(cosmology.velocity_factor(lcdm) - 550.4550) < 5e-4
    assert cosmology.growth(0.0) == 1.0
