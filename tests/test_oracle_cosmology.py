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


def test_transfer_series_at_small_q():
    # Taylor coefficients of T(q) = L(q) G(q) derived by hand:
    # L = ln(1 + a q)/(a q) = 1 - a q/2 + (a q)^2/3 - (a q)^3/4 + ...,
    # G = (1 + x)^(-1/4) = 1 - x/4 + 5 x^2/32 - 15 x^3/128 + ... with
    # x = b1 q + b2 q^2 + b3 q^3 + b4 q^4.  Each of the first three orders
    # brings in one more coefficient of the fit (a and b1, then b2, then b3).
    a, b1, b2, b3 = 2.34, 3.89, 16.1 ** 2, 5.46 ** 3
    l1, l2, l3 = -a / 2, a * a / 3, -a ** 3 / 4
    g1 = -b1 / 4
    g2 = -b2 / 4 + 5 * b1 ** 2 / 32
    g3 = -b3 / 4 + 5 * b1 * b2 / 16 - 15 * b1 ** 3 / 128
    want = [1.0, l1 + g1, l2 + l1 * g1 + g2, l3 + l2 * g1 + l1 * g2 + g3]
    gamma, qmax = 0.21, 0.005
    q = np.linspace(qmax / 400, qmax, 400)
    t = cosmology.bbks_transfer(q * gamma, gamma)
    got = np.polynomial.Polynomial.fit(q, t, 10, domain=[-qmax, qmax]).convert().coef
    for order, tol in enumerate((1e-13, 1e-9, 1e-7, 1e-5)):
        assert abs(got[order] / want[order] - 1.0) < tol, order


def test_transfer_large_q_asymptote():
    # for q -> infinity the bracket tends to (6.71 q)^4 and ln(1 + a q) to
    # ln(a q): T q^2 6.71 a / ln(a q) -> 1, with corrections of order
    # 1/(q ln q)
    a, gamma = 2.34, 0.21
    for q, tol in ((1e6, 2e-8), (1e8, 1e-10)):
        t = cosmology.bbks_transfer(np.array([q * gamma]), gamma)[0]
        assert abs(t * 6.71 * a * q * q / np.log(a * q) - 1.0) < tol


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


def _growth_integral(a, omega_m=1.0):
    # Linear growing mode of a matter + Lambda universe (Heath 1977):
    # D(a) proportional to E(a) int_0^a da' / (a' E(a'))^3, E = H/H0.  It is
    # the growing solution of the linear growth equation, computed here by
    # quadrature, independently of the closed form used by the oracle.
    def e_of(x):
        return math.sqrt(omega_m / x ** 3 + 1.0 - omega_m)

    val = integrate.quad(lambda x: 1.0 / (x * e_of(x)) ** 3, 0.0, a, epsabs=0, epsrel=1e-13, limit=200)[0]
    return e_of(a) * val


@pytest.mark.parametrize("z", [0.0, 1.0, 9.0, 100.0])
def test_growth_is_the_matter_dominated_growing_mode(z):
    # Einstein-de Sitter (Omega_m = 1): the growing mode normalised to D(0) = 1
    # is the scale factor; a wrong power of (1 + z) fails at z = 1 already
    want = _growth_integral(1.0 / (1.0 + z)) / _growth_integral(1.0)
    assert abs(cosmology.growth(z) / want - 1.0) < 1e-10


@pytest.mark.parametrize("z", [0.0, 1.0, 100.0])
def test_sigma8_of_the_spectrum_at_z_init(z):
    # sigma_8 of P(k, z) itself: the z = 0 value 0.8 scaled by the growing
    # mode (a, from the quadrature above), so P carries D^2 and not D
    c = cosmology.Cosmology(z_init=z)
    s = math.sqrt(cosmology.sigma_r_squared(lambda k: cosmology.power(k, c)))
    d = _growth_integral(1.0 / (1.0 + z)) / _growth_integral(1.0)
    assert abs(s / (0.8 * d) - 1.0) < 1e-10
