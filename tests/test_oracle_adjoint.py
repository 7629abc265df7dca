"""Pins for the oracle's gradients of the noise -> displacement map.

The forward map used as ground truth is oracle.pipeline (half-spectrum
transforms, itself pinned by direct DFTs); oracle.adjoint takes the
correlation route with full complex transforms.  A dropped conjugate, a wrong
sign, a swapped component or a missing volume factor in the adjoint fails
the explicit-matrix test; the chain through Eq. (3) and the log-amplitude
derivative are pinned by finite differences and by the closed form
dl/dlog A = l of a loss quadratic in psi.
"""
import numpy as np
import pytest

from oracle import adjoint, cosmology, pipeline
from tests import inputs

COSMO = cosmology.Cosmology()


def _matrix(n, box, j):
    """Columns L_j e_c for every cell c, from the half-spectrum pipeline."""
    cols = np.empty((n ** 3, n ** 3))
    e = np.zeros(n ** 3)
    for c in range(n ** 3):
        e[c] = 1.0
        cols[:, c] = pipeline.displacement_fields(e.reshape(n, n, n), n, box, COSMO, components=(j,))[0].reshape(-1)
        e[c] = 0.0
    return cols


@pytest.fixture(scope="module")
def matrices_8():
    return [_matrix(8, 50.0, j) for j in range(3)]


def test_forward_routes_agree():
    n, box = 16, 80.0
    w = inputs.real_field(n, 11)
    half = pipeline.displacement_fields(w, n, box, COSMO)
    for j in range(3):
        full = adjoint.apply_forward(w, n, box, COSMO, j)
        assert np.abs(full - half[j]).max() < 1e-13 * np.abs(half[j]).max()


def test_gradient_is_explicit_transpose(matrices_8):
    n, box = 8, 50.0
    g = np.stack([inputs.real_field(n, 20 + j) for j in range(3)])
    want = sum(matrices_8[j].T @ g[j].reshape(-1) for j in range(3))
    got = adjoint.noise_gradient(g, n, box, COSMO).reshape(-1)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_kernel_is_odd(matrices_8):
    # L_j^T = -L_j: each displacement operator is antisymmetric
    for m in matrices_8:
        assert np.abs(m + m.T).max() < 1e-13 * np.abs(m).max()
        assert np.abs(m).max() > 0


def test_single_component_gradient_is_minus_forward():
    n, box = 16, 100.0
    g = inputs.real_field(n, 5)
    for j in range(3):
        gj = np.zeros((3, n, n, n))
        gj[j] = g
        got = adjoint.noise_gradient(gj, n, box, COSMO)
        want = -pipeline.displacement_fields(g, n, box, COSMO, components=(j,))[0]
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_dot_product_identity():
    n, box = 32, 200.0
    w = inputs.real_field(n, 7)
    g = np.stack([inputs.real_field(n, 30 + j) for j in range(3)])
    psi = np.stack(pipeline.displacement_fields(w, n, box, COSMO))
    lhs = float(np.sum(psi * g))
    rhs = float(np.sum(w * adjoint.noise_gradient(g, n, box, COSMO)))
    assert abs(lhs - rhs) < 1e-12 * np.sqrt(np.sum(psi * psi) * np.sum(g * g))


def test_amp_scale_multiplies_gradient():
    n, box = 16, 100.0
    g = np.stack([inputs.real_field(n, 40 + j) for j in range(3)])
    a = adjoint.noise_gradient(g, n, box, COSMO)
    b = adjoint.noise_gradient(g, n, box, COSMO, amp_scale=1.75)
    assert np.abs(b - 1.75 * a).max() < 1e-14 * np.abs(a).max()


def _loss_of_noise(w, n, box, cells, weights, amp=None):
    psi = np.stack(pipeline.displacement_fields(w, n, box, COSMO, amp=amp))
    return adjoint.weighted_loss(psi, cells, weights), psi


def test_finite_differences_of_weighted_loss():
    # l = sum_i w_i |psi(c_i)|^2 is quadratic in W, so the central difference
    # is exact apart from rounding
    n, box = 16, 100.0
    w = inputs.real_field(n, 9)
    cells = inputs.cell_sample(n, 300, 42)
    weights = np.random.default_rng(42).uniform(0.0, 1.0, cells.size)
    loss, psi = _loss_of_noise(w, n, box, cells, weights)
    grad = adjoint.noise_gradient(adjoint.weighted_loss_grad(psi, cells, weights), n, box, COSMO)
    eps = 1e-3
    probe = inputs.cell_sample(n, 24, 43)
    for c in probe:
        wp = w.copy().reshape(-1)
        wm = w.copy().reshape(-1)
        wp[c] += eps
        wm[c] -= eps
        fd = (_loss_of_noise(wp.reshape(w.shape), n, box, cells, weights)[0] -
              _loss_of_noise(wm.reshape(w.shape), n, box, cells, weights)[0]) / (2 * eps)
        assert abs(fd - grad.reshape(-1)[c]) < 1e-8 * np.abs(grad).max()
    assert loss > 0


def test_weighted_loss_grad_by_finite_differences():
    n = 8
    psi = np.stack([inputs.real_field(n, 50 + j) for j in range(3)])
    cells = inputs.cell_sample(n, 40, 3)
    weights = np.random.default_rng(4).uniform(0.0, 1.0, cells.size)
    g = adjoint.weighted_loss_grad(psi, cells, weights)
    eps = 1e-4
    for j, c in [(0, cells[0]), (1, cells[7]), (2, cells[-1]), (1, 0 if 0 not in cells else 1)]:
        p = psi.copy().reshape(3, -1)
        p[j, c] += eps
        up = adjoint.weighted_loss(p, cells, weights)
        p[j, c] -= 2 * eps
        dn = adjoint.weighted_loss(p, cells, weights)
        assert abs((up - dn) / (2 * eps) - g.reshape(3, -1)[j, c]) < 1e-8


def test_log_amp_gradient_equals_quadratic_loss():
    n, box = 16, 100.0
    w = inputs.real_field(n, 12)
    cells = inputs.cell_sample(n, 200, 1)
    weights = np.random.default_rng(2).uniform(0.0, 1.0, cells.size)
    amp = cosmology.amplitude(COSMO)
    loss, psi = _loss_of_noise(w, n, box, cells, weights, amp=amp)
    g = adjoint.weighted_loss_grad(psi, cells, weights)
    closed = adjoint.log_amp_gradient(g, psi)
    assert abs(closed - loss) < 1e-13 * loss
    # and by a finite difference in log A, through the spectrum itself
    h = 1e-4
    up = _loss_of_noise(w, n, box, cells, weights, amp=amp * np.exp(h))[0]
    dn = _loss_of_noise(w, n, box, cells, weights, amp=amp * np.exp(-h))[0]
    assert abs((up - dn) / (2 * h) - closed) < 1e-7 * loss


def test_chain_through_particles():
    # x = q + psi has slope 1 and v = aHf psi: a loss on (x, v) evaluated in
    # float64 before the float32 rounding differentiates like one on psi
    n, box = 16, 100.0
    w = inputs.real_field(n, 13)
    vfac = cosmology.velocity_factor(COSMO)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((3, n, n, n))
    b = rng.standard_normal((3, n, n, n))

    def loss(wf):
        psi = np.stack(pipeline.displacement_fields(wf, n, box, COSMO))
        x = np.stack([pipeline.lattice(n, box, 0.5, j) + psi[j] for j in range(3)])
        return float(np.sum(a * x) + 0.5 * np.sum(b * (vfac * psi) ** 2)), psi

    _, psi = loss(w)
    g = adjoint.combine(g_pos=a, g_vel=b * vfac * psi, cosmo=COSMO)
    grad = adjoint.noise_gradient(g, n, box, COSMO)
    eps = 1e-3
    for c in inputs.cell_sample(n, 8, 6):
        wp = w.copy().reshape(-1)
        wm = w.copy().reshape(-1)
        wp[c] += eps
        wm[c] -= eps
        fd = (loss(wp.reshape(w.shape))[0] - loss(wm.reshape(w.shape))[0]) / (2 * eps)
        assert abs(fd - grad.reshape(-1)[c]) < 1e-6 * np.abs(grad).max()


def test_combine_requires_a_gradient():
    with pytest.raises(ValueError):
        adjoint.combine()
