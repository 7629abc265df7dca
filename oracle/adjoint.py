"""Gradients of the noise -> particles map, in float64 (test infrastructure).

The path of Sec. 2.1 (Eq. 1-2) and Sec. 2.2 (Eq. 3) is linear in the white
noise W: psi_j = L_j W, where L_j multiplies the spectrum of W by

    H_j(k) = i k_j / k^2 sqrt(P(k) N^3 / L^3)   (zero at k = 0 and on any
                                                  axis Nyquist plane),

positions are x_j = q_j + psi_j (a periodic wrap, slope 1 almost everywhere)
and velocities v_j = a H f psi_j.  For a loss l(psi, x, v) the gradient with
respect to W is therefore

    dl/dW = sum_j L_j^T g_j,    g_j = dl/dpsi_j + dl/dx_j + a H f dl/dv_j.

L_j is a circular convolution with the real kernel h_j whose transform is
H_j, so its transpose is the circular correlation with h_j, whose transform
is conj(H_j) (the correlation theorem).  This module writes that out with
full complex transforms: it shares no step with the half-spectrum route of
oracle.pipeline, which the pins use as the independent forward map.

The amplitude A of P(k) enters psi as sqrt(A), so dl/dlog A = (1/2) sum g psi
with g as above.  With amp_scale s multiplying psi (A -> s^2 A), dl/dW gains
the factor s.

Pins (tests/test_oracle_adjoint.py): the explicit 512 x 512 matrix of each
L_j, built column by column from oracle.pipeline at 8^3, transposed; the
dot-product identity <L W, g> = <W, L^T g>; oddness of the kernel
(L_j^T = -L_j); central finite differences of a quadratic loss (exact up to
rounding); dl/dlog A = l for a loss quadratic in psi.
"""
import math

import numpy as np

from . import cosmology
from .pipeline import signed_index


def transfer(n, box, cosmo, j, amp=None):
    """H_j on the full (n, n, n) grid of modes, Eq. (1) times Eq. (2)."""
    s = signed_index(n).astype(np.float64)
    s0 = s.reshape(n, 1, 1)
    s1 = s.reshape(1, n, 1)
    s2 = s.reshape(1, 1, n)
    n2 = s0 * s0 + s1 * s1 + s2 * s2
    half = n // 2
    keep = (n2 > 0) & (np.abs(s0) != half) & (np.abs(s1) != half) & (np.abs(s2) != half)
    dk = 2.0 * math.pi / box
    k = dk * np.sqrt(np.where(keep, n2, 1.0))
    p = cosmology.power(k, cosmo, amp)
    sj = (s0, s1, s2)[j]
    ratio = np.where(keep, (dk * sj) / (k * k) * np.sqrt(p * n ** 3 / box ** 3), 0.0)
    return 1j * np.broadcast_to(ratio, (n, n, n))


def apply_forward(w, n, box, cosmo, j, amp_scale=1.0, amp=None):
    """psi_j = amp_scale L_j W by the full complex transform (a second route)."""
    wf = np.fft.fftn(np.asarray(w, dtype=np.float64))
    return amp_scale * np.fft.ifftn(transfer(n, box, cosmo, j, amp) * wf).real


def combine(g_psi=None, g_pos=None, g_vel=None, cosmo=None):
    """g_j = dl/dpsi_j + dl/dx_j + a H f dl/dv_j (Eq. 3 differentiated)."""
    g = None
    for part, factor in ((g_psi, 1.0), (g_pos, 1.0), (g_vel, None)):
        if part is None:
            continue
        if factor is None:
            factor = cosmology.velocity_factor(cosmo)
        term = factor * np.asarray(part, dtype=np.float64)
        g = term if g is None else g + term
    if g is None:
        raise ValueError("no gradient given")
    return g


def noise_gradient(g, n, box, cosmo, amp_scale=1.0, amp=None):
    """dl/dW = amp_scale sum_j L_j^T g_j, g of shape (3, n, n, n)."""
    out = np.zeros((n, n, n), dtype=np.complex128)
    for j in range(3):
        gj = np.fft.fftn(np.asarray(g[j], dtype=np.float64))
        out += np.conj(transfer(n, box, cosmo, j, amp)) * gj
    return amp_scale * np.fft.ifftn(out).real


def log_amp_gradient(g, psi):
    """dl/dlog A = (1/2) sum_j sum_c g_j[c] psi_j[c] (psi grows as sqrt(A))."""
    return 0.5 * float(np.sum(np.asarray(g, dtype=np.float64) * np.asarray(psi, dtype=np.float64)))


def weighted_loss(psi, cells, weights):
    """l = sum_i w_i |psi(c_i)|^2 over flat cell indices c_i."""
    p = np.asarray(psi, dtype=np.float64).reshape(3, -1)[:, cells]
    return float(np.sum(np.asarray(weights, dtype=np.float64) * np.sum(p * p, axis=0)))


def weighted_loss_grad(psi, cells, weights):
    """dl/dpsi of weighted_loss (cells distinct), shape of psi."""
    p = np.asarray(psi, dtype=np.float64).reshape(3, -1)
    g = np.zeros_like(p)
    g[:, cells] = 2.0 * np.asarray(weights, dtype=np.float64) * p[:, cells]
    return g.reshape(np.shape(psi))
