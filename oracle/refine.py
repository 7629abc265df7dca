"""White-noise refinement (App. A) and the combination of low- and high-
resolution velocity fields (Sec. 2.3, Eq. 4-5), in float64 (test
infrastructure).

Refinement.  A patch of N_L parent cells per axis is replaced by N_H child
cells per axis.  With orthonormal 1D bases F_i (N_L points) and E_j (N_H
points), the parent patch V has coefficients a_ijk = sum V(m,n,l) F_i(m)
F_j(n) F_k(l) for i, j, k < N_L; every other coefficient (any index >= N_L)
is a new unit Gaussian; the child patch is sum a_ijk E_i(m) E_j(n) E_k(l)
(the 3D basis is the tensor product, Eq. A.28).  Bases:
    'hr'      N_L = 1, N_H = 2: E = Eq. A.2-A.3 (the Hoffman-Ribak step, A.4)
    '3'       N_L = 2, N_H = 3: E = Eq. A.7-A.9
    '4'       N_L = 2, N_H = 4: E = Eq. A.10-A.13 (the code's default)
    'linear'  N_L = 2, N_H = 4: E = Eq. A.20-A.23
    'sine'    N_L = 2, N_H = 4: E = Eq. A.24-A.27
with F = Eq. A.5-A.6 for N_L = 2 and F_0 = [1] for N_L = 1.
New coefficients: the paper takes them from its generator; here the
coefficient (i, j, k) of patch p (row-major over the patch grid) is the white
noise value (oracle.noise) of index p N_H^3 + (i N_H + j) N_H + k in a given
(seed, stream): one Philox call per coefficient, like one cell of the noise.

Combination (Eq. 4-5, r_s the cutoff scale, f(x) = [x < 1]):
    small scales: psi~_h(k) (1 - f(k r_s)) on the child grid;
    large scales: psi~_l(k) f(k r_s) / W_CiC(k) on the parent grid, inverse
      transformed, then interpolated to the child lattice points by
      cloud-in-cell (trilinear, periodic); W_CiC(k) = prod_j sinc^2(pi s_j / N_p)
      is the transform of that interpolation kernel, divided out beforehand
      (the deconvolution the paper describes);
    psi = small + interpolated large.
Both grids cover the same periodic box here (a full-box resolution increase);
the paper's choice is r_s = 2 parent cells.

Pins (tests/test_oracle_refine.py): orthonormality of every basis (Eq. A.1);
the printed patch formulas A.4, A.15 and A.16-A.19 against the basis
expansion; the 3D tensor product; exact preservation of the parent
coefficients; unit-variance uncorrelated output; CiC interpolation exact for
constants and for linear ramps (inside a period); the split into f and 1 - f
is a partition of the modes; with r_s below one child cell the combination is
the child field alone.
"""
import math

import numpy as np

from . import pipeline
from .noise import noise_cells

S2 = math.sqrt(2.0)
S3 = math.sqrt(3.0)
S6 = math.sqrt(6.0)
S7 = math.sqrt(7.0)
S20 = math.sqrt(20.0)

F_BASIS = {
    1: np.array([[1.0]]),
    2: np.array([[1 / S2, 1 / S2], [-1 / S2, 1 / S2]]),
}

E_BASIS = {
    "hr": np.array([[1 / S2, 1 / S2], [-1 / S2, 1 / S2]]),
    "3": np.array([[1 / S3, 1 / S3, 1 / S3], [-1 / S2, 0.0, 1 / S2], [-1 / S6, 2 / S6, -1 / S6]]),
    "4": np.array([[0.5, 0.5, 0.5, 0.5], [-S7 / 4, -0.25, 0.25, S7 / 4], [-0.5, 0.5, 0.5, -0.5],
                   [0.25, -S7 / 4, S7 / 4, -0.25]]),
    "linear": np.array([[0.5, 0.5, 0.5, 0.5], [-3 / S20, -1 / S20, 1 / S20, 3 / S20], [-0.5, 0.5, 0.5, -0.5],
                        [1 / S20, -3 / S20, 3 / S20, -1 / S20]]),
    "sine": np.array([[0.5, 0.5, 0.5, 0.5], [-0.5, -0.5, 0.5, 0.5], [-0.5, 0.5, 0.5, -0.5], [0.5, -0.5, 0.5, -0.5]]),
}

N_LOW = {"hr": 1, "3": 2, "4": 2, "linear": 2, "sine": 2}


def patch_sizes(variant):
    """(N_L, N_H) of a refinement variant."""
    return N_LOW[variant], E_BASIS[variant].shape[0]


def expand_patches(v, new, variant):
    """Child patches from parent patches v (..., N_L, N_L, N_L) and the full
    coefficient arrays ``new`` (..., N_H, N_H, N_H) whose entries with an index
    >= N_L are used as the new coefficients."""
    nl, nh = patch_sizes(variant)
    f = F_BASIS[nl]
    e = E_BASIS[variant]
    a = np.array(new, dtype=np.float64, copy=True)
    low = np.einsum("...mnl,im,jn,kl->...ijk", np.asarray(v, dtype=np.float64), f, f, f)
    a[..., :nl, :nl, :nl] = low
    return np.einsum("...ijk,im,jn,kl->...mnl", a, e, e, e)


def refine(w_parent, variant, seed, stream):
    """The refined white noise: (P N_H)^3 cells from a parent of (P N_L)^3."""
    w = np.asarray(w_parent, dtype=np.float64)
    nl, nh = patch_sizes(variant)
    npar = w.shape[0]
    if npar % nl:
        raise ValueError("parent size must be a multiple of N_L")
    p = npar // nl
    v = w.reshape(p, nl, p, nl, p, nl).transpose(0, 2, 4, 1, 3, 5)
    idx = np.arange(p ** 3 * nh ** 3, dtype=np.uint64)
    new = noise_cells(idx, seed, stream).reshape(p, p, p, nh, nh, nh)
    child = expand_patches(v, new, variant)
    return child.transpose(0, 3, 1, 4, 2, 5).reshape(p * nh, p * nh, p * nh)


def mode_window(n, box, r_s, part):
    """f(k r_s) ('large') or 1 - f(k r_s) ('small') on the half spectrum."""
    s0 = pipeline.signed_index(n).reshape(n, 1, 1).astype(np.float64)
    s1 = pipeline.signed_index(n).reshape(1, n, 1).astype(np.float64)
    s2 = np.arange(n // 2 + 1).reshape(1, 1, n // 2 + 1).astype(np.float64)
    k = (2.0 * math.pi / box) * np.sqrt(s0 * s0 + s1 * s1 + s2 * s2)
    f = (k * r_s < 1.0).astype(np.float64)
    return f if part == "large" else 1.0 - f


def cic_window(n):
    """W_CiC = prod_j sinc^2(pi s_j / n) on the half spectrum."""
    def sinc2(s):
        x = math.pi * s.astype(np.float64) / n
        return np.where(x == 0.0, 1.0, (np.sin(x) / np.where(x == 0.0, 1.0, x)) ** 2)
    s = pipeline.signed_index(n)
    return (sinc2(s).reshape(n, 1, 1) * sinc2(s).reshape(1, n, 1) *
            sinc2(np.arange(n // 2 + 1)).reshape(1, 1, n // 2 + 1))


def windowed_displacements(w, n, box, cosmo, r_s, part, deconvolve=False, amp=None, workers=None):
    """psi_j (3, n, n, n) from noise w with the Eq. 4 ('small') or Eq. 5
    ('large') window, the large part optionally divided by W_CiC."""
    w_hat = pipeline.forward(np.asarray(w, dtype=np.float64), workers=workers)
    delta_hat = pipeline.density_spectrum(w_hat, n, box, cosmo, amp) * mode_window(n, box, r_s, part)
    if deconvolve:
        delta_hat = delta_hat / cic_window(n)
    return np.stack([pipeline.inverse(pipeline.displacement_spectrum(delta_hat, n, box, j), n, workers=workers)
                     for j in range(3)])


def cic_upsample(field, ratio):
    """Trilinear (cloud-in-cell) interpolation of a periodic field sampled at
    m dx to the points m' dx / ratio (ratio an integer)."""
    f = np.asarray(field, dtype=np.float64)
    n = f.shape[0]
    nc = n * ratio
    u = np.arange(nc) / ratio
    i0 = np.floor(u).astype(np.int64)
    t = u - i0
    i1 = (i0 + 1) % n
    out = f
    for axis in range(3):
        a = np.take(out, i0, axis=axis)
        b = np.take(out, i1, axis=axis)
        shape = [1, 1, 1]
        shape[axis] = nc
        tt = t.reshape(shape)
        out = a * (1.0 - tt) + b * tt
    return out


def cic_resample(field, n_out):
    """Trilinear (cloud-in-cell) interpolation of a periodic field of n^3
    points to the n_out^3 points of the same box (any n_out >= 1): point m
    sits at u = m n / n_out source cells, split exactly into the cell
    floor(m n / n_out) and the weight ((m n) mod n_out) / n_out; axis 0, then
    1, then 2."""
    f = np.asarray(field, dtype=np.float64)
    n = f.shape[0]
    mn = np.arange(n_out, dtype=np.int64) * n
    i0 = mn // n_out
    t = (mn % n_out) / float(n_out)
    i1 = (i0 + 1) % n
    out = f
    for axis in range(3):
        a = np.take(out, i0, axis=axis)
        b = np.take(out, i1, axis=axis)
        shape = [1, 1, 1]
        shape[axis] = n_out
        tt = t.reshape(shape)
        out = a * (1.0 - tt) + b * tt
    return out


def combine(w_parent, w_child, box, cosmo, r_s, workers=None):
    """Full-box resolution increase: psi on the child grid from the parent's
    large scales (Eq. 5, CiC with deconvolution) and the child's small scales
    (Eq. 4).  A child a whole multiple of the parent uses cic_upsample, any
    other size (the 3/2 patches of Eq. A.15) cic_resample."""
    n_p = np.asarray(w_parent).shape[0]
    n_c = np.asarray(w_child).shape[0]
    if n_c < n_p:
        raise ValueError("child lattice smaller than the parent")
    small = windowed_displacements(w_child, n_c, box, cosmo, r_s, "small", workers=workers)
    large = windowed_displacements(w_parent, n_p, box, cosmo, r_s, "large", deconvolve=True, workers=workers)
    if n_c % n_p == 0:
        return small + np.stack([cic_upsample(large[j], n_c // n_p) for j in range(3)])
    return small + np.stack([cic_resample(large[j], n_c) for j in range(3)])
