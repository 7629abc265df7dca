"""Pins for the oracle's white-noise refinement (App. A) and the Eq. 4-5
combination of two resolutions."""
import math

import numpy as np
import pytest

from oracle import cosmology, noise, pipeline, refine
from tests import inputs

COSMO = cosmology.Cosmology()


@pytest.mark.parametrize("variant", ["hr", "3", "4", "linear", "sine"])
def test_bases_are_orthonormal(variant):
    e = refine.E_BASIS[variant]
    assert np.abs(e @ e.T - np.eye(e.shape[0])).max() < 1e-15
    nl, _ = refine.patch_sizes(variant)
    f = refine.F_BASIS[nl]
    assert np.abs(f @ f.T - np.eye(nl)).max() < 1e-15


@pytest.mark.parametrize("variant", ["4", "linear", "sine"])
def test_low_basis_functions_match_parent_symmetry(variant):
    # E_0 constant, E_1 odd about the patch centre (no systematic shift)
    e = refine.E_BASIS[variant]
    assert np.allclose(e[0], e[0][0]) and np.allclose(e[1], -e[1][::-1])


def _patch_1d(v0, v1, rands, variant):
    """1D refinement of two parent cells through the 3D code: a patch whose
    values do not vary along axes 1 and 2 is the 1D patch times F_0 F_0."""
    nl, nh = refine.patch_sizes(variant)
    v = np.zeros((nl, nl, nl))
    f0 = refine.F_BASIS[nl][0]
    for m, val in enumerate([v0, v1][:nl]):
        v[m] = val * np.outer(f0, f0)  # coefficient a_i00 = 1D coefficient a_i
    new = np.zeros((nh, nh, nh))
    for j, r in enumerate(rands):
        new[nl + j, 0, 0] = r
    child = refine.expand_patches(v, new, variant)
    e0 = refine.E_BASIS[variant][0]
    return child[:, 0, 0] / (e0[0] * e0[0])


def test_hoffman_ribak_step():
    # Eq. A.4
    v, r = 0.7, -1.3
    got = _patch_1d(v, None, [r], "hr")
    assert np.allclose(got, [(v - r) / math.sqrt(2), (v + r) / math.sqrt(2)], rtol=0, atol=1e-15)


def test_three_cell_patch_formula():
    # Eq. A.15
    v0, v1, r = 0.31, -1.12, 0.57
    s6 = math.sqrt(6)
    want = [(v0 + v1 - r) / s6 - (v1 - v0) / 2, (v0 + v1 + 2 * r) / s6, (v0 + v1 - r) / s6 + (v1 - v0) / 2]
    assert np.allclose(_patch_1d(v0, v1, [r], "3"), want, rtol=0, atol=1e-15)


def test_four_cell_patch_formula():
    # Eq. A.16-A.19
    v0, v1, r1, r2 = -0.44, 1.9, 0.83, -0.26
    s7, s8, s2 = math.sqrt(7), math.sqrt(8), math.sqrt(2)
    d = v1 - v0
    want = [(v0 + v1) / s8 - s7 * d / (4 * s2) - r1 / 2 + r2 / 4,
            (v0 + v1) / s8 - d / (4 * s2) + r1 / 2 - s7 * r2 / 4,
            (v0 + v1) / s8 + d / (4 * s2) + r1 / 2 + s7 * r2 / 4,
            (v0 + v1) / s8 + s7 * d / (4 * s2) - r1 / 2 - r2 / 4]
    assert np.allclose(_patch_1d(v0, v1, [r1, r2], "4"), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("variant", ["hr", "3", "4", "linear", "sine"])
def test_tensor_product_and_parent_coefficients(variant):
    nl, nh = refine.patch_sizes(variant)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((5, nl, nl, nl))
    new = rng.standard_normal((5, nh, nh, nh))
    child = refine.expand_patches(v, new, variant)
    e = refine.E_BASIS[variant]
    f = refine.F_BASIS[nl]
    # projecting the child patch on E_i E_j E_k gives back every coefficient
    a = np.einsum("pmnl,im,jn,kl->pijk", child, e, e, e)
    low = np.einsum("pmnl,im,jn,kl->pijk", v, f, f, f)
    assert np.abs(a[:, :nl, :nl, :nl] - low).max() < 1e-14
    mask = np.ones((nh, nh, nh), bool)
    mask[:nl, :nl, :nl] = False
    assert np.abs(a[:, mask] - new[:, mask]).max() < 1e-14
    # an explicit triple sum over the 3D basis functions (Eq. A.28)
    full = new.copy()
    full[:, :nl, :nl, :nl] = low
    one = sum(full[0, i, j, k] * np.einsum("m,n,l->mnl", e[i], e[j], e[k])
              for i in range(nh) for j in range(nh) for k in range(nh))
    assert np.abs(one - child[0]).max() < 1e-14


@pytest.mark.parametrize("variant", ["hr", "4", "3"])
def test_refined_noise_is_white(variant):
    nl, nh = refine.patch_sizes(variant)
    parent = noise.noise_grid(32, 5)
    child = refine.refine(parent, variant, seed=11, stream=1)
    assert child.shape == (32 // nl * nh,) * 3
    x = child.ravel()
    m = x.size
    assert abs(x.mean()) < 5 / math.sqrt(m)
    assert abs(x.var() - 1) < 5 * math.sqrt(2 / m)
    for lag in (1, 2, 3, nh, nh * 32 // nl):
        assert abs(np.corrcoef(x[:-lag], x[lag:])[0, 1]) < 5 / math.sqrt(m)


def test_refined_noise_uses_philox_coefficients():
    parent = noise.noise_grid(4, 1)
    child = refine.refine(parent, "4", seed=99, stream=7)
    # patch (0, 0, 1): coefficient (2, 3, 0) is noise value (patch 1) * 64 + 2*16 + 3*4 + 0
    e = refine.E_BASIS["4"]
    blk = child[0:4, 0:4, 4:8]
    a = np.einsum("mnl,im,jn,kl->ijk", blk, e, e, e)
    assert abs(a[2, 3, 0] - noise.noise_cells([64 + 44], 99, 7)[0]) < 1e-14


def test_cic_upsample_exact_cases():
    n = 8
    const = np.full((n, n, n), 1.75)
    assert np.abs(refine.cic_upsample(const, 2) - 1.75).max() < 1e-15
    ramp = np.tile(np.arange(n, dtype=np.float64).reshape(n, 1, 1), (1, n, n))
    up = refine.cic_upsample(ramp, 2)
    # linear inside the period (the last interval wraps from n-1 to 0)
    assert np.abs(up[: 2 * n - 1, 3, 5] - np.arange(2 * n - 1) / 2).max() < 1e-15
    assert abs(up[2 * n - 1, 0, 0] - (n - 1) / 2) < 1e-15
    # even child points are the parent samples
    f = inputs.real_field(n, 2)
    assert np.abs(refine.cic_upsample(f, 2)[::2, ::2, ::2] - f).max() < 1e-15


def test_windows_partition_the_modes():
    n, box, r_s = 32, 100.0, 2 * 100.0 / 16
    big = refine.mode_window(n, box, r_s, "large")
    small = refine.mode_window(n, box, r_s, "small")
    assert np.array_equal(big + small, np.ones_like(big))
    # the cutoff: k r_s < 1 with r_s two parent cells, |n| < N_p / (4 pi)
    s = pipeline.signed_index(n)
    n2 = (s.reshape(n, 1, 1) ** 2 + s.reshape(1, n, 1) ** 2 + np.arange(n // 2 + 1).reshape(1, 1, -1) ** 2)
    assert np.array_equal(big > 0, n2 < (16 / (4 * math.pi)) ** 2)


def test_large_plus_small_is_the_full_field_on_one_grid():
    n, box = 32, 150.0
    w = noise.noise_grid(n, 8)
    r_s = 2 * box / 16
    full = np.stack(pipeline.displacement_fields(w, n, box, COSMO))
    parts = (refine.windowed_displacements(w, n, box, COSMO, r_s, "small") +
             refine.windowed_displacements(w, n, box, COSMO, r_s, "large"))
    assert np.abs(parts - full).max() < 1e-14 * np.abs(full).max()


def test_combine_without_large_scales_is_the_child_field():
    n_p, n_c, box = 16, 32, 120.0
    wp = noise.noise_grid(n_p, 1)
    wc = noise.noise_grid(n_c, 2)
    r_s = box  # k r_s >= 2 pi for every mode but k = 0: no large-scale part
    psi = refine.combine(wp, wc, box, COSMO, r_s)
    full = np.stack(pipeline.displacement_fields(wc, n_c, box, COSMO))
    assert np.abs(psi - full).max() < 1e-14 * np.abs(full).max()


def test_combine_keeps_parent_large_scales():
    # child noise refined from the parent: the combined field's low modes follow
    # the parent's (CiC plus deconvolution reproduces them to a few percent)
    n_p, box = 32, 200.0
    wp = noise.noise_grid(n_p, 4)
    wc = refine.refine(wp, "4", seed=5, stream=1)
    r_s = 2 * box / n_p
    psi = refine.combine(wp, wc, box, COSMO, r_s)
    large_p = refine.windowed_displacements(wp, n_p, box, COSMO, r_s, "large")
    lowc = pipeline.forward(psi[0])[: 3, : 3, : 3] / (2 * n_p) ** 3
    lowp = pipeline.forward(large_p[0])[: 3, : 3, : 3] / n_p ** 3
    sel = np.abs(lowp) > 1e-6 * np.abs(lowp).max()  # modes with k_0 = 0 vanish in psi_0
    rel = np.abs(lowc[sel] - lowp[sel]) / np.abs(lowp[sel])
    assert sel.sum() >= 8 and rel.max() < 0.01


def test_cic_resample_reproduces_cell_linear_fields():
    # trilinear interpolation is exact for a field linear in each source index
    # inside the cells it interpolates (away from the periodic wrap)
    n, n_out = 8, 12
    m = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    f = 1.5 * m[0] - 0.25 * m[1] + 2.0 * m[2] + 0.75
    out = refine.cic_resample(f, n_out)
    u = np.arange(n_out) * n / n_out
    uu = np.meshgrid(u, u, u, indexing="ij")
    want = 1.5 * uu[0] - 0.25 * uu[1] + 2.0 * uu[2] + 0.75
    inner = u <= n - 1
    sel = np.ix_(inner, inner, inner)
    assert np.abs(out[sel] - want[sel]).max() < 1e-13


def test_cic_resample_hits_source_points_and_matches_integer_upsampling():
    f = inputs.real_field(8, 13)
    out = refine.cic_resample(f, 12)
    # output points 0, 3, 6, 9 sit on source points 0, 2, 4, 6 (u = 2m/3)
    assert np.array_equal(out[::3, ::3, ::3], f[::2, ::2, ::2])
    a = refine.cic_resample(f, 16)
    b = refine.cic_upsample(f, 2)
    assert np.abs(a - b).max() <= 2 * np.spacing(np.abs(b).max())


def test_three_halves_combine_whole_box_limit():
    # the 3/2 resolution increase: with r_s so small that Eq. 4 keeps nothing
    # below the child Nyquist the result is the CiC-resampled parent field
    n_p = 16
    box = 40.0
    wp = noise.noise_grid(n_p, 2)
    wc = refine.refine(wp, "3", seed=4, stream=1)
    assert wc.shape == (24, 24, 24)
    r_s = box  # k r_s < 1 keeps only k = 0 in the large part, Eq. 4 keeps everything else
    psi = refine.combine(wp, wc, box, COSMO, r_s)
    full = np.stack(pipeline.displacement_fields(wc, 24, box, COSMO))
    assert np.abs(psi - full).max() < 1e-13 * np.abs(full).max()


def _shape_basis(e1_shape):
    # four-cell basis from its defining shapes (App. A): E_0 constant; E_1 the
    # given shape, odd about the patch centre and increasing like F_1; E_2 the
    # even function orthogonal to E_0; E_3 the odd function orthogonal to E_1
    # (E_2 and E_3 follow from Eq. A.1), signs as printed (E_2(0) < 0 < E_3(0))
    k = np.arange(4) - 1.5
    e0 = np.full(4, 0.5)
    e1 = np.asarray(e1_shape, dtype=np.float64)
    e1 = e1 / np.linalg.norm(e1) * np.sign(e1 @ k)
    e2 = np.array([-1.0, 1.0, 1.0, -1.0]) / 2.0  # even: [a, b, b, a], 2a + 2b = 0
    c, d = e1[0], e1[1]  # odd [c', d', -d', -c'] orthogonal to [c, d, -d, -c]
    e3 = np.array([d, -c, c, -d])
    e3 = e3 / np.linalg.norm(e3) * np.sign(d)
    return np.stack([e0, e1, e2, e3])


def test_linear_basis_from_its_shape():
    # Eq. A.20-A.23: E'_1 varies linearly with the child cell index
    want = _shape_basis(np.arange(4) - 1.5)
    assert np.abs(refine.E_BASIS["linear"] - want).max() < 1e-15


def test_sine_basis_from_its_shape():
    # Eq. A.24-A.27: E''_1 is a sine of period one patch sampled at the four
    # cell centres (k + 1/2)/4 of the patch, with the sign that makes it rise
    x = (np.arange(4) + 0.5) / 4.0
    want = _shape_basis(-np.sin(2.0 * math.pi * x))
    assert np.abs(refine.E_BASIS["sine"] - want).max() < 1e-15


def _fig_a6_curve(variant, n_low):
    # Expected |D(n)|^2 of the difference D = DFT_H(n) / sqrt(r) - DFT_L(n)
    # between a 1D white noise of n_low cells and its refinement (r = N_H/N_L
    # times more cells), for the low-resolution modes 0 < n < n_low/2.  Both
    # DFTs are plain (unnormalised, each lattice indexed from its cell 0).  D
    # is linear in the parent values and the new coefficients, all i.i.d.
    # unit Gaussians, and patches are independent, so E|D|^2 is the patch
    # count times the sum of |coefficient|^2 of one patch's sources.
    nl, nh = refine.patch_sizes(variant)
    e, f = refine.E_BASIS[variant], refine.F_BASIS[nl]
    n = np.arange(1, n_low // 2)
    ph_l = np.exp(-2j * math.pi * np.outer(n, np.arange(nl)) / n_low)
    ph_h = np.exp(-2j * math.pi * np.outer(n, np.arange(nh)) / (n_low * nh // nl)) / math.sqrt(nh / nl)
    total = np.zeros(n.size)
    for m in range(nl):  # parent value V_m enters the child through a_i = sum_m V_m F_i(m)
        total += np.abs(ph_h @ (f[:, m] @ e[:nl]) - ph_l[:, m]) ** 2
    for j in range(nl, nh):  # new coefficient j
        total += np.abs(ph_h @ e[j]) ** 2
    return n, total * (n_low // nl)


def test_fig_a6_relations():
    # App. A, Fig. A.6 (1D noise of 1024 cells refined by a factor 2; the paper
    # averages 10^6 realisations, the expectation is taken exactly here).  The
    # mean amplitude of a circular complex Gaussian is sqrt(pi)/2 times its
    # r.m.s., so ratios of the curves are ratios of sqrt(E|D|^2).  Printed
    # relations: HR and the sine variant identical; A.10-A.13 0.3 % below the
    # linear variant on average and 0.7 % below at k/k_Ny > 0.5; HR and sine
    # 16 % above the other two on average.
    n_low = 1024
    n, lin = _fig_a6_curve("linear", n_low)
    amp = {v: np.sqrt(_fig_a6_curve(v, n_low)[1]) for v in ("hr", "4", "linear", "sine")}
    assert np.abs(amp["hr"] / amp["sine"] - 1.0).max() < 1e-12
    r = amp["4"] / amp["linear"]
    assert 0.0025 < 1.0 - r.mean() < 0.0035
    assert 0.0065 < 1.0 - r[n / (n_low // 2) > 0.5].mean() < 0.0075
    for other in ("4", "linear"):
        assert 0.15 < (amp["hr"] / amp[other]).mean() - 1.0 < 0.17


@pytest.mark.parametrize("variant", ["hr", "4", "sine"])
def test_fig_a6_expectation_matches_realisations(variant):
    # the exact expectation above against realisations refined by the
    # oracle's patch code (1D patches embedded as F_0 F_0 along axes 1, 2)
    n_low, reps = 256, 256
    nl, nh = refine.patch_sizes(variant)
    rng = np.random.default_rng(61)
    lowres = rng.standard_normal((reps, n_low))
    p = n_low // nl
    f0 = refine.F_BASIS[nl][0]
    v = np.einsum("pm,n,l->pmnl", lowres.reshape(reps * p, nl), f0, f0)
    new = np.zeros((reps * p, nh, nh, nh))
    new[:, nl:, 0, 0] = rng.standard_normal((reps * p, nh - nl))
    e0 = refine.E_BASIS[variant][0]
    child = (refine.expand_patches(v, new, variant)[:, :, 0, 0] / (e0[0] * e0[0])).reshape(reps, p * nh)
    d = np.fft.fft(child, axis=1)[:, 1:n_low // 2] / math.sqrt(nh / nl) - np.fft.fft(lowres, axis=1)[:, 1:n_low // 2]
    got = (np.abs(d) ** 2).mean(axis=0)
    _, want = _fig_a6_curve(variant, n_low)
    # bands of 16 modes (n = 1 .. 112): relative standard error 1/sqrt(reps * 16)
    gb, wb = got[:112].reshape(-1, 16).mean(axis=1), want[:112].reshape(-1, 16).mean(axis=1)
    assert np.abs(gb / wb - 1.0).max() < 5.0 / math.sqrt(reps * 16)
