"""Pins for the oracle's zoom levels."""
import numpy as np
import pytest

from oracle import cosmology, noise, pipeline, refine, zoom
from tests import inputs

COSMO = cosmology.Cosmology()


def test_whole_box_level_is_the_full_box_resolution_increase():
    # a level whose sub-box is the whole parent box is Eq. 4-5 on the full box
    n_p, box = 32, 80.0
    wp = noise.noise_grid(n_p, 3)
    wc = refine.refine(wp, "4", seed=3, stream=1)
    psi_p = np.stack(pipeline.displacement_fields(wp, n_p, box, COSMO))
    psi = zoom.level_displacements(wc, 2 * n_p, box, psi_p, n_p, box, (0, 0, 0), COSMO)
    full = refine.combine(wp, wc, box, COSMO, 2 * box / n_p)
    assert np.abs(psi - full).max() < 1e-14 * np.abs(full).max()


def test_lowpass_of_displacements_is_the_windowed_path():
    # Eq. 5 applied to psi equals the filter with the large-scale window (psi is linear in W)
    n, box = 32, 90.0
    w = noise.noise_grid(n, 4)
    psi = np.stack(pipeline.displacement_fields(w, n, box, COSMO))
    r_s = 2 * box / n
    a = np.stack([zoom.lowpass(psi[j], n, box, r_s) for j in range(3)])
    b = refine.windowed_displacements(w, n, box, COSMO, r_s, "large", deconvolve=True)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_cic_at_origin_is_shifted_upsampling():
    n = 12
    f = inputs.real_field(n, 5)
    o = (3, 7, 10)
    shifted = np.roll(f, shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2))
    want = refine.cic_upsample(shifted, 2)[:10, :10, :10]
    assert np.abs(zoom.cic_at(f, o, 2, 10) - want).max() < 1e-15
    assert np.array_equal(zoom.periodic_slice(f, o, 5), shifted[:5, :5, :5])


def test_particles_at_an_origin():
    n, cell, box0 = 8, 0.5, 10.0
    psi = np.zeros((3, n, n, n))
    pos, vel = zoom.particles(psi, n, cell, (9.0, 0.0, 2.0), box0, COSMO)
    # q = origin + (m + 1/2) cell, wrapped into [0, L_0)
    assert pos[0, 0, 0, 0] == np.float32(9.25) and pos[0, 3, 0, 0] == np.float32(0.75)
    assert pos[2, 0, 0, 7] == np.float32(5.75)
    assert np.all(vel == 0)


def test_nested_origins_stay_in_the_inner_half():
    sizes = [192, 160, 96]
    origins = zoom.nested_origins(256, sizes, seed=42)
    parents = [256, 192, 160]
    for lev, (o, n, p) in enumerate(zip(origins, sizes, parents), start=1):
        assert all(0 <= v < p for v in o)
        if lev > 1:
            assert all(p // 4 <= v and v + n // 2 <= p - p // 4 for v in o)
    assert origins == zoom.nested_origins(256, sizes, seed=42)


def test_small_hierarchy_shapes_and_nesting():
    levels = zoom.hierarchy(32, 60.0, [32, 24], [(4, 20, 30), (8, 8, 10)], seed=7, cosmo=COSMO)
    assert [lv["n"] for lv in levels] == [32, 32, 24]
    assert levels[1]["cell"] == 60.0 / 64 and levels[2]["cell"] == 60.0 / 128
    assert levels[2]["origin_box"] == tuple(float(np.fmod(levels[1]["origin_box"][j] + o * levels[1]["cell"], 60.0))
                                            for j, o in enumerate((8, 8, 10)))
    for lv in levels:
        assert lv["pos"].min() >= 0 and lv["pos"].max() < 60.0
    # the level noise is the refinement of the parent's sub-box noise
    w1 = refine.refine(zoom.periodic_slice(levels[0]["w"], (4, 20, 30), 16), "4", 7, 1)
    assert np.array_equal(levels[1]["w"], w1)


def test_fig1_subbox_error_geometry():
    # Sec. 2.3, Fig. 1: a 32 Mpc/h sub-box of 128^3 cells inside a 64 Mpc/h
    # box (parent 128^3, r_s = 2 parent cells), against the full-box resolution
    # increase with the same refined noise.  The error of the sub-box's
    # periodic transforms concentrates at its faces; beyond a quarter of the
    # sub-box from them it is smaller.  Its size is reported in absolute and
    # relative units (the paper does not state the normalisation of its
    # 1e-3), not asserted.
    from tests.gpu_util import report
    box0, n_p, n_sub = 64.0, 128, 128
    wp = noise.noise_grid(n_p, 42, 0)
    o = (32, 32, 32)  # parent cells: the sub-box spans parent cells 32..95
    wc = refine.refine(wp, "4", seed=42, stream=1)
    r_s = 2 * box0 / n_p
    full = refine.combine(wp, wc, box0, COSMO, r_s, workers=8)
    psi_p = np.stack(pipeline.displacement_fields(wp, n_p, box0, COSMO, workers=8))
    w_sub = zoom.periodic_slice(wc, [2 * v for v in o], n_sub)
    psi = zoom.level_displacements(w_sub, n_sub, box0 / 2, psi_p, n_p, box0, o, COSMO, workers=8)
    ref = np.stack([zoom.periodic_slice(full[j], [2 * v for v in o], n_sub) for j in range(3)])
    err = psi - ref
    q = n_sub // 4
    inner = err[:, q:-q, q:-q, q:-q].std()
    rms = np.sqrt((ref ** 2).mean())
    vf = cosmology.velocity_factor(COSMO)
    d = cosmology.growth(COSMO.z_init)
    report(f"Fig. 1 geometry (oracle): sub-box error std beyond 1/4 from the faces {inner:.2e} Mpc/h at z = "
           f"{COSMO.z_init:g} ({inner / d:.2e} Mpc/h scaled to z = 0, {inner * vf:.2f} km/s), {inner / rms:.3f} of rms "
           f"psi, {inner / box0:.1e} of the box; whole sub-box {err.std():.2e} Mpc/h")
    assert inner < 0.7 * err.std()
    assert inner < 0.2 * rms
