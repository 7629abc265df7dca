"""Pins for the oracle's white noise: elementary functions against the
platform's extended-precision libm, Box-Muller against the normal law, and the
cell-to-counter mapping (one Philox call per cell, cosine branch)."""
import numpy as np
import pytest
from scipy import stats

from oracle import noise, normal, philox

LD_TWO_PI = np.longdouble("6.283185307179586476925286766559005768")


def test_log_unit_matches_extended_libm():
    rng = np.random.default_rng(3)
    words = rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64)
    words[:4] = [0, 1, (1 << 32) - 1, 1 << 31]
    u = (words + np.uint64(1)).astype(np.float64) * 2.0 ** -32
    want = np.log(u.astype(np.longdouble))
    got = normal.log_unit(u)
    rel = np.abs((got.astype(np.longdouble) - want) / np.where(want == 0, 1, np.abs(want)))
    assert float(rel.max()) < 4e-16
    assert normal.log_unit(np.array([1.0]))[0] == 0.0


def test_cos_sin_match_extended_libm():
    rng = np.random.default_rng(4)
    w = rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64)
    # quadrant and octant edges
    edges = np.array([0, 1, (1 << 29) - 1, 1 << 29, (1 << 29) + 1, (1 << 30) - 1, 1 << 30,
                      3 << 29, (1 << 31) + 5, (1 << 32) - 1], dtype=np.uint64)
    w = np.concatenate([edges, w])
    c, s = normal.cos_sin_turn(w)
    theta = (w.astype(np.longdouble) * np.longdouble(2.0) ** -32) * LD_TWO_PI
    assert float(np.abs(c - np.cos(theta)).max()) < 6e-16
    assert float(np.abs(s - np.sin(theta)).max()) < 6e-16


def test_reflected_branch_meets_direct_branch():
    # rho = 2^29 is handled by the reflected branch, 2^29 - 1 by the direct one
    c, s = normal.cos_sin_turn(np.array([(1 << 29) - 1, 1 << 29], dtype=np.uint64))
    assert abs(c[0] - c[1]) < 1e-8 and abs(s[0] - s[1]) < 1e-8
    assert abs(c[1] - np.sqrt(0.5)) < 1e-15 and abs(s[1] - np.sqrt(0.5)) < 1e-15


def test_box_muller_matches_libm_formula():
    rng = np.random.default_rng(5)
    wa = rng.integers(0, 1 << 32, 1 << 18, dtype=np.uint64)
    wb = rng.integers(0, 1 << 32, 1 << 18, dtype=np.uint64)
    ga, gb = normal.box_muller(wa, wb)
    u1 = (wa + np.uint64(1)).astype(np.longdouble) * np.longdouble(2.0) ** -32
    th = wb.astype(np.longdouble) * np.longdouble(2.0) ** -32 * LD_TWO_PI
    r = np.sqrt(-2 * np.log(u1))
    assert float(np.abs(ga - r * np.cos(th)).max()) < 1e-14
    assert float(np.abs(gb - r * np.sin(th)).max()) < 1e-14


def test_noise_is_unit_gaussian():
    n = 64
    w = noise.noise_grid(n, 42).ravel()
    m = w.size
    assert abs(w.mean()) < 5 / np.sqrt(m)
    assert abs(w.var() - 1.0) < 5 * np.sqrt(2.0 / m)
    assert abs(stats.kurtosis(w, fisher=False) - 3.0) < 5 * np.sqrt(24.0 / m)
    assert stats.kstest(w, "norm").pvalue > 1e-3
    # even and odd cells (low counter bit) are each N(0, 1)
    for lane in range(2):
        assert stats.kstest(w[lane::2], "norm").pvalue > 1e-4


def test_neighbouring_cells_uncorrelated():
    w = noise.noise_grid(64, 7).ravel()
    for lag in (1, 2, 3, 4, 64):
        r = np.corrcoef(w[:-lag], w[lag:])[0, 1]
        assert abs(r) < 5 / np.sqrt(w.size)


def test_cell_mapping():
    # the noise of cell c only depends on (seed, stream, c): one Philox call
    # with counter (c lo, c hi, stream, 0), words w0 and w1, cosine branch
    seed = 123456789012345
    cells = np.array([0, 1, 2, 3, 4, 1 << 33, (1 << 33) + 3, (1 << 30) - 1], dtype=np.uint64)
    got = noise.noise_cells(cells, seed, stream=2)
    for c, g in zip(cells, got):
        c = int(c)
        w = [int(np.asarray(x).reshape(-1)[0]) for x in philox.philox4x32(
            (c & 0xFFFFFFFF, c >> 32, 2, 0), philox.seed_key(seed))]
        ga, _ = normal.box_muller(np.uint64(w[0]), np.uint64(w[1]))
        assert g == float(ga)
        # the deviate is r cos(theta) of the two words (extended precision)
        u1 = np.longdouble(w[0] + 1) * np.longdouble(2.0) ** -32
        th = np.longdouble(w[1]) * np.longdouble(2.0) ** -32 * LD_TWO_PI
        assert abs(g - float(np.sqrt(-2 * np.log(u1)) * np.cos(th))) < 1e-14


def test_gaussian_is_cosine_branch():
    rng = np.random.default_rng(8)
    wa = rng.integers(0, 1 << 32, 4096, dtype=np.uint64)
    wb = rng.integers(0, 1 << 32, 4096, dtype=np.uint64)
    ga, gb = normal.box_muller(wa, wb)
    assert np.array_equal(normal.gaussian(wa, wb), ga)
    # the sine branch is a different deviate: a mix-up of the branches would show
    assert not np.allclose(ga, gb)


def test_grid_chunking_and_precision():
    a = noise.noise_grid(16, 9, chunk=1000)
    b = noise.noise_grid(16, 9, chunk=1 << 20)
    assert np.array_equal(a, b)
    assert np.array_equal(noise.noise_grid(16, 9, chunk=700, workers=4), a)
    f = noise.noise_grid(16, 9, dtype=np.float32)
    assert f.dtype == np.float32
    # the float32 field is the binary64 field rounded once
    assert np.array_equal(f, a.astype(np.float32))
    assert not np.array_equal(noise.noise_grid(16, 9, stream=1), a)
    assert not np.array_equal(noise.noise_grid(16, 10), a)


@pytest.mark.parametrize("bad", [-1, 1 << 64])
def test_seed_range(bad):
    with pytest.raises(ValueError):
        philox.seed_key(bad)
