"""Pins for the oracle's white noise: elementary functions against the
platform's extended-precision libm, Box-Muller against the normal law, and the
cell-to-counter mapping."""
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
    # each of the four lanes of a Philox group is itself N(0, 1)
    for lane in range(4):
        assert stats.kstest(w[lane::4], "norm").pvalue > 1e-4


def test_neighbouring_cells_uncorrelated():
    w = noise.noise_grid(64, 7).ravel()
    for lag in (1, 2, 3, 4, 64):
        r = np.corrcoef(w[:-lag], w[lag:])[0, 1]
        assert abs(r) < 5 / np.sqrt(w.size)


def test_cell_mapping_and_lanes():
    # the noise of cell c only depends on (seed, stream, c): group c//4, lane c%4
    seed = 123456789012345
    cells = np.array([0, 1, 2, 3, 4, 1 << 33, (1 << 33) + 3], dtype=np.uint64)
    got = noise.noise_cells(cells, seed, stream=2)
    for c, g in zip(cells, got):
        grp = int(c) >> 2
        w = [int(np.asarray(x).reshape(-1)[0]) for x in philox.philox4x32(
            (grp & 0xFFFFFFFF, grp >> 32, 2, 0), philox.seed_key(seed))]
        pair = normal.box_muller(np.uint64(w[0]), np.uint64(w[1])) if int(c) % 4 < 2 else \
            normal.box_muller(np.uint64(w[2]), np.uint64(w[3]))
        assert g == float(pair[int(c) % 2])


def test_grid_chunking_and_precision():
    a = noise.noise_grid(16, 9, chunk=1000)
    b = noise.noise_grid(16, 9, chunk=1 << 20)
    assert np.array_equal(a, b)
    assert np.array_equal(noise.noise_grid(16, 9, chunk=700, workers=4), a)
    f = noise.noise_grid(16, 9, dtype=np.float32)
    assert f.dtype == np.float32
    # the float32 path's deviates are the same realisation to float32 accuracy
    assert np.all(np.abs(f.astype(np.float64) - a) <= 4e-7 * np.maximum(1.0, np.abs(a)))
    assert not np.array_equal(noise.noise_grid(16, 9, stream=1), a)
    assert not np.array_equal(noise.noise_grid(16, 10), a)


@pytest.mark.parametrize("bad", [-1, 1 << 64])
def test_seed_range(bad):
    with pytest.raises(ValueError):
        philox.seed_key(bad)


def test_log_word_f32_matches_extended_libm():
    rng = np.random.default_rng(13)
    w = rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64)
    w[:8] = [0, 1, (1 << 32) - 1, (1 << 32) - 2, normal.W_SPLIT, normal.W_SPLIT - 1, 1 << 31, 12345]
    u = (w.astype(np.longdouble) + 1) * np.longdouble(2.0) ** -32
    want = np.log(u)
    got = normal.log_word_f32(w)
    assert got.dtype == np.float32
    rel = np.abs((got.astype(np.longdouble) - want) / np.where(want == 0, 1, np.abs(want)))
    assert float(rel.max()) < 4e-7
    assert got[2] == 0.0


def test_cos_sin_f32_match_extended_libm():
    rng = np.random.default_rng(14)
    w = rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64)
    w[:6] = [0, (1 << 29) - 1, 1 << 29, 1 << 30, 3 << 30, (1 << 32) - 1]
    c, s = normal.cos_sin_turn_f32(w)
    theta = (w.astype(np.longdouble) * np.longdouble(2.0) ** -32) * LD_TWO_PI
    assert float(np.abs(c - np.cos(theta)).max()) < 3e-7
    assert float(np.abs(s - np.sin(theta)).max()) < 3e-7


def test_box_muller_f32_tracks_binary64():
    rng = np.random.default_rng(15)
    wa = rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64)
    wb = rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64)
    wa[:4] = [0, (1 << 32) - 1, (1 << 32) - 2, normal.W_SPLIT]
    for x32, x64 in zip(normal.box_muller_f32(wa, wb), normal.box_muller(wa, wb)):
        assert x32.dtype == np.float32
        d = np.abs(x32.astype(np.float64) - x64)
        ulp = np.spacing(np.maximum(np.float32(1), np.abs(x64).astype(np.float32))).astype(np.float64)
        assert float((d / ulp).max()) <= 4.0


def test_noise_f32_is_unit_gaussian():
    w = noise.noise_grid(64, 43, dtype=np.float32).ravel().astype(np.float64)
    m = w.size
    assert abs(w.mean()) < 5 / np.sqrt(m)
    assert abs(w.var() - 1.0) < 5 * np.sqrt(2.0 / m)
    assert stats.kstest(w, "norm").pvalue > 1e-3
