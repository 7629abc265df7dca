"""Pins for the oracle's white noise: elementary functions against the
platform's extended-precision libm, Box-Muller against the normal law, and the
cell-to-counter mapping (one Philox call per four cells: two Box-Muller pairs,
cosine branch for the even cell of a pair, sine branch for the odd one)."""
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
    # each of the four cells of a Philox call (cos / sin of either word pair)
    # is N(0, 1) on its own
    for lane in range(4):
        assert stats.kstest(w[lane::4], "norm").pvalue > 1e-4


def test_neighbouring_cells_uncorrelated():
    w = noise.noise_grid(64, 7).ravel()
    for lag in (1, 2, 3, 4, 64):
        r = np.corrcoef(w[:-lag], w[lag:])[0, 1]
        assert abs(r) < 5 / np.sqrt(w.size)


def test_cell_mapping():
    # the noise of cell c = 4q + j only depends on (seed, stream, c): Philox
    # call q with counter (q lo, q hi, stream, 0); words (w0, w1) for j < 2,
    # (w2, w3) for j >= 2; r cos(theta) for even j, r sin(theta) for odd j.
    # Checked against the Box-Muller formula in extended precision.
    seed = 123456789012345
    cells = np.array([0, 1, 2, 3, 4, 7, 1 << 33, (1 << 33) + 1, (1 << 33) + 2, (1 << 33) + 3,
                      (1 << 30) - 1, (1 << 34) + 6], dtype=np.uint64)
    got = noise.noise_cells(cells, seed, stream=2)
    for c, g in zip(cells, got):
        c = int(c)
        q, j = c >> 2, c & 3
        w = [int(np.asarray(x).reshape(-1)[0]) for x in philox.philox4x32(
            (q & 0xFFFFFFFF, q >> 32, 2, 0), philox.seed_key(seed))]
        wa, wb = (w[0], w[1]) if j < 2 else (w[2], w[3])
        u1 = np.longdouble(wa + 1) * np.longdouble(2.0) ** -32
        th = np.longdouble(wb) * np.longdouble(2.0) ** -32 * LD_TWO_PI
        r = np.sqrt(-2 * np.log(u1))
        want = r * (np.sin(th) if j & 1 else np.cos(th))
        assert abs(g - float(want)) < 1e-14
        # the other branch of the same pair is a different deviate
        other = r * (np.cos(th) if j & 1 else np.sin(th))
        assert abs(g - float(other)) > 1e-12


def test_pairs_share_radius_and_are_independent():
    # g(4q)^2 + g(4q+1)^2 = -2 ln u1(w0) and g(4q+2)^2 + g(4q+3)^2 = -2 ln u1(w2)
    # (cos^2 + sin^2 = 1); the two branches and the two pairs are uncorrelated
    n = 1 << 18
    cells = np.arange(n, dtype=np.uint64)
    g = noise.noise_cells(cells, 77, stream=5).reshape(-1, 4)
    q = np.arange(n // 4, dtype=np.uint64)
    w0, _, w2, _ = philox.philox4x32((q, np.zeros_like(q), np.full_like(q, 5), np.zeros_like(q)),
                                    philox.seed_key(77))
    for a, wa in ((0, w0), (2, w2)):
        r2 = -2.0 * np.log((wa + np.uint64(1)).astype(np.longdouble) * np.longdouble(2.0) ** -32)
        s = g[:, a].astype(np.longdouble) ** 2 + g[:, a + 1].astype(np.longdouble) ** 2
        assert float(np.max(np.abs(s - r2) / np.maximum(r2, 1e-30))) < 1e-14
    lim = 5 / np.sqrt(g.shape[0])
    for a, b in ((0, 1), (2, 3), (0, 2), (1, 3), (0, 3), (1, 2)):
        assert abs(np.corrcoef(g[:, a], g[:, b])[0, 1]) < lim
    # independent unit Gaussians: E[g_a^2 g_b^2] = 1 for the two branches of a pair
    assert abs(np.mean(g[:, 0] ** 2 * g[:, 1] ** 2) - 1.0) < 0.05


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
