"""White-noise field W on the N^3 lattice (Sec. 2, step 1; Sec. 2.1).

The paper draws its Gaussian white noise from SPRNG without fixing how cells
map to random numbers.  The reading used here: cell (m0, m1, m2), m_i in
[0, N), has linear index c = (m0 N + m1) N + m2 (row-major, axis 2
contiguous) and is one Philox-4x32-10 call with

    key     = (seed mod 2^32, floor(seed / 2^32))
    counter = (c mod 2^32, floor(c / 2^32), stream, 0).

Of its words (w0, w1, w2, w3), w0 and w1 give the cell's deviate as the
cosine branch of the Box-Muller transform of ``normal.py`` in binary64,
g = sqrt(-2 ln u1) cos(2 pi u2), u1 = (w0 + 1) 2^-32, u2 = w1 2^-32; w2 and
w3 are not used.  The single-precision field is g rounded once to float32,
so both precisions carry the same realisation.  ``stream`` separates
independent fields drawn with the same seed.
"""
import numpy as np

from .philox import philox4x32, seed_key
from .normal import gaussian


def noise_cells(cells, seed, stream=0, dtype=np.float64):
    """Noise values of linear cell indices: binary64 deviates, rounded to
    ``dtype`` (float64 or float32)."""
    cells = np.asarray(cells, dtype=np.uint64)
    key = seed_key(seed)
    w0, w1, _, _ = philox4x32(
        (cells & np.uint64(0xFFFFFFFF), cells >> np.uint64(32), np.uint64(stream), np.uint64(0)), key)
    return gaussian(w0, w1).astype(dtype)


def noise_grid(n, seed, stream=0, dtype=np.float64, chunk=1 << 22, workers=1):
    """The full N^3 noise field, shape (n, n, n), as ``dtype`` (f64 or f32).

    ``workers`` > 1 fills disjoint chunks from a thread pool (numpy releases
    the interpreter lock inside its array loops); the values do not depend on it.
    """
    total = n * n * n
    out = np.empty(total, dtype=dtype)

    def fill(start):
        stop = min(total, start + chunk)
        out[start:stop] = noise_cells(np.arange(start, stop, dtype=np.uint64), seed, stream, dtype)

    starts = range(0, total, chunk)
    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fill, starts))
    else:
        for start in starts:
            fill(start)
    return out.reshape(n, n, n)
