"""White-noise field W on the N^3 lattice (Sec. 2, step 1; Sec. 2.1).

The paper draws its Gaussian white noise from SPRNG without fixing how cells
map to random numbers.  The reading used here: cell (m0, m1, m2), m_i in
[0, N), has linear index c = (m0 N + m1) N + m2 (row-major, axis 2
contiguous).  Four consecutive cells c = 4q + j (j = 0..3) share one
Philox-4x32-10 call with

    key     = (seed mod 2^32, floor(seed / 2^32))
    counter = (q mod 2^32, floor(q / 2^32), stream, 0).

Its words (w0, w1, w2, w3) form two Box-Muller pairs (``normal.py``, binary64):
(w0, w1) gives cells 4q and 4q + 1, (w2, w3) cells 4q + 2 and 4q + 3; of a
pair (wa, wb) the even cell takes r cos(2 pi u2) and the odd cell r sin(2 pi
u2), with r = sqrt(-2 ln u1), u1 = (wa + 1) 2^-32, u2 = wb 2^-32.  The two
deviates of a Box-Muller pair are independent unit Gaussians (Box and
Muller 1958), and the two pairs come from independent words.  The
single-precision field is each deviate rounded once to float32, so both
precisions carry the same realisation.  ``stream`` separates independent
fields drawn with the same seed.
"""
import numpy as np

from .philox import philox4x32, seed_key
from .normal import box_muller


def noise_cells(cells, seed, stream=0, dtype=np.float64):
    """Noise values of linear cell indices: binary64 deviates, rounded to
    ``dtype`` (float64 or float32)."""
    cells = np.asarray(cells, dtype=np.uint64)
    key = seed_key(seed)
    q = cells >> np.uint64(2)
    j = cells & np.uint64(3)
    w0, w1, w2, w3 = philox4x32(
        (q & np.uint64(0xFFFFFFFF), q >> np.uint64(32), np.uint64(stream), np.uint64(0)), key)
    second = j >= np.uint64(2)
    g_cos, g_sin = box_muller(np.where(second, w2, w0), np.where(second, w3, w1))
    return np.where((j & np.uint64(1)) == np.uint64(1), g_sin, g_cos).astype(dtype)


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
