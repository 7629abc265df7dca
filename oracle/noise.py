"""White-noise field W on the N^3 lattice (Sec. 2, step 1; Sec. 2.1).

Cell (m0, m1, m2), m_i in [0, N), has linear index c = (m0 N + m1) N + m2
(row-major, axis 2 contiguous).  Cells are taken four at a time: group
g = floor(c / 4) is one Philox-4x32-10 call with

    key     = (seed mod 2^32, floor(seed / 2^32))
    counter = (g mod 2^32, floor(g / 2^32), stream, 0)

and its words (w0, w1, w2, w3) feed two Box-Muller pairs:
cell 4g   <- r_a cos(theta_a),  cell 4g+1 <- r_a sin(theta_a)  from (w0, w1)
cell 4g+2 <- r_b cos(theta_b),  cell 4g+3 <- r_b sin(theta_b)  from (w2, w3)

``stream`` separates independent fields drawn with the same seed.  The
double precision field uses the binary64 Box-Muller of ``normal.py``; the
single precision field uses its binary32 variant on the same Philox words, so
the two precisions carry the same realisation to float32 accuracy (a few
float32 ulp per cell).
"""
import numpy as np

from .philox import philox4x32, seed_key
from .normal import box_muller, box_muller_f32


def noise_cells(cells, seed, stream=0, dtype=np.float64):
    """Noise values (float64 or float32 arithmetic) for linear cell indices."""
    cells = np.asarray(cells, dtype=np.uint64)
    g = cells >> np.uint64(2)
    lane = (cells & np.uint64(3)).astype(np.int64)
    key = seed_key(seed)
    w0, w1, w2, w3 = philox4x32(
        (g & np.uint64(0xFFFFFFFF), g >> np.uint64(32), np.uint64(stream), np.uint64(0)), key)
    bm = box_muller_f32 if np.dtype(dtype) == np.float32 else box_muller
    ga, gb = bm(w0, w1)
    gc, gd = bm(w2, w3)
    return np.select([lane == 0, lane == 1, lane == 2], [ga, gb, gc], gd).astype(dtype)


def noise_grid(n, seed, stream=0, dtype=np.float64, chunk=1 << 22, workers=1):
    """The full N^3 noise field, shape (n, n, n), computed in ``dtype`` (f64 or f32).

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
