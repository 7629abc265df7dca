"""Nested zoom levels (Sec. 2.3-2.4), in float64 (test infrastructure).

A zoom hierarchy is a base lattice of N_0^3 cells covering the periodic box
L_0 plus levels l = 1, 2, ... of N_l^3 cells, each refining its parent by two
per axis (Delta_l = Delta_{l-1} / 2, the paper's zoom step) over a sub-box of
N_l / 2 parent cells per axis starting at the integer parent cell o_l.  For
every level:

  noise      the parent's noise on the sub-box (periodic slice) refined by
             App. A (4-cell basis, Eq. A.10-A.13) with stream_id = l, so the
             parent's large-scale modes carry over;
  small      Eq. 4 on the level's own periodic sub-box: psi~ (1 - f(k r_s)),
             r_s = 2 Delta_{l-1};
  large      Eq. 5 applied to the parent's final displacement field on the
             parent lattice (periodic on the parent's box): psi~ f(k r_s) /
             W_CiC, inverse transformed, then cloud-in-cell interpolated to the
             level's lattice points o_l Delta_{l-1} + m Delta_l;
  psi        small + large; particles at O_l + (m + 1/2) Delta_l + psi,
             wrapped into [0, L_0), O_l the level's origin in the base box
             (itself taken into [0, L_0)).

The periodic transform inside a sub-box makes psi deviate from the field of a
full-box high-resolution realisation with the same noise; the paper puts the
standard deviation of that error below 1e-3 beyond a quarter of the sub-box
from the faces (Fig. 1) without stating its normalisation.  With the top-hat
window of Eq. 4 the small-scale kernel rings over many r_s, and this oracle
measures about 5% of the rms displacement there (64 Mpc/h box, 32 Mpc/h
sub-box of 128^3 cells): that statement is not used as a pin.

Pins (tests/test_oracle_zoom.py): a level whose sub-box is the whole box
equals the full-box resolution increase of oracle.refine; Eq. 5 on psi equals
the large-scale window of the filter; interpolation at an origin equals
shifted periodic upsampling; particle lattices at an origin; nested origins
inside the parents' inner halves; the level noise is the refinement of the
parent's sub-box noise.
"""
import numpy as np

from . import cosmology, pipeline, refine
from .noise import noise_grid


def periodic_slice(field, origin, count):
    """field[o0:o0+count, o1:o1+count, o2:o2+count] with periodic wrap."""
    f = np.asarray(field)
    n = f.shape[0]
    idx = [(np.arange(count) + o) % n for o in origin]
    return f[np.ix_(*idx)]


def lowpass(field, n, box, r_s, deconvolve=True, workers=None):
    """Eq. 5 on a periodic real field: f(k r_s) (and 1/W_CiC) in Fourier space."""
    spec = pipeline.forward(np.asarray(field, dtype=np.float64), workers=workers)
    spec = spec * refine.mode_window(n, box, r_s, "large")
    if deconvolve:
        spec = spec / refine.cic_window(n)
    return pipeline.inverse(spec, n, workers=workers)


def cic_at(field, origin, ratio, count):
    """Trilinear interpolation of a periodic field at the points
    origin + m / ratio (parent cells), m < count per axis."""
    f = np.asarray(field, dtype=np.float64)
    n = f.shape[0]
    out = f
    for axis in range(3):
        u = origin[axis] + np.arange(count) / ratio
        i0 = np.floor(u).astype(np.int64)
        t = u - i0
        a = np.take(out, i0 % n, axis=axis)
        b = np.take(out, (i0 + 1) % n, axis=axis)
        shape = [1, 1, 1]
        shape[axis] = count
        tt = t.reshape(shape)
        out = a * (1.0 - tt) + b * tt
    return out


def level_displacements(w_level, n_level, box_level, parent_psi, n_parent, box_parent, origin, cosmo,
                        workers=None):
    """psi of one zoom level from its noise and the parent's displacements."""
    delta_parent = box_parent / n_parent
    r_s = 2.0 * delta_parent
    small = refine.windowed_displacements(w_level, n_level, box_level, cosmo, r_s, "small", workers=workers)
    large = np.stack([cic_at(lowpass(parent_psi[j], n_parent, box_parent, r_s, workers=workers), origin, 2, n_level)
                      for j in range(3)])
    return small + large


def particles(psi, n, cell, origin_box, box0, cosmo, offset=0.5):
    """Eq. 3 at the level's lattice: float32 positions in [0, L_0) and velocities."""
    pos = []
    for j in range(3):
        shape = [1, 1, 1]
        shape[j] = n
        q = origin_box[j] + (np.arange(n, dtype=np.float64).reshape(shape) + offset) * cell
        x = q + np.asarray(psi[j], dtype=np.float64)
        x = pipeline.periodic_wrap(x, box0)
        xf = x.astype(np.float32)
        pos.append(np.where(xf >= np.float32(box0), np.float32(0.0), xf))
    vel = (cosmology.velocity_factor(cosmo) * np.asarray(psi, dtype=np.float64)).astype(np.float32)
    return np.stack(pos), vel


def hierarchy(n0, box0, sizes, origins, seed, cosmo, workers=None):
    """All levels: a list of dicts (n, box, cell, origin_box, w, psi, pos, vel).

    ``sizes`` are N_1, N_2, ...; ``origins`` the integer parent-cell origins
    (3-tuples) of levels 1, 2, ...; the base noise is (seed, stream 0).
    """
    w0 = noise_grid(n0, seed, 0, workers=workers or 1)
    psi0 = np.stack(pipeline.displacement_fields(w0, n0, box0, cosmo, workers=workers))
    cell0 = box0 / n0
    pos0, vel0 = particles(psi0, n0, cell0, (0.0, 0.0, 0.0), box0, cosmo)
    levels = [dict(n=n0, box=box0, cell=cell0, origin_box=(0.0, 0.0, 0.0), w=w0, psi=psi0, pos=pos0, vel=vel0)]
    for lev, (n, o) in enumerate(zip(sizes, origins), start=1):
        par = levels[-1]
        if n % 4:
            raise ValueError("level sizes must be multiples of 4")
        cell = par["cell"] / 2.0
        box = n * cell
        w = refine.refine(periodic_slice(par["w"], o, n // 2), "4", seed, lev)
        psi = level_displacements(w, n, box, par["psi"], par["n"], par["box"], o, cosmo, workers=workers)
        origin_box = tuple(float(np.fmod(par["origin_box"][j] + o[j] * par["cell"], box0)) for j in range(3))
        pos, vel = particles(psi, n, cell, origin_box, box0, cosmo)
        levels.append(dict(n=n, box=box, cell=cell, origin_box=origin_box, w=w, psi=psi, pos=pos, vel=vel))
    return levels


def nested_origins(n0, sizes, seed=42):
    """Integer parent-cell origins: level 1 anywhere in the periodic base box;
    deeper levels inside the inner half of their parent (at least a quarter of
    the parent sub-box from its faces, where the sub-box error is small)."""
    rng = np.random.default_rng(seed)
    out = []
    parent = n0
    for lev, n in enumerate(sizes, start=1):
        span = n // 2
        if lev == 1:
            o = tuple(int(v) for v in rng.integers(0, n0, 3))
        else:
            lo = parent // 4
            hi = parent - parent // 4 - span
            if hi < lo:
                raise ValueError("a level does not fit in the inner half of its parent")
            o = tuple(int(v) for v in rng.integers(lo, hi + 1, 3))
        out.append(o)
        parent = n
    return out
