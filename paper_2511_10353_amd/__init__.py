"""MI355X-native initial-conditions path of the Ginnungagap method
(arxiv 2511.10353): seeded white noise -> real-to-complex 3D FFT ->
sqrt(P(k)) i k_j/k^2 filter -> three complex-to-real FFTs -> Zel'dovich
particles, as hand-written HIP kernels for gfx950 behind the C ABI in
include/gg.h.  This package holds the in-tree build of that library and its
ctypes binding."""
from .binding import (Cosmo, GGError, MakeIC, Plan, lib, LIB_PATH, make_ic_autograd, refine_noise,  # noqa: F401
                      interpolate_add, cutoff_n2, increase_resolution, refine_noise_region, interpolate_add_at,
                      Zoom)
