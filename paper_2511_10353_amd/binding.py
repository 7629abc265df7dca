"""ctypes binding of libgg (include/gg.h): argument marshalling only.

Torch tensors supply device memory (``data_ptr``) and the current HIP stream;
every step of the path runs in the library's kernels.  There is no fallback:
if libgg.so is missing or no GPU is present, the calls raise.
"""
import ctypes
import dataclasses
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# GG_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("GG_LIBRARY") or os.path.join(_PKG, "libgg.so")

GG_OK = 0
GG_ERR_INVALID_ARG, GG_ERR_UNSUPPORTED_SIZE, GG_ERR_OUT_OF_MEMORY, GG_ERR_HIP, GG_ERR_INTERNAL = 1, 2, 3, 4, 5
STATUS_NAMES = {0: "GG_OK", 1: "GG_ERR_INVALID_ARG", 2: "GG_ERR_UNSUPPORTED_SIZE",
                3: "GG_ERR_OUT_OF_MEMORY", 4: "GG_ERR_HIP", 5: "GG_ERR_INTERNAL"}
DTYPES = {"f32": 0, "f64": 1}
N_PASSES = 5


class GGError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box", ctypes.c_double)]


class _Cosmo(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("h", ctypes.c_double), ("n_s", ctypes.c_double),
                ("sigma8", ctypes.c_double), ("z_init", ctypes.c_double), ("amp", ctypes.c_double),
                ("lattice_offset", ctypes.c_double)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_int32), ("p1_lines", ctypes.c_int32), ("z_lines", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("box", ctypes.c_double),
                ("amplitude", ctypes.c_double), ("sigma8_integral", ctypes.c_double),
                ("growth", ctypes.c_double), ("velocity_factor", ctypes.c_double),
                ("real_elems", ctypes.c_size_t), ("spectrum_elems", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("chunks", ctypes.c_int32), ("p1_lines", ctypes.c_int32),
                ("z_lines", ctypes.c_int32)]


@dataclasses.dataclass
class Cosmo:
    """Spectrum parameters (defaults: Omega_m 0.3, h 0.7, n_s 0.96, sigma_8 0.8, z 100)."""
    omega_m: float = 0.3
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    z_init: float = 100.0
    amp: float = 0.0
    lattice_offset: float = 0.5

    def _c(self):
        return _Cosmo(self.omega_m, self.h, self.n_s, self.sigma8, self.z_init, self.amp, self.lattice_offset)


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "gg_plan_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(_Grid), ctypes.POINTER(_Cosmo), ctypes.c_int]),
    "gg_plan_destroy": (ctypes.c_int, [_VP]),
    "gg_plan_query": (ctypes.c_int, [_VP, ctypes.POINTER(_Info)]),
    "gg_workspace_bytes": (ctypes.c_size_t, [_VP]),
    "gg_noise": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_uint32, _VP, _VP]),
    "gg_fft3d": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP, _VP]),
    "gg_filter": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "gg_zeldovich": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "gg_make_ic": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP]),
    "gg_make_ic_noalloc": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP]),
    "gg_make_ic_from_noise": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP, _VP]),
    "gg_make_ic_adjoint": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP, _VP]),
    "gg_make_density": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP]),
    "gg_power_spectrum": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "gg_field_stats": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "gg_refine_noise": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_uint64, ctypes.c_uint32,
                                        _VP, _VP]),
    "gg_make_displacements": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _VP, _VP, _VP]),
    "gg_interpolate_add": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _VP, _VP, _VP]),
    "gg_refine_noise_region": (ctypes.c_int, [ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int, ctypes.c_int, _VP,
                                               ctypes.c_uint64, ctypes.c_uint32, _VP, _VP]),
    "gg_interpolate_add_at": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int, _VP, _VP,
                                              _VP]),
    "gg_lowpass": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP, _VP]),
    "gg_cutoff_n2": (ctypes.c_int64, [ctypes.c_double, ctypes.c_double]),
    "gg_increase_resolution": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.c_double, _VP, _VP, _VP, _VP]),
    "gg_zeldovich_at": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, _VP, _VP, _VP]),
    "gg_degrade": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP]),
    "gg_zoom_create": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int]),
    "gg_zoom_destroy": (ctypes.c_int, [_VP]),
    "gg_zoom_workspace_bytes": (ctypes.c_size_t, [_VP]),
    "gg_zoom_query": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, _VP]),
    "gg_zoom_run": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    "gg_zoom_autotune": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP,
                                        ctypes.c_int32, _VP, _VP]),
    "gg_plan_set_tuning": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "gg_plan_autotune": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP, ctypes.c_int32, _VP, _VP]),
    "gg_timing_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
    "gg_timing_read": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]),
    "gg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gg_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libgg.so (built by paper_2511_10353_amd.build) once."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2511_10353_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status):
    if status != GG_OK:
        raise GGError(status, lib().gg_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """One lattice (N, L), cosmology and precision; owns the device tables."""

    def __init__(self, n, box, cosmo=None, dtype="f32"):
        if dtype not in DTYPES:
            raise ValueError("dtype must be 'f32' or 'f64'")
        if not torch.cuda.is_available():
            raise RuntimeError("libgg needs a ROCm GPU; torch.cuda.is_available() is False")
        torch.cuda.init()
        self.n = int(n)
        self.box = float(box)
        self.cosmo = cosmo or Cosmo()
        self.dtype = dtype
        self.real_dtype = torch.float32 if dtype == "f32" else torch.float64
        self.complex_dtype = torch.complex64 if dtype == "f32" else torch.complex128
        self._h = ctypes.c_void_p()
        _check(lib().gg_plan_create(ctypes.byref(self._h), ctypes.byref(_Grid(self.n, self.box)),
                                    ctypes.byref(self.cosmo._c()), DTYPES[dtype]))
        info = _Info()
        _check(lib().gg_plan_query(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.workspace_bytes = int(lib().gg_workspace_bytes(self._h))

    def close(self):
        if self._h:
            lib().gg_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ---------------------------------------------------------------
    def _real_shape(self):
        return (self.n, self.n, self.n)

    def _spec_shape(self):
        return (self.n, self.n, self.n // 2 + 1)

    def _need(self, t, shape, dtype, name):
        if t is None:
            return torch.empty(shape, dtype=dtype, device="cuda")
        if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous cuda tensor {tuple(shape)} {dtype}, "
                             f"got {tuple(t.shape)} {t.dtype} cuda={t.is_cuda}")
        return t

    def workspace(self):
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")

    # -- entry points ------------------------------------------------------------
    def noise(self, seed, out=None, stream_id=0):
        out = self._need(out, self._real_shape(), self.real_dtype, "out")
        _check(lib().gg_noise(self._h, int(seed), int(stream_id), _ptr(out), _stream()))
        return out

    def fft3d(self, x, direction, out=None, work=None):
        if direction == 1:
            x = self._need(x, self._real_shape(), self.real_dtype, "x")
            out = self._need(out, self._spec_shape(), self.complex_dtype, "out")
        elif direction == -1:
            x = self._need(x, self._spec_shape(), self.complex_dtype, "x")
            out = self._need(out, self._real_shape(), self.real_dtype, "out")
            if work is None:
                work = self.workspace()
        else:
            raise ValueError("direction must be +1 or -1")
        _check(lib().gg_fft3d(self._h, int(direction), _ptr(x), _ptr(out), _ptr(work), _stream()))
        return out

    def filter(self, spec, psi=None, delta=None, want_delta=False):
        spec = self._need(spec, self._spec_shape(), self.complex_dtype, "spec")
        psi = self._need(psi, (3,) + self._spec_shape(), self.complex_dtype, "psi")
        if want_delta or delta is not None:
            delta = self._need(delta, self._spec_shape(), self.complex_dtype, "delta")
        _check(lib().gg_filter(self._h, _ptr(spec), _ptr(psi), _ptr(delta), _stream()))
        return (psi, delta) if delta is not None else psi

    def zeldovich(self, psi, pos=None, vel=None):
        psi = self._need(psi, (3,) + self._real_shape(), self.real_dtype, "psi")
        pos = self._need(pos, (3,) + self._real_shape(), torch.float32, "pos")
        vel = self._need(vel, (3,) + self._real_shape(), torch.float32, "vel")
        _check(lib().gg_zeldovich(self._h, _ptr(psi), _ptr(pos), _ptr(vel), _stream()))
        return pos, vel

    def make_ic(self, seed, pos=None, vel=None, psi=None, work=None, want_psi=False):
        pos = self._need(pos, (3,) + self._real_shape(), torch.float32, "pos")
        vel = self._need(vel, (3,) + self._real_shape(), torch.float32, "vel")
        if want_psi or psi is not None:
            psi = self._need(psi, (3,) + self._real_shape(), self.real_dtype, "psi")
        if work is None:
            work = self.workspace()
        elif work.numel() * work.element_size() < self.workspace_bytes or not work.is_cuda:
            raise ValueError("work buffer too small")
        _check(lib().gg_make_ic(self._h, int(seed), _ptr(pos), _ptr(vel), _ptr(psi), _ptr(work), _stream()))
        return (pos, vel, psi) if psi is not None else (pos, vel)

    def make_ic_noalloc(self, seed, pos=None, vel=None, psi=None, want_psi=False):
        """gg_make_ic_noalloc: the fused path on the library's static workspace
        (no workspace argument; lattices up to the library's scratch size)."""
        pos = self._need(pos, (3,) + self._real_shape(), torch.float32, "pos")
        vel = self._need(vel, (3,) + self._real_shape(), torch.float32, "vel")
        if want_psi or psi is not None:
            psi = self._need(psi, (3,) + self._real_shape(), self.real_dtype, "psi")
        _check(lib().gg_make_ic_noalloc(self._h, int(seed), _ptr(pos), _ptr(vel), _ptr(psi), _stream()))
        return (pos, vel, psi) if psi is not None else (pos, vel)

    def make_ic_from_noise(self, w, amp_scale=1.0, pos=None, vel=None, psi=None, work=None, particles=True,
                           want_psi=False):
        """The path from a given noise field w (N^3, path dtype); amp_scale
        multiplies the displacements.  Returns (pos, vel[, psi]) or psi."""
        w = self._need(w, self._real_shape(), self.real_dtype, "w")
        if particles:
            pos = self._need(pos, (3,) + self._real_shape(), torch.float32, "pos")
            vel = self._need(vel, (3,) + self._real_shape(), torch.float32, "vel")
        else:
            pos = vel = None
            want_psi = True
        if want_psi or psi is not None:
            psi = self._need(psi, (3,) + self._real_shape(), self.real_dtype, "psi")
        if work is None:
            work = self.workspace()
        _check(lib().gg_make_ic_from_noise(self._h, _ptr(w), float(amp_scale), _ptr(pos), _ptr(vel), _ptr(psi),
                                           _ptr(work), _stream()))
        if not particles:
            return psi
        return (pos, vel, psi) if psi is not None else (pos, vel)

    def make_ic_adjoint(self, g_psi=None, g_pos=None, g_vel=None, amp_scale=1.0, psi=None, g_w=None, work=None,
                        want_log_amp=False):
        """d loss/d w (and d loss/d log A if want_log_amp, which needs psi)."""
        shape3 = (3,) + self._real_shape()
        if g_psi is not None:
            g_psi = self._need(g_psi, shape3, self.real_dtype, "g_psi")
        if g_pos is not None:
            g_pos = self._need(g_pos, shape3, torch.float32, "g_pos")
        if g_vel is not None:
            g_vel = self._need(g_vel, shape3, torch.float32, "g_vel")
        if psi is not None:
            psi = self._need(psi, shape3, self.real_dtype, "psi")
        g_w = self._need(g_w, self._real_shape(), self.real_dtype, "g_w")
        g_la = torch.empty(1, dtype=torch.float64, device="cuda") if want_log_amp else None
        if work is None:
            work = self.workspace()
        _check(lib().gg_make_ic_adjoint(self._h, _ptr(g_psi), _ptr(g_pos), _ptr(g_vel), float(amp_scale), _ptr(psi),
                                        _ptr(g_la), _ptr(g_w), _ptr(work), _stream()))
        return (g_w, g_la) if want_log_amp else g_w

    def make_density(self, seed=42, w=None, out=None, work=None):
        """delta (Eq. 1) from the noise of ``seed`` or from the field ``w``."""
        if w is not None:
            w = self._need(w, self._real_shape(), self.real_dtype, "w")
        out = self._need(out, self._real_shape(), self.real_dtype, "out")
        if work is None:
            work = self.workspace()
        _check(lib().gg_make_density(self._h, int(seed), _ptr(w), _ptr(out), _ptr(work), _stream()))
        return out

    def power_spectrum(self, field, nbins, work=None):
        """(pk, kmean, counts): float64 device tensors of length nbins."""
        field = self._need(field, self._real_shape(), self.real_dtype, "field")
        res = torch.empty((3, int(nbins)), dtype=torch.float64, device="cuda")
        if work is None:
            work = self.workspace()
        _check(lib().gg_power_spectrum(self._h, _ptr(field), int(nbins), _ptr(res[0]), _ptr(res[1]), _ptr(res[2]),
                                       _ptr(work), _stream()))
        return res[0], res[1], res[2]

    def field_stats(self, field, work=None):
        """float64 device tensor (mean, std, min, max) of the N^3 values."""
        field = self._need(field, self._real_shape(), self.real_dtype, "field")
        out = torch.empty(4, dtype=torch.float64, device="cuda")
        if work is None:
            work = self.workspace()
        _check(lib().gg_field_stats(self._h, _ptr(field), _ptr(out), _ptr(work), _stream()))
        return out

    def make_displacements(self, w, n2_min=0, n2_max=0, deconvolve=False, psi=None, work=None):
        """psi (3, N, N, N) of the noise w with the mode window n2_min <= n^2 <
        n2_max (n2_max <= 0: none) and optional CiC deconvolution (Eq. 4-5)."""
        w = self._need(w, self._real_shape(), self.real_dtype, "w")
        psi = self._need(psi, (3,) + self._real_shape(), self.real_dtype, "psi")
        if work is None:
            work = self.workspace()
        _check(lib().gg_make_displacements(self._h, _ptr(w), int(n2_min), int(n2_max), int(bool(deconvolve)), _ptr(psi),
                                           _ptr(work), _stream()))
        return psi

    def lowpass(self, field, n2_max, deconvolve=True, out=None, work=None):
        """Eq. 5 on a real field: modes n^2 < n2_max kept (optionally / W_CiC)."""
        field = self._need(field, self._real_shape(), self.real_dtype, "field")
        out = self._need(out, self._real_shape(), self.real_dtype, "out")
        if work is None:
            work = self.workspace()
        _check(lib().gg_lowpass(self._h, _ptr(field), int(n2_max), int(bool(deconvolve)), _ptr(out), _ptr(work),
                                _stream()))
        return out

    def degrade(self, fine, factor, shift=(0.5, 0.5, 0.5), out=None, work=None):
        """Sec. 2.3 degrade of a fine (factor n)^3 field onto this plan's lattice:
        nearest-grid-point values, then a Fourier translation by ``shift``
        coarse cells per axis."""
        nf = self.n * int(factor)
        fine = self._need(fine, (nf, nf, nf), self.real_dtype, "fine")
        out = self._need(out, self._real_shape(), self.real_dtype, "out")
        if work is None:
            work = self.workspace()
        sh = (ctypes.c_double * 3)(*[float(v) for v in shift])
        _check(lib().gg_degrade(self._h, _ptr(fine), int(factor), sh, _ptr(out), _ptr(work), _stream()))
        return out

    def zeldovich_at(self, psi, origin, wrap_box, pos=None, vel=None):
        """Eq. 3 for this plan's lattice placed at ``origin`` inside a periodic box."""
        psi = self._need(psi, (3,) + self._real_shape(), self.real_dtype, "psi")
        pos = self._need(pos, (3,) + self._real_shape(), torch.float32, "pos")
        vel = self._need(vel, (3,) + self._real_shape(), torch.float32, "vel")
        o = (ctypes.c_double * 3)(*[float(v) for v in origin])
        _check(lib().gg_zeldovich_at(self._h, _ptr(psi), o, float(wrap_box), _ptr(pos), _ptr(vel), _stream()))
        return pos, vel

    def _refresh_info(self):
        info = _Info()
        _check(lib().gg_plan_query(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}

    def set_tuning(self, chunks=0, p1_lines=0, z_lines=0):
        """Launch configuration of gg_make_ic (0 = keep / built-in)."""
        _check(lib().gg_plan_set_tuning(self._h, int(chunks), int(p1_lines), int(z_lines)))
        self._refresh_info()

    def autotune(self, reps=3, pos=None, vel=None, work=None):
        """Time every valid (chunks, p1_lines, z_lines) for gg_make_ic, keep the
        fastest; returns the list of timed configurations."""
        pos = self._need(pos, (3,) + self._real_shape(), torch.float32, "pos")
        vel = self._need(vel, (3,) + self._real_shape(), torch.float32, "vel")
        if work is None:
            work = self.workspace()
        cap = 64
        res = (_TuneEntry * cap)()
        count = ctypes.c_int32()
        _check(lib().gg_plan_autotune(self._h, _ptr(pos), _ptr(vel), _ptr(work), int(reps), res, cap,
                                      ctypes.byref(count), _stream()))
        self._refresh_info()
        return [dict(chunks=r.chunks, p1_lines=r.p1_lines, z_lines=r.z_lines, ms=r.ms) for r in res[:count.value]]

    def timing_enable(self, on=True):
        _check(lib().gg_timing_enable(self._h, 1 if on else 0))

    def timing_read(self):
        ms = (ctypes.c_double * N_PASSES)()
        calls = ctypes.c_int(0)
        _check(lib().gg_timing_read(self._h, ms, N_PASSES, ctypes.byref(calls)))
        return [ms[i] for i in range(N_PASSES)], calls.value


REFINE_VARIANTS = {"hr": 0, "3": 1, "4": 2, "linear": 3, "sine": 4}
REFINE_SIZES = {"hr": (1, 2), "3": (2, 3), "4": (2, 4), "linear": (2, 4), "sine": (2, 4)}


def _dtype_code(t):
    if t.dtype == torch.float32:
        return DTYPES["f32"]
    if t.dtype == torch.float64:
        return DTYPES["f64"]
    raise ValueError("float32 or float64 tensors only")


def refine_noise(w_parent, variant="4", seed=0, stream_id=1, out=None):
    """White-noise refinement (App. A): a (P N_L)^3 parent field -> (P N_H)^3."""
    if variant not in REFINE_VARIANTS:
        raise ValueError(f"variant must be one of {sorted(REFINE_VARIANTS)}")
    n = int(w_parent.shape[0])
    nl, nh = REFINE_SIZES[variant]
    nc = n // nl * nh
    if tuple(w_parent.shape) != (n, n, n) or not w_parent.is_cuda or not w_parent.is_contiguous():
        raise ValueError("w_parent must be a contiguous cuda tensor (n, n, n)")
    if out is None:
        out = torch.empty((nc, nc, nc), dtype=w_parent.dtype, device=w_parent.device)
    _check(lib().gg_refine_noise(n, _dtype_code(w_parent), REFINE_VARIANTS[variant], _ptr(w_parent), int(seed),
                                 int(stream_id), _ptr(out), _stream()))
    return out


def refine_noise_region(w_parent, origin, count, variant="4", seed=0, stream_id=1, out=None):
    """App. A refinement of the parent cells origin + [0, count) (periodic)."""
    n = int(w_parent.shape[0])
    nl, nh = REFINE_SIZES[variant]
    nc = count // nl * nh
    if out is None:
        out = torch.empty((nc, nc, nc), dtype=w_parent.dtype, device=w_parent.device)
    o = (ctypes.c_int32 * 3)(*[int(v) for v in origin])
    _check(lib().gg_refine_noise_region(n, o, int(count), _dtype_code(w_parent), REFINE_VARIANTS[variant],
                                        _ptr(w_parent), int(seed), int(stream_id), _ptr(out), _stream()))
    return out


def interpolate_add_at(src, dst, origin, ratio=2):
    """dst (3, n_dst^3) += CiC interpolation of src at origin + m / ratio (src cells)."""
    o = (ctypes.c_int32 * 3)(*[int(v) for v in origin])
    _check(lib().gg_interpolate_add_at(int(src.shape[1]), int(ratio), o, int(dst.shape[1]), _dtype_code(src), _ptr(src),
                                       _ptr(dst), _stream()))
    return dst


class _ZoomDesc(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("n", ctypes.c_int32 * 8), ("origin", (ctypes.c_int32 * 3) * 8),
                ("box", ctypes.c_double), ("variant", ctypes.c_int32)]


class _ZoomTuneEntry(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("p1_lines", ctypes.c_int32), ("z_lines", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class Zoom:
    """A zoom hierarchy: base lattice n0^3 over ``box`` plus nested levels of
    ``sizes`` at origins (parent cells); buffers are allocated once and reused."""

    def __init__(self, n0, box, sizes, origins, cosmo=None, dtype="f32", variant="4"):
        if not torch.cuda.is_available():
            raise RuntimeError("libgg needs a ROCm GPU; torch.cuda.is_available() is False")
        torch.cuda.init()
        self.ns = [int(n0)] + [int(v) for v in sizes]
        self.box = float(box)
        self.dtype = dtype
        self.real_dtype = torch.float32 if dtype == "f32" else torch.float64
        d = _ZoomDesc()
        d.levels = len(self.ns)
        for l, n in enumerate(self.ns):
            d.n[l] = n
        for l, o in enumerate(origins, start=1):
            for a in range(3):
                d.origin[l][a] = int(o[a])
        d.box = self.box
        d.variant = REFINE_VARIANTS[variant]
        self._h = ctypes.c_void_p()
        _check(lib().gg_zoom_create(ctypes.byref(self._h), ctypes.byref(d), ctypes.byref((cosmo or Cosmo())._c()),
                                    DTYPES[dtype]))
        self.geometry = []
        for l in range(len(self.ns)):
            b, c, o = ctypes.c_double(), ctypes.c_double(), (ctypes.c_double * 3)()
            _check(lib().gg_zoom_query(self._h, l, ctypes.byref(b), ctypes.byref(c), o))
            self.geometry.append(dict(box=b.value, cell=c.value, origin=tuple(o)))
        self.work = torch.empty(int(lib().gg_zoom_workspace_bytes(self._h)), dtype=torch.uint8, device="cuda")
        self.levels = []
        for n in self.ns:
            self.levels.append(dict(
                w=torch.empty((n, n, n), dtype=self.real_dtype, device="cuda"),
                psi=torch.empty((3, n, n, n), dtype=self.real_dtype, device="cuda"),
                pos=torch.empty((3, n, n, n), dtype=torch.float32, device="cuda"),
                vel=torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")))
        self._ptrs = {k: (ctypes.c_void_p * len(self.ns))(*[lv[k].data_ptr() for lv in self.levels])
                      for k in ("w", "psi", "pos", "vel")}

    def run(self, seed, use_graph=False):
        _check(lib().gg_zoom_run(self._h, int(seed), self._ptrs["w"], self._ptrs["psi"], self._ptrs["pos"],
                                 self._ptrs["vel"], _ptr(self.work), int(bool(use_graph)), _stream()))
        return self.levels

    def autotune(self, seed=42, reps=5):
        """gg_zoom_autotune: per-level tile widths, kept in the zoom; returns
        the timings [{level, p1_lines, z_lines, ms}]."""
        cap = 4 * len(self.ns)
        res = (_ZoomTuneEntry * cap)()
        count = ctypes.c_int32()
        _check(lib().gg_zoom_autotune(self._h, int(seed), self._ptrs["w"], self._ptrs["psi"], self._ptrs["pos"],
                                      self._ptrs["vel"], _ptr(self.work), int(reps), res, cap, ctypes.byref(count),
                                      _stream()))
        return [dict(level=e.level, p1_lines=e.p1_lines, z_lines=e.z_lines, ms=e.ms) for e in res[:count.value]]

    def close(self):
        if self._h:
            lib().gg_zoom_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def interpolate_add(src, dst):
    """dst (3, n_dst^3) += cloud-in-cell interpolation of src (3, n_src^3)."""
    if src.dtype != dst.dtype or src.dim() != 4 or dst.dim() != 4 or src.shape[0] != 3 or dst.shape[0] != 3:
        raise ValueError("src and dst must be (3, n, n, n) tensors of one dtype")
    _check(lib().gg_interpolate_add(int(src.shape[1]), int(dst.shape[1]), _dtype_code(src), _ptr(src), _ptr(dst),
                                    _stream()))
    return dst


def cutoff_n2(box, r_s):
    """gg_cutoff_n2: the mode bound of the top hat [k r_s < 1] (n^2 < cutoff)."""
    cut = lib().gg_cutoff_n2(float(box), float(r_s))
    if cut < 0:
        raise ValueError("box and r_s must be positive and finite")
    return int(cut)


def increase_resolution(parent, child, w_parent, variant="4", seed=0, stream_id=1, r_s=None, w_child=None, psi=None,
                        work=None):
    """gg_increase_resolution (Sec. 2.3, Eq. 4-5): returns (w_child, psi) on
    the child plan's lattice; r_s None selects the library's default (two
    parent cells)."""
    if variant not in REFINE_VARIANTS:
        raise ValueError(f"variant must be one of {sorted(REFINE_VARIANTS)}")
    w_parent = parent._need(w_parent, parent._real_shape(), parent.real_dtype, "w_parent")
    w_child = child._need(w_child, child._real_shape(), child.real_dtype, "w_child")
    psi = child._need(psi, (3,) + child._real_shape(), child.real_dtype, "psi")
    if work is None:
        work = child.workspace()
    _check(lib().gg_increase_resolution(parent._h, child._h, _ptr(w_parent), REFINE_VARIANTS[variant], int(seed),
                                        int(stream_id), 0.0 if r_s is None else float(r_s), _ptr(w_child), _ptr(psi),
                                        _ptr(work), _stream()))
    return w_child, psi


class MakeIC(torch.autograd.Function):
    """Differentiable noise -> (positions, velocities, displacements).

    forward(w, log_amp, plan): w is the white noise (N^3, path dtype),
    log_amp a 0-d tensor shifting ln A (displacements scale as exp(log_amp/2)).
    backward runs the library's adjoint passes (nothing but the forward's
    displacements is kept between the two).
    """

    @staticmethod
    def forward(ctx, w, log_amp, plan):
        scale = float(torch.exp(0.5 * log_amp.detach().double()))
        pos, vel, psi = plan.make_ic_from_noise(w.detach().contiguous(), scale, want_psi=True)
        ctx.plan = plan
        ctx.scale = scale
        ctx.log_amp_dtype = log_amp.dtype
        ctx.set_materialize_grads(False)  # unused outputs pass None, not zeros
        ctx.save_for_backward(psi)
        return pos, vel, psi

    @staticmethod
    def backward(ctx, g_pos, g_vel, g_psi):
        (psi,) = ctx.saved_tensors
        plan = ctx.plan
        if g_pos is None and g_vel is None and g_psi is None:
            return None, None, None
        f = lambda t, dt: None if t is None else t.to(dt).contiguous()
        g_w, g_la = plan.make_ic_adjoint(g_psi=f(g_psi, plan.real_dtype), g_pos=f(g_pos, torch.float32),
                                         g_vel=f(g_vel, torch.float32), amp_scale=ctx.scale, psi=psi,
                                         want_log_amp=True)
        return g_w, g_la.reshape(()).to(ctx.log_amp_dtype), None


def make_ic_autograd(plan, w, log_amp=None):
    """(pos, vel, psi) = MakeIC(w, log_amp); log_amp defaults to 0."""
    if log_amp is None:
        log_amp = torch.zeros((), dtype=torch.float64, device=w.device)
    return MakeIC.apply(w, log_amp, plan)
