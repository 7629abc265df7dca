"""Parity at the measured size: the 1024^3 lattice (box 2000 Mpc/h) in the
launch configuration bench.py times (fused gg_make_ic, pipelined passes).

The float path against the double path over the whole grid, exact mean
removal, positions within one float32 ulp at the box scale; the fused path
against the stand-alone calls; both paths against the full FP64 oracle, on the
whole grid and on a periodic 128^3 sub-box (about two minutes on the host).
"""
import os

import numpy as np
import pytest
import torch

import paper_2511_10353_amd as gg
from tests import inputs
from tests.gpu_util import report, say

pytestmark = pytest.mark.gpu

N, BOX, SEED = 1024, 2000.0, 42


def _rel_rms_t(a, b):
    d = (a.double() - b.double()).pow(2).sum()
    return float(torch.sqrt(d / b.double().pow(2).sum()))


def test_float_noise_is_rounded_double_noise_at_1024():
    # the float path's noise is the binary64 deviate rounded once, for every
    # one of the 2^30 cells (its fast evaluation falls back to the defining
    # sequence near rounding boundaries; a wrong error bound would show here)
    say("[1024] noise f32 vs rounded f64, all cells")
    p64 = gg.Plan(N, BOX, gg.Cosmo(), dtype="f64")
    p32 = gg.Plan(N, BOX, gg.Cosmo(), dtype="f32")
    for seed, stream in ((SEED, 0), (7, 3)):
        w64 = p64.noise(seed, stream_id=stream)
        w32 = p32.noise(seed, stream_id=stream)
        bad = int((w64.float() != w32).sum())
        say(f"[1024] seed {seed} stream {stream}: {bad} mismatching cells")
        assert bad == 0
        del w64, w32
    p64.close()
    p32.close()
    torch.cuda.empty_cache()


def test_plain_transforms_at_1024():
    # the stand-alone r2c / c2r at 1024^3 (its axis-1 passes exchange inside
    # waves; the 513-column half spectrum ends in a ragged tile): sampled modes
    # against direct sums in float64 and the round trip over the whole field
    x = inputs.real_field(N, 31, np.float32)
    p = gg.Plan(N, BOX, gg.Cosmo(), dtype="f32")
    xd = torch.from_numpy(x).cuda()
    spec = p.fft3d(xd, 1)
    torch.cuda.synchronize()
    modes = [(0, 0, 0), (1, 2, 3), (1023, 511, 512), (512, 17, 256), (300, 1000, 511)]
    got = [complex(spec[k].item()) for k in modes]
    xf = x.reshape(N * N, N).astype(np.float64)
    m = np.arange(N)
    for k, g in zip(modes, got):
        e = [np.exp(-2j * np.pi * kk * m / N) for kk in k]
        t2 = xf @ e[2].real + 1j * (xf @ e[2].imag)  # axis 2 (real matrix, no complex copy of it)
        t1 = t2.reshape(N, N) @ e[1]         # axis 1
        want = t1 @ e[0]                     # axis 0
        rms = np.sqrt(N ** 3)                # |X| scale of unit white noise
        say(f"[1024 fft] mode {k}: |got - want| / sqrt(N^3) = {abs(g - want) / rms:.3e}")
        assert abs(g - want) < 2e-5 * rms
    del xf
    y = p.fft3d(spec, -1)
    torch.cuda.synchronize()
    err = _rel_rms_t(y, xd)
    say(f"[1024 fft] round trip rel rms {err:.3e}")
    assert err < 1e-6
    del spec, y, xd
    p.close()
    torch.cuda.empty_cache()


def test_launch_configurations_agree_bitwise_at_1024():
    # the benchmark's autotuned configuration (one chunk, 8-line first pass,
    # 16-line last pass) against the built-in one and a pipelined one
    p = gg.Plan(N, BOX, gg.Cosmo(), dtype="f32")
    ref = p.make_ic(SEED)
    torch.cuda.synchronize()
    for tuning in ((1, 8, 16), (4, 16, 8)):
        say(f"[1024] make_ic at tuning {tuning}")
        p.set_tuning(*tuning)
        got = p.make_ic(SEED)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), tuning
        del got
    del ref
    p.close()
    torch.cuda.empty_cache()


def test_fp32_matches_fp64_at_1024():
    say(f"[1024] FP64 make_ic")
    p64 = gg.Plan(N, BOX, gg.Cosmo(), dtype="f64")
    pos64, vel64, psi64 = p64.make_ic(SEED, want_psi=True)
    torch.cuda.synchronize()
    p64.close()
    torch.cuda.empty_cache()
    say("[1024] FP32 make_ic")
    p32 = gg.Plan(N, BOX, gg.Cosmo(), dtype="f32")
    pos32, vel32, psi32 = p32.make_ic(SEED, want_psi=True)
    torch.cuda.synchronize()
    for j in range(3):
        e = _rel_rms_t(psi32[j], psi64[j])
        ev = _rel_rms_t(vel32[j], vel64[j])
        rms = float(psi64[j].pow(2).mean().sqrt())
        mean64 = float(psi64[j].mean())
        d = (pos32[j].double() - pos64[j].double()).abs()
        dper = torch.minimum(d, BOX - d)
        say(f"[1024] j={j} psi rel_rms f32 vs f64 = {e:.3e}  vel {ev:.3e}  rms psi {rms:.4f} Mpc/h  "
            f"mean/rms {mean64 / rms:.2e}  max |dpos| {float(dper.max()):.3e}")
        assert e < 2e-6 and ev < 2e-6
        assert abs(mean64) < 1e-10 * rms
        assert float(dper.max()) <= float(np.spacing(np.float32(BOX)))
    assert float(pos32.min()) >= 0 and float(pos32.max()) < BOX
    del pos64, vel64, psi64, pos32, vel32, psi32
    torch.cuda.empty_cache()


def _oracle_noise(n, seed, dtype, workers, slabs=16):
    """The oracle's noise field, filled slab by slab (axis 0) with a line per slab."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import noise as onoise
    out = np.empty((n, n, n), dtype=dtype)
    flat = out.reshape(-1)
    per = n // slabs * n * n
    chunk = 1 << 22
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for s in range(slabs):
            def fill(a, s=s):
                b = min(a + chunk, (s + 1) * per)
                flat[a:b] = onoise.noise_cells(np.arange(a, b, dtype=np.uint64), seed, 0, dtype)
            list(ex.map(fill, range(s * per, (s + 1) * per, chunk)))
            say(f"[1024 oracle] noise slab {s + 1}/{slabs}")
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def test_1024_against_fp64_oracle():
    # The headline lattice against the FP64 oracle (Eq. 1-3): both GPU paths,
    # on the whole grid and on a periodic 128^3 sub-box.  The oracle's float
    # noise is its binary64 noise rounded once (its definition), so the
    # binary64 field is computed once.  Stage times of the oracle are printed
    # as the CPU reference at this size.
    import time
    from oracle import cosmology as ocosmo
    from oracle import pipeline as opipe
    workers = min(16, os.cpu_count() or 1)
    c = ocosmo.Cosmology()
    origin = inputs.subbox_origin(N, 42)
    idx = [np.arange(o, o + 128) % N for o in origin]
    say(f"[1024 oracle] host: {_cpu_model()}, os.cpu_count() = {os.cpu_count()}, workers = {workers}")
    t0 = time.perf_counter()
    w64 = _oracle_noise(N, SEED, np.float64, workers)
    t_noise = time.perf_counter() - t0
    results = {}
    for dtype in ("f64", "f32"):
        say(f"[1024 oracle] GPU {dtype}")
        p = gg.Plan(N, BOX, gg.Cosmo(), dtype=dtype)
        _, _, psi = p.make_ic(SEED, want_psi=True)
        torch.cuda.synchronize()
        p.close()
        w = w64 if dtype == "f64" else w64.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        w_hat = opipe.forward(w, workers=workers)
        t_fwd = time.perf_counter() - t0
        del w
        t0 = time.perf_counter()
        d_hat = opipe.density_spectrum(w_hat, N, BOX, c)
        del w_hat
        t_inv = 0.0
        for j in range(3):
            t1 = time.perf_counter()
            want = opipe.inverse(opipe.displacement_spectrum(d_hat, N, BOX, j), N, workers=workers)
            t_inv += time.perf_counter() - t1
            got = psi[j].cpu().numpy().astype(np.float64)
            full = float(np.linalg.norm(got - want) / np.linalg.norm(want))
            sb = np.ix_(*idx)
            sub = float(np.linalg.norm(got[sb] - want[sb]) / np.linalg.norm(want[sb]))
            results[(dtype, j)] = (full, sub)
            say(f"[1024 oracle] {dtype} j={j} rel_rms full grid {full:.3e}  128^3 sub-box at {origin} {sub:.3e}")
            del want, got
        if dtype == "f64":
            total = t_noise + t_fwd + t_inv
            report(f"FP64 oracle at 1024^3 on {_cpu_model()} ({workers} threads): noise {t_noise:.1f} s, forward r2c "
                   f"{t_fwd:.1f} s, filter + 3 inverse c2r {t_inv:.1f} s; {N ** 3 / total:.3e} cells/s without the "
                   f"particle step")
        del psi, d_hat
        torch.cuda.empty_cache()
    del w64
    for dtype in ("f64", "f32"):
        full = max(results[(dtype, j)][0] for j in range(3))
        sub = max(results[(dtype, j)][1] for j in range(3))
        report(f"1024^3 / 2000 Mpc/h {dtype} path vs FP64 oracle, psi rel_rms (worst component): full grid "
               f"{full:.3e}, 128^3 sub-box at {origin} {sub:.3e} (bar {1e-12 if dtype == 'f64' else 2e-6:g})")
    for (dtype, j), (full, sub) in results.items():
        bar = 1e-12 if dtype == "f64" else 2e-6
        assert full < bar and sub < bar


def test_fused_equals_standalone_chain_at_1024():
    # the fused path (blocked spectrum rows, in-wave exchanges, persistent
    # passes) against the stand-alone calls (public half-spectrum layout, plain
    # rows, their own kernels) over the whole 1024^3 float grid
    say("[1024] fused make_ic vs gg_noise + gg_fft3d + gg_filter + 3 gg_fft3d + gg_zeldovich, FP32")
    p = gg.Plan(N, BOX, gg.Cosmo(), dtype="f32")
    pos, vel, psi = p.make_ic(SEED, want_psi=True)
    torch.cuda.synchronize()
    w = p.noise(SEED)
    spec = p.fft3d(w, 1)
    del w
    psi_spec = p.filter(spec)
    del spec
    work = p.workspace()
    psi2 = torch.empty_like(psi)
    for j in range(3):
        psi2[j] = p.fft3d(psi_spec[j].contiguous(), -1, work=work)
    del psi_spec, work
    pos2, vel2 = p.zeldovich(psi2)
    torch.cuda.synchronize()
    worst = 0.0
    for j in range(3):
        e = _rel_rms_t(psi[j], psi2[j])
        ev = _rel_rms_t(vel[j], vel2[j])
        d = (pos[j].double() - pos2[j].double()).abs()
        dper = float(torch.minimum(d, BOX - d).max())
        say(f"[1024] j={j} fused vs stand-alone: psi rel_rms {e:.3e}  vel {ev:.3e}  max |dpos| {dper:.3e}")
        worst = max(worst, e)
        assert e < 1e-6 and ev < 1e-6
        assert dper <= float(np.spacing(np.float32(BOX)))
    report(f"1024^3 FP32 fused make_ic vs stand-alone calls: psi rel_rms {worst:.3e} (worst component)")
    del pos, vel, psi, pos2, vel2, psi2
    p.close()
    torch.cuda.empty_cache()
