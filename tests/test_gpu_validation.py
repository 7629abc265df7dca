"""Argument validation on the GPU: every entry point that takes device
buffers rejects a misaligned one with GG_ERR_INVALID_ARG before launching
anything, and accepts the same call with aligned buffers.

Each buffer is its own 1 MiB allocation (far more than the 16^3 lattice
needs), and the misaligned pointer is that allocation's start + 4 bytes, so
even a launch that got through would stay inside its buffer."""
import ctypes

import pytest
import torch

import paper_2511_10353_amd as gg
from paper_2511_10353_amd import binding
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

VP = ctypes.c_void_p
MIB = 1 << 20
N = 16


@pytest.fixture(scope="module")
def env():
    plan = gg.Plan(N, 50.0, gg.Cosmo(), dtype="f32")
    child = gg.Plan(2 * N, 50.0, gg.Cosmo(), dtype="f32")
    bufs = [torch.zeros(MIB, dtype=torch.uint8, device="cuda") for _ in range(8)]
    yield plan, child, bufs
    plan.close()
    child.close()


def _calls(plan, child):
    """(name, function, argument builder, indices of device-buffer arguments,
    required alignment of each); the builder takes the list of buffer
    pointers to use."""
    lib = binding.lib()
    h, hc = plan._h, child._h
    s = VP(torch.cuda.current_stream().cuda_stream)
    o3 = (ctypes.c_int32 * 3)(1, 2, 3)
    sh = (ctypes.c_double * 3)(0.5, 0.5, 0.5)
    org = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    A = 256
    return [
        ("gg_noise", lambda b: lib.gg_noise(h, 42, 0, b[0], s), [A]),
        ("gg_fft3d+", lambda b: lib.gg_fft3d(h, 1, b[0], b[1], None, s), [A, A]),
        ("gg_fft3d-", lambda b: lib.gg_fft3d(h, -1, b[0], b[1], b[2], s), [A, A, A]),
        ("gg_filter", lambda b: lib.gg_filter(h, b[0], b[1], b[2], s), [A, A, A]),
        ("gg_zeldovich", lambda b: lib.gg_zeldovich(h, b[0], b[1], b[2], s), [A, A, A]),
        ("gg_make_ic", lambda b: lib.gg_make_ic(h, 42, b[0], b[1], b[2], b[3], s), [A, A, A, A]),
        ("gg_make_ic_from_noise", lambda b: lib.gg_make_ic_from_noise(h, b[0], 1.0, b[1], b[2], b[3], b[4], s),
         [A] * 5),
        ("gg_make_ic_adjoint", lambda b: lib.gg_make_ic_adjoint(h, b[0], b[1], b[2], 1.0, b[3], b[4], b[5], b[6], s),
         [A, A, A, A, 8, A, A]),
        ("gg_make_density", lambda b: lib.gg_make_density(h, 42, b[0], b[1], b[2], s), [A, A, A]),
        ("gg_power_spectrum", lambda b: lib.gg_power_spectrum(h, b[0], 8, b[1], b[2], b[3], b[4], s),
         [A, 8, 8, 8, A]),
        ("gg_field_stats", lambda b: lib.gg_field_stats(h, b[0], b[1], b[2], s), [A, 8, A]),
        ("gg_make_displacements", lambda b: lib.gg_make_displacements(h, b[0], 3, 0, 0, b[1], b[2], s), [A, A, A]),
        ("gg_lowpass", lambda b: lib.gg_lowpass(h, b[0], 9, 1, b[1], b[2], s), [A, A, A]),
        ("gg_degrade", lambda b: lib.gg_degrade(h, b[0], 2, sh, b[1], b[2], s), [A, A, A]),
        ("gg_zeldovich_at", lambda b: lib.gg_zeldovich_at(h, b[0], org, 100.0, b[1], b[2], s), [A, A, A]),
        ("gg_increase_resolution",
         lambda b: lib.gg_increase_resolution(h, hc, b[0], 2, 7, 1, 0.0, b[1], b[2], b[3], s), [A, A, A, A]),
        ("gg_refine_noise", lambda b: lib.gg_refine_noise(N, 0, 2, b[0], 7, 1, b[1], s), [A, A]),
        ("gg_refine_noise_region", lambda b: lib.gg_refine_noise_region(N, o3, 8, 0, 2, b[0], 7, 1, b[1], s), [A, A]),
        ("gg_interpolate_add", lambda b: lib.gg_interpolate_add(N, 2 * N, 0, b[0], b[1], s), [A, A]),
        ("gg_interpolate_add_at", lambda b: lib.gg_interpolate_add_at(N, 2, o3, N, 0, b[0], b[1], s), [A, A]),
    ]


@pytest.mark.parametrize("idx", range(20))
def test_misaligned_buffers_rejected(env, idx):
    plan, child, bufs = env
    name, call, aligns = _calls(plan, child)[idx]
    good = [VP(t.data_ptr()) for t in bufs[:len(aligns)]]
    assert all(p.value % 256 == 0 for p in good)
    for k, a in enumerate(aligns):
        args = list(good)
        args[k] = VP(good[k].value + 4)  # 4 bytes off: breaks both the 256- and the 8-byte rule
        say(f"[validation] {name}: argument {k} misaligned")
        st = call(args)
        assert st == binding.GG_ERR_INVALID_ARG, (name, k, st)
        assert "align" in binding.lib().gg_last_error().decode()
    say(f"[validation] {name}: aligned call")
    assert call(good) == 0, binding.lib().gg_last_error().decode()
    torch.cuda.synchronize()
