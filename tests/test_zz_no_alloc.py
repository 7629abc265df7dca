"""gg_make_ic_noalloc (static device workspace, no allocation) against
gg_make_ic with a caller workspace: bit-identical positions, velocities and
displacements on two calls in a row, the second on a smaller lattice, so the
second call runs on the first one's leftover scratch contents."""
import ctypes

import pytest
import torch

import paper_2511_10353_amd as gg
from paper_2511_10353_amd import binding
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _noalloc_vs_workspace(n, box, dtype, seed):
    say(f"[noalloc] n={n} box={box} dtype={dtype} seed={seed}")
    p = gg.Plan(n, box, gg.Cosmo(), dtype=dtype)
    # the reference: a workspace filled with NaN bytes, so a read-before-write
    # of the workspace in either call would show up as a difference
    work = torch.full((p.workspace_bytes,), 0xFF, dtype=torch.uint8, device="cuda")
    want = p.make_ic(seed, work=work, want_psi=True)
    got = p.make_ic_noalloc(seed, want_psi=True)
    torch.cuda.synchronize()
    for a, b, name in zip(got, want, ("pos", "vel", "psi")):
        assert torch.equal(a, b), (n, dtype, name)
    p.close()


@pytest.mark.parametrize("dtype,sizes", [("f32", (160, 64)), ("f64", (128, 32))])
def test_noalloc_matches_make_ic_twice(dtype, sizes):
    big, small = sizes
    _noalloc_vs_workspace(big, 300.0, dtype, 42)
    _noalloc_vs_workspace(small, 100.0, dtype, 7)


def test_noalloc_rejects_lattices_beyond_the_scratch():
    for n, dtype in ((192, "f32"), (160, "f64")):
        p = gg.Plan(n, 300.0, gg.Cosmo(), dtype=dtype)
        assert p.workspace_bytes > (48 << 20)
        pos = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        vel = torch.empty_like(pos)
        st = binding.lib().gg_make_ic_noalloc(p._h, 1, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()),
                                              None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == binding.GG_ERR_UNSUPPORTED_SIZE
        assert "scratch" in binding.lib().gg_last_error().decode()
        p.close()
