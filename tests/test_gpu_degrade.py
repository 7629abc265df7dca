"""GPU parity of the resolution degrade (Sec. 2.3: nearest-grid-point values
on the coarse lattice, then a Fourier translation) against the FP64 oracle.

Bars: FP64 1e-12, FP32 2e-6 relative r.m.s.; the decimation alone (shift 0)
within the same bars (it passes through a forward and an inverse transform).
"""
import numpy as np
import pytest
import torch

import paper_2511_10353_amd as gg
from oracle import degrade as odeg
from tests import inputs
from tests.gpu_util import rel_rms, say

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-6, "f64": 1e-12}
NPDT = {"f32": np.float32, "f64": np.float64}


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n_lo,factor", [(32, 2), (16, 4), (32, 3), (96, 2), (8, 1)])
@pytest.mark.parametrize("shift", [(0.5, 0.5, 0.5), (0.25, -0.5, 1.75), (0.0, 0.0, 0.0)])
def test_degrade_against_oracle(dtype, n_lo, factor, shift):
    fine = inputs.real_field(n_lo * factor, 11 + factor, NPDT[dtype])
    p = gg.Plan(n_lo, 100.0, gg.Cosmo(), dtype=dtype)
    got = p.degrade(torch.from_numpy(fine).cuda(), factor, shift).cpu().numpy()
    want = odeg.degrade(fine.astype(np.float64), factor, shift)
    err = rel_rms(got, want)
    say(f"[degrade] {dtype} {n_lo * factor}->{n_lo} shift {shift}: rel rms {err:.3e}")
    assert err < TOL[dtype]


def test_degrade_512_to_256_f32():
    fine = inputs.real_field(512, 21, np.float32)
    p = gg.Plan(256, 500.0, gg.Cosmo(), dtype="f32")
    got = p.degrade(torch.from_numpy(fine).cuda(), 2).cpu().numpy()
    want = odeg.degrade(fine.astype(np.float64), 2)
    err = rel_rms(got, want)
    say(f"[degrade] f32 512->256 rel rms {err:.3e}")
    assert err < TOL["f32"]


def test_unshifted_degrade_of_displacements_samples_the_fine_field():
    # a make_ic displacement field degraded without translation gives the
    # fine field's values at the coarse lattice points
    n_lo, factor = 32, 2
    p_hi = gg.Plan(n_lo * factor, 200.0, gg.Cosmo(), dtype="f64")
    _, _, psi = p_hi.make_ic(5, want_psi=True)
    p_lo = gg.Plan(n_lo, 200.0, gg.Cosmo(), dtype="f64")
    for j in range(3):
        got = p_lo.degrade(psi[j].contiguous(), factor, (0.0, 0.0, 0.0)).cpu().numpy()
        want = psi[j].cpu().numpy()[::factor, ::factor, ::factor]
        assert rel_rms(got, want) < 1e-12


def test_degrade_rejects_bad_arguments():
    import ctypes
    from paper_2511_10353_amd import binding
    p = gg.Plan(16, 100.0, gg.Cosmo(), dtype="f32")
    fine = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda")
    out = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    work = p.workspace()
    sh = (ctypes.c_double * 3)(0.5, 0.5, 0.5)
    for factor in (0, -2):  # straight to the C entry point: the library rejects it
        st = binding.lib().gg_degrade(p._h, fine.data_ptr(), factor, sh, out.data_ptr(), work.data_ptr(), None)
        assert st == 1
    st = binding.lib().gg_degrade(p._h, fine.data_ptr(), 2, sh, fine.data_ptr(), work.data_ptr(), None)
    assert st == 1  # out overlaps fine
    big = torch.zeros((16 * 17,) * 3, dtype=torch.float32, device="cuda")
    with pytest.raises(gg.GGError):
        p.degrade(big, 17)
    with pytest.raises(gg.GGError):
        p.degrade(fine, 2, (float("nan"), 0.0, 0.0))
    with pytest.raises(ValueError):
        p.degrade(fine, 3)  # wrong fine shape for the factor
