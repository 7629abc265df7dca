"""GPU parity of the diagnostics: density field (Eq. 1 alone), binned power
spectrum and field statistics, against the FP64 oracle.

Bars: density FP64 1e-12 / FP32 2e-6 relative r.m.s.; power spectrum counts
exact, kmean 1e-13, P_b 1e-12 (FP64) / 2e-6 (FP32, transform in float)
relative per bin; statistics: min and max exact, mean and standard deviation
1e-12 relative to the standard deviation.
"""
import math

import numpy as np
import pytest
import torch

import paper_2511_10353_amd as gg
from oracle import cosmology as ocosmo
from oracle import pipeline as opipe
from oracle import stats as ostats
from tests import inputs
from tests.gpu_util import oracle_cosmo, oracle_noise, rel_rms, say

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-6, "f64": 1e-12}
NPDT = {"f32": np.float32, "f64": np.float64}
TDT = {"f32": torch.float32, "f64": torch.float64}


def _plan(n, box, dtype):
    say(f"[plan] n={n} box={box} dtype={dtype}")
    return gg.Plan(n, box, gg.Cosmo(), dtype=dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 32, 128])
def test_density_from_seed_against_oracle(dtype, n):
    box = 3.125 * n
    p = _plan(n, box, dtype)
    d = p.make_density(42).cpu().numpy()
    w = oracle_noise(n, 42, dtype)
    want = opipe.density_field(w.astype(np.float64), n, box, oracle_cosmo(p.cosmo), workers=8)
    err = rel_rms(d, want)
    say(f"[density] n={n} {dtype} rel rms {err:.3e}")
    assert err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_density_from_field_equals_seed_path(dtype):
    n, box = 64, 200.0
    p = _plan(n, box, dtype)
    for seed in (7, 2**64 - 1):
        # the first pass's own noise equals gg_noise's, bit for bit
        a = p.make_density(seed)
        b = p.make_density(w=p.noise(seed))
        torch.cuda.synchronize()
        assert torch.equal(a, b), seed


def test_density_is_minus_divergence_of_displacements():
    # spectral check on the GPU outputs: div psi = -delta (Eq. 2)
    n, box = 64, 150.0
    p = _plan(n, box, "f64")
    d = p.make_density(5).cpu().numpy()
    _, _, psi = p.make_ic(5, want_psi=True)
    psi = psi.cpu().numpy()
    kf = 2 * np.pi / box
    ks = kf * opipe.signed_index(n).astype(np.float64)
    ks[n // 2] = 0.0  # Nyquist modes are zero in both fields
    kz = kf * np.arange(n // 2 + 1, dtype=np.float64)
    kz[n // 2] = 0.0
    div = 1j * (ks.reshape(n, 1, 1) * opipe.forward(psi[0]) + ks.reshape(1, n, 1) * opipe.forward(psi[1]) +
                kz.reshape(1, 1, n // 2 + 1) * opipe.forward(psi[2]))
    err = rel_rms(opipe.inverse(div, n), -d)
    say(f"[div] rel rms {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,nbins", [(8, 8), (32, 28), (128, 100), (64, 1024), (256, 200)])
def test_power_spectrum_against_oracle(dtype, n, nbins):
    box = 7.0 * n
    p = _plan(n, box, dtype)
    f = inputs.real_field(n, 600 + n, NPDT[dtype])
    pk, km, ct = [t.cpu().numpy() for t in p.power_spectrum(torch.from_numpy(f).cuda(), nbins)]
    wpk, wkm, wct = ostats.power_spectrum(f.astype(np.float64), box, nbins)
    assert np.array_equal(ct, wct)
    nz = wct > 0
    # binary64 sums of up to ~10^7 terms per bin, in another order than numpy's
    assert np.abs(km[nz] / wkm[nz] - 1).max() < 1e-12
    rel = np.abs(pk[nz] / wpk[nz] - 1)
    say(f"[pk] n={n} {dtype} max rel {rel.max():.3e}")
    assert rel.max() < TOL[dtype]


def test_power_spectrum_deterministic_and_validated():
    n, box = 64, 100.0
    p = _plan(n, box, "f32")
    f = p.noise(3)
    a = torch.stack(p.power_spectrum(f, 40))
    b = torch.stack(p.power_spectrum(f, 40))
    assert torch.equal(a, b)
    for bad in (0, 1025):
        with pytest.raises(gg.GGError):
            p.power_spectrum(f, bad)


def test_density_power_spectrum_recovers_input_spectrum():
    # Eq. (1) normalisation measured on the GPU: the binned P(k) of the density
    # field at 256^3 (box 500) averages the analytic P(k) within 5 sigma per bin
    n, box, nbins = 256, 500.0, 64
    p = _plan(n, box, "f32")
    c = oracle_cosmo(p.cosmo)
    acc = np.zeros(nbins)
    nseed = 4
    for sd in range(nseed):
        pk, km, ct = p.power_spectrum(p.make_density(100 + sd), nbins)
        acc += pk.cpu().numpy()
    acc /= nseed
    ct = ct.cpu().numpy()
    b, kn, w, n2 = ostats.mode_bins(n)
    worst = 0.0
    for bb in range(2, nbins):
        sel = (b == bb) & (n2 > 0) & (np.abs(opipe.signed_index(n)).reshape(n, 1, 1) != n // 2)
        sel &= (np.abs(opipe.signed_index(n)).reshape(1, n, 1) != n // 2) & (np.arange(n // 2 + 1) != n // 2)
        pw = ocosmo.power(kn[sel] * 2 * math.pi / box, c)
        expect = float(np.sum(w[sel] * pw) / ct[bb])  # Nyquist modes are zero but counted
        sigma = expect / math.sqrt(ct[bb] * nseed / 2)
        worst = max(worst, abs(acc[bb] - expect) / sigma)
    say(f"[pk recovery] worst deviation {worst:.2f} sigma")
    assert worst < 5


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_field_stats_against_oracle(dtype):
    n, box = 128, 400.0
    p = _plan(n, box, dtype)
    f = inputs.real_field(n, 77, NPDT[dtype]) * NPDT[dtype](0.3) + NPDT[dtype](1.25)
    got = p.field_stats(torch.from_numpy(f).cuda()).cpu().numpy()
    mean, sd, lo, hi = ostats.field_stats(f.astype(np.float64))
    say(f"[stats] {dtype} {got} vs {(mean, sd, lo, hi)}")
    assert got[2] == lo and got[3] == hi
    assert abs(got[0] - mean) < 1e-12 * sd and abs(got[1] - sd) < 1e-12 * sd


def test_field_stats_of_the_ic_displacements():
    # rms of psi per component at 256^3 / 500 Mpc/h (about 0.05 Mpc/h)
    n, box = 256, 500.0
    p = _plan(n, box, "f32")
    _, _, psi = p.make_ic(42, want_psi=True)
    for j in range(3):
        st = p.field_stats(psi[j]).cpu().numpy()
        say(f"[psi stats] comp {j}: mean {st[0]:.3e} std {st[1]:.4f} min {st[2]:.4f} max {st[3]:.4f}")
        assert abs(st[0]) < 1e-6 * st[1] * n ** 1.5 and 0.02 < st[1] < 0.1
