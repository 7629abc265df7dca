"""GPU parity of the differentiable path: gg_make_ic_from_noise and
gg_make_ic_adjoint (through the C ABI and the autograd Function) against the
oracle's gradients.

Bars: FP64 1e-12 relative r.m.s., FP32 2e-6 relative r.m.s. against the
oracle fed the same inputs; the dot-product identity <L W, g> = <W, L^T g>
to the same bars; central finite differences of the weighted loss on the FP64
path (the loss is quadratic in W, so the difference is exact up to rounding).
"""
import numpy as np
import pytest
import torch

import paper_2511_10353_amd as gg
from oracle import adjoint as oadj
from oracle import cosmology as ocosmo
from oracle import pipeline as opipe
from tests import inputs
from tests.gpu_util import oracle_cosmo, oracle_ic, rel_rms, say

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-6, "f64": 1e-12}
NPDT = {"f32": np.float32, "f64": np.float64}


def _plan(n, box, dtype):
    say(f"[plan] n={n} box={box} dtype={dtype}")
    return gg.Plan(n, box, gg.Cosmo(), dtype=dtype)


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype,n", [("f64", 32), ("f32", 64), ("f32", 256), ("f64", 256)])
def test_from_noise_of_generated_noise_is_make_ic(dtype, n):
    box = 100.0 * n / 32
    p = _plan(n, box, dtype)
    pos0, vel0, psi0 = p.make_ic(42, want_psi=True)
    w = p.noise(42)
    pos1, vel1, psi1 = p.make_ic_from_noise(w, 1.0, want_psi=True)
    torch.cuda.synchronize()
    assert torch.equal(psi0, psi1)
    assert torch.equal(pos0, pos1)
    assert torch.equal(vel0, vel1)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [16, 128])
def test_from_noise_amp_scale_against_oracle(dtype, n):
    box = 6.25 * n
    p = _plan(n, box, dtype)
    w = inputs.real_field(n, 100 + n, NPDT[dtype])
    scale = 1.3
    psi = _host(p.make_ic_from_noise(_dev(w, p.real_dtype), scale, particles=False))
    c = oracle_cosmo(p.cosmo)
    want = np.stack(opipe.displacement_fields(w.astype(np.float64), n, box, c, amp=ocosmo.amplitude(c) * scale ** 2,
                                              workers=8))
    for j in range(3):
        err = rel_rms(psi[j], want[j])
        say(f"[from_noise] n={n} {dtype} comp {j} rel rms {err:.3e}")
        assert err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 32, 128])
def test_adjoint_of_psi_gradient_against_oracle(dtype, n):
    box = 3.125 * n
    p = _plan(n, box, dtype)
    g = np.stack([inputs.real_field(n, 200 + j, NPDT[dtype]) for j in range(3)])
    scale = 0.7
    gw = _host(p.make_ic_adjoint(g_psi=_dev(g, p.real_dtype), amp_scale=scale))
    want = oadj.noise_gradient(g.astype(np.float64), n, box, oracle_cosmo(p.cosmo), amp_scale=scale)
    err = rel_rms(gw, want)
    say(f"[adjoint psi] n={n} {dtype} rel rms {err:.3e}")
    assert err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_adjoint_of_particle_gradients_against_oracle(dtype):
    n, box = 64, 300.0
    p = _plan(n, box, dtype)
    c = oracle_cosmo(p.cosmo)
    gp = np.stack([inputs.real_field(n, 300 + j, np.float32) for j in range(3)])
    gv = np.stack([inputs.real_field(n, 310 + j, np.float32) for j in range(3)]) * np.float32(1e-3)
    gs = np.stack([inputs.real_field(n, 320 + j, NPDT[dtype]) for j in range(3)])
    cases = [
        (dict(g_pos=gp), dict(g_pos=gp)),
        (dict(g_vel=gv), dict(g_vel=gv)),
        (dict(g_psi=gs, g_pos=gp, g_vel=gv), dict(g_psi=gs, g_pos=gp, g_vel=gv)),
    ]
    for dev_args, ora_args in cases:
        kw = {k: _dev(v, p.real_dtype if k == "g_psi" else torch.float32) for k, v in dev_args.items()}
        gw = _host(p.make_ic_adjoint(**kw))
        want = oadj.noise_gradient(oadj.combine(cosmo=c, **ora_args), n, box, c)
        err = rel_rms(gw, want)
        say(f"[adjoint particles] {dtype} {sorted(dev_args)} rel rms {err:.3e}")
        assert err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_log_amp_gradient_against_oracle(dtype):
    n, box = 64, 300.0
    p = _plan(n, box, dtype)
    c = oracle_cosmo(p.cosmo)
    psi = np.stack([inputs.real_field(n, 400 + j, NPDT[dtype]) for j in range(3)])
    gs = np.stack([inputs.real_field(n, 410 + j, NPDT[dtype]) for j in range(3)])
    gv = np.stack([inputs.real_field(n, 420 + j, np.float32) for j in range(3)])
    gw, gla = p.make_ic_adjoint(g_psi=_dev(gs, p.real_dtype), g_vel=_dev(gv, torch.float32),
                                psi=_dev(psi, p.real_dtype), want_log_amp=True)
    want = oadj.log_amp_gradient(oadj.combine(g_psi=gs, g_vel=gv, cosmo=c), psi)
    got = float(gla.item())
    say(f"[log A] {dtype} got {got!r} want {want!r}")
    assert abs(got - want) <= 1e-11 * np.sum(np.abs(oadj.combine(g_psi=gs, g_vel=gv, cosmo=c) * psi))


def _dot(a, b):
    """sum a*b in float64, one axis-0 slab block at a time (bounded temporaries)."""
    total = 0.0
    step = max(1, a.shape[0] // 8)
    for i in range(0, a.shape[0], step):
        total += float((a[i:i + step].double() * b[i:i + step].double()).sum())
    return total


@pytest.mark.parametrize("dtype,n", [("f64", 64), ("f32", 64), ("f32", 1024)])
def test_dot_product_identity(dtype, n):
    # <L W, g> = <W, L^T g> at any size; at 1024^3 this is the check that
    # runs in the launch configuration of the full-size workload
    box = 2000.0 * n / 1024
    p = _plan(n, box, dtype)
    w = p.noise(7)
    psi = p.make_ic_from_noise(w, 1.0, particles=False)
    g = torch.empty_like(psi)
    g.copy_(p.noise(8).unsqueeze(0).expand(3, -1, -1, -1))
    g[1].mul_(-0.5)
    g[2] = torch.roll(g[2], shifts=1, dims=0)
    gw = p.make_ic_adjoint(g_psi=g)
    lhs = sum(_dot(psi[j], g[j]) for j in range(3))
    rhs = _dot(w, gw)
    norm = float(np.sqrt(sum(_dot(psi[j], psi[j]) for j in range(3)) * sum(_dot(g[j], g[j]) for j in range(3))))
    say(f"[dot] n={n} {dtype} lhs {lhs:.15e} rhs {rhs:.15e} rel {abs(lhs - rhs) / norm:.3e}")
    assert abs(lhs - rhs) < (1e-12 if dtype == "f64" else 2e-6) * norm
    del psi, g, gw, w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_adjoint_is_minus_forward(dtype):
    # each L_j is odd: the gradient of <g, psi_j> is -L_j g
    n, box = 128, 400.0
    p = _plan(n, box, dtype)
    g = p.noise(11)
    for j in range(3):
        gp = torch.zeros((3, n, n, n), dtype=p.real_dtype, device="cuda")
        gp[j] = g
        gw = p.make_ic_adjoint(g_psi=gp)
        fwd = p.make_ic_from_noise(g, 1.0, particles=False)[j]
        err = rel_rms(_host(gw), -_host(fwd))
        say(f"[odd] {dtype} comp {j} rel rms {err:.3e}")
        assert err < (1e-13 if dtype == "f64" else 1e-6)


def _loss(psi, cells, weights):
    q = psi.reshape(3, -1)[:, cells].double()
    return (weights * (q * q).sum(0)).sum()


@pytest.fixture(scope="module")
def weighted_cells():
    n = 256
    cells = inputs.cell_sample(n, 4096, 42)
    weights = np.random.default_rng(42).uniform(0.0, 1.0, cells.size)
    return n, cells, weights


def test_weighted_loss_gradient_fp32_against_oracle(weighted_cells):
    # the differentiable workload: 256^3 FP32, loss sum_i w_i |psi(c_i)|^2 over
    # 4096 cells, gradients with respect to W (float32) and log A
    n, cells, weights = weighted_cells
    box = 500.0
    p = _plan(n, box, "f32")
    w = p.noise(42).requires_grad_(True)
    log_amp = torch.zeros((), dtype=torch.float64, device="cuda", requires_grad=True)
    pos, vel, psi = gg.make_ic_autograd(p, w, log_amp)
    cl = torch.from_numpy(cells).cuda()
    wl = torch.from_numpy(weights).cuda()
    loss = _loss(psi, cl, wl)
    loss.backward()
    gw = _host(w.grad)
    gla = float(log_amp.grad)
    c = oracle_cosmo(p.cosmo)
    _, _, psi_o = oracle_ic(n, box, 42, "f32")
    loss_o = oadj.weighted_loss(psi_o, cells, weights)
    want = oadj.noise_gradient(oadj.weighted_loss_grad(psi_o, cells, weights), n, box, c)
    err = rel_rms(gw, want)
    say(f"[cfg grad] loss {loss.item():.9e} oracle {loss_o:.9e}; dW rel rms {err:.3e}; dlogA {gla:.9e}")
    assert abs(loss.item() / loss_o - 1) < 2e-6
    assert err < TOL["f32"]
    assert abs(gla / loss_o - 1) < 2e-6  # dl/dlog A = l for a loss quadratic in psi
    assert pos.dtype == torch.float32 and vel.dtype == torch.float32


def test_weighted_loss_finite_differences_fp64(weighted_cells):
    n, cells, weights = weighted_cells
    box = 500.0
    p = _plan(n, box, "f64")
    w = p.noise(42)
    cl = torch.from_numpy(cells).cuda()
    wl = torch.from_numpy(weights).cuda()
    psi = p.make_ic_from_noise(w, 1.0, particles=False)
    loss0 = float(_loss(psi, cl, wl))
    g = torch.zeros_like(psi)
    q = psi.reshape(3, -1)[:, cl]
    g.reshape(3, -1)[:, cl] = 2.0 * wl * q
    gw, gla = p.make_ic_adjoint(g_psi=g, psi=psi, want_log_amp=True)
    gmax = float(gw.abs().max())
    eps = 1e-3
    probe = inputs.cell_sample(n, 64, 43)
    wf = w.reshape(-1)
    work = p.workspace()
    worst = 0.0
    for c in probe:
        v = float(wf[c])
        wf[c] = v + eps
        up = float(_loss(p.make_ic_from_noise(w, 1.0, psi=psi, work=work, particles=False), cl, wl))
        wf[c] = v - eps
        dn = float(_loss(p.make_ic_from_noise(w, 1.0, psi=psi, work=work, particles=False), cl, wl))
        wf[c] = v
        fd = (up - dn) / (2 * eps)
        worst = max(worst, abs(fd - float(gw.reshape(-1)[c])) / gmax)
    say(f"[fd] max |fd - grad| / max|grad| = {worst:.3e} over {probe.size} cells (eps {eps})")
    assert worst < 1e-6
    h = 1e-3
    up = float(_loss(p.make_ic_from_noise(w, float(np.exp(h / 2)), particles=False), cl, wl))
    dn = float(_loss(p.make_ic_from_noise(w, float(np.exp(-h / 2)), particles=False), cl, wl))
    fd = (up - dn) / (2 * h)
    say(f"[fd logA] fd {fd:.12e} adjoint {float(gla):.12e} loss {loss0:.12e}")
    assert abs(fd / float(gla) - 1) < 1e-6
    assert abs(float(gla) / loss0 - 1) < 1e-12


def test_autograd_through_particles_against_oracle():
    n, box = 64, 300.0
    p = _plan(n, box, "f64")
    c = oracle_cosmo(p.cosmo)
    a = inputs.real_field(n, 500, np.float32)
    b = inputs.real_field(n, 501, np.float32)
    w = torch.from_numpy(inputs.real_field(n, 502)).cuda().requires_grad_(True)
    pos, vel, psi = gg.make_ic_autograd(p, w)
    ta = _dev(np.stack([a, -a, 2 * a]), torch.float32)
    tb = _dev(np.stack([b, b, -b]), torch.float32)
    ((ta.double() * pos.double()).sum() + (tb.double() * vel.double()).sum()).backward()
    want = oadj.noise_gradient(oadj.combine(g_pos=_host(ta), g_vel=_host(tb), cosmo=c), n, box, c)
    err = rel_rms(_host(w.grad), want)
    say(f"[autograd particles] rel rms {err:.3e}")
    assert err < TOL["f64"]


def test_adjoint_rejects_bad_arguments():
    p = _plan(16, 50.0, "f32")
    g = torch.zeros((3, 16, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(gg.GGError):
        p.make_ic_adjoint()
    with pytest.raises(gg.GGError):
        p.make_ic_adjoint(g_psi=g, want_log_amp=True)  # needs psi
    with pytest.raises(gg.GGError):
        p.make_ic_adjoint(g_psi=g, amp_scale=0.0)
    with pytest.raises(gg.GGError):
        p.make_ic_from_noise(torch.zeros((16, 16, 16), device="cuda"), -1.0)
