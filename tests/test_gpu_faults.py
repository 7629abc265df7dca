"""Error paths forced from the host (GG_FAULT_INJECT): an allocation failure in
plan creation and a failed launch surface as status codes, leave nothing
behind, and the next call works."""
import pytest
import torch

import paper_2511_10353_amd as gg
from paper_2511_10353_amd import binding

pytestmark = pytest.mark.gpu


def test_plan_allocation_failure_is_out_of_memory(monkeypatch):
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    monkeypatch.setenv("GG_FAULT_INJECT", "plan_alloc")
    for dtype in ("f32", "f64"):
        with pytest.raises(gg.GGError) as err:
            gg.Plan(64, 100.0, gg.Cosmo(), dtype=dtype)
        assert err.value.status == binding.GG_ERR_OUT_OF_MEMORY
    monkeypatch.delenv("GG_FAULT_INJECT")
    torch.cuda.synchronize()
    # the tables allocated before the failing one were released
    assert torch.cuda.mem_get_info()[0] >= before - (64 << 20)
    p = gg.Plan(64, 100.0, gg.Cosmo(), dtype="f32")
    pos, vel = p.make_ic(1)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(pos).all())


def test_failed_launch_is_a_hip_error(monkeypatch):
    p = gg.Plan(32, 100.0, gg.Cosmo(), dtype="f32")
    ref = p.make_ic(3)
    torch.cuda.synchronize()
    monkeypatch.setenv("GG_FAULT_INJECT", "launch")
    with pytest.raises(gg.GGError) as err:
        p.make_ic(3)
    assert err.value.status == binding.GG_ERR_HIP
    monkeypatch.delenv("GG_FAULT_INJECT")
    again = p.make_ic(3)
    torch.cuda.synchronize()
    assert torch.equal(again[0], ref[0]) and torch.equal(again[1], ref[1])
