"""The persistent passes (P3 of float plans, P5) give the same bits whatever
their grid: with GG_CUS=1 a single P3 work-group and 16 P5 work-groups loop
over every tile (many tiles per work-group, the prefetch crossing line
blocks, column blocks and components), against the default grids.  The
lattices include uneven ones (96, 160, 192) whose tile counts leave a
ragged last round, and the FP64 path (its P5 is persistent too)."""
import os

import pytest
import torch

import paper_2511_10353_amd as gg
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _run(n, box, dtype, cus):
    old = os.environ.get("GG_CUS")
    if cus is None:
        os.environ.pop("GG_CUS", None)
    else:
        os.environ["GG_CUS"] = str(cus)
    try:
        p = gg.Plan(n, box, gg.Cosmo(), dtype=dtype)
    finally:
        if old is None:
            os.environ.pop("GG_CUS", None)
        else:
            os.environ["GG_CUS"] = old
    pos, vel, psi = p.make_ic(7, want_psi=True)
    torch.cuda.synchronize()
    out = [t.clone() for t in (pos, vel, psi)]
    p.close()
    return out


@pytest.mark.parametrize("n,box,dtype", [(64, 100.0, "f32"), (96, 150.0, "f32"), (192, 300.0, "f32"),
                                         (256, 500.0, "f32"), (160, 250.0, "f64"), (128, 200.0, "f64")])
@pytest.mark.parametrize("cus", [1, 3])
def test_persistent_grids_agree_bitwise(n, box, dtype, cus):
    ref = _run(n, box, dtype, None)
    got = _run(n, box, dtype, cus)
    say(f"[persistent] {dtype} {n}^3 GG_CUS={cus}")
    for name, a, b in zip(("pos", "vel", "psi"), got, ref):
        assert torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else a.view(torch.int64),
                           b.view(torch.int32) if b.dtype == torch.float32 else b.view(torch.int64)), name
