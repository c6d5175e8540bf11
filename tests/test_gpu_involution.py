"""The paper's benchmark protocol as a test (Section 4: every run composes 12
transposes of one dataset; Section 3: the transpose is an involution).

Twelve transposes are composed on device-resident ping-pong buffers, each
call reading the previous call's outputs. The generator emits rows in column
order (the canonical form), so T^12(A) must equal A exactly; T^1 and T^11 must
both equal the oracle's T(A), element by element.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

from .common import to_device

pytestmark = pytest.mark.gpu


def _arrays(x):
    return {"row_ptr": x.row_ptr, "col": x.col, "payload_off": x.payload_off,
            "payload": x.payload}


@pytest.mark.parametrize("perm_plan", [False, True], ids=["packed", "wide"])
def test_twelve_composed_transposes(perm_plan):
    from paper_2012_06012_amd import mgt
    a = gen.large(seed=3, scale=5)  # 2^18 x 2^18, 2^24 cells
    ref = oracle.transpose(a)
    d = to_device(a)
    orig = {k: v.clone() for k, v in _arrays(d).items()}
    # two partition passes and a gathering finish (the benchmark's path);
    # the wide form carries the cell index, which perm needs
    plan = mgt.plan_for(d, mgt.EMIT_PERM if perm_plan else 0)
    plan.set_schedule(8, 7, 0)
    assert plan.schedule()["passes"] == 2, plan.schedule()
    ws = mgt.workspace_for(plan, d.col.device)
    bufs = [mgt.alloc_outputs(d, perm=perm_plan), mgt.alloc_outputs(d, perm=perm_plan)]
    status = torch.empty(1, dtype=torch.int32, device=d.col.device)
    x = d
    seen = {}
    for i in range(1, 13):
        o = bufs[(i - 1) & 1]
        mgt.transpose(x, plan=plan, workspace=ws, out=o, perm=perm_plan, status=status)
        torch.cuda.synchronize()
        assert int(status.cpu()[0]) == mgt.OK, i
        x = mgt.DeviceCsr(x.n_cols, x.n_rows, o["t_row_ptr"], o["t_col"], o["t_payload_off"],
                          o["t_payload"], x.bounds, x.offset_width)
        if i in (1, 11):
            seen[i] = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
    for i in (1, 11):
        h = seen[i]
        assert np.array_equal(h["t_row_ptr"], ref.t_row_ptr), i
        assert np.array_equal(h["t_col"], ref.t_col), i
        assert np.array_equal(h["t_payload_off"], ref.t_payload_off), i
        assert np.array_equal(h["t_payload"], ref.t_payload), i
        if perm_plan:  # T^11 reads T^10(A) = A, so its perm is T(A)'s as well
            assert np.array_equal(h["perm"].view(np.uint32), ref.perm), i
    for k, v in _arrays(x).items():
        assert torch.equal(v, orig[k]), f"T^12(A) differs from A in {k}"
