"""GPU tests of mgt_transpose_noalloc, the transpose that allocates nothing
(its workspace is the library's own device array), through the C ABI.

Each case makes two calls in a row on the same device array, the second with
a smaller input, and checks every output array against the same call through
mgt_transpose / mgt_transpose_partitioned with a workspace of its own, and
against the oracle (bit for bit: the transpose is integer index work and byte
moves). Schedules of one, two (packed and wide records) and three passes are
forced so every kernel path runs on the array.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

from .common import to_device

pytestmark = pytest.mark.gpu

_KEYS = ("t_row_ptr", "t_col", "t_payload_off", "t_payload", "perm", "xfer_cells", "xfer_bytes",
         "part_cell_off", "part_byte_off", "sdispls", "rdispls")


def _noalloc(d, plan, partitioned, perm):
    from paper_2012_06012_amd import mgt
    out = mgt.alloc_outputs(d, perm=perm, partitioned=partitioned)
    for v in out.values():  # poison: every element must be written
        if v is not None:
            v.fill_(-7 if v.dtype != torch.uint8 else 0xA5)
    st = torch.full((1,), 12345, dtype=torch.int32, device=d.col.device)
    mgt.mgt_transpose_noalloc(plan, partitioned, d.row_ptr, d.col, d.payload_off, d.payload,
                              out["t_row_ptr"], out["t_col"], out["t_payload_off"],
                              out["t_payload"], out["perm"], out.get("xfer_cells"),
                              out.get("xfer_bytes"), out.get("part_cell_off"),
                              out.get("part_byte_off"), out.get("sdispls"), out.get("rdispls"),
                              d_status=st)
    torch.cuda.synchronize()
    return out, int(st.cpu()[0])


def _check(a, d, plan, partitioned, perm):
    from paper_2012_06012_amd import mgt
    assert plan.workspace_bytes <= mgt.NOALLOC_SCRATCH_BYTES, plan.workspace_bytes
    ref, st = mgt.transpose(d, plan=plan, perm=perm, partitioned=partitioned)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == mgt.OK
    out, st2 = _noalloc(d, plan, partitioned, perm)
    assert st2 == mgt.OK
    for k in _KEYS:
        if ref.get(k) is not None:
            assert torch.equal(out[k], ref[k]), k
    t = oracle.transpose(a)
    assert np.array_equal(out["t_col"].cpu().numpy(), t.t_col)
    assert np.array_equal(out["t_payload"].cpu().numpy(), t.t_payload)
    assert np.array_equal(out["t_payload_off"].cpu().numpy(), t.t_payload_off)
    if perm:
        assert np.array_equal(out["perm"].cpu().numpy().view(np.uint32), t.perm)


@pytest.mark.parametrize("sched", [None, (5, 4, 0), (4, 3, 0), (8, 4, 4096)],
                         ids=["rule", "2pass", "3pass", "slim12"])
@pytest.mark.parametrize("partitioned", [False, True], ids=["plain", "part"])
@pytest.mark.parametrize("perm", [False, True], ids=["noperm", "perm"])
def test_noalloc_equals_workspace_call(sched, partitioned, perm):
    from paper_2012_06012_amd import mgt
    # 2^14 x 2^14 with 2^20 cells (2^13 x 2^13 with 2^19 cells for three passes,
    # whose workspace is larger), R = 64; then 1,000 x 1,000 with about 2e4
    # cells, R = 4. slim12: 4,096-cell tiles, so the records-only pass runs in
    # its slim form and, without perm, writes 12-byte records
    big = gen.large(seed=1, scale=10 if sched == (4, 3, 0) else 9)
    small = gen.tiny(seed=2)
    for a in (big, small):             # the second call is the smaller one
        d = to_device(a)
        plan = mgt.plan_for(d, mgt.EMIT_PERM if perm else 0)
        if sched and a is big:
            plan.set_schedule(*sched)
            assert plan.schedule(partitioned)["passes"] >= 2
        _check(a, d, plan, partitioned, perm)


def test_noalloc_refuses_oversize_and_timing_plans():
    from paper_2012_06012_amd import mgt
    a = gen.large(seed=0, scale=6)     # 2^23 cells: about 280 MB of workspace
    d = to_device(a)
    plan = mgt.plan_for(d)
    assert plan.workspace_bytes > mgt.NOALLOC_SCRATCH_BYTES
    out = mgt.alloc_outputs(d)
    with pytest.raises(mgt.MgtError) as e:
        mgt.mgt_transpose_noalloc(plan, False, d.row_ptr, d.col, d.payload_off, d.payload,
                                  out["t_row_ptr"], out["t_col"], out["t_payload_off"],
                                  out["t_payload"], None)
    assert e.value.code == mgt.ENOMEM
    t = gen.tiny(seed=0)
    dt = to_device(t)
    tplan = mgt.plan_for(dt, mgt.DEBUG_TIMING)
    o = mgt.alloc_outputs(dt)
    with pytest.raises(mgt.MgtError) as e:
        mgt.mgt_transpose_noalloc(tplan, False, dt.row_ptr, dt.col, dt.payload_off, dt.payload,
                                  o["t_row_ptr"], o["t_col"], o["t_payload_off"], o["t_payload"],
                                  None)
    assert e.value.code == mgt.EINVAL
