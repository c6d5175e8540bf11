"""The debug guard words (MGT_DEBUG=1, set for the whole test session): every
output and workspace buffer of the binding's helpers is followed by a guard
zone that the call helpers check after each call. Here: the zones are in
place, survive real calls, and a planted change inside one (an in-bounds
write to the guard bytes themselves) is reported."""
import pytest
import torch

from workloads import gen

from .common import to_device

pytestmark = pytest.mark.gpu


def test_guards_survive_calls_and_catch_a_planted_overwrite():
    from paper_2012_06012_amd import mgt
    assert mgt._debug()
    a = gen.large(seed=9, scale=7)
    d = to_device(a)
    for part in (False, True):
        out, st = mgt.transpose(d, partitioned=part)   # checks its guards itself
        assert int(st.cpu()[0]) == mgt.OK
        assert all(hasattr(v, "_mgt_guard") for v in out.values() if v is not None)
    base, off = out["t_col"]._mgt_guard
    base[off + 7] = 0                                  # inside the guard zone
    with pytest.raises(mgt.GuardError):
        mgt.check_guards([out["t_col"]], "planted")
    mats = [to_device(gen.random_small(s, n_rows=200, n_cols=300, deg_mean=5.0)) for s in range(3)]
    outs, st, _, ws = mgt.batch_transpose(mats)       # checks its guards itself
    assert (st.cpu().numpy() == 0).all() and hasattr(ws, "_mgt_guard")
