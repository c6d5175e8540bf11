"""GPU parity of recorded transposes (mgt_graph_create / mgt_graph_launch).

A graph holds every stage of one call with fixed buffers. Each replay must
write the transpose of the inputs as they are at replay time, so the tests
change the inputs in place between replays (new payload bytes, new columns
with the same row structure), poison the outputs and the status word, run
other eager library work on the same device in between, and compare every
replay with the oracle.
"""
import numpy as np
import pytest
import torch

from workloads import gen

from .common import assert_matches_oracle, host, to_device

pytestmark = pytest.mark.gpu


def _variant(a, k):
    """Same rows, nnz, widths and bounds as a; other columns and payload bytes."""
    if k == 0:
        return a
    rng = np.random.default_rng(100 + k)
    col = rng.integers(0, a.n_cols, size=a.nnz).astype(np.int32)
    for i in range(a.n_rows):  # keep the rows' sortedness like the generator's
        lo, hi = int(a.row_ptr[i]), int(a.row_ptr[i + 1])
        if k % 2:
            col[lo:hi].sort()
    pay = rng.integers(0, 256, size=a.payload_bytes, dtype=np.uint8)
    return gen.from_arrays(a.n_rows, a.n_cols, a.row_ptr, col, np.diff(a.payload_off), pay,
                           a.offset_width, a.bounds)


def _load(d, b):
    d.col.copy_(torch.from_numpy(np.ascontiguousarray(b.col)))
    d.payload.copy_(torch.from_numpy(np.ascontiguousarray(b.payload)))


def _poison(out, status):
    for v in out.values():
        if v is not None and v.numel():
            v.view(torch.uint8).fill_(0xA5)
    status.fill_(77)


def _replays(a, partitioned, n_replays=4):
    from paper_2012_06012_amd import mgt
    d = to_device(a)
    g, out, status = mgt.transpose_graph(d, perm=True, partitioned=partitioned)
    other = to_device(gen.random_small(9, n_rows=700, n_cols=500, deg_mean=5.0))
    for k in range(n_replays):
        b = _variant(a, k)
        _load(d, b)
        _poison(out, status)
        # eager work of the program between replays
        eo, es = mgt.transpose(other, perm=True)
        torch.cuda.synchronize()
        g.launch()
        h = host(out)
        assert int(status.cpu()[0]) == 0
        assert_matches_oracle(b, h, partitioned=partitioned)
        assert int(es.cpu()[0]) == 0
    g.close()


@pytest.mark.parametrize("partitioned", [False, True])
def test_graph_replays_small(partitioned):
    _replays(gen.random_small(1, n_rows=3000, n_cols=3000, deg_mean=6.0, w_lo=0, w_hi=11,
                              parts=7), partitioned)


def test_graph_replays_tiny_recipe():
    _replays(gen.tiny(seed=2), False)


@pytest.mark.parametrize("caps", [(4, 4), (3, 3)])
def test_graph_replays_long_schedules(monkeypatch, caps):
    # the schedule is fixed when the graph is recorded: record under the caps,
    # replay after they are gone
    monkeypatch.setenv("MGT_MAX_PASS_BITS", str(caps[0]))
    monkeypatch.setenv("MGT_MAX_FINISH_BITS", str(caps[1]))
    from paper_2012_06012_amd import mgt
    a = gen.random_small(4, n_rows=4000, n_cols=4000, deg_mean=5.0, w_lo=0, w_hi=9, parts=5)
    d = to_device(a)
    g, out, status = mgt.transpose_graph(d, perm=True, partitioned=True)
    monkeypatch.delenv("MGT_MAX_PASS_BITS")
    monkeypatch.delenv("MGT_MAX_FINISH_BITS")
    for k in range(3):
        b = _variant(a, k)
        _load(d, b)
        _poison(out, status)
        torch.cuda.synchronize()
        g.launch()
        h = host(out)
        assert int(status.cpu()[0]) == 0
        assert_matches_oracle(b, h, partitioned=True)


def test_graph_on_a_side_stream_and_plan_destroyed():
    from paper_2012_06012_amd import mgt
    a = gen.random_small(5, n_rows=2000, n_cols=1500, deg_mean=4.0, w_lo=1, w_hi=6)
    d = to_device(a)
    plan = mgt.plan_for(d, mgt.EMIT_PERM)
    g, out, status = mgt.transpose_graph(d, plan=plan, perm=True)
    plan.close()  # the graph does not need the plan after recording
    s = torch.cuda.Stream()
    for _ in range(2):
        _poison(out, status)
        torch.cuda.synchronize()
        g.launch(stream=s)
        s.synchronize()
        h = host(out)
        assert int(status.cpu()[0]) == 0
        assert_matches_oracle(a, h)


def test_graph_validate_reports_bad_columns():
    from paper_2012_06012_amd import mgt
    a = gen.random_small(6, n_rows=500, n_cols=500, deg_mean=4.0)
    d = to_device(a)
    g, out, status = mgt.transpose_graph(d, perm=True, validate=True)
    g.launch()
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 0
    bad = d.col.clone()
    bad[3] = a.n_cols + 5
    d.col.copy_(bad)
    g.launch()
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == mgt.ERANGE
    d.col.copy_(torch.from_numpy(np.ascontiguousarray(a.col)))
    g.launch()
    h = host(out)
    assert int(status.cpu()[0]) == 0
    assert_matches_oracle(a, h)


def test_batch_graph_replays():
    # one recorded batch submit: replays after in-place input changes, with
    # outputs and statuses poisoned in between, each against the oracle
    from paper_2012_06012_amd import mgt
    base = [gen.tiny(seed=3),
            gen.random_small(11, n_rows=2000, n_cols=2000, deg_mean=5.0, w_lo=0, w_hi=9, parts=4),
            gen.random_small(12, n_rows=50, n_cols=70, deg_mean=3.0, w_lo=0, w_hi=3),
            gen.large(seed=4, scale=10)]
    base = [b if b.offset_width == 8 else
            gen.from_arrays(b.n_rows, b.n_cols, b.row_ptr, b.col, np.diff(b.payload_off), b.payload,
                            8, b.bounds) for b in base]
    mats = [to_device(a) for a in base]
    g, outs, status, plan, ws = mgt.batch_graph(mats, perm=True)
    for k in range(3):
        cur = [_variant(a, k) for a in base]
        for d, b in zip(mats, cur):
            _load(d, b)
        for o in outs:
            for v in o.values():
                if v is not None and v.numel():
                    v.view(torch.uint8).fill_(0xA5)
        status.fill_(77)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert (status.cpu().numpy() == 0).all()
        for b, o in zip(cur, outs):
            assert_matches_oracle(b, host(o), partitioned=b.n_parts > 1)
    g.close()
