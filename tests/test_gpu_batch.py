"""GPU parity of the batched entry point (mgt_batch_submit): every item of a
batch must equal the oracle's transpose of that item, bit for bit, and equal
what the single-matrix entry points produce for it."""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen
from workloads.gen import from_arrays

from .common import assert_matches_oracle, host, to_device

pytestmark = pytest.mark.gpu


def _mixed_items(seed, n_items, n_lo=100, n_hi=20000):
    items = []
    for i in range(n_items):
        n, deg, width = gen.batch_item_params(seed, i, n_lo, n_hi)
        a = gen.generate(n, n, seed=(seed << 20) + i, deg_law=gen.DEG_POISSON,
                         deg_mean=float(min(deg, 20)), pay_law=gen.PAY_BYTES, w_lo=width,
                         w_hi=width, offset_width=8, name=f"item{i}")
        if i % 3 == 1:  # some items partitioned, R in 2..9
            a.bounds = gen.equal_bounds(n, min(n, 2 + i % 8))
        items.append(a)
    return items


def _run_batch(items, perm=True, validate=False):
    from paper_2012_06012_amd import mgt
    mats = [to_device(a) for a in items]
    outs, status, plan, ws = mgt.batch_transpose(mats, perm=perm, validate=validate)
    torch.cuda.synchronize()
    return [host(o) for o in outs], status.cpu().numpy()


@pytest.mark.parametrize("seed,n_items", [(0, 7), (1, 40)])
def test_batch_matches_oracle(seed, n_items):
    items = _mixed_items(seed, n_items)
    outs, st = _run_batch(items)
    assert (st == 0).all()
    for a, h in zip(items, outs):
        assert_matches_oracle(a, h, partitioned=a.n_parts > 1)


def test_batch_with_empty_and_tiny_items():
    items = [from_arrays(0, 0, [0], [], [], None, 8),
             from_arrays(3, 3, [0, 0, 0, 0], [], [], None, 8),
             from_arrays(1, 1, [0, 2], [0, 0], [3, 0], None, 8),
             gen.random_small(3, n_rows=64, n_cols=64, deg_mean=3.0, w_lo=0, w_hi=16),
             gen.random_small(4, n_rows=5000, n_cols=70000, deg_mean=9.0, w_lo=0, w_hi=3)]
    outs, st = _run_batch(items)
    assert (st == 0).all()
    for a, h in zip(items, outs):
        assert_matches_oracle(a, h)


def test_batch_equals_single_calls():
    from paper_2012_06012_amd import mgt
    items = _mixed_items(5, 12)
    outs, _ = _run_batch(items, perm=False)
    for a, hb in zip(items, outs):
        d = to_device(a)
        o, s = mgt.transpose(d, perm=False, partitioned=a.n_parts > 1)
        hs = host(o)
        for k, v in hs.items():
            if v is not None:
                assert np.array_equal(v, hb[k]), k


def test_batch_validation_isolates_bad_item():
    items = _mixed_items(9, 5)
    bad = items[2]
    bad.col = bad.col.copy()
    bad.col[0] = bad.n_cols + 5
    _, st = _run_batch(items, validate=True)
    assert st[2] == -2                   # MGT_ERANGE for the bad item
    assert all(st[i] == -6 for i in (0, 1, 3, 4))  # the rest were cancelled, not transposed


def test_batch_repeated_submits_reuse_plan_and_workspace():
    from paper_2012_06012_amd import mgt
    items = _mixed_items(11, 6)
    mats = [to_device(a) for a in items]
    outs, status, plan, ws = mgt.batch_transpose(mats)
    for _ in range(3):
        outs2, status2, _, _ = mgt.batch_transpose(mats, plan=plan, workspace=ws)
    torch.cuda.synchronize()
    for o1, o2 in zip(outs, outs2):
        for k in o1:
            if o1[k] is not None:
                assert torch.equal(o1[k], o2[k]), k
    ref = oracle.transpose(items[0])
    assert np.array_equal(outs2[0]["t_col"].cpu().numpy(), ref.t_col)


@pytest.mark.parametrize("wide_cell", [False, True])
def test_batch_packed_records(wide_cell, monkeypatch):
    # a batch whose widest item needs two passes runs every item through one
    # records-only pass; without perm its records are packed (per item column
    # bits) unless some cell's payload does not fit beside its column
    items = _mixed_items(13, 9)
    items.append(gen.random_small(14, n_rows=60000, n_cols=1 << 21, deg_mean=5.0, w_lo=0, w_hi=11))
    if wide_cell:  # 2^21 columns leave 11 bits: a 2,048-byte cell cannot be packed
        a = items[3]
        w = np.diff(a.payload_off).astype(np.int64)
        w[len(w) // 2] = 2048
        items[3] = from_arrays(a.n_rows, a.n_cols, a.row_ptr, a.col, w, None, 8, a.bounds, 3)
    outs, st = _run_batch(items, perm=False)
    assert (st == 0).all()
    for a, h in zip(items, outs):
        assert_matches_oracle(a, h, partitioned=a.n_parts > 1)
    monkeypatch.setenv("MGT_NO_PACK", "1")
    outs2, st2 = _run_batch(items, perm=False)
    assert (st2 == 0).all()
    for h, h2 in zip(outs, outs2):
        for k, v in h.items():
            if v is not None:
                assert np.array_equal(v, h2[k]), k


def test_batch_items_take_the_padded_passes():
    # every item of a batch makes as many passes as the item that needs the
    # most; an item whose fewest passes would come from wide finish buckets
    # (100,000 columns of ~60 cells: one pass and 512-column buckets of about
    # 30,000 cells) takes the second pass's bits instead and keeps buckets
    # of up to 8,192 cells; packed 12-byte records through the 512-thread pass
    from paper_2012_06012_amd import mgt
    items = [gen.random_small(31, n_rows=1 << 19, n_cols=1 << 19, deg_mean=8.0, w_lo=0, w_hi=13),
             gen.random_small(32, n_rows=100000, n_cols=100000, deg_mean=60.0, w_lo=0, w_hi=9),
             gen.random_small(33, n_rows=3000, n_cols=3000, deg_mean=5.0, w_lo=0, w_hi=20)]
    outs, st = _run_batch(items, perm=False)
    assert (st == 0).all()
    for a, h in zip(items, outs):
        assert_matches_oracle(a, h)
        o, s1 = mgt.transpose(to_device(a), perm=False)
        hs = host(o)
        for k, v in hs.items():
            if v is not None:
                assert np.array_equal(v, h[k]), k


def test_batch_packed_with_fixed_width_items():
    # fixed-width items beside variable ones in one packed two-pass batch: the
    # first pass then reads columns and offsets (or k * width) for every item
    from paper_2012_06012_amd import mgt
    items = _mixed_items(17, 5)
    items.append(gen.random_small(18, n_rows=50000, n_cols=1 << 21, deg_mean=5.0, w_lo=0, w_hi=9))
    fixed = [gen.random_small(19 + k, n_rows=3000, n_cols=3000, deg_mean=6.0, w_lo=w, w_hi=w)
             for k, w in enumerate((12, 0, 28))]
    mats = [to_device(a) for a in items] + [to_device(a, fixed_width=True) for a in fixed]
    outs, status, plan, ws = mgt.batch_transpose(mats, perm=False)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    for a, o in zip(items + fixed, outs):
        h = host(o)
        if h.get("t_payload_off") is None:
            w = a.payload_bytes // max(a.nnz, 1)
            h = dict(h, t_payload_off=np.arange(a.nnz + 1, dtype=a.payload_off.dtype) * w)
        assert_matches_oracle(a, h, partitioned=a.n_parts > 1)
