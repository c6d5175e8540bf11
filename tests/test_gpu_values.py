"""GPU parity of the value-list conversions (mgt_coalesce, mgt_expand,
mgt_counts_to_offsets) against the oracle's definitions (oracle/values.py),
and the commutation of the transpose with coalescing on the device."""
import numpy as np
import pytest
import torch

from oracle import values
from workloads import gen
from workloads.gen import from_arrays

from .common import to_device

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _check_coalesce(a):
    from paper_2012_06012_amd import mgt
    d = to_device(a)
    out, m = mgt.coalesce(d)
    want = values.coalesce(a.row_ptr, a.col, a.payload_off)
    assert m == want.col.shape[0]
    assert np.array_equal(_np(out["row_ptr"]).astype(np.int64), want.row_ptr)
    assert np.array_equal(_np(out["col"]), want.col)
    assert np.array_equal(_np(out["payload_off"]).astype(np.int64), want.payload_off)
    assert np.array_equal(_np(out["counts"]).view(np.uint32).astype(np.int64), want.counts)


@pytest.mark.parametrize("seed,n,deg,ow,sort_rows", [
    (0, 300, 6.0, 8, True), (1, 300, 6.0, 4, False), (2, 5000, 9.0, 8, True),
    (3, 40000, 8.0, 4, True),   # over 16 K cells: the multi-block scan
    (4, 30000, 12.0, 8, False),
])
def test_coalesce_matches_oracle(seed, n, deg, ow, sort_rows):
    _check_coalesce(gen.random_small(seed, n_rows=n, n_cols=max(8, n // 10), deg_mean=deg,
                                     w_lo=0, w_hi=7, offset_width=ow, sort_rows=sort_rows))


def test_coalesce_edge_cases():
    _check_coalesce(from_arrays(3, 3, [0, 0, 0, 0], [], [], None, 8))            # no cells
    _check_coalesce(from_arrays(1, 1, [0, 5], [0] * 5, [1, 0, 2, 0, 3], None, 4))  # one run
    _check_coalesce(from_arrays(4, 4, [0, 3, 3, 7, 10], [1, 1, 3, 0, 2, 2, 2, 2, 1, 2],
                                [1] * 10, None, 8))                               # runs across rows
    _check_coalesce(gen.hetero(seed=1, scale=10))                                # U{1..50} repeats


@pytest.mark.parametrize("w,ow", [(4, 8), (12, 4), (1, 8)])
def test_expand_matches_oracle(w, ow):
    from paper_2012_06012_amd import mgt
    rng = np.random.default_rng(w)
    n = 3000
    rp = np.concatenate([[0], np.cumsum(rng.integers(0, 7, size=n))])
    col = rng.integers(0, 500, size=rp[-1]).astype(np.int32)
    cnt = rng.integers(0, 6, size=rp[-1])
    a = from_arrays(n, 500, rp, col, cnt * w, None, ow)
    out, st = mgt.expand(to_device(a), w)
    want = values.expand(a.row_ptr, a.col, a.payload_off, w)
    assert int(st.cpu()[0]) == 0
    assert np.array_equal(_np(out["row_ptr"]).astype(np.int64), want.row_ptr)
    assert np.array_equal(_np(out["col"]), want.col)
    assert np.array_equal(_np(out["payload_off"]).astype(np.int64), want.payload_off)


def test_expand_reports_partial_values():
    from paper_2012_06012_amd import mgt
    a = from_arrays(2, 3, [0, 2, 3], [0, 2, 1], [4, 6, 2], None, 8)  # 12 bytes, a 6-byte cell
    out, st = mgt.expand(to_device(a), 4)
    assert int(st.cpu()[0]) == mgt.ERANGE


def test_counts_to_offsets_matches_oracle():
    from paper_2012_06012_amd import mgt
    for nnz, w, ow in ((0, 4, 8), (1000, 4, 8), (70000, 12, 4)):
        cnt = np.random.default_rng(nnz).integers(0, 9, size=nnz).astype(np.uint32)
        odt = torch.int32 if ow == 4 else torch.int64
        poff = torch.empty(nnz + 1, dtype=odt, device="cuda")
        ws = torch.empty(max(mgt.mgt_value_lists_workspace(nnz), 256), dtype=torch.uint8,
                         device="cuda")
        c = torch.from_numpy(cnt.view(np.int32)).cuda()
        mgt.mgt_counts_to_offsets(nnz, c, w, ow, poff, ws)
        assert np.array_equal(_np(poff).astype(np.int64), values.counts_to_offsets(cnt, w))


def test_transpose_commutes_with_coalesce_on_device():
    # T(coalesce(A)) == coalesce(T(A)) for column-sorted rows, payload bytes included
    from paper_2012_06012_amd import mgt
    a = gen.random_small(8, n_rows=20000, n_cols=3000, deg_mean=10.0, w_lo=0, w_hi=9)
    d = to_device(a)
    c, m = mgt.coalesce(d)
    dc = mgt.DeviceCsr(a.n_rows, a.n_cols, c["row_ptr"], c["col"].contiguous(),
                       c["payload_off"].contiguous(), d.payload, a.bounds, a.offset_width)
    lhs, st1 = mgt.transpose(dc)
    ta, st2 = mgt.transpose(d)
    ta_csr = mgt.DeviceCsr(a.n_cols, a.n_rows, ta["t_row_ptr"], ta["t_col"], ta["t_payload_off"],
                           ta["t_payload"], np.array([0, a.n_cols]), a.offset_width)
    rhs, m2 = mgt.coalesce(ta_csr)
    assert int(st1.cpu()[0]) == 0 and int(st2.cpu()[0]) == 0 and m == m2
    assert torch.equal(lhs["t_row_ptr"], rhs["row_ptr"])
    assert torch.equal(lhs["t_col"], rhs["col"])
    assert torch.equal(lhs["t_payload_off"], rhs["payload_off"])
    assert torch.equal(lhs["t_payload"], ta["t_payload"])
