"""GPU parity of LocalTranspose and ViewSwap (mgt_view_transform, Section 3)
against the oracle's definitions (oracle/views.py), bit for bit. On the
device as in the oracle, the compositions of the two must equal the
transpose (mgt_transpose), which the paper's composition claim requires."""
import numpy as np
import pytest
import torch

from oracle import views
from workloads import gen

from .common import assert_matches_oracle, gpu_transpose

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(x: views.ViewCsr, op, perm=True, validate=False, fixed=False):
    from paper_2012_06012_amd import mgt
    out, st = mgt.view_transform(_dev(x.row_ptr), _dev(x.col),
                                 None if fixed else _dev(x.payload_off), _dev(x.payload),
                                 x.n_rows, x.n_cols, x.bounds, x.row_ptr.dtype.itemsize, op,
                                 x.view, perm=perm, validate=validate, fixed_width=fixed)
    torch.cuda.synchronize()
    h = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    return h, int(st.cpu()[0])


def _check(h, want: views.ViewCsr, perm=None):
    assert np.array_equal(h["row_ptr"].astype(np.int64), np.asarray(want.row_ptr, np.int64))
    assert np.array_equal(h["col"], want.col)
    if h["payload_off"] is not None:
        assert np.array_equal(h["payload_off"].astype(np.int64),
                              np.asarray(want.payload_off, np.int64))
    assert np.array_equal(h["payload"], want.payload)
    if perm is not None and h["perm"] is not None:
        assert np.array_equal(h["perm"].view(np.uint32), perm)


def _as_view(h, like: views.ViewCsr, n_rows, n_cols, view):
    return views.ViewCsr(n_rows, n_cols, view, like.bounds, h["row_ptr"], h["col"],
                         h["payload_off"], h["payload"])


CASES = [
    ("tiny", lambda: gen.tiny(seed=2)),
    ("r7", lambda: gen.random_small(5, n_rows=3000, n_cols=3000, deg_mean=6.0, w_lo=0, w_hi=11,
                                    parts=7)),
    ("r5-unsorted-ow4", lambda: gen.random_small(6, n_rows=2000, n_cols=2000, deg_mean=5.0,
                                                 w_lo=0, w_hi=7, sort_rows=False,
                                                 offset_width=4, parts=5)),
    ("r1-rect", lambda: gen.random_small(7, n_rows=1500, n_cols=900, deg_mean=4.0, w_lo=1,
                                         w_hi=3)),
    ("large-r64", lambda: gen.large(seed=3, scale=8)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("op", [views.LOCAL_TRANSPOSE, views.VIEW_SWAP])
def test_view_ops_match_oracle_both_views(name, make, op):
    a = make()
    x = views.from_csr(a)
    want, perm = views.apply(op, x)              # row view in
    h, st = _run(x, op)
    assert st == 0
    _check(h, want, perm)
    # and back from the column view (the oracle's own column-view result)
    back, perm2 = views.apply(op, want)
    h2, st = _run(want, op)
    assert st == 0
    _check(h2, back, perm2)


@pytest.mark.parametrize("name,make", CASES[1:3], ids=[c[0] for c in CASES[1:3]])
def test_device_compositions_equal_the_transpose(name, make):
    a = make()
    x = views.from_csr(a)
    h_t, st = gpu_transpose(a, perm=False)
    assert st == 0
    assert_matches_oracle(a, h_t, check_perm=False)
    for first, second in ((views.LOCAL_TRANSPOSE, views.VIEW_SWAP),
                          (views.VIEW_SWAP, views.LOCAL_TRANSPOSE)):
        h1, st = _run(x, first, perm=False)
        assert st == 0
        y = (_as_view(h1, x, a.n_cols, a.n_rows, views.COLUMN_VIEW) if first == views.LOCAL_TRANSPOSE
             else _as_view(h1, x, a.n_rows, a.n_cols, views.COLUMN_VIEW))
        h2, st = _run(y, second, perm=False)
        assert st == 0
        assert np.array_equal(h2["row_ptr"], h_t["t_row_ptr"])
        assert np.array_equal(h2["col"], h_t["t_col"])
        assert np.array_equal(h2["payload_off"], h_t["t_payload_off"])
        assert np.array_equal(h2["payload"], h_t["t_payload"])


def test_view_ops_fixed_width():
    a = gen.random_small(8, n_rows=4000, n_cols=4000, deg_mean=5.0, w_lo=12, w_hi=12, parts=9)
    x = views.from_csr(a)
    for op in (views.LOCAL_TRANSPOSE, views.VIEW_SWAP):
        want, perm = views.apply(op, x)
        h, st = _run(x, op, fixed=True)
        assert st == 0
        _check(h, want, perm)


def test_view_validate_flags_column_outside_its_partition():
    a = gen.random_small(9, n_rows=600, n_cols=600, deg_mean=4.0, w_lo=0, w_hi=3, parts=3)
    x = views.from_csr(a)
    cv, _ = views.view_swap(x)                   # a valid column view ...
    h, st = _run(cv, views.VIEW_SWAP, validate=True)
    assert st == 0
    bad = views.ViewCsr(cv.n_rows, cv.n_cols, cv.view, cv.bounds, cv.row_ptr, cv.col.copy(),
                        cv.payload_off, cv.payload)
    bad.col[0] = int(cv.bounds[-1]) - 1          # ... with a cell of partition 0 given a column
    h, st = _run(bad, views.VIEW_SWAP, validate=True)  # owned by the last partition
    assert st == -2
