"""Pins of the LocalTranspose / ViewSwap oracle (oracle/views.py), CPU only.

What pins it, other than itself:
* hand-worked values of both operations on the 6-vertex, 3-rank example
  (tests/golden/views_6v_3ranks.json);
* the counting-sort transpose oracle (oracle.c): the paper's composition
  claim Transpose = LocalTranspose . ViewSwap = ViewSwap . LocalTranspose
  (Section 3) must reproduce it, as must LocalTranspose alone with one
  partition;
* the involution claims of Section 3 (each operation applied twice gives the
  matrix back, with rows column-sorted as the transpose's T(T(A)) does),
  checked against T(T(A)) from oracle.c;
* closed forms: with one partition ViewSwap is the identity; a block-diagonal
  matrix keeps its cells in place under ViewSwap.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import views
from workloads import gen
from workloads.gen import from_arrays

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_input():
    with open(os.path.join(GOLDEN, "xcsr_6v_3ranks.json")) as f:
        g = json.load(f)
    vals = [v.encode() for v in g["values"]]
    return from_arrays(g["n_rows"], g["n_cols"], g["row_ptr"], g["col"], [len(v) for v in vals],
                       np.frombuffer(b"".join(vals), np.uint8), 8, g["bounds"])


def _same(x, y):
    assert x.view == y.view and x.n_rows == y.n_rows and x.n_cols == y.n_cols
    assert np.array_equal(np.asarray(x.row_ptr, np.int64), np.asarray(y.row_ptr, np.int64))
    assert np.array_equal(x.col, y.col)
    assert np.array_equal(np.asarray(x.payload_off, np.int64), np.asarray(y.payload_off, np.int64))
    assert np.array_equal(x.payload, y.payload)


def _row_view(t, a, n_rows, n_cols):
    return views.ViewCsr(n_rows, n_cols, views.ROW_VIEW, np.asarray(a.bounds, np.int64),
                         t.t_row_ptr, t.t_col, t.t_payload_off, t.t_payload)


def test_golden_local_transpose_and_view_swap():
    a = _golden_input()
    with open(os.path.join(GOLDEN, "views_6v_3ranks.json")) as f:
        g = json.load(f)
    for op, name in ((views.LOCAL_TRANSPOSE, "local_transpose"), (views.VIEW_SWAP, "view_swap")):
        out, perm = views.apply(op, views.from_csr(a))
        e = g[name]
        assert out.view == views.COLUMN_VIEW
        assert np.asarray(out.row_ptr).tolist() == e["row_ptr"], name
        assert out.col.tolist() == e["col"], name
        assert perm.tolist() == e["perm"], name
        assert np.asarray(out.payload_off).tolist() == e["payload_off"], name
        assert bytes(out.payload) == "".join(e["values"]).encode(), name


def _cases():
    yield gen.tiny(seed=1)
    yield gen.random_small(3, n_rows=300, n_cols=300, deg_mean=5.0, w_lo=0, w_hi=9, parts=7)
    yield gen.random_small(4, n_rows=200, n_cols=200, deg_mean=4.0, w_lo=0, w_hi=5,
                           sort_rows=False, parts=5)
    yield gen.large(seed=2, scale=12)


@pytest.mark.parametrize("a", list(_cases()), ids=lambda a: f"{a.name}-{a.n_rows}-{a.n_parts}")
def test_compositions_equal_the_transpose(a):
    # Transpose = LocalTranspose . ViewSwap = ViewSwap . LocalTranspose
    t = oracle.transpose(a)
    want = _row_view(t, a, a.n_cols, a.n_rows)
    x = views.from_csr(a)
    lt, _ = views.local_transpose(x)
    vs, _ = views.view_swap(x)
    _same(views.view_swap(lt)[0], want)
    _same(views.local_transpose(vs)[0], want)


@pytest.mark.parametrize("a", list(_cases()), ids=lambda a: f"{a.name}-{a.n_rows}-{a.n_parts}")
def test_both_are_involutions(a):
    # LocalTranspose twice gives back the matrix with column-sorted rows, as
    # T(T(A)) does; so does ViewSwap twice when the rows were column-sorted.
    # Unsorted rows come back grouped by the partition of their columns,
    # which a further round trip keeps.
    tt = oracle.transpose(a)
    ttt = oracle.transpose(gen.from_arrays(a.n_cols, a.n_rows, tt.t_row_ptr, tt.t_col,
                                           np.diff(tt.t_payload_off), tt.t_payload,
                                           a.offset_width, a.bounds))
    canon = _row_view(ttt, a, a.n_rows, a.n_cols)
    x = views.from_csr(a)
    once, _ = views.local_transpose(x)
    assert once.view == views.COLUMN_VIEW
    _same(views.local_transpose(once)[0], canon)
    once, _ = views.view_swap(x)
    assert once.view == views.COLUMN_VIEW
    twice, _ = views.view_swap(once)
    rows_sorted = all((np.diff(a.col[a.row_ptr[i]:a.row_ptr[i + 1]]) >= 0).all()
                      for i in range(a.n_rows))
    if rows_sorted:
        _same(twice, canon)
    else:
        _same(views.view_swap(views.view_swap(twice)[0])[0], twice)
        # and the cells of every row are those of A's row, in a partition-grouped order
        assert np.array_equal(np.asarray(twice.row_ptr, np.int64), np.asarray(a.row_ptr, np.int64))
        for i in range(a.n_rows):
            lo, hi = int(a.row_ptr[i]), int(a.row_ptr[i + 1])
            assert sorted(twice.col[lo:hi].tolist()) == sorted(a.col[lo:hi].tolist())
            own = views.owner(a.bounds, twice.col[lo:hi].astype(np.int64))
            assert (np.diff(own) >= 0).all()


def test_one_partition_local_transpose_is_the_transpose_and_view_swap_the_identity():
    a = gen.random_small(7, n_rows=150, n_cols=90, deg_mean=6.0, w_lo=0, w_hi=7)
    t = oracle.transpose(a)
    lt, perm = views.local_transpose(views.from_csr(a))
    assert np.array_equal(np.asarray(lt.row_ptr, np.int64), np.asarray(t.t_row_ptr, np.int64))
    assert np.array_equal(lt.col, t.t_col)
    assert np.array_equal(perm, t.perm)
    assert np.array_equal(lt.payload, t.t_payload)
    vs, perm = views.view_swap(views.from_csr(a))
    assert np.array_equal(np.asarray(vs.row_ptr, np.int64), np.asarray(a.row_ptr, np.int64))
    assert np.array_equal(vs.col, a.col)
    assert np.array_equal(perm, np.arange(a.nnz))
    assert np.array_equal(vs.payload, a.payload)


def test_block_diagonal_matrix_keeps_its_order_under_view_swap():
    # every cell's column is owned by its row's partition: the column view
    # lists the same cells in the same order
    rng = np.random.default_rng(3)
    b = np.array([0, 40, 70, 120], np.int64)
    rows, cols = [], []
    for p in range(3):
        for i in range(b[p], b[p + 1]):
            c = np.sort(rng.integers(b[p], b[p + 1], size=rng.integers(0, 6)))
            rows.append(len(c))
            cols.extend(c.tolist())
    rp = np.concatenate([[0], np.cumsum(rows)])
    a = from_arrays(120, 120, rp, cols, rng.integers(0, 5, size=len(cols)), None, 8, b)
    vs, perm = views.view_swap(views.from_csr(a))
    assert np.array_equal(perm, np.arange(a.nnz))
    assert np.array_equal(vs.payload, a.payload)


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 40), st.integers(1, 6), st.integers(0, 2**31 - 1))
def test_random_tiny_views(n, R, seed):
    R = min(R, n)
    a = gen.random_small(seed % 1000, n_rows=n, n_cols=n, deg_mean=3.0, w_lo=0, w_hi=4,
                         sort_rows=bool(seed & 1), parts=R)
    t = oracle.transpose(a)
    want = _row_view(t, a, a.n_cols, a.n_rows)
    x = views.from_csr(a)
    _same(views.view_swap(views.local_transpose(x)[0])[0], want)
    _same(views.local_transpose(views.view_swap(x)[0])[0], want)
