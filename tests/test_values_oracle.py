"""Pins of the value-list conversions of the oracle (oracle/values.py), CPU only.

What pins them, other than themselves:
* a hand-worked example (tests/golden/value_lists_4rows.json);
* brute force with per-row grouping loops on small random matrices;
* round trips: expanding the coalesced form of one-value cells gives the
  cells back, and coalescing the expanded form of cells without adjacent equal
  columns gives them back;
* the counting-sort transpose (oracle.c): transposing commutes with both
  conversions, since the transpose keeps the cells of one (row, column) pair
  adjacent and in order (Section 2 definition, stable order of repeats).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import values
from workloads import gen
from workloads.gen import from_arrays

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_coalesce_and_expand():
    with open(os.path.join(GOLDEN, "value_lists_4rows.json")) as f:
        g = json.load(f)
    rc, vl = g["repeated_cells"], g["value_lists"]
    poff = np.arange(len(rc["col"]) + 1)  # one byte per cell
    out = values.coalesce(rc["row_ptr"], rc["col"], poff)
    assert out.row_ptr.tolist() == vl["row_ptr"]
    assert out.col.tolist() == vl["col"]
    assert out.payload_off.tolist() == vl["payload_off"]
    assert out.counts.tolist() == vl["counts"]
    pay = "".join(rc["values"])
    assert [pay[a:b] for a, b in zip(vl["payload_off"][:-1], vl["payload_off"][1:])] == \
        ["ab", "c", "d", "efg", "h", "i", "j"]
    back = values.expand(out.row_ptr, out.col, out.payload_off, 1)
    assert back.row_ptr.tolist() == rc["row_ptr"]
    assert back.col.tolist() == rc["col"]
    assert back.payload_off.tolist() == poff.tolist()


def _brute_coalesce(rp, col, poff):
    out_rp, out_col, out_poff, cnt = [0], [], [], []
    for i in range(len(rp) - 1):
        cells = list(range(rp[i], rp[i + 1]))
        for c, grp in itertools.groupby(cells, key=lambda k: int(col[k])):
            grp = list(grp)
            out_col.append(c)
            out_poff.append(int(poff[grp[0]]))
            cnt.append(len(grp))
        out_rp.append(len(out_col))
    out_poff.append(int(poff[-1]))
    return out_rp, out_col, out_poff, cnt


@pytest.mark.parametrize("seed,sort_rows", [(0, True), (1, False), (2, True), (3, False)])
def test_coalesce_brute_force(seed, sort_rows):
    a = gen.random_small(seed, n_rows=200, n_cols=30, deg_mean=6.0, w_lo=0, w_hi=5,
                         sort_rows=sort_rows)
    out = values.coalesce(a.row_ptr, a.col, a.payload_off)
    rp, col, poff, cnt = _brute_coalesce(np.asarray(a.row_ptr, np.int64), a.col,
                                         np.asarray(a.payload_off, np.int64))
    assert out.row_ptr.tolist() == rp
    assert out.col.tolist() == col
    assert out.payload_off.tolist() == poff
    assert out.counts.tolist() == cnt


def test_expand_brute_force():
    rng = np.random.default_rng(4)
    n, w = 50, 4
    rp = np.concatenate([[0], np.cumsum(rng.integers(0, 5, size=n))])
    col = rng.integers(0, 9, size=rp[-1]).astype(np.int32)
    cnt = rng.integers(0, 4, size=rp[-1])
    poff = values.counts_to_offsets(cnt, w)
    out = values.expand(rp, col, poff, w)
    exp_col, exp_rp = [], [0]
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            exp_col += [int(col[k])] * int(cnt[k])
        exp_rp.append(len(exp_col))
    assert out.col.tolist() == exp_col
    assert out.row_ptr.tolist() == exp_rp
    assert out.payload_off.tolist() == [w * q for q in range(len(exp_col) + 1)]
    assert out.counts.tolist() == cnt.tolist()
    assert values.offsets_to_counts(poff, w).tolist() == cnt.tolist()


def test_round_trips():
    # one w-byte value per repeated cell: expand(coalesce(A)) == A
    a = gen.random_small(5, n_rows=300, n_cols=40, deg_mean=8.0, w_lo=4, w_hi=4)
    c = values.coalesce(a.row_ptr, a.col, a.payload_off)
    assert (c.counts >= 1).all() and c.counts.sum() == a.nnz
    e = values.expand(c.row_ptr, c.col, c.payload_off, 4)
    assert np.array_equal(e.row_ptr, np.asarray(a.row_ptr, np.int64))
    assert np.array_equal(e.col, a.col)
    assert np.array_equal(e.payload_off, np.asarray(a.payload_off, np.int64))
    # cells with no adjacent equal columns: coalesce(expand(X)) == X
    c2 = values.coalesce(e.row_ptr, e.col, e.payload_off)
    assert np.array_equal(c2.row_ptr, c.row_ptr) and np.array_equal(c2.col, c.col)
    assert np.array_equal(c2.payload_off, c.payload_off)


def test_expand_rejects_partial_values():
    with pytest.raises(ValueError):
        values.expand([0, 2], [0, 1], [0, 4, 6], 4)


def _as_csr(n_rows, n_cols, rp, col, poff, payload, ow=8):
    return from_arrays(n_rows, n_cols, rp, col, np.diff(np.asarray(poff, np.int64)), payload, ow)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transpose_commutes_with_coalesce(seed):
    # T(coalesce(A)) == coalesce(T(A)), payload bytes included
    a = gen.random_small(seed, n_rows=400, n_cols=60, deg_mean=7.0, w_lo=0, w_hi=6,
                         sort_rows=seed % 2 == 0)
    c = values.coalesce(a.row_ptr, a.col, a.payload_off)
    ta = oracle.transpose(a)
    lhs = oracle.transpose(_as_csr(a.n_rows, a.n_cols, c.row_ptr, c.col, c.payload_off, a.payload))
    rhs = values.coalesce(ta.t_row_ptr, ta.t_col, ta.t_payload_off)
    # coalesced cells stay merged when transposed only if the input rows kept
    # equal columns adjacent; the transpose output always does
    if seed % 2 == 0:
        assert np.array_equal(np.asarray(lhs.t_row_ptr, np.int64), rhs.row_ptr)
        assert np.array_equal(lhs.t_col, rhs.col)
        assert np.array_equal(np.asarray(lhs.t_payload_off, np.int64), rhs.payload_off)
        assert np.array_equal(lhs.t_payload, ta.t_payload)
    # coalescing the transpose merges every (row, column) pair of the input
    pairs = {(int(r), int(j)) for r, j in zip(np.repeat(np.arange(a.n_rows), np.diff(a.row_ptr)), a.col)}
    assert rhs.col.shape[0] == len(pairs)


def test_transpose_commutes_with_expand():
    rng = np.random.default_rng(7)
    n, w = 120, 4
    rp = np.concatenate([[0], np.cumsum(rng.integers(0, 6, size=n))])
    col = np.sort(rng.integers(0, 80, size=rp[-1]).reshape(-1))
    col = np.concatenate([np.sort(col[rp[i]:rp[i + 1]]) for i in range(n)]).astype(np.int32)
    cnt = rng.integers(0, 5, size=rp[-1])
    poff = values.counts_to_offsets(cnt, w)
    pay = rng.integers(0, 256, size=int(poff[-1]), dtype=np.uint8)
    x = _as_csr(n, 80, rp, col, poff, pay)
    tx = oracle.transpose(x)
    lhs = values.expand(tx.t_row_ptr, tx.t_col, tx.t_payload_off, w)
    e = values.expand(rp, col, poff, w)
    rhs = oracle.transpose(_as_csr(n, 80, e.row_ptr, e.col, e.payload_off, pay))
    assert np.array_equal(lhs.row_ptr, np.asarray(rhs.t_row_ptr, np.int64))
    assert np.array_equal(lhs.col, rhs.t_col)
    assert np.array_equal(lhs.payload_off, np.asarray(rhs.t_payload_off, np.int64))
    assert np.array_equal(tx.t_payload, rhs.t_payload)


def test_empty():
    c = values.coalesce([0, 0, 0], np.zeros(0, np.int32), [0])
    assert c.row_ptr.tolist() == [0, 0, 0] and c.col.size == 0 and c.payload_off.tolist() == [0]
    e = values.expand([0, 0], np.zeros(0, np.int32), [0], 4)
    assert e.row_ptr.tolist() == [0, 0] and e.col.size == 0 and e.payload_off.tolist() == [0]
