"""Pins of the oracle for unordered multigraphs stored as one triangle
(oracle/symmetric.py; paper Section 2: M_ij = M_ji = e, one triangle stored)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import symmetric
from workloads import gen
from workloads.gen import from_arrays

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "symmetric_5v.json")) as f:
        return json.load(f)


def _csr(n, part, ow=8):
    vals = [v.encode() for v in part["values"]]
    return from_arrays(n, n, part["row_ptr"], part["col"], [len(v) for v in vals],
                       np.frombuffer(b"".join(vals), np.uint8), ow)


def _values(s):
    po = np.asarray(s.payload_off, np.int64)
    return [bytes(s.payload[po[k]:po[k + 1]]).decode() for k in range(s.nnz)]


@pytest.mark.parametrize("ow", [4, 8])
@pytest.mark.parametrize("lower", [True, False])
def test_hand_worked_example(lower, ow):
    g = _golden()
    a = _csr(g["n"], g["lower" if lower else "upper"], ow)
    s = symmetric.symmetrize(a, lower=lower)
    assert s.row_ptr.tolist() == g["expected"]["row_ptr"]
    assert s.col.tolist() == g["expected"]["col"]
    assert _values(s) == g["expected"]["values"]
    assert s.row_ptr.dtype == (np.int32 if ow == 4 else np.int64)


def test_the_two_stored_triangles_are_transposes():
    g = _golden()
    lo, up = _csr(g["n"], g["lower"]), _csr(g["n"], g["upper"])
    t = oracle.transpose(lo)
    assert t.t_row_ptr.tolist() == up.row_ptr.tolist()
    assert t.t_col.tolist() == up.col.tolist()
    assert bytes(t.t_payload) == bytes(up.payload)


def _random_symmetric(seed, n, deg, w_hi, ow=8):
    """A random matrix, its lower triangle stored (column-sorted rows)."""
    a = gen.random_small(seed, n_rows=n, n_cols=n, deg_mean=deg, w_lo=0, w_hi=w_hi, offset_width=ow)
    return symmetric.triangle(a, lower=True)


@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    lo = _random_symmetric(seed, 40 + 7 * seed, 5.0, 9, ow=4 if seed % 2 else 8)
    s = symmetric.symmetrize(lo, lower=True)
    rp = np.asarray(lo.row_ptr, np.int64)
    row_of = np.repeat(np.arange(lo.n_rows), np.diff(rp))
    diag = int((np.asarray(lo.col) == row_of).sum())
    diag_bytes = int(sum(lo.payload_off[k + 1] - lo.payload_off[k] for k in range(lo.nnz)
                         if lo.col[k] == row_of[k]))
    # every off-diagonal cell twice, every diagonal cell once
    assert s.nnz == 2 * lo.nnz - diag
    assert s.payload_bytes == 2 * lo.payload_bytes - diag_bytes
    # S is symmetric as a multiset of (row, col, payload)
    sp = np.asarray(s.payload_off, np.int64)
    srow = np.repeat(np.arange(s.n_rows), np.diff(np.asarray(s.row_ptr, np.int64)))
    cells = sorted((int(srow[k]), int(s.col[k]), bytes(s.payload[sp[k]:sp[k + 1]]))
                   for k in range(s.nnz))
    mirror = sorted((c, r, e) for r, c, e in cells)
    assert cells == mirror
    # rows come out in column order, and the lower triangle of S is the input
    assert all(np.all(np.diff(s.col[int(s.row_ptr[i]):int(s.row_ptr[i + 1])]) >= 0)
               for i in range(s.n_rows))
    back = symmetric.triangle(s, lower=True)
    assert np.array_equal(back.row_ptr.astype(np.int64), np.asarray(lo.row_ptr, np.int64))
    assert np.array_equal(back.col, lo.col)
    assert bytes(back.payload) == bytes(lo.payload)
    # upper storage of the same graph (the transposed triangle) gives the same S
    t = oracle.transpose(lo)
    up = from_arrays(lo.n_rows, lo.n_cols, t.t_row_ptr, t.t_col, np.diff(t.t_payload_off),
                     t.t_payload, lo.offset_width)
    su = symmetric.symmetrize(up, lower=False)
    assert np.array_equal(np.asarray(su.row_ptr), np.asarray(s.row_ptr))
    assert np.array_equal(su.col, s.col)
    assert bytes(su.payload) == bytes(s.payload)
    # S is its own transpose up to the order of equal cells: T(S) is canonical
    # and equals S when S's equal cells are in an order the transpose keeps
    ts = oracle.transpose(s)
    assert np.array_equal(np.asarray(ts.t_row_ptr), np.asarray(s.row_ptr))
    assert np.array_equal(ts.t_col, s.col)


def test_closed_forms():
    # diagonal only: S is the stored matrix itself
    d = from_arrays(4, 4, [0, 1, 3, 3, 4], [0, 1, 1, 3], [2, 1, 0, 3],
                    np.arange(6, dtype=np.uint8), 8)
    s = symmetric.symmetrize(d)
    assert s.row_ptr.tolist() == [0, 1, 3, 3, 4] and s.col.tolist() == [0, 1, 1, 3]
    assert bytes(s.payload) == bytes(d.payload)
    # one off-diagonal cell: two cells with the same payload
    e = from_arrays(3, 3, [0, 0, 0, 1], [1], [3], np.array([7, 8, 9], np.uint8), 8)
    s = symmetric.symmetrize(e)
    assert s.row_ptr.tolist() == [0, 0, 1, 2] and s.col.tolist() == [2, 1]
    assert s.payload.tolist() == [7, 8, 9, 7, 8, 9]
    # empty
    z = from_arrays(3, 3, [0, 0, 0, 0], [], None, None, 8)
    assert symmetric.symmetrize(z).nnz == 0


def test_rejects_cells_outside_the_triangle():
    a = from_arrays(3, 3, [0, 1, 1, 2], [2, 0], None, None, 8)  # row 0 holds column 2
    with pytest.raises(symmetric.NotATriangle):
        symmetric.symmetrize(a, lower=True)
    b = from_arrays(3, 3, [0, 0, 1, 1], [0], None, None, 8)     # row 1 holds column 0
    with pytest.raises(symmetric.NotATriangle):
        symmetric.symmetrize(b, lower=False)
