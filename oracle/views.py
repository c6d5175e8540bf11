"""LocalTranspose and ViewSwap (Section 3) on host arrays -- TEST INFRASTRUCTURE ONLY.

Only the test suite may use this module (it is part of the oracle package).

A distributed matrix X (n_rows x n_cols) with R partitions (bounds b, shared by
rows and columns, so R > 1 needs a square matrix) is held in one of two views
(Section 3, "view"; layouts of Fig. 1):

* row view: partition r holds the rows [b_r, b_r+1) of X with all their cells.
  Stored as one CSR over the n_rows rows, since the partitions are consecutive
  row ranges.
* column view: partition s holds the columns [b_s, b_s+1) of X, for every row.
  Each partition is a CSR over the n_rows rows, and the R of them are stored
  one after another: one CSR over R * n_rows virtual rows, virtual row
  s * n_rows + i being row i of partition s.

Inside a row, cells keep their order: every operation below is a stable sort
of the cells by a key, carrying each cell's payload bytes.

* LocalTranspose (first definition of Section 3): every partition transposes
  its own block. Row view of X in, column view of X^T out (partition r holds
  the block of X's rows in V_r, transposed), and back.
* ViewSwap (second definition): the same matrix in the orthogonal view.

The paper's claims, which the tests check: both are involutions, and
Transpose = LocalTranspose . ViewSwap = ViewSwap . LocalTranspose. Applied
twice, LocalTranspose returns every row column-sorted (as T(T(A)) does) and
ViewSwap returns every row grouped by its columns' partitions, so both give
the matrix back exactly when its rows are column-sorted.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ROW_VIEW, COLUMN_VIEW = 0, 1
LOCAL_TRANSPOSE, VIEW_SWAP = 0, 1


@dataclass
class ViewCsr:
    n_rows: int            # rows of the matrix X it represents
    n_cols: int
    view: int              # ROW_VIEW or COLUMN_VIEW
    bounds: np.ndarray     # R + 1 partition bounds (int64)
    row_ptr: np.ndarray    # n_rows + 1 (row view) or R * n_rows + 1 (column view)
    col: np.ndarray        # int32 column of X of every cell
    payload_off: np.ndarray
    payload: np.ndarray

    @property
    def n_parts(self) -> int:
        return len(self.bounds) - 1

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def owner(bounds: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Partition holding index v: the largest p with bounds[p] <= v."""
    return np.searchsorted(bounds, v, side="right") - 1


def from_csr(a) -> ViewCsr:
    """A workloads Csr (row view, its own bounds)."""
    return ViewCsr(a.n_rows, a.n_cols, ROW_VIEW, np.asarray(a.bounds, np.int64), a.row_ptr,
                   a.col, a.payload_off, a.payload)


def _stable_by_key(x: ViewCsr, key: np.ndarray, value: np.ndarray, n_out: int):
    """Cells sorted stably by key (ties keep input order): row offsets over
    n_out output rows, the carried value, payload offsets and bytes, and the
    input cell of every output position."""
    order = np.argsort(key, kind="stable")
    counts = np.bincount(key, minlength=n_out) if key.size else np.zeros(n_out, np.int64)
    dt = x.row_ptr.dtype
    row_ptr = np.zeros(n_out + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    sizes = (x.payload_off[1:] - x.payload_off[:-1]).astype(np.int64)[order]
    poff = np.zeros(order.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=poff[1:])
    starts = x.payload_off[:-1].astype(np.int64)[order]
    # output byte b of cell p is input byte starts[p] + (b - poff[p])
    src = np.repeat(starts - poff[:-1], sizes) + np.arange(int(poff[-1]), dtype=np.int64)
    payload = x.payload[src] if src.size else np.empty(0, dtype=np.uint8)
    return (row_ptr.astype(dt), value[order].astype(np.int32), poff.astype(dt), payload,
            order.astype(np.uint32))


def _rows(x: ViewCsr) -> np.ndarray:
    n_virtual = x.row_ptr.shape[0] - 1
    return np.repeat(np.arange(n_virtual, dtype=np.int64),
                     np.diff(x.row_ptr.astype(np.int64)))


def local_transpose(x: ViewCsr):
    """LocalTranspose (Section 3, first definition). Returns (ViewCsr, perm)."""
    R = x.n_parts
    v = _rows(x)
    j = x.col.astype(np.int64)
    if x.view == ROW_VIEW:
        # partition r = owner(i) transposes its rows: output partition r, row j
        i = v
        key = owner(x.bounds, i) * x.n_cols + j
        rp, col, poff, pay, perm = _stable_by_key(x, key, i, R * x.n_cols)
        return ViewCsr(x.n_cols, x.n_rows, COLUMN_VIEW, x.bounds, rp, col, poff, pay), perm
    # column view: partition s holds X[:, V_s]; its transpose is rows V_s of X^T
    i = v % x.n_rows
    key = j
    rp, col, poff, pay, perm = _stable_by_key(x, key, i, x.n_cols)
    return ViewCsr(x.n_cols, x.n_rows, ROW_VIEW, x.bounds, rp, col, poff, pay), perm


def view_swap(x: ViewCsr):
    """ViewSwap (Section 3, second definition). Returns (ViewCsr, perm)."""
    R = x.n_parts
    v = _rows(x)
    j = x.col.astype(np.int64)
    if x.view == ROW_VIEW:
        # cell (i, j) moves to partition owner(j), row i
        i = v
        key = owner(x.bounds, j) * x.n_rows + i
        rp, col, poff, pay, perm = _stable_by_key(x, key, j, R * x.n_rows)
        return ViewCsr(x.n_rows, x.n_cols, COLUMN_VIEW, x.bounds, rp, col, poff, pay), perm
    i = v % x.n_rows
    rp, col, poff, pay, perm = _stable_by_key(x, i, j, x.n_rows)
    return ViewCsr(x.n_rows, x.n_cols, ROW_VIEW, x.bounds, rp, col, poff, pay), perm


def apply(op: int, x: ViewCsr):
    return local_transpose(x) if op == LOCAL_TRANSPOSE else view_swap(x)
