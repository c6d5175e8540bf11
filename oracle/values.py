"""XCSR value lists and repeated cells (Section 2) -- TEST INFRASTRUCTURE ONLY.

Only the test suite may use this module (it is part of the oracle package).

The paper's XCSR keeps one cell per (row, column) pair whose value is a list
of N_ij values of one type, serialised as all values back to back plus a
count of values per cell (the extra cell_counts argument of the Transpose
signature, Section 2). A multigraph can instead keep every edge as a cell of
its own, so a pair with N_ij edges appears as N_ij repeated cells. Both forms
are CSRs with byte payloads here (cell k owns payload[payload_off[k] ..
payload_off[k+1])), and the conversions between them are written from those
definitions:

* coalesce: every run of consecutive cells of one row with the same column
  becomes one cell whose payload is the run's payloads in order; its count is
  the run's length (the value count when every repeated cell holds one value).
  The payload bytes keep their order, so the payload array is unchanged.
* expand: a cell whose payload is a list of w-byte values becomes one cell per
  value (same row and column), in order; the payload array is unchanged.
* counts_to_offsets / offsets_to_counts: value counts per cell and byte
  offsets of w-byte values, each the other's exclusive scan / difference.

Coalescing merges only consecutive equal columns, so a row whose equal columns
are not adjacent keeps one cell per run. Rows sorted by column (every
transpose output) have one cell per distinct (row, column) pair after it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ValueLists:
    row_ptr: np.ndarray      # n_rows + 1 (int64)
    col: np.ndarray          # int32, one entry per cell
    payload_off: np.ndarray  # n_cells + 1 (int64), offsets into the unchanged payload
    counts: np.ndarray       # int64 per cell: cells merged into it (coalesce) or values (expand)


def _rows_of(row_ptr: np.ndarray) -> np.ndarray:
    rp = np.asarray(row_ptr, np.int64)
    return np.repeat(np.arange(rp.shape[0] - 1, dtype=np.int64), np.diff(rp))


def coalesce(row_ptr, col, payload_off) -> ValueLists:
    """Merge runs of consecutive equal columns inside each row (see module doc)."""
    rp = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int32)
    poff = np.asarray(payload_off, np.int64)
    nnz = col.shape[0]
    rows = _rows_of(rp)
    head = np.ones(nnz, dtype=bool)
    if nnz > 1:
        head[1:] = (rows[1:] != rows[:-1]) | (col[1:] != col[:-1])
    starts = np.flatnonzero(head)                     # first input cell of every output cell
    m = starts.shape[0]
    ends = np.append(starts[1:], nnz)
    out_rp = np.searchsorted(starts, rp, side="left").astype(np.int64)  # output cells before each row start
    out_poff = np.append(poff[starts], poff[-1] if poff.size else 0).astype(np.int64)
    return ValueLists(out_rp, col[starts].copy(), out_poff, (ends - starts).astype(np.int64))


def expand(row_ptr, col, payload_off, value_bytes: int) -> ValueLists:
    """One cell per value_bytes-wide value (see module doc). Raises ValueError
    if a cell's payload is not a whole number of values."""
    if value_bytes <= 0:
        raise ValueError("value_bytes must be positive")
    rp = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int32)
    poff = np.asarray(payload_off, np.int64)
    if np.any(poff % value_bytes):
        raise ValueError("a cell's payload is not a whole number of values")
    vstart = poff // value_bytes                       # values before each cell
    counts = np.diff(vstart)
    out_col = np.repeat(col, counts)
    total = int(vstart[-1]) if vstart.size else 0
    out_rp = vstart[rp] if rp.size else rp
    return ValueLists(out_rp.astype(np.int64), out_col.astype(np.int32),
                      np.arange(total + 1, dtype=np.int64) * value_bytes, counts.astype(np.int64))


def counts_to_offsets(counts, value_bytes: int) -> np.ndarray:
    c = np.asarray(counts, np.int64)
    out = np.zeros(c.shape[0] + 1, dtype=np.int64)
    np.cumsum(c * value_bytes, out=out[1:])
    return out


def offsets_to_counts(payload_off, value_bytes: int) -> np.ndarray:
    d = np.diff(np.asarray(payload_off, np.int64))
    if np.any(d % value_bytes):
        raise ValueError("a cell's payload is not a whole number of values")
    return d // value_bytes
