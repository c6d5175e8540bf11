"""Unordered multigraphs stored as one triangle -- TEST INFRASTRUCTURE ONLY
(part of the oracle; only tests/, the smoke check and the benchmark's CPU
leg use it; it shares no code with the GPU library).

Paper, Section 2: an edge {i, j, e} of an unordered graph gives M_ij = M_ji = e,
so the connectivity matrix is symmetric and storing its lower triangle (every
cell with column <= row) or its upper triangle (column >= row) is enough; the
unordered case is a sub-problem of the ordered one. Here a multigraph keeps
every edge as a cell of its own with an opaque byte payload, as in the rest of
the library.

``symmetrize(a, lower)`` builds the full symmetric matrix S of such a stored
triangle, straight from that definition: every stored off-diagonal cell
(i, j, e) appears in S as (i, j, e) and as (j, i, e); a stored diagonal cell
(i, i, e) appears once. Reading (the paper gives no order for S): row i of S
lists, for lower storage, the stored cells of row i in their stored order and
then the mirrored cells (i, r) in the order of their source cells (source row
r ascending, then stored order); for upper storage the mirrored cells (whose
sources lie in rows r < i) come first, then the stored row. With rows stored
in column order both give rows in column order, and symmetrize(L, lower)
equals symmetrize(T(L), upper) cell for cell.
"""
from __future__ import annotations

import numpy as np

from workloads.gen import Csr


class NotATriangle(ValueError):
    pass


def symmetrize(a: Csr, lower: bool = True) -> Csr:
    """Full symmetric matrix of the stored triangle `a` (plain loops)."""
    if a.n_rows != a.n_cols:
        raise ValueError("an unordered graph's matrix is square")
    n = a.n_rows
    rp = np.asarray(a.row_ptr, dtype=np.int64)
    col = np.asarray(a.col, dtype=np.int64)
    po = np.asarray(a.payload_off, dtype=np.int64)
    pay = np.asarray(a.payload, dtype=np.uint8)
    row_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    bad = (col > row_of) if lower else (col < row_of)
    if bad.any():
        raise NotATriangle(f"cell {int(np.argmax(bad))} lies outside the stored triangle")
    # the mirrored cells of every row: sources k with col[k] == i and row(k) != i,
    # in source order (k ascending is row ascending, then stored order)
    mirrored = [[] for _ in range(n)]
    for k in range(a.nnz):
        if col[k] != row_of[k]:
            mirrored[col[k]].append(k)
    out_rp = [0]
    out_col, out_src = [], []
    for i in range(n):
        stored = list(range(rp[i], rp[i + 1]))
        parts = [(stored, False), (mirrored[i], True)] if lower else \
                [(mirrored[i], True), (stored, False)]
        for ks, mirror in parts:
            for k in ks:
                out_col.append(int(row_of[k]) if mirror else int(col[k]))
                out_src.append(k)
        out_rp.append(len(out_col))
    sizes = [int(po[k + 1] - po[k]) for k in out_src]
    out_po = np.zeros(len(out_src) + 1, dtype=np.int64)
    out_po[1:] = np.cumsum(sizes, dtype=np.int64)
    out_pay = (np.concatenate([pay[po[k]:po[k + 1]] for k in out_src]) if out_src
               else np.zeros(0, np.uint8))
    dt = np.int32 if a.offset_width == 4 else np.int64
    return Csr(n, n, np.asarray(out_rp, dtype=dt), np.asarray(out_col, dtype=np.int32),
               out_po.astype(dt), out_pay.astype(np.uint8), np.asarray(a.bounds, np.int64),
               a.offset_width, "symmetrized")


def triangle(a: Csr, lower: bool = True) -> Csr:
    """The cells of `a` on and below (lower) or above the diagonal, in their
    order: the stored triangle of a symmetric matrix."""
    rp = np.asarray(a.row_ptr, dtype=np.int64)
    col = np.asarray(a.col, dtype=np.int64)
    po = np.asarray(a.payload_off, dtype=np.int64)
    row_of = np.repeat(np.arange(a.n_rows, dtype=np.int64), np.diff(rp))
    keep = (col <= row_of) if lower else (col >= row_of)
    ks = np.nonzero(keep)[0]
    cnt = np.bincount(row_of[ks], minlength=a.n_rows)
    new_rp = np.zeros(a.n_rows + 1, dtype=np.int64)
    new_rp[1:] = np.cumsum(cnt)
    sizes = po[ks + 1] - po[ks]
    new_po = np.zeros(len(ks) + 1, dtype=np.int64)
    new_po[1:] = np.cumsum(sizes)
    pay = (np.concatenate([a.payload[po[k]:po[k + 1]] for k in ks]) if len(ks)
           else np.zeros(0, np.uint8))
    dt = np.int32 if a.offset_width == 4 else np.int64
    return Csr(a.n_rows, a.n_cols, new_rp.astype(dt), col[ks].astype(np.int32),
               new_po.astype(dt), pay.astype(np.uint8), np.asarray(a.bounds, np.int64),
               a.offset_width, "triangle")
