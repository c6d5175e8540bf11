"""Rank-by-rank simulation of the paper's staged transpose -- TEST INFRASTRUCTURE ONLY.

Follows Section 2 (sparse transpose in three steps) and Section 3 (local
transpose, view swap in two steps, final row-column ordering), with R ranks
simulated as separate arrays in one process. numpy's stable argsort is the only
library step. It shares nothing with oracle.c, so equality of the two pins the
counting-sort oracle to the paper's staged algorithm, including the transfer
matrices and displacements.

Stages, for ranks r = 0..R-1 owning rows [bounds[r], bounds[r+1]):
  1. Allgather of row counts -> rank row offsets (Section 2 step 1; Section 3
     intervals, 0-based).
  2. LocalTranspose (Section 3, eq. for LocalTranspose; Fig. 4): rank r orders
     its own cells by column, keeping original order among equal columns, and
     builds per-cell metadata (row id, column id, value count).
  3. Counts matrix X[r][s] and its Alltoall transpose (Section 2 step 2, Fig. 5).
  4. Alltoallv of metadata: rank r's cells for rank s are one contiguous run of
     its locally transposed order (columns of s form one interval).
  5. Value counts B[r][s], their Alltoall, and Alltoallv of the values
     (Section 3 / Fig. 6).
  6. Receiving rank s orders what it received by column (row-column ordering,
     Fig. 6); a stable sort keeps source-rank order, i.e. original row order.
  7. The distributed transpose is the vertical concatenation of the ranks'
     results (Section 3 concatenation; layout (d) of Fig. 1).
"""
from __future__ import annotations

import numpy as np


def run(a):
    R = a.n_parts
    bounds = np.asarray(a.bounds, dtype=np.int64)
    rp = np.asarray(a.row_ptr, dtype=np.int64)
    po = np.asarray(a.payload_off, dtype=np.int64)
    col = np.asarray(a.col, dtype=np.int64)
    # step 1: Allgather of row counts, offsets = exclusive scan
    row_counts = np.diff(bounds)
    offsets = np.concatenate([[0], np.cumsum(row_counts)])
    assert np.array_equal(offsets, bounds)
    owner_of = lambda v: np.searchsorted(offsets, v, side="right") - 1  # noqa: E731

    send_meta, send_vals, X, B = [], [], np.zeros((R, R), np.int64), np.zeros((R, R), np.int64)
    for r in range(R):
        k0, k1 = rp[offsets[r]], rp[offsets[r + 1]]
        ks = np.arange(k0, k1)
        rows = np.repeat(np.arange(offsets[r], offsets[r + 1]), np.diff(rp[offsets[r]:offsets[r + 1] + 1]))
        # step 2: local transpose = stable order by column
        order = np.argsort(col[ks], kind="stable")
        meta = np.stack([rows[order], col[ks][order], po[ks + 1][order] - po[ks][order], ks[order]], 1)
        vals = [a.payload[po[k]:po[k + 1]] for k in ks[order]]
        dst = owner_of(meta[:, 1]) if len(meta) else np.zeros(0, np.int64)
        # step 3: counts per destination (one row of X); bytes likewise (step 5)
        X[r] = np.bincount(dst, minlength=R) if len(meta) else 0
        B[r] = np.bincount(dst, weights=meta[:, 2], minlength=R).astype(np.int64) if len(meta) else 0
        send_meta.append(meta)
        send_vals.append(vals)
    recv_counts = X.T.copy()            # Alltoall of the counts matrix
    recv_bytes = B.T.copy()
    sdispls = np.zeros((R, R), np.int64)
    rdispls = np.zeros((R, R), np.int64)
    sdispls[:, 1:] = np.cumsum(X, axis=1)[:, :-1]
    rdispls[:, 1:] = np.cumsum(recv_counts, axis=1)[:, :-1]

    out_meta, out_vals = [], []
    for s in range(R):
        # step 4 + 5: Alltoallv of metadata and values into rank s
        blocks_m, blocks_v = [], []
        for r in range(R):
            lo = sdispls[r, s]
            hi = lo + X[r, s]
            blocks_m.append(send_meta[r][lo:hi])
            blocks_v.extend(send_vals[r][lo:hi])
        m = np.concatenate(blocks_m) if blocks_m else np.zeros((0, 4), np.int64)
        assert len(m) == recv_counts[s].sum()
        # step 6: the receiver orders what it got by column, then row (Fig. 6)
        order = np.argsort(m[:, 1], kind="stable")
        out_meta.append(m[order])
        out_vals.extend(blocks_v[i] for i in order)

    meta = np.concatenate(out_meta) if out_meta else np.zeros((0, 4), np.int64)
    t_row_ptr = np.zeros(a.n_cols + 1, np.int64)
    np.add.at(t_row_ptr, meta[:, 1] + 1, 1)
    t_row_ptr = np.cumsum(t_row_ptr)
    t_poff = np.concatenate([[0], np.cumsum(meta[:, 2])]).astype(np.int64)
    t_payload = np.concatenate(out_vals) if out_vals else np.zeros(0, np.uint8)
    part_cell_off = np.concatenate([[0], np.cumsum(recv_counts.sum(axis=1))])
    part_byte_off = np.concatenate([[0], np.cumsum(recv_bytes.sum(axis=1))])
    return dict(t_row_ptr=t_row_ptr, t_col=meta[:, 0].astype(np.int32),
                t_payload_off=t_poff, t_payload=t_payload.astype(np.uint8),
                perm=meta[:, 3].astype(np.uint32), xfer_cells=X, xfer_bytes=B,
                part_cell_off=part_cell_off, part_byte_off=part_byte_off,
                sdispls=sdispls, rdispls=rdispls)
