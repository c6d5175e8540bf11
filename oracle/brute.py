"""Brute-force transpose for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Independent of oracle.c: lists every cell as an edge (row i, column j, cell
position k, payload e) and sorts the edges by their transposed key (j, i, k).
Section 2 defines the transpose edge by edge, E* = {(j, i, e) : (i, j, e) in E};
ordering by (j, i, k) places each transposed row's cells by original row and
keeps repeated (i, j) cells in their original order. Pure Python loops: use
only on inputs of a few hundred cells.
"""
from __future__ import annotations

import numpy as np


def edges(a):
    """(row, col, k, payload bytes) for every cell of a workloads.Csr."""
    out = []
    rp = [int(x) for x in a.row_ptr]
    po = [int(x) for x in a.payload_off]
    for i in range(a.n_rows):
        for k in range(rp[i], rp[i + 1]):
            out.append((i, int(a.col[k]), k, bytes(a.payload[po[k]:po[k + 1]])))
    return out


def transpose(a):
    """Returns (t_row_ptr, t_col, t_payload_off, t_payload, perm) as numpy arrays."""
    e = edges(a)
    e.sort(key=lambda t: (t[1], t[0], t[2]))
    t_row_ptr = [0] * (a.n_cols + 1)
    for (_, j, _, _) in e:
        t_row_ptr[j + 1] += 1
    for c in range(a.n_cols):
        t_row_ptr[c + 1] += t_row_ptr[c]
    t_col = [i for (i, _, _, _) in e]
    perm = [k for (_, _, k, _) in e]
    t_poff = [0]
    blob = bytearray()
    for (_, _, _, pay) in e:
        blob += pay
        t_poff.append(len(blob))
    return (np.array(t_row_ptr, dtype=np.int64), np.array(t_col, dtype=np.int32),
            np.array(t_poff, dtype=np.int64), np.frombuffer(bytes(blob), dtype=np.uint8),
            np.array(perm, dtype=np.uint32))
