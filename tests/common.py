"""Helpers shared by the GPU tests: move inputs to the device, run the C ABI
through the binding, bring results back and compare them with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from workloads.gen import Csr


def to_device(a: Csr, device="cuda", fixed_width=False):
    """Device copy of `a`. fixed_width: every cell has the same width, and the
    payload offsets are left on the host (the library must not need them)."""
    from paper_2012_06012_amd import mgt
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device)  # noqa: E731
    if fixed_width:
        w = np.diff(a.payload_off)
        assert w.size == 0 or (w == w[0]).all(), "cells of unequal width"
    return mgt.DeviceCsr(a.n_rows, a.n_cols, t(a.row_ptr), t(a.col),
                         None if fixed_width else t(a.payload_off), t(a.payload),
                         np.asarray(a.bounds, np.int64), a.offset_width, fixed_width)


def host(out: dict) -> dict:
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def gpu_transpose(a: Csr, partitioned=False, perm=True, validate=False):
    from paper_2012_06012_amd import mgt
    d = to_device(a)
    out, status = mgt.transpose(d, perm=perm, partitioned=partitioned, validate=validate)
    h = host(out)
    return h, int(status.cpu()[0])


def assert_matches_oracle(a: Csr, h: dict, check_perm=True, partitioned=False):
    t = oracle.transpose(a)
    assert np.array_equal(h["t_row_ptr"], t.t_row_ptr), "t_row_ptr"
    assert np.array_equal(h["t_col"], t.t_col), "t_col"
    assert np.array_equal(h["t_payload_off"], t.t_payload_off), "t_payload_off"
    assert np.array_equal(h["t_payload"], t.t_payload), "t_payload"
    if check_perm and h.get("perm") is not None:
        assert np.array_equal(h["perm"].view(np.uint32), t.perm), "perm"
    if partitioned:
        pc = oracle.partition_counts(a)
        for key in ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls",
                    "rdispls"):
            assert np.array_equal(h[key], getattr(pc, key)), key


def first_mismatch(x: np.ndarray, y: np.ndarray):
    if x.shape != y.shape:
        return f"shape {x.shape} vs {y.shape}"
    idx = np.nonzero(x != y)[0]
    return None if idx.size == 0 else (int(idx[0]), x[idx[0]], y[idx[0]], int(idx.size))
