"""GPU parity at the full sizes of the benchmark workloads, on the launch
configuration bench.py times (default plan, one call), checked on outputs the
oracle can produce piece by piece:

* every column's degree (the transposed row offsets) against a bincount of the
  input columns (torch's, on the device);
* complete transposed rows (ids, payload offsets relative to the row, payload
  bytes) for sampled column ranges, including the first and the last, from
  the oracle's column-range mode;
* for the partitioned form, the partition offsets against the transposed row
  offsets at the bounds, and the transfer-matrix sums against the cells per
  source and destination partition.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

from .common import to_device

pytestmark = pytest.mark.gpu


def _sampled_parity(a, d, out, ranges):
    deg = torch.bincount(d.col.long(), minlength=a.n_cols)
    assert torch.equal(torch.diff(out["t_row_ptr"].long()), deg)
    t_row_ptr = out["t_row_ptr"].cpu().numpy()
    assert int(t_row_ptr[-1]) == a.nnz
    for lo, hi in ranges:
        s = oracle.transpose_columns(a, lo, hi)
        p0, p1 = int(t_row_ptr[lo]), int(t_row_ptr[hi])
        assert np.array_equal(t_row_ptr[lo:hi + 1] - p0, s.t_row_ptr)
        assert np.array_equal(out["t_col"][p0:p1].cpu().numpy(), s.t_col)
        po = out["t_payload_off"][p0:p1 + 1].cpu().numpy()
        assert np.array_equal(po - po[0], s.t_payload_off)
        assert np.array_equal(out["t_payload"][int(po[0]):int(po[-1])].cpu().numpy(), s.t_payload)
    return t_row_ptr


def _ranges(n, width, seed):
    rng = np.random.default_rng(seed)
    return [(0, width), (n - width, n)] + [(int(c), int(c) + width)
                                           for c in rng.integers(0, n - width, size=3)]


def test_large_plain_full_size():
    from paper_2012_06012_amd import mgt
    a = gen.large(seed=0)                      # 2^23 x 2^23, 2^29 cells
    d = to_device(a)
    out, status = mgt.transpose(d)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 0
    _sampled_parity(a, d, out, _ranges(a.n_cols, 48, 1))
    del d, out
    torch.cuda.empty_cache()


def test_hetero_partitioned_full_size():
    from paper_2012_06012_amd import mgt
    a = gen.hetero(seed=0)                     # 2^21 x 2^21, 2^30 cells, R = 256
    d = to_device(a)
    out, status = mgt.transpose(d, partitioned=True)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 0
    t_row_ptr = _sampled_parity(a, d, out, _ranges(a.n_cols, 16, 2)[:4])
    b = np.asarray(a.bounds, np.int64)
    assert np.array_equal(out["part_cell_off"].cpu().numpy(), t_row_ptr[b])
    x = out["xfer_cells"].cpu().numpy()
    rows_per_part = np.diff(np.asarray(a.row_ptr, np.int64)[b])
    assert np.array_equal(x.sum(axis=1), rows_per_part)       # cells each source sends
    assert np.array_equal(x.sum(axis=0), np.diff(t_row_ptr[b]))  # cells each destination gets
    assert int(out["xfer_bytes"].cpu().numpy().sum()) == a.payload_bytes
    del d, out
    torch.cuda.empty_cache()
