"""GPU parity at the full sizes of the benchmark workloads, element by element.

Each test builds the whole workload on the host, runs the oracle once over the
whole matrix (``oracle.transpose_sliced``: the oracle's column-range mode over
disjoint column ranges in host threads, pinned against ``oracle.transpose``;
and ``oracle.partition_counts``), then runs
the library in the launch configurations the benchmarks time and compares
every output array in full: the transposed row offsets, column ids, payload
offsets and payload bytes, the cell permutation where one is emitted, and for
the partitioned form the transfer matrices, partition offsets and both
displacement matrices (paper Section 2: M^T_ij = M_ji with repeated cells in
input order; Section 3: the receiver's ordering by column, then row).

The large multigraph (2^29 cells) carries 9.66 GB of payload and the
heterogeneous one (2^30 cells) 30 GB, so payload offsets above 2^32 (the
high word of the records' offsets) are compared in full here.
"""
import gc

import numpy as np
import pytest
import torch

import oracle
from workloads import gen

from .common import first_mismatch, to_device

pytestmark = pytest.mark.gpu

_PART_KEYS = ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls", "rdispls")


def _log(msg):
    print(msg, flush=True)


def compare_full(out: dict, ref, pc=None, what: str = ""):
    """Every output array against the oracle's; arrays come to the host one at
    a time."""
    torch.cuda.synchronize()
    for k in ("t_row_ptr", "t_col", "t_payload_off", "t_payload", "perm"):
        t = out.get(k)
        if t is None:
            continue
        h = t.cpu().numpy()
        r = getattr(ref, k)
        if k == "perm":
            h = h.view(np.uint32)
        assert h.shape == r.shape and np.array_equal(h, r), (what, k, first_mismatch(h, r))
        del h
    if pc is not None:
        for k in _PART_KEYS:
            if out.get(k) is None:
                continue
            h = out[k].cpu().numpy()
            assert np.array_equal(h, getattr(pc, k)), (what, k)
    gc.collect()


def _run(d, *, partitioned, perm, what):
    from paper_2012_06012_amd import mgt
    _log(f"[fullsize] {what}: transpose")
    out, status = mgt.transpose(d, perm=perm, partitioned=partitioned)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == mgt.OK, what
    return out


def test_large_full_size():
    """Large multigraph (2^23 x 2^23, 2^29 cells, int64 offsets): the plain
    call the headline bench times (packed records, no perm), then the
    partitioned call with R = 64 and perm (wide records)."""
    a = gen.large(seed=0)
    _log(f"[fullsize] large: {a.nnz} cells, {a.payload_bytes} payload bytes")
    ref = oracle.transpose_sliced(a, slices=2 * oracle.host_threads())
    pc = oracle.partition_counts(a)
    d = to_device(a)
    out = _run(d, partitioned=False, perm=False, what="large plain")
    compare_full(out, ref, what="large plain")
    del out
    torch.cuda.empty_cache()
    out = _run(d, partitioned=True, perm=True, what="large partitioned R=64, perm")
    compare_full(out, ref, pc, what="large partitioned")
    del out, d, ref, pc, a
    gc.collect()
    torch.cuda.empty_cache()


def test_hetero_full_size():
    """Heterogeneous multigraph (2^21 x 2^21, 2^30 cells, 28-byte payload,
    R = 256): the partitioned call of its bench mode, then the fixed-width
    form (no payload offsets read on the device)."""
    a = gen.hetero(seed=0)
    _log(f"[fullsize] hetero: {a.nnz} cells, {a.payload_bytes} payload bytes")
    ref = oracle.transpose_sliced(a, slices=2 * oracle.host_threads())
    pc = oracle.partition_counts(a)
    ref.perm = None  # neither call below emits perm; frees 4 GB
    d = to_device(a)
    out = _run(d, partitioned=True, perm=False, what="hetero partitioned")
    compare_full(out, ref, pc, what="hetero partitioned")
    del out, d
    gc.collect()
    torch.cuda.empty_cache()
    from paper_2012_06012_amd import mgt
    d = to_device(a, fixed_width=True)
    _log("[fullsize] hetero fixed-width partitioned: transpose")
    out, status = mgt.transpose(d, partitioned=True)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == mgt.OK
    compare_full(out, ref, pc, what="hetero fixed-width")
    del out, d, ref, pc, a
    gc.collect()
    torch.cuda.empty_cache()


def test_payload_offsets_above_4g():
    """A mid-size matrix whose payload offsets cross 2^32 (2^20 x 2^20,
    about 8.4e7 cells of 48-80 bytes, 5.4 GB of payload), compared in full
    in every record form: packed (no perm), wide (perm), partitioned, and a
    forced three-pass schedule whose middle pass moves payload too."""
    from paper_2012_06012_amd import mgt
    n = 1 << 20
    a = gen.generate(n, n, seed=17, deg_law=gen.DEG_POISSON, deg_mean=80.0,
                     pay_law=gen.PAY_BYTES, w_lo=48, w_hi=80, offset_width=8,
                     bounds=gen.equal_bounds(n, 16))
    assert a.payload_bytes > 2**32, a.payload_bytes
    _log(f"[fullsize] >4G: {a.nnz} cells, {a.payload_bytes} payload bytes")
    ref = oracle.transpose_sliced(a, slices=2 * oracle.host_threads())
    pc = oracle.partition_counts(a)
    d = to_device(a)
    for perm, part in ((False, False), (True, False), (False, True)):
        what = f">4G perm={perm} partitioned={part}"
        out = _run(d, partitioned=part, perm=perm, what=what)
        compare_full(out, ref, pc if part else None, what=what)
        del out
        torch.cuda.empty_cache()
    plan = mgt.plan_for(d, 0)
    plan.set_schedule(6, 6, 0)  # 20 column bits: 14 over three passes, 6 in the finish
    assert plan.schedule()["passes"] == 3, plan.schedule()
    _log("[fullsize] >4G three passes: transpose")
    out, status = mgt.transpose(d, plan=plan)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == mgt.OK
    compare_full(out, ref, what=">4G three passes")
    del out, d, ref, pc, a
    gc.collect()
    torch.cuda.empty_cache()


def test_last_pass_segment_over_2g():
    """Packed records of a single large matrix are 12 bytes, the payload offset
    stored relative to the finish bucket's first byte in 32 bits. Here every
    cell lies in one first-pass segment of about 2.3 GB (2^24 columns, all
    cells in the lowest 2^16), too wide for that, so the call keeps 16-byte
    records; compared in full with the oracle."""
    from paper_2012_06012_amd import mgt
    n_rows, n_cols, deg = 1 << 20, 1 << 24, 32
    rng = np.random.default_rng(23)
    rp = np.arange(n_rows + 1, dtype=np.int64) * deg
    col = np.sort(rng.integers(0, 1 << 16, size=(n_rows, deg)), axis=1).astype(np.int32).ravel()
    widths = np.full(col.shape[0], 68, dtype=np.int64)
    a = gen.from_arrays(n_rows, n_cols, rp, col, widths=widths, fill_seed=23)
    assert a.payload_bytes >= 2**31, a.payload_bytes
    d = to_device(a)
    sc = mgt.plan_for(d, 0).schedule()
    assert sc["passes"] == 2 and sc["tile_cells"] >= 4096, sc  # the 12-byte record path
    _log(f"[fullsize] >2G segment: {a.nnz} cells, {a.payload_bytes} payload bytes, {sc}")
    ref = oracle.transpose_sliced(a, slices=2 * oracle.host_threads())
    out = _run(d, partitioned=False, perm=False, what=">2G segment")
    compare_full(out, ref, what=">2G segment")
    del out, d, ref, a
    gc.collect()
    torch.cuda.empty_cache()
