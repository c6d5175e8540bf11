"""GPU parity of the packed record form.

A call whose schedule has one records-only pass, made without a permutation
output, carries each cell as (column | size << column bits,
row) after the first pass and (column | size << column bits, row, payload
offset) after the second, instead of separate (column, size), (row, cell
index) and offset records. The first histogram checks that every payload
size fits beside the column; if one does not, the call keeps the wide
records. Either way the result must be the oracle's, bit for bit, and equal
to the same call with packing switched off (MGT_NO_PACK=1) and to the call
with a permutation output.
"""
import numpy as np
import pytest
import torch

from workloads import gen
from workloads.gen import from_arrays

from .common import assert_matches_oracle, host, to_device

pytestmark = pytest.mark.gpu


def _two_pass(a, partitioned, tile=0):
    """(pass bits, finish bits) of a schedule with exactly two partition
    passes for `a`, or None."""
    from paper_2012_06012_amd import mgt
    plan = mgt.plan_for(to_device(a), 0)
    for pb in (6, 5, 7, 4, 8, 3):
        for fb in (3, 4, 2, 5, 1, 6, 0, 7, 8):
            try:
                plan.set_schedule(pb, fb, tile)
            except mgt.MgtError:
                continue
            if plan.schedule(partitioned)["passes"] == 2:
                return pb, fb
    return None


def _run(a, partitioned, pass_bits, finish_bits, tile, perm=False):
    from paper_2012_06012_amd import mgt
    d = to_device(a)
    plan = mgt.plan_for(d, mgt.EMIT_PERM if perm else 0)
    plan.set_schedule(pass_bits, finish_bits, tile)
    sc = plan.schedule(partitioned)
    out, status = mgt.transpose(d, plan=plan, perm=perm, partitioned=partitioned)
    h = host(out)
    return h, int(status.cpu()[0]), sc


def _check(a, partitioned, tile, monkeypatch):
    pass_bits, finish_bits = _two_pass(a, partitioned, tile)
    h, st, sc = _run(a, partitioned, pass_bits, finish_bits, tile)
    assert sc["passes"] == 2, sc  # the schedule the packed form applies to
    assert st == 0
    assert_matches_oracle(a, h, partitioned=partitioned)
    monkeypatch.setenv("MGT_NO_PACK", "1")
    h2, st2, _ = _run(a, partitioned, pass_bits, finish_bits, tile)
    monkeypatch.delenv("MGT_NO_PACK")
    assert st2 == 0
    for k in h:
        if h[k] is not None:
            assert np.array_equal(h[k], h2[k]), k
    h3, st3, _ = _run(a, partitioned, pass_bits, finish_bits, tile, perm=True)
    assert st3 == 0
    assert_matches_oracle(a, h3, partitioned=partitioned)



@pytest.mark.parametrize("tile", [2048, 8192])  # 256-thread and 512-thread records-only pass
@pytest.mark.parametrize("partitioned", [False, True])
def test_large_recipe_two_passes(tile, partitioned, monkeypatch):
    a = gen.large(seed=3, scale=7)  # 2^16 columns, 2^22 cells
    _check(a, partitioned, tile, monkeypatch)


@pytest.mark.parametrize("seed,n_rows,n_cols,deg,wlo,whi,ow,sort_rows,parts", [
    (0, 3000, 5000, 10.0, 0, 33, 8, False, 1),
    (1, 4096, 4096, 30.0, 4, 4, 4, True, 16),
    (2, 20000, 20000, 4.0, 0, 9, 8, True, 64),
    (3, 9000, 9000, 6.0, 0, 0, 8, True, 3),     # no payload at all
    (4, 4096, 4096, 8.0, 0, 9, 8, False, 1024),
])
def test_random_shapes(seed, n_rows, n_cols, deg, wlo, whi, ow, sort_rows, parts, monkeypatch):
    a = gen.random_small(seed, n_rows=n_rows, n_cols=n_cols, deg_mean=deg, w_lo=wlo, w_hi=whi,
                         sort_rows=sort_rows, offset_width=ow, parts=parts)
    for partitioned in ((False, True) if parts > 1 else (False,)):
        _check(a, partitioned, 0, monkeypatch)


def test_hetero_fixed_width(monkeypatch):
    from paper_2012_06012_amd import mgt
    a = gen.hetero(seed=1, scale=9)  # 28-byte cells, 2^12 columns
    d = to_device(a)
    fixed = mgt.DeviceCsr(d.n_rows, d.n_cols, d.row_ptr, d.col, None, d.payload, a.bounds,
                          a.offset_width, True)
    for part in (False, True):
        sched = _two_pass(a, part)
        if sched is None:
            assert part  # 16-row partitions leave no room for two passes
            continue
        plan = mgt.plan_for(fixed, 0)
        plan.set_schedule(sched[0], sched[1], 0)
        assert plan.schedule(part)["passes"] == 2
        out, st = mgt.transpose(fixed, plan=plan, partitioned=part)
        h = host(out)
        assert int(st.cpu()[0]) == 0
        ref_h, _, _ = _run(a, part, sched[0], sched[1], 0, perm=True)
        for k in ("t_row_ptr", "t_col", "t_payload"):
            assert np.array_equal(h[k], ref_h[k]), k
        assert_matches_oracle(a, ref_h, partitioned=part)


def test_size_too_wide_to_pack_falls_back(monkeypatch):
    # 2^20 columns leave 12 bits for sizes: one cell of 5,000 bytes keeps the
    # whole call on the wide records; a cell of 4,095 bytes still packs
    for big in (5000, 4095, 4096):
        rng = np.random.default_rng(big)
        n_rows, n_cols = 3000, 1 << 20
        deg = rng.poisson(5.0, size=n_rows)
        rp = np.zeros(n_rows + 1, dtype=np.int64)
        np.cumsum(deg, out=rp[1:])
        nnz = int(rp[-1])
        col = np.sort(rng.integers(0, n_cols, size=nnz)).astype(np.int32)
        for i in range(n_rows):
            col[rp[i]:rp[i + 1]].sort()
        widths = rng.integers(0, 9, size=nnz)
        widths[nnz // 3] = big
        a = from_arrays(n_rows, n_cols, rp, col, widths=widths, fill_seed=big)
        _check(a, False, 0, monkeypatch)


@pytest.mark.parametrize("tile", [0, 4096])  # 4,096: the slim pass and 12-byte records
def test_graph_replays_packed(tile):
    # a recorded packed call: replays after the inputs change in place
    from paper_2012_06012_amd import mgt
    a = gen.random_small(21, n_rows=5000, n_cols=6000, deg_mean=6.0, w_lo=0, w_hi=17)
    d = to_device(a)
    plan = mgt.plan_for(d, 0)
    plan.set_schedule(*_two_pass(a, False, tile), tile)
    assert plan.schedule(False)["passes"] == 2
    g, out, status = mgt.transpose_graph(d, plan=plan)
    for k in range(3):
        rng = np.random.default_rng(k)
        col = a.col.copy()
        if k:
            col = rng.integers(0, a.n_cols, size=a.nnz).astype(np.int32)
            for i in range(a.n_rows):
                col[a.row_ptr[i]:a.row_ptr[i + 1]].sort()
        pay = rng.integers(0, 256, size=a.payload_bytes, dtype=np.uint8)
        b = gen.from_arrays(a.n_rows, a.n_cols, a.row_ptr, col, np.diff(a.payload_off), pay,
                            a.offset_width, a.bounds)
        d.col.copy_(torch.from_numpy(col))
        d.payload.copy_(torch.from_numpy(pay))
        for v in out.values():
            if v is not None and v.numel():
                v.view(torch.uint8).fill_(0xA5)
        status.fill_(77)
        torch.cuda.synchronize()
        g.launch()
        h = host(out)
        assert int(status.cpu()[0]) == 0
        assert_matches_oracle(b, h)
    g.close()


def test_validate_with_packed_records():
    # validation stops a packed call on a bad column exactly as a wide one
    from paper_2012_06012_amd import mgt
    a = gen.random_small(31, n_rows=4000, n_cols=5000, deg_mean=5.0, w_lo=0, w_hi=9)
    pb, fb = _two_pass(a, False)
    d = to_device(a)
    plan = mgt.plan_for(d, mgt.VALIDATE)
    plan.set_schedule(pb, fb, 0)
    out, st = mgt.transpose(d, plan=plan, validate=True)
    assert int(st.cpu()[0]) == 0
    assert_matches_oracle(a, host(out))
    bad = d.col.clone()
    bad[7] = a.n_cols + 3
    d.col.copy_(bad)
    out, st = mgt.transpose(d, plan=plan, validate=True)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == mgt.ERANGE


def test_hot_columns_packed(monkeypatch):
    # two hot columns: buckets of over 12,000 cells (many sub-chunks) beside
    # small ones, in one packed call
    rng = np.random.default_rng(41)
    n_rows, n_cols = 30000, 1 << 16
    deg = rng.poisson(3.0, size=n_rows) + 1
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    nnz = int(rp[-1])
    col = rng.integers(0, n_cols, size=nnz).astype(np.int32)
    hot = rng.random(nnz)
    col[hot < 0.25] = 777
    col[(hot >= 0.25) & (hot < 0.45)] = 40000
    for i in range(n_rows):
        col[rp[i]:rp[i + 1]].sort()
    a = from_arrays(n_rows, n_cols, rp, col, widths=rng.integers(0, 13, size=nnz), fill_seed=5)
    assert (col == 777).sum() > 12288
    _check(a, False, 0, monkeypatch)


@pytest.mark.parametrize("threads", [None, "512", "1024"])
def test_whole_bucket_forms(threads, monkeypatch):
    # packed buckets of every size class in one call: up to 4,608 cells (the
    # 512-thread whole-bucket finish, two workgroups per CU), up to 10,240 (the
    # 1,024-thread form, which runs after it and takes what it left) and more
    # (k_finish). Unset: both forms in turn; "512" or "1024": that form alone.
    if threads is not None:
        monkeypatch.setenv("MGT_BUCKET_THREADS", threads)
    rng = np.random.default_rng(43)
    n_rows, n_cols = 40000, 1 << 16
    deg = rng.poisson(2.0, size=n_rows) + 1
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    nnz = int(rp[-1])
    col = rng.integers(0, n_cols, size=nnz).astype(np.int32)
    hot = rng.random(nnz)
    col[hot < 0.06] = 1234                    # a bucket of 4,608 to 10,240 cells
    col[(hot >= 0.06) & (hot < 0.17)] = 50000  # a bucket of more than 10,240
    col[(hot >= 0.17) & (hot < 0.25)] = 20000  # one of 9,216 to 10,240 (1,024 threads only)
    for i in range(n_rows):
        col[rp[i]:rp[i + 1]].sort()
    assert 4608 < (col == 1234).sum() <= 9216 - 200 and (col == 50000).sum() > 10240
    assert 9216 < (col == 20000).sum() <= 10240 - 400
    a = from_arrays(n_rows, n_cols, rp, col, widths=rng.integers(0, 13, size=nnz) * 4,
                    fill_seed=7)
    _check(a, False, 0, monkeypatch)


@pytest.mark.parametrize("tile", [4096, 16384])
def test_nine_bit_records_pass(tile):
    # 2^23 columns with 6-bit finish buckets: 17 bits in two passes, the
    # second (records only, 512-thread form) taking 9
    from paper_2012_06012_amd import mgt
    n = 1 << 23
    a = gen.generate(1 << 16, n, seed=11, deg_law=gen.DEG_POISSON, deg_mean=64.0,
                     col_law=gen.COL_UNIFORM, mult_law=gen.MULT_GEOMETRIC, pay_law=gen.PAY_FLOATS,
                     w_lo=1, w_hi=8, offset_width=8, name="wide-columns")
    d = to_device(a)
    plan = mgt.plan_for(d, 0)
    plan.set_schedule(8, 6, tile)
    assert plan.schedule() == {"passes": 2, "bits": [8, 9], "finish_bits": 6, "tile_cells": tile,
                               "partition_pass": False}
    out, status = mgt.transpose(d, plan=plan)
    assert int(status.cpu()[0]) == 0
    assert_matches_oracle(a, host(out))


@pytest.mark.parametrize("threads", [None, "512", "1024"])
def test_twelve_byte_records_all_finish_forms(threads, monkeypatch):
    # a single matrix whose tiles hold 4,096 cells or more: its records-only
    # pass runs in the slim form and writes 12-byte records (payload offset
    # relative to the finish bucket's first byte), read back by every finish
    # path: buckets of up to 4,608 cells, up to 10,240, and more (k_finish)
    if threads is not None:
        monkeypatch.setenv("MGT_BUCKET_THREADS", threads)
    rng = np.random.default_rng(47)
    n_rows, n_cols = 200000, 1 << 16
    deg = rng.poisson(20.0, size=n_rows) + 1
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    nnz = int(rp[-1])
    col = rng.integers(0, n_cols, size=nnz).astype(np.int32)
    hot = rng.random(nnz)
    col[hot < 0.0017] = 1234
    col[(hot >= 0.0017) & (hot < 0.0047)] = 50000
    for i in range(n_rows):
        col[rp[i]:rp[i + 1]].sort()
    assert 4608 < (col == 1234).sum() <= 9000 and (col == 50000).sum() > 10240
    a = from_arrays(n_rows, n_cols, rp, col, widths=rng.integers(0, 13, size=nnz) * 4,
                    fill_seed=9)
    from paper_2012_06012_amd import mgt
    assert mgt.plan_for(to_device(a), 0).schedule()["tile_cells"] >= 4096
    _check(a, False, 0, monkeypatch)


@pytest.mark.parametrize("form", ["packed", "wide", "perm", "partitioned"])
def test_unaligned_cells_every_offset(form, monkeypatch):
    # cell sizes 0..40 bytes in a cycle, so source offsets take every value
    # modulo 16 and destination offsets every value modulo 4: cells of up to
    # 16 bytes (one or two aligned source blocks held in registers), 17 to 32
    # (copied in two halves) and longer (copied piece by piece), through the
    # first pass, the records-only pass and every finish form
    from paper_2012_06012_amd import mgt
    rng = np.random.default_rng(91)
    n_rows, n_cols = 30000, 1 << 14
    deg = rng.poisson(12.0, size=n_rows)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    nnz = int(rp[-1])
    col = rng.integers(0, n_cols, size=nnz).astype(np.int32)
    for i in range(n_rows):
        col[rp[i]:rp[i + 1]].sort()
    widths = (np.arange(nnz) * 7 + rng.integers(0, 3, size=nnz)) % 41
    parts = 8 if form == "partitioned" else 1
    bounds = None
    if parts > 1:
        bounds = np.linspace(0, n_rows, parts + 1).astype(np.int64)
        n_cols = n_rows  # partitioned matrices are square
        col = (col.astype(np.int64) * n_rows // (1 << 14)).astype(np.int32)
        for i in range(n_rows):
            col[rp[i]:rp[i + 1]].sort()
    a = from_arrays(n_rows, n_cols, rp, col, widths=widths, fill_seed=92, bounds=bounds)
    if form == "wide":
        monkeypatch.setenv("MGT_NO_PACK", "1")
    d = to_device(a)
    for tile in (0, 4096):
        plan = mgt.plan_for(d, mgt.EMIT_PERM if form == "perm" else 0)
        plan.set_schedule(8, -1, tile)
        out, st = mgt.transpose(d, plan=plan, perm=form == "perm", partitioned=parts > 1)
        assert int(st.cpu()[0]) == 0
        assert_matches_oracle(a, host(out), partitioned=parts > 1)


@pytest.mark.parametrize("ow", [8, 4])
@pytest.mark.parametrize("threads", [None, "512", "1024"])
def test_unaligned_small_cells_staged_finish(threads, ow, monkeypatch):
    # every cell of 0 to 16 bytes at any alignment: whole rounds of the
    # bucket finish take the staged path for unaligned cells (bytes shifted
    # into the wave's run in LDS), the first pass the register copy
    if threads is not None:
        monkeypatch.setenv("MGT_BUCKET_THREADS", threads)
    rng = np.random.default_rng(93)
    n_rows, n_cols = 60000, 1 << 15
    deg = rng.poisson(16.0, size=n_rows)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    nnz = int(rp[-1])
    col = rng.integers(0, n_cols, size=nnz).astype(np.int32)
    for i in range(n_rows):
        col[rp[i]:rp[i + 1]].sort()
    widths = rng.integers(0, 17, size=nnz)
    a = from_arrays(n_rows, n_cols, rp, col, widths=widths, offset_width=ow, fill_seed=94)
    from paper_2012_06012_amd import mgt
    d = to_device(a)
    for tile in (0, 4096):
        plan = mgt.plan_for(d, 0)
        plan.set_schedule(8, -1, tile)
        out, st = mgt.transpose(d, plan=plan)
        assert int(st.cpu()[0]) == 0
        assert_matches_oracle(a, host(out))
