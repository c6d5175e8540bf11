"""C ABI checks that need no GPU: the library loads, exports every entry point
include/mgt.h declares, and rejects bad descriptors / arguments on the host
before anything is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2012_06012_amd import mgt
    return mgt


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "mgt.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(mgt_\w+)\(", txt, re.M)))


def test_header_symbols_exported():
    mgt = _lib()
    lib = ctypes.CDLL(mgt.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) <= set(mgt.EXPORTED)


def test_version():
    assert "gfx950" in _lib().version()


def test_plan_host_only_and_workspace_grows():
    mgt = _lib()
    p1 = mgt.mgt_plan(1000, 1000, 20000, 200000, 4, [0, 250, 500, 750, 1000])
    p2 = mgt.mgt_plan(1 << 20, 1 << 20, 1 << 24, 1 << 28, 8, None)
    assert 0 < p1.workspace_bytes < p2.workspace_bytes


def test_schedule_caps_from_environment(monkeypatch):
    # a longer schedule needs a second level buffer and the per-cell payload
    # offsets of its last pass: the workspace grows; out-of-range caps are ignored
    mgt = _lib()
    args = (30000, 30000, 150000, 1500000, 8, None)
    base = mgt.mgt_plan(*args).workspace_bytes
    monkeypatch.setenv("MGT_MAX_PASS_BITS", "4")
    monkeypatch.setenv("MGT_MAX_FINISH_BITS", "4")
    longer = mgt.mgt_plan(*args).workspace_bytes
    assert longer > base + 16 * 150000
    monkeypatch.setenv("MGT_MAX_PASS_BITS", "0")
    monkeypatch.setenv("MGT_MAX_FINISH_BITS", "11")
    assert mgt.mgt_plan(*args).workspace_bytes == base


@pytest.mark.parametrize("args,code", [
    ((-1, 10, 0, 0, 8, None), -1),                 # negative rows
    ((10, 10, 5, 0, 3, None), -1),                 # bad offset width
    ((10, 12, 5, 0, 8, [0, 5, 10]), -1),           # partitioned but not square
    ((10, 10, 5, 0, 8, [0, 6, 5, 10]), -1),        # decreasing bounds
    ((10, 10, 5, 0, 8, [1, 5, 10]), -1),           # bounds[0] != 0
    ((10, 10, 5, 0, 8, [0, 5, 9]), -1),            # bounds[R] != n_rows
    ((1 << 31, 10, 5, 0, 8, None), -5),            # too many rows
    ((10, 10, 1 << 32, 0, 8, None), -5),           # nnz beyond 2^32
    ((10, 10, 1 << 31, 0, 4, None), -5),           # int32 offsets overflow
    ((0, 10, 5, 0, 8, None), -1),                  # cells but no rows
])
def test_plan_rejects(args, code):
    mgt = _lib()
    with pytest.raises(mgt.MgtError) as e:
        mgt.mgt_plan(*args)
    assert e.value.code == code


def test_plan_rejects_too_many_parts():
    mgt = _lib()
    b = np.linspace(0, 5000, 1026).astype(np.int64)
    with pytest.raises(mgt.MgtError):
        mgt.mgt_plan(5000, 5000, 10, 0, 8, b)


def test_transpose_rejects_null_pointers_before_launch():
    mgt = _lib()
    p = mgt.mgt_plan(10, 10, 5, 0, 8, None)
    lib = ctypes.CDLL(mgt.LIB_PATH)
    lib.mgt_transpose.argtypes = [ctypes.c_void_p] * 10 + [ctypes.c_void_p, ctypes.c_size_t,
                                                          ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(4096)
    # missing col with nnz > 0
    rc = lib.mgt_transpose(p.handle, fake, None, fake, None, fake, fake, fake, None, None, fake,
                           1 << 20, None, None)
    assert rc == -1
    # perm given without MGT_EMIT_PERM
    rc = lib.mgt_transpose(p.handle, fake, fake, fake, None, fake, fake, fake, None, fake, fake,
                           1 << 20, None, None)
    assert rc == -1
    # misaligned workspace
    rc = lib.mgt_transpose(p.handle, fake, fake, fake, None, fake, fake, fake, None, None,
                           ctypes.c_void_p(4097), 1 << 20, None, None)
    assert rc == -1
    # workspace too small
    rc = lib.mgt_transpose(p.handle, fake, fake, fake, None, fake, fake, fake, None, None, fake,
                           16, None, None)
    assert rc == -3


def test_fixed_width_descriptor_and_offset_pointers():
    mgt = _lib()
    # payload bytes must split evenly over the cells; any size when there are none
    with pytest.raises(mgt.MgtError) as e:
        mgt.mgt_plan(10, 10, 4, 10, 8, None, mgt.FIXED_WIDTH)
    assert e.value.code == -1
    mgt.mgt_plan(10, 10, 0, 0, 8, None, mgt.FIXED_WIDTH)
    assert mgt.mgt_plan(10, 10, 4, 12, 8, None, mgt.FIXED_WIDTH).workspace_bytes > 0
    lib = ctypes.CDLL(mgt.LIB_PATH)
    lib.mgt_transpose.argtypes = [ctypes.c_void_p] * 10 + [ctypes.c_void_p, ctypes.c_size_t,
                                                          ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(4096)
    # without the flag the offset arrays are required ...
    p = mgt.mgt_plan(10, 10, 4, 12, 8, None)
    rc = lib.mgt_transpose(p.handle, fake, fake, None, fake, fake, fake, fake, fake, None, fake,
                           1 << 20, None, None)
    assert rc == -1
    rc = lib.mgt_transpose(p.handle, fake, fake, fake, fake, fake, fake, None, fake, None, fake,
                           1 << 20, None, None)
    assert rc == -1
    # ... with it both may be NULL (a too-small workspace is then the first error)
    p = mgt.mgt_plan(10, 10, 4, 12, 8, None, mgt.FIXED_WIDTH)
    rc = lib.mgt_transpose(p.handle, fake, fake, None, fake, fake, fake, None, fake, None, fake,
                           16, None, None)
    assert rc == -3


def test_view_plans():
    mgt = _lib()
    b = [0, 30, 100]
    for op in (mgt.LOCAL_TRANSPOSE, mgt.VIEW_SWAP):
        for view in (mgt.ROW_VIEW, mgt.COLUMN_VIEW):
            assert mgt.mgt_view_plan(100, 100, 500, 2000, 8, b, op, view).workspace_bytes > 0
    for args, code in [((100, 90, 500, 2000, 8, b, 0, 0), -1),     # partitioned, not square
                       ((100, 100, 500, 2000, 8, b, 2, 0), -1),    # unknown operation
                       ((100, 100, 500, 2000, 8, b, 0, 2), -1),    # unknown view
                       ((1 << 21, 1 << 21, 10, 0, 8,               # R * n_cols >= 2^31
                         np.linspace(0, 1 << 21, 1025).astype(np.int64), 0, 0), -5)]:
        with pytest.raises(mgt.MgtError) as e:
            mgt.mgt_view_plan(*args)
        assert e.value.code == code
    # with one partition the matrix may be rectangular
    assert mgt.mgt_view_plan(50, 80, 100, 0, 4, None, mgt.VIEW_SWAP, mgt.ROW_VIEW).workspace_bytes
    # a view plan is not a transpose plan
    p = mgt.mgt_view_plan(10, 10, 5, 0, 8, None, mgt.LOCAL_TRANSPOSE, mgt.ROW_VIEW)
    lib = ctypes.CDLL(mgt.LIB_PATH)
    lib.mgt_transpose.argtypes = [ctypes.c_void_p] * 10 + [ctypes.c_void_p, ctypes.c_size_t,
                                                          ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(4096)
    rc = lib.mgt_transpose(p.handle, fake, fake, fake, None, fake, fake, fake, None, None, fake,
                           1 << 30, None, None)
    assert rc == -1


def test_partitioned_rejects_missing_outputs():
    mgt = _lib()
    p = mgt.mgt_plan(10, 10, 5, 0, 8, [0, 5, 10])
    lib = ctypes.CDLL(mgt.LIB_PATH)
    lib.mgt_transpose_partitioned.argtypes = [ctypes.c_void_p] * 16 + [
        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(4096)
    rc = lib.mgt_transpose_partitioned(p.handle, fake, fake, fake, None, fake, fake, fake, None,
                                       None, None, fake, fake, fake, None, None, fake, 1 << 30,
                                       None, None)
    assert rc == -1


def test_graph_create_rejects_before_recording():
    mgt = _lib()
    lib = ctypes.CDLL(mgt.LIB_PATH)
    lib.mgt_graph_create.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 16 + [
        ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.mgt_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.mgt_graph_destroy.argtypes = [ctypes.c_void_p]
    fake = ctypes.c_void_p(4096)
    g = ctypes.c_void_p()

    def create(plan, part=0, col=fake, out=True):
        return lib.mgt_graph_create(plan, part, fake, col, fake, None, fake, fake, fake, None,
                                    None, fake, fake, fake, fake, None, None, fake, 1 << 30, None,
                                    ctypes.byref(g) if out else None)

    assert create(None) == -1
    assert create(mgt.mgt_plan(10, 10, 5, 0, 8, None).handle, out=False) == -1
    assert create(mgt.mgt_plan(10, 10, 5, 0, 8, None).handle, col=None) == -1   # missing col
    assert create(mgt.mgt_plan(10, 10, 5, 0, 8, None, flags=mgt.DEBUG_TIMING).handle) == -1
    assert create(mgt.mgt_view_plan(10, 10, 5, 0, 8, None, mgt.VIEW_SWAP,
                                    mgt.ROW_VIEW).handle) == -1
    assert g.value is None
    assert lib.mgt_graph_launch(None, None) == -1
    assert lib.mgt_graph_destroy(None) == -1


def test_batch_plan_limits_and_exact_workspace():
    mgt = _lib()
    with pytest.raises(mgt.MgtError):
        mgt.mgt_batch_plan(0, 1, 1, 1, 1, 1, 1)
    bp = mgt.mgt_batch_plan(4, 10**6, 10**5, 10**5, 64, 10**6, 10**5)
    fake = ctypes.c_void_p(4096)

    class T:  # minimal stand-in with a data_ptr for host-only sizing
        def __init__(self, n):
            self.n = n

        def numel(self):
            return self.n

        def data_ptr(self):
            return 4096

    entries = []
    for n, nnz in [(1000, 8000), (3000, 50000)]:
        d = mgt.Desc(n, n, nnz, nnz * 3, 8, 1, None, 0)
        e = dict(desc=d)
        for k in ("row_ptr", "col", "payload_off", "payload", "t_row_ptr", "t_col",
                  "t_payload_off", "t_payload"):
            e[k] = T(8)
        entries.append(e)
    items = mgt.make_items(entries)
    ws = mgt.mgt_batch_workspace(bp, items)
    assert ws > (16 + 3) * 58000  # records + payload of every cell, at least once
    # too many items for the plan
    items5 = mgt.make_items(entries * 3)
    with pytest.raises(mgt.MgtError):
        mgt.mgt_batch_workspace(bp, items5)


def test_value_list_calls_reject_before_launch():
    mgt = _lib()
    lib = ctypes.CDLL(mgt.LIB_PATH)
    assert mgt.mgt_value_lists_workspace(0) >= 256
    assert mgt.mgt_value_lists_workspace(1 << 20) > mgt.mgt_value_lists_workspace(1 << 10)
    with pytest.raises(mgt.MgtError):
        mgt.mgt_value_lists_workspace(1 << 32)
    v, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.mgt_coalesce.argtypes = [i64, i64, i32] + [v] * 9 + [sz, v]
    lib.mgt_expand.argtypes = [i64, i64, i64, i32, i32] + [v] * 8
    lib.mgt_counts_to_offsets.argtypes = [i64, v, i32, i32, v, v, sz, v]
    fake = ctypes.c_void_p(4096)
    ws = mgt.mgt_value_lists_workspace(100)
    # bad offset width, missing outputs, misaligned or short workspace
    assert lib.mgt_coalesce(10, 100, 2, fake, fake, fake, fake, fake, fake, None, None, fake, ws,
                            None) == -1
    assert lib.mgt_coalesce(10, 100, 8, fake, fake, fake, fake, None, fake, None, None, fake, ws,
                            None) == -1
    assert lib.mgt_coalesce(10, 100, 8, fake, fake, fake, fake, fake, fake, None, None,
                            ctypes.c_void_p(4097), ws, None) == -1
    assert lib.mgt_coalesce(10, 100, 8, fake, fake, fake, fake, fake, fake, None, None, fake, 16,
                            None) == -3
    # payload not a whole number of values; zero value width; too many values
    assert lib.mgt_expand(10, 100, 401, 8, 4, fake, fake, fake, fake, fake, None, None, None) == -1
    assert lib.mgt_expand(10, 100, 400, 8, 0, fake, fake, fake, fake, fake, None, None, None) == -1
    assert lib.mgt_expand(10, 100, 1 << 40, 8, 4, fake, fake, fake, fake, fake, None, None,
                          None) == -5
    assert lib.mgt_counts_to_offsets(100, None, 4, 8, fake, fake, ws, None) == -1


def test_plan_schedule_settings():
    mgt = _lib()
    b = [i * (1 << 17) for i in range(65)]
    p = mgt.mgt_plan(1 << 23, 1 << 23, 1 << 29, 9663557316, 8, b)
    # the records-only pass of a single large matrix takes 9 bits (its 512-thread
    # form), so two passes reach finish buckets of 2^6 columns, ~4,096 cells
    assert p.schedule() == {"passes": 2, "bits": [8, 9], "finish_bits": 6, "tile_cells": 16384,
                            "partition_pass": False}
    # 64 partitions x 4: a fan-out of 256, whose segments hold 38 MB of payload on average
    assert p.schedule(True)["partition_pass"] and p.schedule(True)["bits"] == [2, 9]
    # 30 GB over 256 partitions: 256 segments would average 117 MB, so the
    # partition pass takes a fan-out of 512 (256 x 2)
    h = mgt.mgt_plan(1 << 21, 1 << 21, 1 << 30, 28 << 30, 8, [i * (1 << 13) for i in range(257)])
    # (a 9-bit last pass would leave finish buckets of 8 columns: kept at 8 bits)
    assert h.schedule(True) == {"passes": 2, "bits": [1, 8], "finish_bits": 4, "tile_cells": 16384,
                                "partition_pass": True}
    # tiles under 4,096 cells keep the last pass at 8 bits
    p.set_schedule(8, -1, 2048)
    assert p.schedule()["bits"] == [8, 8] and p.schedule()["finish_bits"] == 7
    p.set_schedule()
    h2 = mgt.mgt_plan(1 << 21, 1 << 21, 1 << 30, 8 << 30, 8, [i * (1 << 13) for i in range(257)])
    assert h2.schedule(True)["bits"][0] == 0  # 8 GB: 256 segments of 32 MB
    ws0 = p.workspace_bytes
    p.set_schedule(7, 9, 8192)
    assert p.schedule() == {"passes": 2, "bits": [7, 7], "finish_bits": 9, "tile_cells": 8192,
                            "partition_pass": False}
    assert p.schedule(True)["bits"] == [2, 6]          # 17 column bits per partition: 2 + 6 + 9
    with pytest.raises(mgt.MgtError) as e:            # 20 bits in passes of at most 4: five passes
        p.set_schedule(4, 3, 0)
    assert e.value.code == -5
    assert p.schedule()["finish_bits"] == 9           # a refused setting changes nothing
    p.set_schedule(5, 8, 0)                            # 15 bits in passes of at most 5: three
    assert p.schedule()["passes"] == 3 and sum(p.schedule()["bits"]) == 15
    assert p.set_schedule() == ws0 and p.schedule()["finish_bits"] == 6
    for bad in ((9, -1, 0), (-1, -1, 0), (0, 11, 0), (0, -2, 0), (0, -1, 1000), (0, -1, 32768)):
        with pytest.raises(mgt.MgtError):
            p.set_schedule(*bad)
    v = mgt.mgt_view_plan(10, 10, 5, 0, 8, None, mgt.VIEW_SWAP, mgt.ROW_VIEW)
    with pytest.raises(mgt.MgtError):
        v.set_schedule(8, -1, 0)


def test_batch_plan_takes_a_schedule():
    mgt = _lib()
    bp = mgt.mgt_batch_plan(8, 1 << 20, 1 << 20, 1 << 20, 8, 1 << 20, 1 << 20, 8)
    est = bp.workspace_bytes
    for setting in ((4, -1, 8192), (6, -1, 16384), (8, -1, 0), (0, -1, 0)):
        assert bp.set_schedule(*setting) == est      # the plan's estimate, unchanged
    for bad in ((9, -1, 0), (-1, -1, 0), (0, 11, 0), (0, -1, 1000)):
        with pytest.raises(mgt.MgtError):
            bp.set_schedule(*bad)
    with pytest.raises(mgt.MgtError):                 # schedules are read on single-matrix plans
        bp.schedule()


def test_autotune_shape_classes():
    import numpy as np
    from paper_2012_06012_amd import autotune
    mgt = _lib()

    class Fake:  # the fields shape_key reads (no device needed)
        def __init__(self, nnz, n_cols, pbytes):
            self.nnz, self.n_cols, self.n_rows, self.payload_bytes = nnz, n_cols, n_cols, pbytes
            self.offset_width, self.bounds, self.fixed_width = 8, np.array([0, n_cols]), False
            self.n_parts = 1
            self.col = type("C", (), {"device": "cpu"})()
    k1 = autotune.shape_key(Fake(1 << 29, 1 << 23, 9 << 30), False, False)
    k2 = autotune.shape_key(Fake((1 << 29) + 12345, (1 << 23) - 7, (9 << 30) + 99), False, False)
    k3 = autotune.shape_key(Fake(1 << 27, 1 << 23, 9 << 28), False, False)
    assert k1 == k2 and k1 != k3   # one class for nearby shapes, another for 4x fewer cells
    b1 = autotune.batch_shape_key([Fake(1000, 100, 8000), Fake(3000, 300, 24000)], False)
    b2 = autotune.batch_shape_key([Fake(1100, 110, 8800), Fake(2900, 290, 23000)], False)
    assert b1 == b2
