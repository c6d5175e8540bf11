"""CPU oracle for the XCSR multigraph transpose -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It wraps ``oracle.c`` (a plain single-threaded
counting-sort transpose written from the paper's definitions) and adds two
pure-Python/numpy cross-checks: ``brute`` (sort every cell by its transposed
key) and ``staged`` (a rank-by-rank simulation of the paper's staged
algorithm), ``views`` (the Section 3 LocalTranspose and ViewSwap on their
own) and ``values`` (XCSR value lists against repeated cells, Section 2).
``scantrans.c`` is the multi-threaded CPU baseline the benchmark reports
beside the oracle (``transpose_mt``); the tests pin it against ``oracle.c``.
The GPU library shares no code with anything here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_MT_SRC = os.path.join(_HERE, "scantrans.c")
_MT_LIB = os.path.join(_HERE, "libscantrans.so")

OK, EINVAL, ERANGE, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -5

# MGT_HOST_SANITIZE=1 builds and loads copies instrumented with the address
# and undefined-behaviour sanitizers instead (the process must then preload
# the address sanitizer's runtime; tests/test_sanitizers.py does).
SANITIZE = os.environ.get("MGT_HOST_SANITIZE", "") == "1"
SANITIZE_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]
if SANITIZE:
    _LIB = _LIB.replace(".so", "_san.so")
    _MT_LIB = _MT_LIB.replace(".so", "_san.so")


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, gcc) in place."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        opt = SANITIZE_FLAGS if SANITIZE else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=c99", "-Wall", "-fPIC", "-shared", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_MT_LIB) or \
            os.path.getmtime(_MT_LIB) < os.path.getmtime(_MT_SRC):
        tmp = _MT_LIB + ".tmp"
        opt = SANITIZE_FLAGS if SANITIZE else ["-O3"]
        subprocess.check_call(["gcc", *opt, "-std=gnu99", "-Wall", "-fPIC", "-shared", "-pthread",
                               _MT_SRC, "-o", tmp])
        os.replace(tmp, _MT_LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.mgo_validate.argtypes = [i64, i64, i32, vp, vp, vp, i32, vp]
        lib.mgo_transpose.argtypes = [i64, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.mgo_partition_counts.argtypes = [i64, i64, i32, vp, vp, vp, i32, vp, vp, vp, vp,
                                             vp, vp, vp]
        lib.mgo_transpose_columns.argtypes = [i64, i64, i32, vp, vp, vp, vp, i64, i64, vp, vp,
                                              vp, vp, vp, vp, vp]
        for f in (lib.mgo_validate, lib.mgo_transpose, lib.mgo_partition_counts,
                  lib.mgo_transpose_columns):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data if a.size else None


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle rejected the input (status {code})")
        self.code = code


@dataclass
class Transposed:
    """Transposed XCSR: t_row_ptr has n_cols+1 entries; t_col holds original row ids."""
    t_row_ptr: np.ndarray
    t_col: np.ndarray
    t_payload_off: np.ndarray
    t_payload: np.ndarray
    perm: np.ndarray


@dataclass
class PartitionCounts:
    xfer_cells: np.ndarray   # [R, R], [src, dst]
    xfer_bytes: np.ndarray   # [R, R]
    part_cell_off: np.ndarray  # [R+1]
    part_byte_off: np.ndarray  # [R+1]
    sdispls: np.ndarray      # [R, R]: send displacement of block src->dst inside src's send buffer
    rdispls: np.ndarray      # [R, R]: [dst, src] receive displacement inside dst's receive buffer


def validate(a, n_parts: int = 0) -> int:
    b = np.ascontiguousarray(a.bounds, dtype=np.int64) if n_parts else None
    return _load().mgo_validate(a.n_rows, a.n_cols, a.offset_width, _p(a.row_ptr), _p(a.col),
                                _p(a.payload_off), n_parts, _p(b))


def alloc_transposed(a) -> Transposed:
    """Output arrays for ``transpose(a, out=...)``, written once so their pages
    are resident before a timed call."""
    dt = np.int32 if a.offset_width == 4 else np.int64
    t = Transposed(np.empty(a.n_cols + 1, dtype=dt), np.empty(a.nnz, dtype=np.int32),
                   np.empty(a.nnz + 1, dtype=dt), np.empty(a.payload_bytes, dtype=np.uint8),
                   np.empty(a.nnz, dtype=np.uint32))
    for x in (t.t_row_ptr, t.t_col, t.t_payload_off, t.t_payload, t.perm):
        x.fill(0)
    return t


def transpose(a, out: Optional[Transposed] = None) -> Transposed:
    """Transpose of a workloads.Csr (plain definition, Gustavson counting sort).
    ``out`` (from ``alloc_transposed``) receives the result when given."""
    if out is None:
        dt = np.int32 if a.offset_width == 4 else np.int64
        nnz = a.nnz
        out = Transposed(np.zeros(a.n_cols + 1, dtype=dt), np.zeros(nnz, dtype=np.int32),
                         np.zeros(nnz + 1, dtype=dt), np.zeros(a.payload_bytes, dtype=np.uint8),
                         np.zeros(nnz, dtype=np.uint32))
    t_row_ptr, t_col, t_poff, t_payload, perm = (out.t_row_ptr, out.t_col, out.t_payload_off,
                                                 out.t_payload, out.perm)
    st = _load().mgo_transpose(a.n_rows, a.n_cols, a.offset_width, _p(a.row_ptr), _p(a.col),
                               _p(a.payload_off), _p(a.payload), _p(t_row_ptr), _p(t_col),
                               _p(t_poff), _p(t_payload), _p(perm))
    if st != OK:
        raise OracleError(st)
    return out


_mt_lib = None


def host_threads(cap: int = 16) -> int:
    """CPUs this process may run on, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def transpose_mt(a, threads: int, perm: bool = True) -> Transposed:
    """The multi-threaded scan-based CPU baseline (``scantrans.c``); same
    result as ``transpose``."""
    global _mt_lib
    if _mt_lib is None:
        if not os.path.exists(_MT_LIB):
            build(force=False)
        lib = ctypes.CDLL(_MT_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.mgs_transpose.argtypes = [i64, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]
        lib.mgs_transpose.restype = ctypes.c_int
        _mt_lib = lib
    dt = np.int32 if a.offset_width == 4 else np.int64
    nnz = a.nnz
    t_row_ptr = np.empty(a.n_cols + 1, dtype=dt)
    t_col = np.empty(nnz, dtype=np.int32)
    t_poff = np.empty(nnz + 1, dtype=dt)
    t_payload = np.empty(a.payload_bytes, dtype=np.uint8)
    pm = np.empty(nnz, dtype=np.uint32) if perm else None
    st = _mt_lib.mgs_transpose(a.n_rows, a.n_cols, a.offset_width, _p(a.row_ptr), _p(a.col),
                               _p(a.payload_off), _p(a.payload), _p(t_row_ptr), _p(t_col),
                               _p(t_poff), _p(t_payload), _p(pm), int(threads))
    if st != OK:
        raise OracleError(st)
    return Transposed(t_row_ptr, t_col, t_poff, t_payload, pm)


def partition_counts(a) -> PartitionCounts:
    R = a.n_parts
    bounds = np.ascontiguousarray(a.bounds, dtype=np.int64)
    x = np.zeros((R, R), dtype=np.int64)
    b = np.zeros((R, R), dtype=np.int64)
    pc = np.zeros(R + 1, dtype=np.int64)
    pb = np.zeros(R + 1, dtype=np.int64)
    sd = np.zeros((R, R), dtype=np.int64)
    rd = np.zeros((R, R), dtype=np.int64)
    st = _load().mgo_partition_counts(a.n_rows, a.n_cols, a.offset_width, _p(a.row_ptr),
                                      _p(a.col), _p(a.payload_off), R, _p(bounds), _p(x), _p(b),
                                      _p(pc), _p(pb), _p(sd), _p(rd))
    if st != OK:
        raise OracleError(st)
    return PartitionCounts(x, b, pc, pb, sd, rd)


def transpose_columns(a, c_lo: int, c_hi: int) -> Transposed:
    """Transpose restricted to output rows [c_lo, c_hi); offsets relative to the slice."""
    lib = _load()
    cells = ctypes.c_int64(0)
    nbytes = ctypes.c_int64(0)
    args = (a.n_rows, a.n_cols, a.offset_width, _p(a.row_ptr), _p(a.col), _p(a.payload_off),
            _p(a.payload), c_lo, c_hi)
    st = lib.mgo_transpose_columns(*args, None, None, None, None, None, ctypes.byref(cells),
                                   ctypes.byref(nbytes))
    if st != OK:
        raise OracleError(st)
    t_row_ptr = np.zeros(c_hi - c_lo + 1, dtype=np.int64)
    t_col = np.zeros(cells.value, dtype=np.int32)
    t_poff = np.zeros(cells.value + 1, dtype=np.int64)
    t_payload = np.zeros(nbytes.value, dtype=np.uint8)
    perm = np.zeros(cells.value, dtype=np.uint32)
    st = lib.mgo_transpose_columns(*args, _p(t_row_ptr), _p(t_col), _p(t_poff[:-1]) if cells.value else None,
                                   _p(t_payload), _p(perm), None, None)
    if st != OK:
        raise OracleError(st)
    t_poff[-1] = nbytes.value
    return Transposed(t_row_ptr, t_col, t_poff, t_payload, perm)


def transpose_sliced(a, slices: int = 16, threads: int = 0) -> Transposed:
    """The whole transpose assembled from ``slices`` column ranges, each made
    by the oracle's column-range mode (``mgo_transpose_columns``) in a thread
    of its own; the same arrays as ``transpose``. Output row block
    [c_lo, c_hi) of the transpose depends only on the input cells whose
    column lies in it, so the slices are independent: each lands at the
    cells and bytes of all earlier slices. For full-size checks on hosts with
    many cores; pinned against ``transpose`` by the tests."""
    from concurrent.futures import ThreadPoolExecutor
    lib = _load()
    n_cols, nnz = int(a.n_cols), int(a.nnz)
    slices = max(1, min(int(slices), max(n_cols, 1)))
    edges = [n_cols * s // slices for s in range(slices + 1)]
    ranges = [(edges[s], edges[s + 1]) for s in range(slices)]
    base = (a.n_rows, a.n_cols, a.offset_width, _p(a.row_ptr), _p(a.col), _p(a.payload_off),
            _p(a.payload))
    threads = threads or host_threads()

    def size(r):
        cells, nbytes = ctypes.c_int64(0), ctypes.c_int64(0)
        st = lib.mgo_transpose_columns(*base, r[0], r[1], None, None, None, None, None,
                                       ctypes.byref(cells), ctypes.byref(nbytes))
        if st != OK:
            raise OracleError(st)
        return cells.value, nbytes.value

    with ThreadPoolExecutor(threads) as ex:
        sizes = list(ex.map(size, ranges))
    cell0 = np.concatenate([[0], np.cumsum([c for c, _ in sizes])]).astype(np.int64)
    byte0 = np.concatenate([[0], np.cumsum([b for _, b in sizes])]).astype(np.int64)
    if int(cell0[-1]) != nnz:
        raise OracleError(ERANGE)
    dt = np.int32 if a.offset_width == 4 else np.int64
    t_row_ptr = np.empty(n_cols + 1, dtype=dt)
    t_col = np.empty(nnz, dtype=np.int32)
    t_poff = np.empty(nnz + 1, dtype=dt)
    t_payload = np.empty(int(byte0[-1]), dtype=np.uint8)
    perm = np.empty(nnz, dtype=np.uint32)

    def fill(s):
        (lo, hi), c0, b0 = ranges[s], int(cell0[s]), int(byte0[s])
        cells = int(cell0[s + 1]) - c0
        rp = np.empty(hi - lo + 1, dtype=np.int64)
        po = np.empty(cells, dtype=np.int64)
        st = lib.mgo_transpose_columns(*base, lo, hi, _p(rp), _p(t_col[c0:c0 + cells]),
                                       _p(po), _p(t_payload[b0:int(byte0[s + 1])]),
                                       _p(perm[c0:c0 + cells]), None, None)
        if st != OK:
            raise OracleError(st)
        t_row_ptr[lo:hi] = (rp[:-1] + c0).astype(dt)
        t_poff[c0:c0 + cells] = (po + b0).astype(dt)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, range(slices)))
    t_row_ptr[n_cols] = nnz
    t_poff[nnz] = int(byte0[-1])
    return Transposed(t_row_ptr, t_col, t_poff, t_payload, perm)
