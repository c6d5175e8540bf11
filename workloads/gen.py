"""Seeded synthetic XCSR multigraph workloads (inputs only).

The arrays produced here are the *inputs* of a transpose: row offsets, column
ids, per-cell payload offsets and payload bytes, plus partition bounds. Nothing
in this module computes any part of the transpose; the CPU oracle and the GPU
library both consume these arrays unchanged.

XCSR (the paper's Section 2, "eXtended Compressed Sparse Row") stores a matrix
as CSR plus a per-cell value count. Here every cell's values are an opaque byte
string, so the value count becomes a byte width and the value list a byte
range: ``payload[payload_off[k]:payload_off[k+1]]`` belongs to cell ``k``.

Workload recipes (all seeded, all synthetic):

* ``tiny``: 1,000 x 1,000, row degree Poisson(20), uniform columns, each drawn
  column repeated Geometric(1/2) times, rows sorted by column; payload is 1-3
  float32 in [0,1) followed by an int32 tag equal to the cell's index; int32
  offsets; R = 4 equal row blocks.
* ``large``: 2^23 x 2^23 with exactly 2^29 cells, 2^23 per each of R = 64
  equal row blocks; degrees drawn from a power law (alpha 2.1, d >= 10, capped
  at 10^5) then rescaled inside each block to its exact total; uniform columns,
  Geometric(1/2) multiplicity; payload 1-8 float32; int64 offsets.
* ``hetero``: 2^21 x 2^21 with 2^30 cells over R = 256 equal row blocks whose
  totals are proportional to 10^u, u ~ U[0,1); rows of a block share its total
  evenly; each drawn column lies in a +/-5% window around the row (wrapping),
  repeated U{1..50} times; fixed 28-byte payload (5 float32, int32 source row,
  int32 source column); int64 offsets.
* ``batch`` / ``served`` item generators: per-item sizes drawn log-uniformly,
  Poisson degrees with an integer mean U{8..64}, Geometric(1/2) multiplicity,
  random-byte payloads of one width per item.

Every recipe takes ``scale`` (a right shift applied to rows and cells) so tests
can run the same shape at a size the oracle finishes in seconds.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "libmgtgen.so")

DEG_POISSON, DEG_POWERLAW_BALANCED, DEG_PART_WEIGHTED, DEG_FIXED, DEG_UNIFORM = range(5)
COL_UNIFORM, COL_WINDOW = range(2)
MULT_GEOMETRIC, MULT_UNIFORM, MULT_ONE = range(3)
PAY_FLOATS_TAG, PAY_FLOATS, PAY_FLOATS_ROWCOL, PAY_BYTES, PAY_TAG64 = range(5)


class _Spec(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("seed", ctypes.c_uint64),
        ("deg_law", ctypes.c_int32), ("deg_mean", ctypes.c_double),
        ("deg_min", ctypes.c_int64), ("deg_max", ctypes.c_int64),
        ("target_nnz", ctypes.c_int64), ("n_parts", ctypes.c_int32),
        ("col_law", ctypes.c_int32), ("window", ctypes.c_int64),
        ("mult_law", ctypes.c_int32), ("mult_max", ctypes.c_int32),
        ("sort_rows", ctypes.c_int32), ("pay_law", ctypes.c_int32),
        ("w_lo", ctypes.c_int32), ("w_hi", ctypes.c_int32), ("threads", ctypes.c_int32),
    ]


# MGT_HOST_SANITIZE=1 builds and loads a copy instrumented with the address
# and undefined-behaviour sanitizers instead (the process must then preload
# the address sanitizer's runtime; tests/test_sanitizers.py does).
SANITIZE = os.environ.get("MGT_HOST_SANITIZE", "") == "1"
SANITIZE_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]
if SANITIZE:
    _LIB = _LIB.replace(".so", "_san.so")


def build(force: bool = True) -> str:
    """Compile the generator library in place (g++, host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        opt = SANITIZE_FLAGS if SANITIZE else ["-O2"]
        subprocess.check_call(["g++", *opt, "-std=c++17", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Spec)
        vp = ctypes.c_void_p
        lib.mgg_degrees.argtypes = [P, vp]
        lib.mgg_degrees.restype = ctypes.c_int64
        lib.mgg_fill_cols.argtypes = [P, vp, vp]
        lib.mgg_fill_cols.restype = ctypes.c_int
        lib.mgg_widths.argtypes = [P, vp, vp]
        lib.mgg_widths.restype = ctypes.c_int64
        lib.mgg_fill_payload.argtypes = [P, vp, vp, vp, vp]
        lib.mgg_fill_payload.restype = ctypes.c_int
        lib.mgg_draw.argtypes = [ctypes.c_uint64] * 4
        lib.mgg_draw.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


@dataclass
class Csr:
    """A row-distributed XCSR matrix held in host memory.

    ``bounds`` are the partition (rank) row bounds: partition r owns rows
    ``[bounds[r], bounds[r+1])`` (the paper's rank row intervals, Section 3,
    with 0-based ranks).
    """
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col: np.ndarray
    payload_off: np.ndarray
    payload: np.ndarray
    bounds: np.ndarray
    offset_width: int = 8
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def payload_bytes(self) -> int:
        return int(self.payload.shape[0])

    @property
    def n_parts(self) -> int:
        return int(self.bounds.shape[0]) - 1

    def algorithmic_bytes(self, partitioned: bool = False, emit_perm: bool = False) -> int:
        """Compulsory traffic: every input read once, every output written once."""
        o = self.offset_width
        one_way = ((self.n_rows + 1) * o + 4 * self.nnz + (self.nnz + 1) * o + self.payload_bytes)
        other_way = ((self.n_cols + 1) * o + 4 * self.nnz + (self.nnz + 1) * o + self.payload_bytes)
        b = one_way + other_way
        if partitioned:
            r = self.n_parts
            b += 2 * r * r * 8 + 2 * (r + 1) * 8
        if emit_perm:
            b += 4 * self.nnz
        return int(b)


def equal_bounds(n: int, r: int) -> np.ndarray:
    """R equal row blocks (the first n % R blocks get one extra row)."""
    base, rem = divmod(n, r)
    sizes = np.full(r, base, dtype=np.int64)
    sizes[:rem] += 1
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def generate(n_rows: int, n_cols: int, *, seed: int = 0, deg_law: int = DEG_POISSON,
             deg_mean: float = 8.0, deg_min: int = 0, deg_max: int = 0, target_nnz: int = 0,
             n_parts_gen: int = 1, col_law: int = COL_UNIFORM, window: int = 0,
             mult_law: int = MULT_GEOMETRIC, mult_max: int = 1, sort_rows: bool = True,
             pay_law: int = PAY_BYTES, w_lo: int = 0, w_hi: int = 0, offset_width: int = 8,
             bounds: Optional[np.ndarray] = None, threads: int = 0, name: str = "") -> Csr:
    lib = _load()
    s = _Spec(n_rows, n_cols, seed & (2**64 - 1), deg_law, float(deg_mean), deg_min, deg_max,
              target_nnz, n_parts_gen, col_law, window, mult_law, mult_max, int(sort_rows),
              pay_law, w_lo, w_hi, threads)
    row_ptr = np.empty(n_rows + 1, dtype=np.int64)
    nnz = lib.mgg_degrees(ctypes.byref(s), _ptr(row_ptr))
    if nnz < 0:
        raise ValueError("bad generator spec")
    col = np.empty(nnz, dtype=np.int32)
    if lib.mgg_fill_cols(ctypes.byref(s), _ptr(row_ptr), _ptr(col)) != 0:
        raise ValueError("bad generator spec (columns)")
    poff = np.empty(nnz + 1, dtype=np.int64)
    pbytes = lib.mgg_widths(ctypes.byref(s), _ptr(row_ptr), _ptr(poff))
    payload = np.empty(pbytes, dtype=np.uint8)
    lib.mgg_fill_payload(ctypes.byref(s), _ptr(row_ptr), _ptr(col), _ptr(poff), _ptr(payload))
    if offset_width == 4:
        if nnz >= 2**31 or pbytes >= 2**31:
            raise ValueError("int32 offsets cannot hold this matrix")
        row_ptr = row_ptr.astype(np.int32)
        poff = poff.astype(np.int32)
    if bounds is None:
        bounds = np.array([0, n_rows], dtype=np.int64)
    return Csr(n_rows, n_cols, row_ptr, col, poff, payload, np.asarray(bounds, dtype=np.int64),
               offset_width, name)


def draw(seed: int, stream: int, index: int, ctr: int = 0) -> int:
    """One counter-based 64-bit draw, for workload-level parameters."""
    return int(_load().mgg_draw(seed & (2**64 - 1), stream, index, ctr))


def _unit(u: int) -> float:
    return (u >> 11) * 2.0 ** -53


# --------------------------------------------------------------------------- recipes

def tiny(seed: int = 0, scale: int = 0) -> Csr:
    n = max(4, 1000 >> scale)
    return generate(n, n, seed=seed, deg_law=DEG_POISSON, deg_mean=20.0, col_law=COL_UNIFORM,
                    mult_law=MULT_GEOMETRIC, pay_law=PAY_FLOATS_TAG, w_lo=1, w_hi=3,
                    offset_width=4, bounds=equal_bounds(n, 4), name="tiny")


def large(seed: int = 0, scale: int = 0, parts: int = 64) -> Csr:
    n = (1 << 23) >> scale
    nnz = (1 << 29) >> scale
    return generate(n, n, seed=seed, deg_law=DEG_POWERLAW_BALANCED, deg_mean=2.1, deg_min=10,
                    deg_max=100000, target_nnz=nnz, n_parts_gen=parts, col_law=COL_UNIFORM,
                    mult_law=MULT_GEOMETRIC, pay_law=PAY_FLOATS, w_lo=1, w_hi=8, offset_width=8,
                    bounds=equal_bounds(n, parts), name="large")


def hetero(seed: int = 0, scale: int = 0, parts: int = 256) -> Csr:
    n = (1 << 21) >> scale
    nnz = (1 << 30) >> scale
    return generate(n, n, seed=seed, deg_law=DEG_PART_WEIGHTED, target_nnz=nnz, n_parts_gen=parts,
                    col_law=COL_WINDOW, window=int(math.floor(0.05 * n)), mult_law=MULT_UNIFORM,
                    mult_max=50, pay_law=PAY_FLOATS_ROWCOL, w_lo=5, offset_width=8,
                    bounds=equal_bounds(n, parts), name="hetero")


def batch_item_params(seed: int, index: int, n_lo: float = 1e3, n_hi: float = 1e6):
    """Per-matrix parameters of the batched workload: (n, mean degree, payload width)."""
    u = _unit(draw(seed, 0, index, 0))
    n = int(round(10 ** (math.log10(n_lo) + u * (math.log10(n_hi) - math.log10(n_lo)))))
    deg = 8 + (draw(seed, 0, index, 1) % 57)          # integer mean in U{8..64}
    width = draw(seed, 0, index, 2) % 17              # bytes in U{0..16}
    return n, int(deg), int(width)


def batch_item(seed: int, index: int, n_lo: float = 1e3, n_hi: float = 1e6,
               threads: int = 0) -> Csr:
    n, deg, width = batch_item_params(seed, index, n_lo, n_hi)
    return generate(n, n, seed=(seed << 20) + index, deg_law=DEG_POISSON, deg_mean=float(deg),
                    mult_law=MULT_GEOMETRIC, pay_law=PAY_BYTES, w_lo=width, w_hi=width,
                    offset_width=8, threads=threads, name=f"batch[{index}]")


def served_request_params(seed: int, index: int, c_lo: float = 1e4, c_hi: float = 1e8):
    """Per-request parameters: (cells target, n, mean degree, payload width, R)."""
    u = _unit(draw(seed, 1, index, 0))
    cells = 10 ** (math.log10(c_lo) + u * (math.log10(c_hi) - math.log10(c_lo)))
    deg = 8 + (draw(seed, 1, index, 1) % 57)
    n = max(1, int(round(cells / deg)))
    width = draw(seed, 1, index, 2) % 33               # bytes in U{0..32}
    r = 1 + (draw(seed, 1, index, 3) % 64)             # partitions in U{1..64}
    r = min(r, n)
    return int(cells), n, int(deg), int(width), int(r)


def served_request(seed: int, index: int, c_lo: float = 1e4, c_hi: float = 1e8,
                   threads: int = 0) -> Csr:
    _, n, deg, width, r = served_request_params(seed, index, c_lo, c_hi)
    return generate(n, n, seed=(1 << 40) + (seed << 24) + index, deg_law=DEG_POISSON,
                    deg_mean=float(deg), mult_law=MULT_GEOMETRIC, pay_law=PAY_BYTES, w_lo=width,
                    w_hi=width, offset_width=8, bounds=equal_bounds(n, r), threads=threads,
                    name=f"served[{index}]")


def random_small(seed: int, n_rows: int, n_cols: int, deg_mean: float = 4.0,
                 w_lo: int = 0, w_hi: int = 7, sort_rows: bool = True, offset_width: int = 8,
                 parts: int = 1, pay_law: int = PAY_BYTES) -> Csr:
    """Small random multigraph for edge-case tests (any widths, optional unsorted rows)."""
    bounds = equal_bounds(n_rows, parts) if n_rows >= parts else None
    return generate(n_rows, n_cols, seed=seed, deg_law=DEG_POISSON, deg_mean=deg_mean,
                    mult_law=MULT_GEOMETRIC, sort_rows=sort_rows, pay_law=pay_law, w_lo=w_lo,
                    w_hi=w_hi, offset_width=offset_width, bounds=bounds, name="random_small")


def from_arrays(n_rows: int, n_cols: int, row_ptr, col, widths=None, payload=None,
                offset_width: int = 8, bounds=None, fill_seed: int = 0) -> Csr:
    """Build a Csr from explicit arrays (hand-written cases and closed forms).

    ``widths`` gives each cell's payload byte count; bytes default to a
    deterministic pattern unless ``payload`` is given.
    """
    dt = np.int32 if offset_width == 4 else np.int64
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int32)
    nnz = col.shape[0]
    if widths is None:
        widths = np.zeros(nnz, dtype=np.int64)
    widths = np.asarray(widths, dtype=np.int64)
    poff = np.zeros(nnz + 1, dtype=np.int64)
    np.cumsum(widths, out=poff[1:])
    if payload is None:
        rng = np.random.default_rng(fill_seed)
        payload = rng.integers(0, 256, size=int(poff[-1]), dtype=np.uint8)
    payload = np.asarray(payload, dtype=np.uint8)
    if bounds is None:
        bounds = np.array([0, n_rows], dtype=np.int64)
    return Csr(n_rows, n_cols, row_ptr.astype(dt), col, poff.astype(dt), payload,
               np.asarray(bounds, dtype=np.int64), offset_width, "explicit")


def poisson_arrivals(n: int, rate: float, seed: int = 0):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    t, out = 0.0, []
    for i in range(n):
        u = _unit(draw(seed, 9, i))
        t += -math.log(1.0 - u) / rate
        out.append(t)
    return out


CONFIGS = {
    "tiny": tiny,
    "large": large,
    "hetero": hetero,
}
