"""Thin Python binding of libmgt (the C ABI in include/mgt.h).

Argument marshalling only: every step of the transpose runs in the library's
HIP kernels. PyTorch provides device memory and the stream. The same names as
the C entry points are exposed (``mgt_plan``, ``mgt_transpose``,
``mgt_transpose_partitioned``, ``mgt_batch_plan``, ``mgt_batch_workspace``,
``mgt_batch_submit``), plus small conveniences that allocate the outputs.

If libmgt.so has not been built this module raises on import: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgt.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP, EUNSUPPORTED, ECANCELED = 0, -1, -2, -3, -4, -5, -6
VALIDATE, EMIT_PERM, DEBUG_TIMING, FIXED_WIDTH = 1, 2, 4, 8
LOCAL_TRANSPOSE, VIEW_SWAP = 0, 1
ROW_VIEW, COLUMN_VIEW = 0, 1
_NAMES = {0: "MGT_OK", -1: "MGT_EINVAL", -2: "MGT_ERANGE", -3: "MGT_ENOMEM", -4: "MGT_EHIP",
          -5: "MGT_EUNSUPPORTED", -6: "MGT_ECANCELED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmgt.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                      "python -m paper_2012_06012_amd.build")


class MgtError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"{what}: {_NAMES.get(code, code)}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("payload_bytes", ctypes.c_int64), ("offset_width", ctypes.c_int32),
                ("n_parts", ctypes.c_int32), ("part_bounds", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


class Limits(ctypes.Structure):
    _fields_ = [("max_items", ctypes.c_int32), ("offset_width", ctypes.c_int32),
                ("max_total_nnz", ctypes.c_int64), ("max_total_cols", ctypes.c_int64),
                ("max_total_rows", ctypes.c_int64), ("max_total_parts", ctypes.c_int64),
                ("max_item_nnz", ctypes.c_int64), ("max_item_cols", ctypes.c_int64),
                ("flags", ctypes.c_uint32)]


class Item(ctypes.Structure):
    _fields_ = [("desc", Desc)] + [(n, ctypes.c_void_p) for n in (
        "row_ptr", "col", "payload_off", "payload", "t_row_ptr", "t_col", "t_payload_off",
        "t_payload", "perm", "xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off",
        "sdispls", "rdispls")]


_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
_lib.mgt_plan.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(_vp), ctypes.POINTER(_sz)]
_lib.mgt_plan_destroy.argtypes = [_vp]
_lib.mgt_transpose.argtypes = [_vp] * 10 + [_vp, _sz, _vp, _vp]
_lib.mgt_transpose_partitioned.argtypes = [_vp] * 16 + [_vp, _sz, _vp, _vp]
_lib.mgt_batch_plan.argtypes = [ctypes.POINTER(Limits), ctypes.POINTER(_vp), ctypes.POINTER(_sz)]
_lib.mgt_batch_workspace.argtypes = [_vp, ctypes.POINTER(Item), _i32, ctypes.POINTER(_sz)]
_lib.mgt_batch_submit.argtypes = [_vp, ctypes.POINTER(Item), _i32, _vp, _sz, _vp, _vp, _vp]
_lib.mgt_plan_stage_times.argtypes = [_vp, ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_char_p), _i32, ctypes.POINTER(_i32)]
_lib.mgt_view_plan.argtypes = [ctypes.POINTER(Desc), _i32, _i32, ctypes.POINTER(_vp),
                               ctypes.POINTER(_sz)]
_lib.mgt_view_transform.argtypes = [_vp] * 10 + [_vp, _sz, _vp, _vp]
_lib.mgt_graph_create.argtypes = [_vp, _i32] + [_vp] * 16 + [_sz, _vp, ctypes.POINTER(_vp)]
_lib.mgt_graph_launch.argtypes = [_vp, _vp]
_lib.mgt_batch_graph_create.argtypes = [_vp, ctypes.POINTER(Item), _i32, _vp, _sz, _vp,
                                        ctypes.POINTER(_vp)]
_lib.mgt_graph_destroy.argtypes = [_vp]
_i64 = ctypes.c_int64
_lib.mgt_value_lists_workspace.argtypes = [_i64, ctypes.POINTER(_sz)]
_lib.mgt_plan_set_schedule.argtypes = [_vp, _i32, _i32, _i32, ctypes.POINTER(_sz)]
_lib.mgt_plan_schedule.argtypes = [_vp, _i32, ctypes.POINTER(_i32)]
_lib.mgt_coalesce.argtypes = [_i64, _i64, _i32] + [_vp] * 9 + [_sz, _vp]
_lib.mgt_expand.argtypes = [_i64, _i64, _i64, _i32, _i32] + [_vp] * 7 + [_vp]
_lib.mgt_counts_to_offsets.argtypes = [_i64, _vp, _i32, _i32, _vp, _vp, _sz, _vp]
_lib.mgt_transpose_noalloc.argtypes = [_vp, _i32] + [_vp] * 17
_lib.mgt_symmetrize_workspace.argtypes = [_vp, ctypes.POINTER(_sz)]
_lib.mgt_symmetrize.argtypes = [_vp, _i32] + [_vp] * 10 + [_sz, _vp, _vp]
_lib.mgt_version.restype = ctypes.c_char_p
for _f in ("mgt_plan", "mgt_plan_destroy", "mgt_transpose", "mgt_transpose_partitioned",
           "mgt_batch_plan", "mgt_batch_workspace", "mgt_batch_submit", "mgt_plan_stage_times",
           "mgt_view_plan", "mgt_view_transform", "mgt_graph_create", "mgt_graph_launch",
           "mgt_graph_destroy", "mgt_value_lists_workspace", "mgt_coalesce", "mgt_expand",
           "mgt_counts_to_offsets", "mgt_batch_graph_create", "mgt_plan_set_schedule",
           "mgt_plan_schedule", "mgt_transpose_noalloc", "mgt_symmetrize_workspace",
           "mgt_symmetrize"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("mgt_plan", "mgt_plan_destroy", "mgt_transpose", "mgt_transpose_partitioned",
            "mgt_batch_plan", "mgt_batch_workspace", "mgt_batch_submit", "mgt_plan_stage_times",
            "mgt_version", "mgt_view_plan", "mgt_view_transform", "mgt_graph_create",
            "mgt_graph_launch", "mgt_graph_destroy", "mgt_value_lists_workspace", "mgt_coalesce",
            "mgt_expand", "mgt_counts_to_offsets", "mgt_batch_graph_create", "mgt_plan_set_schedule",
            "mgt_plan_schedule", "mgt_transpose_noalloc", "mgt_symmetrize_workspace",
            "mgt_symmetrize")
LOWER, UPPER = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20  # MGT_NOALLOC_SCRATCH_BYTES


def version() -> str:
    return _lib.mgt_version().decode()


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return t.data_ptr() if t.numel() else None


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check(code: int, what: str):
    if code != OK:
        raise MgtError(code, what)


# ----------------------------------------------------------------------------- plans

class Plan:
    """Owns an mgt plan (host object)."""

    def __init__(self, handle: int, workspace_bytes: int, desc: Optional[Desc], batch: bool,
                 bounds: Optional[np.ndarray] = None):
        self.handle = handle
        self.workspace_bytes = workspace_bytes
        self.desc = desc
        self.batch = batch
        self._bounds = bounds

    def close(self):
        if self.handle:
            _lib.mgt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, pass_bits: int = 0, finish_bits: int = -1, tile_cells: int = 0) -> int:
        """mgt_plan_set_schedule; updates and returns workspace_bytes."""
        ws = _sz()
        _check(_lib.mgt_plan_set_schedule(self.handle, pass_bits, finish_bits, tile_cells,
                                          ctypes.byref(ws)), "mgt_plan_set_schedule")
        self.workspace_bytes = ws.value
        return ws.value

    def schedule(self, partitioned: bool = False) -> dict:
        """The schedule a call uses (mgt_plan_schedule)."""
        o = (_i32 * 8)()
        _check(_lib.mgt_plan_schedule(self.handle, 1 if partitioned else 0, o), "mgt_plan_schedule")
        return {"passes": o[0], "bits": [o[1 + l] for l in range(o[0])], "finish_bits": o[5],
                "tile_cells": o[6], "partition_pass": bool(o[7])}

    def stage_times(self):
        ms = (ctypes.c_float * 64)()
        names = (ctypes.c_char_p * 64)()
        n = _i32(0)
        _check(_lib.mgt_plan_stage_times(self.handle, ms, names, 64, ctypes.byref(n)), "stage_times")
        return [(names[i].decode(), ms[i]) for i in range(min(n.value, 64))]


def mgt_plan(n_rows: int, n_cols: int, nnz: int, payload_bytes: int, offset_width: int = 8,
             part_bounds: Optional[Sequence[int]] = None, flags: int = 0) -> Plan:
    b = None if part_bounds is None else np.ascontiguousarray(part_bounds, dtype=np.int64)
    d = Desc(n_rows, n_cols, nnz, payload_bytes, offset_width,
             1 if b is None else len(b) - 1, None if b is None else b.ctypes.data, flags)
    h = _vp()
    ws = _sz()
    _check(_lib.mgt_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws)), "mgt_plan")
    return Plan(h.value, ws.value, d, False, b)


def mgt_batch_plan(max_items: int, max_total_nnz: int, max_total_cols: int,
                   max_total_rows: int, max_total_parts: int, max_item_nnz: int,
                   max_item_cols: int, offset_width: int = 8, flags: int = 0) -> Plan:
    lim = Limits(max_items, offset_width, max_total_nnz, max_total_cols, max_total_rows,
                 max_total_parts, max_item_nnz, max_item_cols, flags)
    h = _vp()
    ws = _sz()
    _check(_lib.mgt_batch_plan(ctypes.byref(lim), ctypes.byref(h), ctypes.byref(ws)),
           "mgt_batch_plan")
    return Plan(h.value, ws.value, None, True)


# ----------------------------------------------------------------------------- raw entry points

def mgt_transpose(plan: Plan, row_ptr, col, payload_off, payload, t_row_ptr, t_col,
                  t_payload_off, t_payload, perm, workspace, d_status=None, stream=None) -> None:
    _check(_lib.mgt_transpose(plan.handle, _ptr(row_ptr), _ptr(col), _ptr(payload_off),
                              _ptr(payload), _ptr(t_row_ptr), _ptr(t_col), _ptr(t_payload_off),
                              _ptr(t_payload), _ptr(perm), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _ptr(d_status),
                              _stream(stream)), "mgt_transpose")


def mgt_symmetrize_workspace(plan: Plan) -> int:
    ws = _sz()
    _check(_lib.mgt_symmetrize_workspace(plan.handle, ctypes.byref(ws)), "mgt_symmetrize_workspace")
    return ws.value


def mgt_symmetrize(plan: Plan, triangle: int, row_ptr, col, payload_off, payload, s_row_ptr, s_col,
                   s_payload_off, s_payload, d_sizes, workspace, d_status=None,
                   stream=None) -> None:
    _check(_lib.mgt_symmetrize(plan.handle, triangle, _ptr(row_ptr), _ptr(col), _ptr(payload_off),
                               _ptr(payload), _ptr(s_row_ptr), _ptr(s_col), _ptr(s_payload_off),
                               _ptr(s_payload), _ptr(d_sizes), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _ptr(d_status),
                               _stream(stream)), "mgt_symmetrize")


def symmetrize(a: "DeviceCsr", lower: bool = True, validate: bool = False, stream=None):
    """Full symmetric matrix of the stored triangle `a` (mgt_symmetrize).
    Returns (outputs sized to S, status tensor); synchronises to read S's size."""
    plan = plan_for(a, VALIDATE if validate else 0)
    dev = a.col.device
    ws = _empty(max(mgt_symmetrize_workspace(plan), 256), torch.uint8, dev)
    odt = torch.int32 if a.offset_width == 4 else torch.int64
    out = dict(row_ptr=_empty(a.n_rows + 1, odt, dev),
               col=_empty(2 * a.nnz, torch.int32, dev),
               payload_off=_empty(2 * a.nnz + 1, odt, dev),
               payload=_empty(2 * a.payload_bytes, torch.uint8, dev))
    sizes = torch.zeros(2, dtype=torch.int64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    mgt_symmetrize(plan, LOWER if lower else UPPER, a.row_ptr, a.col, a.payload_off, a.payload,
                   out["row_ptr"], out["col"], out["payload_off"], out["payload"], sizes, ws,
                   status, stream)
    torch.cuda.synchronize()
    if _debug():
        check_guards(list(out.values()) + [ws], "symmetrize")
    m, b = (int(x) for x in sizes.cpu().tolist())
    out["col"], out["payload_off"], out["payload"] = (out["col"][:m], out["payload_off"][:m + 1],
                                                      out["payload"][:b])
    return out, status


def mgt_transpose_noalloc(plan: Plan, partitioned: bool, row_ptr, col, payload_off, payload,
                          t_row_ptr, t_col, t_payload_off, t_payload, perm, xfer_cells=None,
                          xfer_bytes=None, part_cell_off=None, part_byte_off=None, sdispls=None,
                          rdispls=None, d_status=None, stream=None) -> None:
    _check(_lib.mgt_transpose_noalloc(
        plan.handle, 1 if partitioned else 0, _ptr(row_ptr), _ptr(col), _ptr(payload_off),
        _ptr(payload), _ptr(t_row_ptr), _ptr(t_col), _ptr(t_payload_off), _ptr(t_payload),
        _ptr(perm), _ptr(xfer_cells), _ptr(xfer_bytes), _ptr(part_cell_off), _ptr(part_byte_off),
        _ptr(sdispls), _ptr(rdispls), _ptr(d_status), _stream(stream)), "mgt_transpose_noalloc")


def mgt_transpose_partitioned(plan: Plan, row_ptr, col, payload_off, payload, t_row_ptr, t_col,
                              t_payload_off, t_payload, perm, xfer_cells, xfer_bytes,
                              part_cell_off, part_byte_off, sdispls, rdispls, workspace,
                              d_status=None, stream=None) -> None:
    _check(_lib.mgt_transpose_partitioned(
        plan.handle, _ptr(row_ptr), _ptr(col), _ptr(payload_off), _ptr(payload), _ptr(t_row_ptr),
        _ptr(t_col), _ptr(t_payload_off), _ptr(t_payload), _ptr(perm), _ptr(xfer_cells),
        _ptr(xfer_bytes), _ptr(part_cell_off), _ptr(part_byte_off), _ptr(sdispls), _ptr(rdispls),
        _ptr(workspace), workspace.numel() * workspace.element_size(), _ptr(d_status),
        _stream(stream)), "mgt_transpose_partitioned")


class Graph:
    """Owns an mgt graph: one recorded transpose call, replayed by launch().

    Keeps the tensors it was recorded with alive for as long as it exists."""

    def __init__(self, handle: int, keep: tuple):
        self.handle = handle
        self._keep = keep

    def launch(self, stream=None) -> None:
        _check(_lib.mgt_graph_launch(self.handle, _stream(stream)), "mgt_graph_launch")

    def close(self):
        if self.handle:
            _lib.mgt_graph_destroy(self.handle)
            self.handle = None
        self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mgt_graph_create(plan: Plan, partitioned: bool, row_ptr, col, payload_off, payload,
                     t_row_ptr, t_col, t_payload_off, t_payload, perm, xfer_cells, xfer_bytes,
                     part_cell_off, part_byte_off, sdispls, rdispls, workspace,
                     d_status=None) -> Graph:
    args = (row_ptr, col, payload_off, payload, t_row_ptr, t_col, t_payload_off, t_payload, perm,
            xfer_cells, xfer_bytes, part_cell_off, part_byte_off, sdispls, rdispls, workspace,
            d_status)
    h = _vp()
    _check(_lib.mgt_graph_create(
        plan.handle, 1 if partitioned else 0, *[_ptr(t) for t in args[:16]],
        workspace.numel() * workspace.element_size(), _ptr(d_status), ctypes.byref(h)),
        "mgt_graph_create")
    return Graph(h.value, args)


def mgt_value_lists_workspace(nnz: int) -> int:
    ws = _sz()
    _check(_lib.mgt_value_lists_workspace(nnz, ctypes.byref(ws)), "mgt_value_lists_workspace")
    return ws.value


def mgt_coalesce(n_rows: int, nnz: int, offset_width: int, row_ptr, col, payload_off, o_row_ptr,
                 o_col, o_payload_off, o_counts, d_m, workspace, stream=None) -> None:
    _check(_lib.mgt_coalesce(n_rows, nnz, offset_width, _ptr(row_ptr), _ptr(col),
                             _ptr(payload_off), _ptr(o_row_ptr), _ptr(o_col),
                             _ptr(o_payload_off), _ptr(o_counts), _ptr(d_m), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream)),
           "mgt_coalesce")


def mgt_expand(n_rows: int, nnz: int, payload_bytes: int, offset_width: int, value_bytes: int,
               row_ptr, col, payload_off, o_row_ptr, o_col, o_payload_off, d_status=None,
               stream=None) -> None:
    _check(_lib.mgt_expand(n_rows, nnz, payload_bytes, offset_width, value_bytes, _ptr(row_ptr),
                           _ptr(col), _ptr(payload_off), _ptr(o_row_ptr), _ptr(o_col),
                           _ptr(o_payload_off), _ptr(d_status), _stream(stream)), "mgt_expand")


def mgt_counts_to_offsets(nnz: int, counts, value_bytes: int, offset_width: int, payload_off,
                          workspace, stream=None) -> None:
    _check(_lib.mgt_counts_to_offsets(nnz, _ptr(counts), value_bytes, offset_width,
                                      _ptr(payload_off), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(),
                                      _stream(stream)), "mgt_counts_to_offsets")


def mgt_batch_graph_create(plan: Plan, items: ctypes.Array, workspace, d_status=None,
                           keep: tuple = ()) -> Graph:
    h = _vp()
    _check(_lib.mgt_batch_graph_create(plan.handle, items, len(items), _ptr(workspace),
                                       workspace.numel() * workspace.element_size(),
                                       _ptr(d_status), ctypes.byref(h)), "mgt_batch_graph_create")
    return Graph(h.value, (items, workspace, d_status) + tuple(keep))


def mgt_view_plan(n_rows: int, n_cols: int, nnz: int, payload_bytes: int, offset_width: int,
                  part_bounds: Optional[Sequence[int]], op: int, in_view: int,
                  flags: int = 0) -> Plan:
    b = None if part_bounds is None else np.ascontiguousarray(part_bounds, dtype=np.int64)
    d = Desc(n_rows, n_cols, nnz, payload_bytes, offset_width,
             1 if b is None else len(b) - 1, None if b is None else b.ctypes.data, flags)
    h = _vp()
    ws = _sz()
    _check(_lib.mgt_view_plan(ctypes.byref(d), op, in_view, ctypes.byref(h), ctypes.byref(ws)),
           "mgt_view_plan")
    return Plan(h.value, ws.value, d, False, b)


def mgt_view_transform(plan: Plan, row_ptr, col, payload_off, payload, o_row_ptr, o_col,
                       o_payload_off, o_payload, perm, workspace, d_status=None,
                       stream=None) -> None:
    _check(_lib.mgt_view_transform(plan.handle, _ptr(row_ptr), _ptr(col), _ptr(payload_off),
                                   _ptr(payload), _ptr(o_row_ptr), _ptr(o_col),
                                   _ptr(o_payload_off), _ptr(o_payload), _ptr(perm),
                                   _ptr(workspace), workspace.numel(), _ptr(d_status),
                                   _stream(stream)), "mgt_view_transform")


def make_items(entries) -> ctypes.Array:
    """entries: list of dicts with 'desc' (Desc) and tensor fields named as in mgt_item."""
    arr = (Item * len(entries))()
    for i, e in enumerate(entries):
        arr[i].desc = e["desc"]
        for name in ("row_ptr", "col", "payload_off", "payload", "t_row_ptr", "t_col",
                     "t_payload_off", "t_payload", "perm", "xfer_cells", "xfer_bytes",
                     "part_cell_off", "part_byte_off", "sdispls", "rdispls"):
            setattr(arr[i], name, _ptr(e.get(name)))
    return arr


def mgt_batch_workspace(plan: Plan, items: ctypes.Array) -> int:
    ws = _sz()
    _check(_lib.mgt_batch_workspace(plan.handle, items, len(items), ctypes.byref(ws)),
           "mgt_batch_workspace")
    return ws.value


def mgt_batch_submit(plan: Plan, items: ctypes.Array, workspace, d_status=None, stream=None,
                     done_event=None) -> None:
    ev = None
    if done_event is not None:
        ev = done_event.cuda_event if hasattr(done_event, "cuda_event") else int(done_event)
    _check(_lib.mgt_batch_submit(plan.handle, items, len(items), _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), _ptr(d_status),
                                 _stream(stream), ev), "mgt_batch_submit")


# ----------------------------------------------------------------------------- conveniences

@dataclass
class DeviceCsr:
    """A matrix resident in device memory (torch tensors)."""
    n_rows: int
    n_cols: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    payload_off: Optional[torch.Tensor]   # may be None when fixed_width
    payload: torch.Tensor
    bounds: np.ndarray
    offset_width: int
    fixed_width: bool = False             # every cell carries payload_bytes / nnz bytes

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def payload_bytes(self) -> int:
        return int(self.payload.numel())

    @property
    def n_parts(self) -> int:
        return int(len(self.bounds)) - 1


# Debug guard words (MGT_DEBUG=1 in the environment): every output and
# workspace buffer the helpers below allocate is followed by GUARD_BYTES of a
# fixed pattern, and the call helpers check, after each call, that no byte of
# those zones changed (a write past the end of an array). Off by default.
GUARD_BYTES = 4096
GUARD_PATTERN = 0xA5


def _debug() -> bool:
    return os.environ.get("MGT_DEBUG", "") == "1"


def _empty(shape, dtype, device) -> torch.Tensor:
    """torch.empty, with a guard zone after the tensor's bytes under MGT_DEBUG."""
    if not _debug():
        return torch.empty(shape, dtype=dtype, device=device)
    n = 1
    for x in (shape if isinstance(shape, tuple) else (shape,)):
        n *= int(x)
    item = torch.empty(0, dtype=dtype).element_size()
    base = torch.empty(n * item + GUARD_BYTES, dtype=torch.uint8, device=device)
    base[n * item:].fill_(GUARD_PATTERN)
    t = base[:n * item].view(dtype).view(shape)
    t._mgt_guard = (base, n * item)
    return t


class GuardError(RuntimeError):
    pass


def check_guards(tensors, what: str = "") -> None:
    """Raises GuardError if a guard zone after any of `tensors` changed
    (tensors without one are skipped). Synchronises the device."""
    gs = [t._mgt_guard for t in tensors if t is not None and hasattr(t, "_mgt_guard")]
    if not gs:
        return
    torch.cuda.synchronize()
    for base, off in gs:
        z = base[off:]
        if not bool((z == GUARD_PATTERN).all()):
            bad = int(torch.nonzero(z != GUARD_PATTERN)[0])
            raise GuardError(f"{what}: byte {bad} past the end of a {off}-byte buffer was written")


def alloc_outputs(a: DeviceCsr, perm: bool = False, partitioned: bool = False, device=None,
                  payload_off: bool = True):
    """Output tensors for `a`. payload_off=False leaves out t_payload_off (only
    for fixed-width matrices, whose payload offsets are implied)."""
    dev = device or a.col.device
    odt = torch.int32 if a.offset_width == 4 else torch.int64
    out = dict(
        t_row_ptr=_empty(a.n_cols + 1, odt, dev),
        t_col=_empty(a.nnz, torch.int32, dev),
        t_payload_off=(_empty(a.nnz + 1, odt, dev) if payload_off or not a.fixed_width else None),
        t_payload=_empty(a.payload_bytes, torch.uint8, dev),
        perm=_empty(a.nnz, torch.int32, dev) if perm else None,
    )
    if partitioned:
        R = a.n_parts
        out.update(xfer_cells=_empty((R, R), torch.int64, dev),
                   xfer_bytes=_empty((R, R), torch.int64, dev),
                   part_cell_off=_empty(R + 1, torch.int64, dev),
                   part_byte_off=_empty(R + 1, torch.int64, dev),
                   sdispls=_empty((R, R), torch.int64, dev),
                   rdispls=_empty((R, R), torch.int64, dev))
    return out


def plan_for(a: DeviceCsr, flags: int = 0) -> Plan:
    return mgt_plan(a.n_rows, a.n_cols, a.nnz, a.payload_bytes, a.offset_width,
                    a.bounds if a.n_parts >= 1 else None,
                    flags | (FIXED_WIDTH if a.fixed_width else 0))


def workspace_for(plan: Plan, device) -> torch.Tensor:
    # torch's caching allocator returns 256-byte aligned blocks
    return _empty(max(plan.workspace_bytes, 256), torch.uint8, device)


def transpose(a: DeviceCsr, plan: Optional[Plan] = None, workspace=None, perm: bool = False,
              partitioned: bool = False, validate: bool = False, stream=None, out=None,
              status=None):
    """Allocates outputs and runs mgt_transpose / mgt_transpose_partitioned.

    Returns (outputs dict, status tensor). Asynchronous: read the tensors after
    synchronising the stream. `status` (one int32 on the device) may be passed
    to reuse it; otherwise one is taken from torch's allocator uninitialised
    (the library writes it on every call it launches, so no fill kernel runs).
    """
    flags = (EMIT_PERM if perm else 0) | (VALIDATE if validate else 0)
    if plan is None:
        plan = plan_for(a, flags)  # adds FIXED_WIDTH for fixed-width matrices
    dev = a.col.device
    if workspace is None:
        workspace = workspace_for(plan, dev)
    if out is None:
        out = alloc_outputs(a, perm, partitioned, dev)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
    if partitioned:
        mgt_transpose_partitioned(plan, a.row_ptr, a.col, a.payload_off, a.payload,
                                  out["t_row_ptr"], out["t_col"], out["t_payload_off"],
                                  out["t_payload"], out["perm"], out["xfer_cells"],
                                  out["xfer_bytes"], out["part_cell_off"], out["part_byte_off"],
                                  out["sdispls"], out["rdispls"], workspace, status, stream)
    else:
        mgt_transpose(plan, a.row_ptr, a.col, a.payload_off, a.payload, out["t_row_ptr"],
                      out["t_col"], out["t_payload_off"], out["t_payload"], out["perm"],
                      workspace, status, stream)
    if _debug():
        check_guards(list(out.values()) + [workspace], "transpose")
    return out, status


def transpose_graph(a: DeviceCsr, plan: Optional[Plan] = None, workspace=None, perm: bool = False,
                    partitioned: bool = False, validate: bool = False, out=None):
    """Records the transpose of a into fixed outputs as a graph.

    Returns (Graph, outputs dict, status tensor); every Graph.launch() writes
    the transpose of a's current contents into the same outputs."""
    flags = (EMIT_PERM if perm else 0) | (VALIDATE if validate else 0)
    if plan is None:
        plan = plan_for(a, flags)
    dev = a.col.device
    if workspace is None:
        workspace = workspace_for(plan, dev)
    if out is None:
        out = alloc_outputs(a, perm, partitioned, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    g = mgt_graph_create(plan, partitioned, a.row_ptr, a.col, a.payload_off, a.payload,
                         out["t_row_ptr"], out["t_col"], out["t_payload_off"], out["t_payload"],
                         out["perm"], out.get("xfer_cells"), out.get("xfer_bytes"),
                         out.get("part_cell_off"), out.get("part_byte_off"), out.get("sdispls"),
                         out.get("rdispls"), workspace, status)
    return g, out, status


def coalesce(a: DeviceCsr, stream=None):
    """Runs of repeated (row, column) cells merged into XCSR value-list cells.

    Returns (outputs dict with row_ptr, col, payload_off, counts trimmed to the
    m output cells, m). The payload tensor of `a` is the payload of the result.
    Synchronises to read m."""
    dev = a.col.device
    odt = torch.int32 if a.offset_width == 4 else torch.int64
    if a.payload_off is None:
        raise ValueError("coalesce needs the payload offsets")
    o_rp = torch.empty(a.n_rows + 1, dtype=odt, device=dev)
    o_col = torch.empty(a.nnz, dtype=torch.int32, device=dev)
    o_poff = torch.empty(a.nnz + 1, dtype=odt, device=dev)
    o_cnt = torch.empty(a.nnz, dtype=torch.int32, device=dev)
    d_m = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(mgt_value_lists_workspace(a.nnz), 256), dtype=torch.uint8, device=dev)
    mgt_coalesce(a.n_rows, a.nnz, a.offset_width, a.row_ptr, a.col, a.payload_off, o_rp, o_col,
                 o_poff, o_cnt, d_m, ws, stream)
    m = int(d_m.cpu()[0])
    return dict(row_ptr=o_rp, col=o_col[:m], payload_off=o_poff[:m + 1], counts=o_cnt[:m]), m


def expand(a: DeviceCsr, value_bytes: int, payload_off: bool = True, stream=None):
    """One cell per value_bytes-wide value. Returns (outputs dict, status tensor)."""
    dev = a.col.device
    odt = torch.int32 if a.offset_width == 4 else torch.int64
    if a.payload_off is None:
        raise ValueError("expand needs the payload offsets")
    nv = a.payload_bytes // value_bytes
    out = dict(row_ptr=torch.empty(a.n_rows + 1, dtype=odt, device=dev),
               col=torch.empty(nv, dtype=torch.int32, device=dev),
               payload_off=torch.empty(nv + 1, dtype=odt, device=dev) if payload_off else None)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    mgt_expand(a.n_rows, a.nnz, a.payload_bytes, a.offset_width, value_bytes, a.row_ptr, a.col,
               a.payload_off, out["row_ptr"], out["col"], out["payload_off"], status, stream)
    return out, status


def batch_entries(mats: Sequence[DeviceCsr], outs: Sequence[dict], perm: bool = False,
                  flags: int = 0):
    """Item table entries for mgt_batch_submit (items with R > 1 are partitioned)."""
    entries = []
    keep = []
    for a, o in zip(mats, outs):
        b = np.ascontiguousarray(a.bounds, dtype=np.int64)
        keep.append(b)
        d = Desc(a.n_rows, a.n_cols, a.nnz, a.payload_bytes, a.offset_width, a.n_parts,
                 b.ctypes.data, flags | (FIXED_WIDTH if a.fixed_width else 0))
        e = dict(desc=d, row_ptr=a.row_ptr, col=a.col, payload_off=a.payload_off,
                 payload=a.payload, **{k: o.get(k) for k in (
                     "t_row_ptr", "t_col", "t_payload_off", "t_payload", "perm", "xfer_cells",
                     "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls", "rdispls")})
        entries.append(e)
    return entries, keep


def batch_plan_for(mats: Sequence[DeviceCsr], perm: bool = False, validate: bool = False) -> Plan:
    """A batch plan whose limits are these matrices' totals."""
    flags = (EMIT_PERM if perm else 0) | (VALIDATE if validate else 0)
    return mgt_batch_plan(len(mats), sum(a.nnz for a in mats), sum(a.n_cols for a in mats),
                          sum(a.n_rows for a in mats), sum(a.n_parts for a in mats),
                          max(a.nnz for a in mats), max(a.n_cols for a in mats),
                          mats[0].offset_width, flags)


def batch_transpose(mats: Sequence[DeviceCsr], plan: Optional[Plan] = None, perm: bool = False,
                    validate: bool = False, stream=None, outs=None, workspace=None,
                    done_event=None):
    """Transposes every matrix of `mats` with one mgt_batch_submit call.

    Returns (outputs per item, per-item status tensor, plan, workspace)."""
    flags = (EMIT_PERM if perm else 0) | (VALIDATE if validate else 0)
    dev = mats[0].col.device
    if outs is None:
        outs = [alloc_outputs(a, perm, a.n_parts > 1, dev) for a in mats]
    if plan is None:
        plan = batch_plan_for(mats, perm, validate)
    entries, keep = batch_entries(mats, outs, perm, flags)
    items = make_items(entries)
    need = mgt_batch_workspace(plan, items)
    if workspace is None or workspace.numel() < need:
        workspace = _empty(max(need, 256), torch.uint8, dev)
    status = torch.empty(len(mats), dtype=torch.int32, device=dev)  # written by the call
    mgt_batch_submit(plan, items, workspace, status, stream, done_event)
    del keep
    if _debug():
        check_guards([t for o in outs for t in o.values()] + [workspace], "batch_transpose")
    return outs, status, plan, workspace


def batch_graph(mats: Sequence[DeviceCsr], plan: Optional[Plan] = None, perm: bool = False,
                validate: bool = False, outs=None, workspace=None):
    """Records one batch transpose of `mats` into fixed outputs as a graph.

    Returns (Graph, outputs per item, per-item status tensor, plan, workspace);
    every Graph.launch() transposes the matrices' current contents."""
    flags = (EMIT_PERM if perm else 0) | (VALIDATE if validate else 0)
    dev = mats[0].col.device
    if outs is None:
        outs = [alloc_outputs(a, perm, a.n_parts > 1, dev) for a in mats]
    if plan is None:
        plan = batch_plan_for(mats, perm, validate)
    entries, keep = batch_entries(mats, outs, perm, flags)
    items = make_items(entries)
    need = mgt_batch_workspace(plan, items)
    if workspace is None or workspace.numel() < need:
        workspace = _empty(max(need, 256), torch.uint8, dev)
    status = torch.zeros(len(mats), dtype=torch.int32, device=dev)
    g = mgt_batch_graph_create(plan, items, workspace, status, keep=(keep, outs, tuple(mats)))
    return g, outs, status, plan, workspace


def view_out_rows(n_rows: int, n_cols: int, n_parts: int, op: int, in_view: int) -> int:
    """Rows of a view operation's output CSR (see mgt_view_plan)."""
    if op == LOCAL_TRANSPOSE:
        return n_parts * n_cols if in_view == ROW_VIEW else n_cols
    return n_parts * n_rows if in_view == ROW_VIEW else n_rows


def view_transform(row_ptr, col, payload_off, payload, n_rows: int, n_cols: int, bounds,
                   offset_width: int, op: int, in_view: int, perm: bool = False,
                   validate: bool = False, fixed_width: bool = False, plan: Optional[Plan] = None,
                   workspace=None, stream=None):
    """Allocates outputs and runs mgt_view_transform (LocalTranspose or
    ViewSwap of the matrix X, n_rows x n_cols, with the given partition bounds,
    held in view in_view). Returns (outputs dict, status tensor)."""
    flags = ((EMIT_PERM if perm else 0) | (VALIDATE if validate else 0)
             | (FIXED_WIDTH if fixed_width else 0))
    nnz, nbytes = int(col.numel()), int(payload.numel())
    b = np.ascontiguousarray(bounds, dtype=np.int64)
    if plan is None:
        plan = mgt_view_plan(n_rows, n_cols, nnz, nbytes, offset_width, b, op, in_view, flags)
    dev = col.device
    if workspace is None:
        workspace = workspace_for(plan, dev)
    odt = torch.int32 if offset_width == 4 else torch.int64
    n_out = view_out_rows(n_rows, n_cols, len(b) - 1, op, in_view)
    out = dict(row_ptr=torch.empty(n_out + 1, dtype=odt, device=dev),
               col=torch.empty(nnz, dtype=torch.int32, device=dev),
               payload_off=(None if fixed_width else torch.empty(nnz + 1, dtype=odt, device=dev)),
               payload=torch.empty(nbytes, dtype=torch.uint8, device=dev),
               perm=torch.empty(nnz, dtype=torch.int32, device=dev) if perm else None)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    mgt_view_transform(plan, row_ptr, col, payload_off, payload, out["row_ptr"], out["col"],
                       out["payload_off"], out["payload"], out["perm"], workspace, status, stream)
    return out, status
