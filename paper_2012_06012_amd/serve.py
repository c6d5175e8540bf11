"""Continuous-batching request loop for transposes on one device.

Requests arrive over time (each names an input matrix already resident in
device memory). The loop:

* admits requests FIFO while the sum of the footprints (outputs + workspace)
  of everything admitted and not yet finished stays within an HBM budget;
  a request larger than the whole budget is rejected;
* whenever one of its slots (streams) is free, submits every admitted request
  that is waiting (up to ``max_batch``) as one ``mgt_batch_submit`` on that
  slot's stream, so requests that arrive while others run join the next
  submit and their work overlaps on the device;
* polls completion events, returns each request's memory to the budget as it
  finishes, and records its latency (arrival -> completion observed);
* isolates failures: if a batch reports an error, the items it cancelled are
  resubmitted, and a failing item does not take the others down.

The executor does the device work; ``GpuExecutor`` drives libmgt, and tests
can plug in any object with the same three methods.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

OK, ECANCELED = 0, -6


@dataclass
class Request:
    rid: int
    mat: object                  # input matrix (device-resident for GpuExecutor)
    arrival: float               # seconds, on the server's clock
    partitioned: bool = False
    footprint: int = 0
    nnz: int = 0
    # filled by the server
    admit_t: Optional[float] = None
    submit_t: Optional[float] = None
    done_t: Optional[float] = None
    status: Optional[int] = None
    outputs: Optional[dict] = None
    attempts: int = 0
    rejected: bool = False

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_t is None else self.done_t - self.arrival


@dataclass
class Stats:
    completed: int = 0
    rejected: int = 0
    failed: int = 0
    batches: int = 0
    resubmits: int = 0
    cells: int = 0
    first_arrival: float = 0.0
    last_done: float = 0.0
    latencies: List[float] = field(default_factory=list)
    max_inflight_bytes: int = 0

    def percentile(self, q: float) -> float:
        if not self.latencies:
            return float("nan")
        xs = sorted(self.latencies)
        k = max(0, min(len(xs) - 1, int(math.ceil(q / 100.0 * len(xs))) - 1))
        return xs[k]

    @property
    def cells_per_s(self) -> float:
        span = self.last_done - self.first_arrival
        return self.cells / span if span > 0 else float("nan")

    def summary(self) -> dict:
        return {"completed": self.completed, "rejected": self.rejected, "failed": self.failed,
                "batches": self.batches, "resubmits": self.resubmits,
                "p50_ms": self.percentile(50) * 1e3, "p99_ms": self.percentile(99) * 1e3,
                "cells_per_s": self.cells_per_s, "max_inflight_bytes": self.max_inflight_bytes}


class Server:
    def __init__(self, executor, budget_bytes: int, max_batch: int = 64, n_slots: int = 2,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, max_attempts: int = 3,
                 on_done: Optional[Callable[[Request], None]] = None):
        # on_done(request) runs when a request completes (or fails): where its
        # outputs are handed over. The budget counts a request's footprint
        # until then only, so a caller that keeps every output must size the
        # budget for that.
        self.on_done = on_done
        self.ex = executor
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.n_slots = n_slots
        self.clock = clock
        self.sleep = sleep
        self.max_attempts = max_attempts

    def run(self, requests: List[Request]) -> Stats:
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.footprint = self.ex.footprint(r)
        st = Stats()
        t0 = self.clock()
        st.first_arrival = reqs[0].arrival if reqs else 0.0
        nxt = 0                      # next request to arrive
        queue: List[Request] = []    # arrived, not admitted (FIFO)
        ready: List[Request] = []    # admitted, not submitted
        inflight = {}                # slot -> (handle, [requests])
        used = 0
        free_slots = list(range(self.n_slots))
        while nxt < len(reqs) or queue or ready or inflight:
            now = self.clock() - t0
            progressed = False
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
                progressed = True
            # admission, FIFO by footprint
            while queue:
                r = queue[0]
                if r.footprint > self.budget:
                    queue.pop(0)
                    r.rejected = True
                    st.rejected += 1
                    progressed = True
                    continue
                if used + r.footprint > self.budget:
                    break
                queue.pop(0)
                used += r.footprint
                st.max_inflight_bytes = max(st.max_inflight_bytes, used)
                r.admit_t = now
                ready.append(r)
                progressed = True
            # submit to free slots
            while free_slots and ready:
                slot = free_slots.pop(0)
                # up to max_batch requests, and within the executor's cells per
                # batch (a request larger than that goes alone)
                cap = getattr(self.ex, "max_batch_cells", None)
                take, cells = 0, 0
                while take < len(ready) and take < self.max_batch:
                    c = ready[take].nnz
                    if take and cap is not None and cells + c > cap:
                        break
                    cells += c
                    take += 1
                batch, ready = ready[:take], ready[take:]
                for r in batch:
                    r.submit_t = now
                    r.attempts += 1
                inflight[slot] = (self.ex.submit(batch, slot), batch)
                st.batches += 1
                progressed = True
            # completions
            for slot in list(inflight):
                handle, batch = inflight[slot]
                if not self.ex.poll(handle):
                    continue
                statuses = self.ex.finish(handle)
                done_t = self.clock() - t0
                del inflight[slot]
                free_slots.append(slot)
                progressed = True
                retry = []
                for r, s in zip(batch, statuses):
                    if s == ECANCELED and r.attempts < self.max_attempts:
                        retry.append(r)         # cancelled by another item's failure
                        continue
                    r.status = s
                    r.done_t = done_t
                    used -= r.footprint
                    if self.on_done is not None:
                        self.on_done(r)
                    if s == OK:
                        st.completed += 1
                        st.cells += r.nnz
                        st.latencies.append(done_t - r.arrival)
                        st.last_done = max(st.last_done, done_t)
                    else:
                        st.failed += 1
                if retry:
                    # the failing item is reported; the items it cancelled go
                    # again, ahead of newer work
                    st.resubmits += len(retry)
                    ready = retry + ready
            if not progressed:
                wait = 2e-4
                if nxt < len(reqs) and not inflight:
                    wait = max(0.0, min(wait * 10, reqs[nxt].arrival - (self.clock() - t0)))
                self.sleep(wait)
        return st


# ----------------------------------------------------------------------------- GPU executor

class GpuExecutor:
    """Runs batches with mgt_batch_submit, one batch plan, stream and workspace
    per slot (a plan's staging buffer must not be shared by concurrent
    submits). Outputs are allocated per request and kept on the request."""

    def __init__(self, n_slots: int, offset_width: int = 8, perm: bool = False,
                 validate: bool = False, max_items: int = 256, max_cells: int = 1 << 31,
                 max_cols: int = 1 << 30, batch_cells: Optional[int] = None):
        import torch
        from . import mgt
        self.torch = torch
        self.mgt = mgt
        self.perm = perm
        self.flags = (mgt.EMIT_PERM if perm else 0) | (mgt.VALIDATE if validate else 0)
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.plans = [mgt.mgt_batch_plan(max_items, max_cells, max_cols, max_cols, 1 << 20,
                                         max_cells, max_cols, offset_width, self.flags)
                      for _ in range(n_slots)]
        # the server forms batches within this many cells (a larger request
        # still runs, alone); the plans take up to max_cells
        self.max_batch_cells = min(batch_cells or max_cells, max_cells)
        self.ws = [None] * n_slots

    def footprint(self, r: Request) -> int:
        a = r.mat
        o = a.offset_width
        out = (a.n_cols + 1) * o + 4 * a.nnz + (a.nnz + 1) * o + a.payload_bytes
        if self.perm:
            out += 4 * a.nnz
        r.nnz = a.nnz
        ws = 2 * (16 * a.nnz + a.payload_bytes) + 64 * (a.nnz // 1024 + 64) + (1 << 20)
        return int(out + ws)

    def submit(self, batch: List[Request], slot: int):
        torch, mgt = self.torch, self.mgt
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            mats = [r.mat for r in batch]
            outs = [mgt.alloc_outputs(a, self.perm, r.partitioned and a.n_parts > 1)
                    for a, r in zip(mats, batch)]
            entries, keep = mgt.batch_entries(mats, outs, self.perm, self.flags)
            items = mgt.make_items(entries)
            need = mgt.mgt_batch_workspace(self.plans[slot], items)
            if self.ws[slot] is None or self.ws[slot].numel() < need:
                self.ws[slot] = None
                self.ws[slot] = torch.empty(max(need, 256), dtype=torch.uint8, device=mats[0].col.device)
            status = torch.zeros(len(batch), dtype=torch.int32, device=mats[0].col.device)
            ev = torch.cuda.Event()
            mgt.mgt_batch_submit(self.plans[slot], items, self.ws[slot], status, stream)
            ev.record(stream)
        for r, o in zip(batch, outs):
            r.outputs = o
        return (ev, status, keep, items)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> List[int]:
        handle[0].synchronize()
        return [int(x) for x in handle[1].cpu().tolist()]


class PlainExecutor(GpuExecutor):
    """Comparator: every request runs alone with mgt_transpose /
    mgt_transpose_partitioned on one stream (no batching)."""

    def __init__(self, offset_width: int = 8, perm: bool = False):
        import torch
        from . import mgt
        self.torch = torch
        self.mgt = mgt
        self.perm = perm
        self.flags = mgt.EMIT_PERM if perm else 0
        self.streams = [torch.cuda.Stream()]
        self.ws = [None]
        self._plans = {}

    def submit(self, batch: List[Request], slot: int):
        torch, mgt = self.torch, self.mgt
        stream = self.streams[0]
        statuses = []
        with torch.cuda.stream(stream):
            for r in batch:
                a = r.mat
                plan = mgt.plan_for(a, self.flags)
                if self.ws[0] is None or self.ws[0].numel() < plan.workspace_bytes:
                    self.ws[0] = None
                    self.ws[0] = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8,
                                             device=a.col.device)
                part = r.partitioned and a.n_parts > 1
                out, status = mgt.transpose(a, plan=plan, workspace=self.ws[0], perm=self.perm,
                                            partitioned=part, stream=stream)
                r.outputs = out
                statuses.append(status)
                self._plans[r.rid] = plan
            ev = torch.cuda.Event()
            ev.record(stream)
        return (ev, statuses)

    def finish(self, handle) -> List[int]:
        handle[0].synchronize()
        self._plans.clear()
        return [int(s.cpu()[0]) for s in handle[1]]
