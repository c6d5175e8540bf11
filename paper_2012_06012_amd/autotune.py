"""Autotuner for single-matrix and batched transposes.

The library's default schedule is a rule: the fewest partition passes, then
the narrowest finish buckets of about 4,096 cells, with tiles sized for the
call. The autotuner times candidate schedules (digit width of the passes,
finish bucket width, tile size; ``mgt_plan_set_schedule``) on the caller's
own matrix, or on a sample batch for batch plans, and leaves the fastest on
the plan. Every candidate's output is compared with the default schedule's,
bit for bit, before its time counts. Results are cached per device
architecture and shape class (powers of two of the cell count, column bits
and payload bytes per cell), in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import mgt

_CACHE: Dict[str, dict] = {}


@dataclass
class TuneResult:
    best: dict                       # pass_bits, finish_bits, tile_cells, ms, schedule
    default_ms: float
    default_schedule: dict
    trials: List[dict] = field(default_factory=list)


def _arch(dev) -> str:
    try:
        return torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _lg(x: float) -> int:
    return int(round(math.log2(max(float(x), 1.0))))


def _class(a: mgt.DeviceCsr) -> list:
    """Shape class of one matrix: rounded log2 of its cells, its column bits,
    rounded log2 of (1 + payload bytes per cell)."""
    return [_lg(a.nnz), int(math.ceil(math.log2(max(a.n_cols, 1)))),
            _lg(1 + a.payload_bytes / max(a.nnz, 1))]


def shape_key(a: mgt.DeviceCsr, partitioned: bool, perm: bool) -> str:
    return json.dumps([_arch(a.col.device), "single"] + _class(a) +
                      [a.offset_width, _lg(a.n_parts), bool(partitioned), bool(perm),
                       bool(a.fixed_width)])


def batch_shape_key(mats: Sequence[mgt.DeviceCsr], perm: bool) -> str:
    """Shape class of a batch: item count, total cells, and the mean of the
    items' classes (rounded)."""
    cls = [_class(a) for a in mats]
    mean = [int(round(sum(c[i] for c in cls) / max(len(cls), 1))) for i in range(3)]
    return json.dumps([_arch(mats[0].col.device), "batch", _lg(len(mats)),
                       _lg(sum(a.nnz for a in mats))] + mean +
                      [mats[0].offset_width, bool(perm)])


def load_cache(path: str) -> None:
    with open(path) as f:
        _CACHE.update(json.load(f))


def save_cache(path: str) -> None:
    with open(path, "w") as f:
        json.dump(_CACHE, f, indent=1, sort_keys=True)


def _grid(plan: mgt.Plan, partitioned: bool, pass_bits: Sequence[int],
          finish_span: Sequence[int], tiles: Sequence[int]) -> List[Tuple[int, int, int]]:
    """Candidate settings whose schedules differ from each other."""
    plan.set_schedule()
    fb0 = plan.schedule(partitioned)["finish_bits"]
    seen, out = set(), []
    for pb in pass_bits:
        for d in finish_span:
            fb = fb0 + d
            if fb < 0 or fb > 10:
                continue
            for t in tiles:
                try:
                    plan.set_schedule(pb, fb, t)
                except mgt.MgtError:
                    continue
                sc = plan.schedule(partitioned)
                key = (tuple(sc["bits"]), sc["finish_bits"], sc["tile_cells"])
                if key not in seen:
                    seen.add(key)
                    out.append((pb, fb, t))
    plan.set_schedule()
    return out


def _run(a, plan, ws, out, partitioned, perm):
    return mgt.transpose(a, plan=plan, workspace=ws, perm=perm, partitioned=partitioned, out=out)


def _time(a, plan, ws, out, partitioned, perm, reps) -> float:
    _run(a, plan, ws, out, partitioned, perm)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        _run(a, plan, ws, out, partitioned, perm)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(a: mgt.DeviceCsr, plan: Optional[mgt.Plan] = None, partitioned: bool = False,
             perm: bool = False, reps: int = 3, pass_bits: Sequence[int] = (6, 7, 8),
             finish_span: Sequence[int] = (-1, 0, 1, 2), tiles: Sequence[int] = (8192, 16384),
             use_cache: bool = True) -> Tuple[mgt.Plan, TuneResult]:
    """Times the default and every candidate schedule on `a`; sets the fastest
    (whose output equals the default's) on the plan and returns it."""
    if plan is None:
        plan = mgt.plan_for(a, mgt.EMIT_PERM if perm else 0)
    key = shape_key(a, partitioned, perm)
    if use_cache and key in _CACHE:
        b = _CACHE[key]
        plan.set_schedule(b["pass_bits"], b["finish_bits"], b["tile_cells"])
        return plan, TuneResult(best=dict(b), default_ms=b.get("default_ms", float("nan")),
                                default_schedule=b.get("default_schedule", {}))
    cands = _grid(plan, partitioned, pass_bits, finish_span, tiles)
    need = plan.workspace_bytes
    for pb, fb, t in cands:
        need = max(need, plan.set_schedule(pb, fb, t))
    plan.set_schedule()
    dev = a.col.device
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    out = mgt.alloc_outputs(a, perm, partitioned, dev)
    default_ms = _time(a, plan, ws, out, partitioned, perm, reps)
    default_sched = plan.schedule(partitioned)
    ref = {k: v.clone() for k, v in out.items() if v is not None}
    res = TuneResult(best={"pass_bits": 0, "finish_bits": -1, "tile_cells": 0, "ms": default_ms,
                           "schedule": default_sched},
                     default_ms=default_ms, default_schedule=default_sched)
    for pb, fb, t in cands:
        plan.set_schedule(pb, fb, t)
        ms = _time(a, plan, ws, out, partitioned, perm, reps)
        same = all(torch.equal(out[k], ref[k]) for k in ref)
        trial = {"pass_bits": pb, "finish_bits": fb, "tile_cells": t, "ms": ms,
                 "schedule": plan.schedule(partitioned), "bit_exact": bool(same)}
        res.trials.append(trial)
        if not same:
            raise RuntimeError(f"schedule {trial['schedule']} changed the result")
        if ms < res.best["ms"]:
            res.best = trial
    b = res.best
    plan.set_schedule(b["pass_bits"], b["finish_bits"], b["tile_cells"])
    _CACHE[key] = {"pass_bits": b["pass_bits"], "finish_bits": b["finish_bits"],
                   "tile_cells": b["tile_cells"], "ms": b["ms"], "default_ms": default_ms,
                   "default_schedule": default_sched}
    return plan, res


def _time_batch(mats, plan, ws, outs, perm, reps) -> float:
    mgt.batch_transpose(mats, plan=plan, perm=perm, workspace=ws, outs=outs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mgt.batch_transpose(mats, plan=plan, perm=perm, workspace=ws, outs=outs)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune_batch(mats: Sequence[mgt.DeviceCsr], plan: Optional[mgt.Plan] = None,
                   perm: bool = False, reps: int = 3, pass_bits: Sequence[int] = (4, 6, 8),
                   tiles: Sequence[int] = (8192, 16384),
                   use_cache: bool = True) -> Tuple[mgt.Plan, TuneResult]:
    """Times the default and every candidate (digit width of the passes, tile
    size; each item keeps the rule's finish width) on the sample batch `mats`;
    sets the fastest whose outputs equal the default's on the batch plan."""
    if plan is None:
        plan = mgt.batch_plan_for(mats, perm)
    key = batch_shape_key(mats, perm)
    if use_cache and key in _CACHE:
        b = _CACHE[key]
        plan.set_schedule(b["pass_bits"], -1, b["tile_cells"])
        return plan, TuneResult(best=dict(b), default_ms=b.get("default_ms", float("nan")),
                                default_schedule=b.get("default_schedule", {}))
    dev = mats[0].col.device
    cands = [(pb, t) for pb in pass_bits for t in tiles]
    items_need = 0
    outs = [mgt.alloc_outputs(a, perm, a.n_parts > 1) for a in mats]
    entries, keep = mgt.batch_entries(mats, outs, perm, mgt.EMIT_PERM if perm else 0)
    items = mgt.make_items(entries)
    for pb, t in [(0, 0)] + cands:
        plan.set_schedule(pb, -1, t)
        items_need = max(items_need, mgt.mgt_batch_workspace(plan, items))
    del keep
    ws = torch.empty(max(items_need, 256), dtype=torch.uint8, device=dev)
    plan.set_schedule()
    default_ms = _time_batch(mats, plan, ws, outs, perm, reps)
    ref = [{k: v.clone() for k, v in o.items() if v is not None} for o in outs]
    res = TuneResult(best={"pass_bits": 0, "finish_bits": -1, "tile_cells": 0, "ms": default_ms,
                           "schedule": "rule"},
                     default_ms=default_ms, default_schedule={"rule": True})
    for pb, t in cands:
        plan.set_schedule(pb, -1, t)
        ms = _time_batch(mats, plan, ws, outs, perm, reps)
        same = all(torch.equal(o[k], r[k]) for o, r in zip(outs, ref) for k in r)
        trial = {"pass_bits": pb, "finish_bits": -1, "tile_cells": t, "ms": ms,
                 "schedule": f"pass bits <= {pb}, tiles of {t} cells", "bit_exact": bool(same)}
        res.trials.append(trial)
        if not same:
            raise RuntimeError(f"batch schedule {trial['schedule']} changed the result")
        if ms < res.best["ms"]:
            res.best = trial
    b = res.best
    plan.set_schedule(b["pass_bits"], -1, b["tile_cells"])
    _CACHE[key] = {"pass_bits": b["pass_bits"], "finish_bits": -1, "tile_cells": b["tile_cells"],
                   "ms": b["ms"], "default_ms": default_ms, "default_schedule": {"rule": True}}
    return plan, res
