"""Autotuner for single-matrix transposes.

The library's default schedule is a rule: the fewest partition passes, then
the narrowest finish buckets of about 4,096 cells, with tiles sized for the
call. The autotuner times candidate schedules (digit width of the passes,
finish bucket width, tile size; ``mgt_plan_set_schedule``) on the caller's
own matrix and leaves the fastest on the plan. Every candidate's output is
compared with the default schedule's, bit for bit, before its time counts.
Results are cached per matrix shape, in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
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


def shape_key(a: mgt.DeviceCsr, partitioned: bool, perm: bool) -> str:
    return json.dumps([a.n_rows, a.n_cols, a.nnz, a.payload_bytes, a.offset_width, int(a.n_parts),
                       bool(partitioned), bool(perm), bool(a.fixed_width)])


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
