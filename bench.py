#!/usr/bin/env python3
"""Benchmark: plain XCSR multigraph transpose on one MI355X.

Workload (default): 2^23 x 2^23 multigraph with exactly 2^29 cells (2^23 per
each of 64 equal row blocks), power-law row degrees (alpha 2.1, d >= 10,
capped at 10^5), uniform columns, Geometric(1/2) multiplicity, 1-8 float32 of
payload per cell, int64 offsets, int32 column ids; synthetic and seeded.

A step is one mgt_transpose call (every stage of the hot path) on inputs
already resident in HBM. Prints one JSON line with cells/s, the fraction of
the 8 TB/s HBM peak reached in algorithmic bytes, the dominant kernel's
roofline, a CPU-oracle baseline on a bounded sample of the same workload and
a bit-exactness verdict from sampled output rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(a, stage: str, pass_idx: int, perm: bool) -> int:
    """Algorithmic bytes of one launch of a stage: its inputs read once and its
    outputs written once (records are 16 bytes per cell in the level buffers)."""
    nnz, P, o = a.nnz, a.payload_bytes, a.offset_width
    if stage == "scatter" and pass_idx == 0:
        return nnz * (4 + 2 * o) + (a.n_rows + 1) * o + P + nnz * 16 + P
    if stage == "scatter":
        return 2 * (nnz * 16 + P)
    if stage == "finish":
        return nnz * 16 + P + nnz * (4 + o + (4 if perm else 0)) + (a.n_cols + 1) * o + P
    if stage == "hist" and pass_idx == 0:
        return nnz * (4 + 2 * o)
    if stage == "hist":
        return nnz * 8
    return 0


def copy_calibration(mib: int):
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_bytes_each_way": n, "ms": ms, "GBps_read_plus_write": 2 * n / ms / 1e6}))


def _device(a, dev):
    import torch
    from paper_2012_06012_amd import mgt
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    return mgt.DeviceCsr(a.n_rows, a.n_cols, t(a.row_ptr), t(a.col), t(a.payload_off),
                         t(a.payload), a.bounds, a.offset_width)


def bench_batch(args):
    """Many independent matrices: one mgt_batch_submit versus one mgt_transpose
    per matrix on one stream (same matrices, bit-exact outputs compared)."""
    import torch
    from workloads import gen
    from paper_2012_06012_amd import mgt
    dev = torch.device("cuda:0")
    t0 = time.time()
    host = [gen.batch_item(args.seed, i, 1e3, 1e5) for i in range(args.items)]
    mats = [_device(a, dev) for a in host]
    cells = sum(a.nnz for a in host)
    log(f"[batch] {len(host)} matrices, {cells} cells, generated in {time.time() - t0:.1f}s")
    outs, status, plan, ws = mgt.batch_transpose(mats)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        mgt.batch_transpose(mats, plan=plan, workspace=ws, outs=outs)
    ev1.record()
    torch.cuda.synchronize()
    ms_batch = ev0.elapsed_time(ev1) / args.steps
    plans = [mgt.plan_for(a) for a in mats]
    wsz = max(p.workspace_bytes for p in plans)
    ws1 = torch.empty(wsz, dtype=torch.uint8, device=dev)
    outs1 = [mgt.alloc_outputs(a) for a in mats]
    for a, p, o in zip(mats, plans, outs1):
        mgt.transpose(a, plan=p, workspace=ws1, out=o)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        for a, p, o in zip(mats, plans, outs1):
            mgt.transpose(a, plan=p, workspace=ws1, out=o)
    ev1.record()
    torch.cuda.synchronize()
    ms_plain = ev0.elapsed_time(ev1) / args.steps
    same = all(torch.equal(o1[k], o2[k]) for o1, o2 in zip(outs, outs1) for k in o1
               if o1[k] is not None)
    res = {"metric": "cells/s, batched vs per-matrix plain launches", "mode": "batch",
           "matrices": len(host), "cells": cells, "ms_batched": ms_batch, "ms_per_matrix_plain": ms_plain,
           "cells_per_s_batched": cells / (ms_batch * 1e-3),
           "cells_per_s_plain": cells / (ms_plain * 1e-3), "speedup": ms_plain / ms_batch,
           "bit_exact_batched_vs_plain": bool(same),
           "config": {"workload": "batch of matrices, n log-uniform 1e3-1e5, mean degree U{8..64}, "
                                  "payload U{0..16} bytes per matrix", "seed": args.seed}}
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Served requests: Poisson arrivals into the continuous-batching loop,
    then the same stream through per-request plain launches."""
    import torch
    from workloads import gen
    from paper_2012_06012_amd import serve
    from paper_2012_06012_amd.serve import Request, Server
    dev = torch.device("cuda:0")
    t0 = time.time()
    pool_n = 32
    host = []
    for i in range(pool_n):
        cells, n, deg, width, r = gen.served_request_params(args.seed, i, 1e4, 1e7)
        host.append(gen.generate(n, n, seed=(args.seed << 24) + i + 11, deg_law=gen.DEG_POISSON,
                                 deg_mean=float(deg), pay_law=gen.PAY_BYTES, w_lo=width,
                                 w_hi=width, offset_width=8, bounds=gen.equal_bounds(n, min(r, n))))
    pool = [_device(a, dev) for a in host]
    log(f"[serve] pool of {pool_n} inputs, {sum(a.nnz for a in host)} cells, "
        f"{time.time() - t0:.1f}s")
    n_req = args.items

    def make(rate):
        arr = gen.poisson_arrivals(n_req, rate, args.seed + 3)
        return [Request(rid=i, mat=pool[i % pool_n], arrival=t, partitioned=pool[i % pool_n].n_parts > 1)
                for i, t in enumerate(arr)]

    budget = 200 << 30
    # capacity of the plain path: back-to-back, no arrivals gaps
    plain = Server(serve.PlainExecutor(), budget, max_batch=1, n_slots=1)
    st = plain.run([Request(rid=i, mat=pool[i % pool_n], arrival=0.0,
                            partitioned=pool[i % pool_n].n_parts > 1) for i in range(64)])
    mu = 64 / st.last_done
    log(f"[serve] plain capacity {mu:.1f} req/s")
    out = {}
    for frac in (0.7, 1.2):
        rate = frac * mu
        sb = Server(serve.GpuExecutor(n_slots=2, max_items=64), budget, max_batch=32, n_slots=2).run(make(rate))
        sp = Server(serve.PlainExecutor(), budget, max_batch=1, n_slots=1).run(make(rate))
        out[f"{frac}mu"] = {"batched": sb.summary(), "plain": sp.summary()}
        log(f"[serve] rate {rate:.1f}/s: batched {sb.summary()} plain {sp.summary()}")
    res = {"metric": "served p50/p99 latency and sustained cells/s, batched vs plain",
           "mode": "serve", "requests": n_req, "plain_capacity_req_s": mu, "results": out,
           "config": {"workload": "requests of log-uniform 1e4-1e7 cells, widths U{0..32}, "
                                  "R U{1..64}, Poisson arrivals", "budget_bytes": budget}}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=0, help="right shift of rows and cells (tests)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--partitioned", action="store_true",
                    help="time mgt_transpose_partitioned (R = 64) instead of the plain form")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device-to-device copy of this size (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters and measures copy bandwidth)")
    ap.add_argument("--mode", choices=["plain", "batch", "serve"], default="plain",
                    help="plain: the headline line; batch: many matrices in one mgt_batch_submit "
                         "vs per-matrix launches; serve: the continuous-batching request loop vs "
                         "per-request plain launches")
    ap.add_argument("--items", type=int, default=512, help="batch / serve: matrices or requests")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): this build has no "
              "multi-GPU path; see DESIGN.md for how the transpose would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import gen
    from paper_2012_06012_amd import mgt

    t0 = time.time()
    log(f"[bench] generating large multigraph (scale {args.scale})")
    a = gen.large(seed=args.seed, scale=args.scale)
    log(f"[bench] generated nnz={a.nnz} payload={a.payload_bytes} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(x).to(dev)  # noqa: E731
    d = mgt.DeviceCsr(a.n_rows, a.n_cols, t(a.row_ptr), t(a.col), t(a.payload_off),
                      t(a.payload), a.bounds, a.offset_width)
    torch.cuda.synchronize()
    log(f"[bench] uploaded in {time.time() - t0:.1f}s")

    part = args.partitioned
    plan = mgt.plan_for(d, 0)
    ws = mgt.workspace_for(plan, dev)
    out = mgt.alloc_outputs(d, perm=False, partitioned=part)
    stream = torch.cuda.current_stream()

    def step(p=plan):
        mgt.transpose(d, plan=p, workspace=ws, partitioned=part, out=out, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms)")

    # per-stage device times (events recorded by the library on the same stream)
    tplan = mgt.plan_for(d, mgt.DEBUG_TIMING)
    acc = {}
    n_t = max(3, min(args.steps, 5))
    for _ in range(n_t):
        step(tplan)
        times = tplan.stage_times()
        pi = {}
        for name, v in times:
            k = pi.get(name, 0)
            pi[name] = k + 1
            acc.setdefault((name, k), []).append(v)
    stages = {f"{n}{k}": float(np.mean(v)) for (n, k), v in acc.items()}
    log(f"[bench] stages (ms): {json.dumps({k: round(v, 3) for k, v in stages.items()})}")
    dom_key = max((k for k in stages if k.startswith(("scatter", "finish", "hist"))),
                  key=lambda k: stages[k])
    dom_stage = dom_key.rstrip("0123456789")
    dom_pass = int(dom_key[len(dom_stage):] or 0)
    dom_bytes = kernel_bytes(a, dom_stage, dom_pass, False)
    dom_ms = stages[dom_key]
    kname = {"scatter": "k_pass_scatter", "finish": "k_finish", "hist": "k_pass_hist"}[dom_stage]

    b_alg = a.algorithmic_bytes(partitioned=part)
    value = a.nnz / (ms * 1e-3)
    achieved_step = b_alg / (ms * 1e-3) / 1e9

    # bit-exactness on sampled output rows + global invariants
    exact = None
    if not args.no_check:
        import oracle
        torch.cuda.synchronize()
        t_row_ptr = out["t_row_ptr"].cpu().numpy()
        ok = np.array_equal(np.diff(t_row_ptr), np.bincount(a.col, minlength=a.n_cols))
        ok &= int(t_row_ptr[-1]) == a.nnz
        rng = np.random.default_rng(args.seed + 7)
        ranges = [(0, 64), (a.n_cols - 64, a.n_cols)]
        ranges += [(int(c), int(c) + 64) for c in rng.integers(0, a.n_cols - 64, size=4)]
        t_poff = out["t_payload_off"]
        for lo, hi in ranges:
            s = oracle.transpose_columns(a, lo, hi)
            p0, p1 = int(t_row_ptr[lo]), int(t_row_ptr[hi])
            ok &= np.array_equal(t_row_ptr[lo:hi + 1] - p0, s.t_row_ptr)
            ok &= np.array_equal(out["t_col"][p0:p1].cpu().numpy(), s.t_col)
            po = t_poff[p0:p1 + 1].cpu().numpy()
            ok &= np.array_equal(po - po[0], s.t_payload_off)
            ok &= np.array_equal(out["t_payload"][int(po[0]):int(po[-1])].cpu().numpy(),
                                 s.t_payload)
        exact = bool(ok)
        log(f"[bench] sampled parity: {exact}")

    cpu = None
    if not args.no_cpu:
        import oracle
        # bounded sample: the first 1/16 of the row blocks as a matrix of its own
        rows = a.n_rows // 16
        k1 = int(a.row_ptr[rows])
        sub = gen.Csr(rows, a.n_cols, a.row_ptr[:rows + 1].copy(), a.col[:k1],
                      a.payload_off[:k1 + 1].copy(), a.payload[:int(a.payload_off[k1])],
                      np.array([0, rows]), a.offset_width)
        c0 = time.perf_counter()
        oracle.transpose(sub)
        cs = time.perf_counter() - c0
        cpu = {"value": sub.nnz / cs, "unit": "cells/s", "cores": 1, "kind": "oracle",
               "sample": f"first {rows} rows ({sub.nnz} cells, {sub.payload_bytes} payload bytes) "
                         f"of the same matrix, all {a.n_cols} columns; {cs:.1f} s single-threaded"}
        log(f"[bench] cpu oracle: {cpu['value']:.3e} cells/s")

    res = {
        "metric": "cells/s (plain transpose, bit-exact) and % of HBM peak",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "large multigraph 2^23 x 2^23, 2^29 cells, int64 offsets, "
                               "1-8 float32 payload per cell" + (", partitioned R=64" if part else ""),
                   "n": a.n_rows, "nnz": a.nnz, "payload_bytes": a.payload_bytes,
                   "partitions": 64 if part else 1, "scale_shift": args.scale},
        "hbm_frac_step": achieved_step / HBM_PEAK_GBS,
        "algorithmic_GBps_step": achieved_step,
        "algorithmic_bytes_step": b_alg,
        "bit_exact_sampled": exact,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "roofline": {"bound": "hbm", "kernel": kname, "launch": dom_key,
                     "achieved": dom_bytes / (dom_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom_bytes / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": dom_bytes, "ms_per_launch": dom_ms},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
