#!/usr/bin/env python3
"""Benchmark: plain XCSR multigraph transpose on one MI355X.

Workload (default): 2^23 x 2^23 multigraph with exactly 2^29 cells (2^23 per
each of 64 equal row blocks), power-law row degrees (alpha 2.1, d >= 10,
capped at 10^5), uniform columns, Geometric(1/2) multiplicity, 1-8 float32 of
payload per cell, int64 offsets, int32 column ids; synthetic and seeded.

A step is one mgt_transpose call (every stage of the hot path) on inputs
already resident in HBM. Prints one JSON line with cells/s, the fraction of
the 8 TB/s HBM peak reached in algorithmic bytes, the dominant kernel's
roofline, the CPU oracle's time on the same matrix (the CPU baseline) and a
bit-exactness verdict from comparing every output array with the oracle's.
"""
from __future__ import annotations

import argparse
import hashlib
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


def packs_records(a, perm: bool, n_passes: int) -> bool:
    """Whether the library carries this single-matrix call's records packed:
    one records-only pass, no perm, at most 28 column bits and every payload
    size below 2^(32 - column bits) bytes."""
    cb = max(int(a.n_cols) - 1, 0).bit_length()
    if perm or n_passes != 2 or cb > 28:
        return False
    if a.nnz == 0:
        return True
    return int(np.diff(np.asarray(a.payload_off, dtype=np.int64)).max()) < (1 << (32 - cb))


def kernel_bytes(a, stage: str, pass_idx: int, perm: bool, n_passes: int,
                 packed: bool = False) -> int:
    """Algorithmic bytes of one launch of a stage: each array it reads counted
    once and each array it writes counted once. Level-buffer records are 16
    bytes per cell (column, size, row, cell index); with two or more passes the
    last one moves records only and adds an 8-byte payload offset per cell,
    which the finish reads to fetch each payload. Packed records (one
    records-only pass, no perm) are 8 bytes after the first pass (column and
    size in one word, row) and 12 after the second (plus the payload offset
    relative to the finish bucket's first byte) where the 512-thread
    records-only pass writes them, as on the single-matrix workloads."""
    nnz, P, o = a.nnz, a.payload_bytes, a.offset_width
    rec = nnz * 16
    deferred = n_passes >= 2
    if packed:
        # the first histogram writes a 4-byte (column | size) word per cell,
        # which the first pass reads instead of the columns and offsets
        if stage == "scatter" and pass_idx == 0:
            return 4 * nnz + (a.n_rows + 1) * o + P + 8 * nnz + P
        if stage == "hist" and pass_idx == 0:
            return 4 * nnz + (nnz + 1) * o + 4 * nnz
        if stage == "scatter":
            return 8 * nnz + 12 * nnz
        if stage == "finish":
            return 12 * nnz + P + 4 * nnz + (nnz + 1) * o + (a.n_cols + 1) * o + P
    if stage == "scatter" and pass_idx == 0:
        return 4 * nnz + (nnz + 1) * o + (a.n_rows + 1) * o + P + rec + P
    if stage == "scatter" and deferred and pass_idx == n_passes - 1:
        return rec + 8 * nnz + 16 * nnz  # (column, size) and (row, index, payload offset) out
    if stage == "scatter":
        return 2 * (rec + P)
    if stage == "finish":  # after a records-only pass its records are 8 + 16 bytes
        return (rec + (8 * nnz if deferred else 0) + P + nnz * (4 + (4 if perm else 0))
                + (nnz + 1) * o + (a.n_cols + 1) * o + P)
    if stage == "hist" and pass_idx == 0:
        return 4 * nnz + (nnz + 1) * o
    if stage == "hist":
        return nnz * 8
    return 0


# HBM bytes of one whole step on the default workload (plain transpose of the
# large multigraph, seed 0), from two profiler counter runs: FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch, summed over every kernel of one step, each
# scaled by what the same counter reads for a plain device copy of known size.
# A reading holds only for the kernel sources it was taken on; after any change
# to them the traffic figure is reported as null.
MEASURED_TRAFFIC = {
    "step": {"sources_sha256": "b41429b62f1f5cab6b118842d51ceb6f2ebb66d48b303e4b12531d3a1c783382",
             "fetch_kib": 43052224.2, "write_kib": 44266422.2},
}
COPY_SCALE = {"fetch": 2.0, "write": 1.0}


def profiler_kernel_name(stage: str, pass_idx: int, n_passes: int, partitioned: bool,
                         packed: bool = False) -> str:
    """The profiler's name of the kernel behind a stage of one single-matrix
    call (template arguments as the library instantiates them). A packed
    first pass runs in the slim 256-thread kernel (its partition form when
    partitioned), and a packed records-only pass in the slim 512-thread
    kernel (the plain ones launched beside them return at once)."""
    if stage == "hist":
        return "mgt::geo256::k_pass_hist"
    if stage == "finishs":  # the 512-thread whole-bucket finish, two workgroups per CU
        return "mgt::geo256::k_finish_bucket<512>"
    if stage == "finishb":
        return "mgt::geo256::k_finish_bucket<1024>"
    if stage == "finish":
        return "mgt::geo256::k_finish<%s>" % ("true" if n_passes >= 2 else "false")
    if stage == "scatter":
        if pass_idx == 0:
            if packed:  # (the bench's variable-width matrices: the key-word form)
                return "mgt::geo256::k_pass_scatter<true, false, false, true, %s, false>" % (
                    "true" if partitioned else "false")
            return "mgt::geo256::k_pass_scatter<true, false, false, false, false, false>"
        if pass_idx == n_passes - 1:  # records only; 512-thread form for single matrices
            return "mgt::geo512::k_pass_scatter<false, true, false, %s, false, false>" % (
                "true" if packed else "false")
        return "mgt::geo256::k_pass_scatter<false, false, false, false, false, false>"
    return stage


# The sources that build the transpose's kernels and launches (the value-list
# conversions in values.hip are not part of it).
TRANSPOSE_SOURCES = ("kernels.h", "kernels.hip", "kernels_wide.hip", "mgt_internal.h", "prims.h",
                     "runtime.cpp")


def kernel_sources_digest() -> str:
    d = os.path.join(ROOT, "paper_2012_06012_amd", "csrc")
    h = hashlib.sha256()
    for name in TRANSPOSE_SOURCES:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def host_info() -> dict:
    """CPU count, the CPUs this process may use, CPU model and RAM of the host."""
    model, ram = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model, "ram_gib": ram}


def measured_traffic(kname: str, args):
    m = MEASURED_TRAFFIC.get(kname)
    if (m is None or args.partitioned or args.scale or args.seed
            or m["sources_sha256"] != kernel_sources_digest()):
        return None
    return int((m["fetch_kib"] * COPY_SCALE["fetch"] + m["write_kib"] * COPY_SCALE["write"]) * 1024)


def copy_rate(mib: int, reps: int = 5) -> dict:
    """A plain device-to-device copy of `mib` MiB, timed with events: the
    achievable HBM rate (read plus write) on this part."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_bytes_each_way": n, "ms": ms, "GBps_read_plus_write": 2 * n / ms / 1e6}


def copy_calibration(mib: int):
    print(json.dumps(copy_rate(mib)))


def _device(a, dev, fixed_width=False):
    import torch
    from paper_2012_06012_amd import mgt
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    return mgt.DeviceCsr(a.n_rows, a.n_cols, t(a.row_ptr), t(a.col),
                         None if fixed_width else t(a.payload_off), t(a.payload), a.bounds,
                         a.offset_width, fixed_width)


def _oracle_check(makers, outs, threads: int = 8, partition: bool = False) -> bool:
    """Every output array of item j (outs[j], device tensors) against the
    oracle's transpose of makers[j]() (a host matrix), in parallel threads;
    with `partition`, also the partition arrays of items that have them."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    def one(j):
        a = makers[j]()
        ref = oracle.transpose(a)
        o = outs[j]
        ok = all(np.array_equal(o[k].cpu().numpy(), getattr(ref, k)) for k in
                 ("t_row_ptr", "t_col", "t_payload_off", "t_payload") if o.get(k) is not None)
        if partition and o.get("xfer_cells") is not None:
            pc = oracle.partition_counts(a)
            ok = ok and all(np.array_equal(o[k].cpu().numpy(), getattr(pc, k)) for k in
                            ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off",
                             "sdispls", "rdispls") if o.get(k) is not None)
        return ok
    with ThreadPoolExecutor(threads) as ex:
        return all(ex.map(one, range(len(makers))))


def bench_batch(args):
    """Many independent matrices: mgt_batch_submit against one mgt_transpose per
    matrix on one stream, on the same matrices with bit-exact outputs compared.

    The 4,096-matrix workload holds about 2e10 cells, more than HBM: it is
    streamed in waves whose estimated footprint (inputs, outputs, workspace)
    stays within --batch-budget bytes. Each wave is generated, uploaded and
    then timed on the device with its inputs resident (HIP events around the
    submits only); cells/s is the sum of cells over the sum of timed wave
    times."""
    import torch
    from workloads import gen
    from paper_2012_06012_amd import mgt
    dev = torch.device("cuda:0")
    n_items = args.batch_items
    # ~100 bytes per cell: inputs and outputs (col, offsets, payload) plus the
    # batch workspace's level buffers
    est = [gen.batch_item_params(args.seed, i, 1e3, args.batch_n_hi) for i in range(n_items)]
    waves, cur, cur_b = [], [], 0.0
    for i, (n, deg, w) in enumerate(est):
        b = n * deg * (100.0 + 2 * w)
        if cur and cur_b + b > args.batch_budget:
            waves.append(cur)
            cur, cur_b = [], 0.0
        cur.append(i)
        cur_b += b
    if cur:
        waves.append(cur)
    log(f"[batch] {n_items} matrices in {len(waves)} waves (budget {args.batch_budget:.3g} B)")
    from paper_2012_06012_amd import autotune
    tot_cells, ms_b_tot, ms_g_tot, ms_p_tot, same_all = 0, 0.0, 0.0, 0.0, True
    ms_d_tot = 0.0
    oracle_all = True
    tuned, tune_report = None, None
    tot_bytes = 0  # algorithmic bytes of every matrix (inputs read once, outputs written once)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for wi, idx in enumerate(waves):
        t0 = time.time()
        mats = []
        for i in idx:
            h = gen.batch_item(args.seed, i, 1e3, args.batch_n_hi)
            tot_bytes += h.algorithmic_bytes()
            mats.append(_device(h, dev))
            del h
        cells = sum(a.nnz for a in mats)
        log(f"[batch] wave {wi}: {len(mats)} matrices, {cells} cells, ready in {time.time() - t0:.1f}s")
        outs, status, plan, ws = mgt.batch_transpose(mats)  # warm-up, allocations
        torch.cuda.synchronize()
        if tuned is None:
            # the autotuner on a sample batch (the first wave's first matrices,
            # up to 3e8 cells): digit widths 4/6/8 and tile sizes, every
            # candidate bit-identical to the rule; its setting runs every wave
            k, c = 0, 0
            while k < len(mats) and c + mats[k].nnz <= 3e8:
                c += mats[k].nnz
                k += 1
            _, tr = autotune.autotune_batch(mats[:max(k, 1)], reps=2, use_cache=False)
            torch.cuda.empty_cache()
            tuned = (tr.best["pass_bits"], tr.best["tile_cells"])
            tune_report = {"setting": {"pass_bits": tuned[0], "tile_cells": tuned[1]},
                           "sample": f"{max(k, 1)} matrices, {c} cells",
                           "default_ms_wave0": tr.default_ms, "best_ms_wave0": tr.best["ms"],
                           "candidates": [{k: t[k] for k in ("pass_bits", "tile_cells", "ms",
                                                             "bit_exact")} for t in tr.trials]}
            log(f"[batch] tuned on wave 0: {tune_report}")
        ev0.record()
        for _ in range(args.steps):
            mgt.batch_transpose(mats, plan=plan, workspace=ws, outs=outs)
        ev1.record()
        torch.cuda.synchronize()
        ms_d = ev0.elapsed_time(ev1) / args.steps
        ok_status = bool((status.cpu().numpy() == 0).all())
        # the tuned setting on the same matrices and outputs
        plan_t = mgt.batch_plan_for(mats)
        plan_t.set_schedule(tuned[0], -1, tuned[1])
        _, st_t, _, ws = mgt.batch_transpose(mats, plan=plan_t, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        ok_status = ok_status and bool((st_t.cpu().numpy() == 0).all())
        ev0.record()
        for _ in range(args.steps):
            mgt.batch_transpose(mats, plan=plan_t, workspace=ws, outs=outs)
        ev1.record()
        torch.cuda.synchronize()
        ms_b = ev0.elapsed_time(ev1) / args.steps
        plan = plan_t
        # the same submit recorded once as a graph and replayed (same outputs)
        g, _, gst, _, _ = mgt.batch_graph(mats, plan=plan, workspace=ws, outs=outs)
        g.launch()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            g.launch()
        ev1.record()
        torch.cuda.synchronize()
        ms_g = ev0.elapsed_time(ev1) / args.steps
        ok_status = ok_status and bool((gst.cpu().numpy() == 0).all())
        g.close()
        # one mgt_transpose per matrix into one scratch output set
        plans = [mgt.plan_for(a) for a in mats]
        ws1 = torch.empty(max(max(p.workspace_bytes for p in plans), 256), dtype=torch.uint8,
                          device=dev)
        odt = torch.int32 if mats[0].offset_width == 4 else torch.int64
        flat = dict(t_row_ptr=torch.empty(max(a.n_cols for a in mats) + 1, dtype=odt, device=dev),
                    t_col=torch.empty(max(a.nnz for a in mats), dtype=torch.int32, device=dev),
                    t_payload_off=torch.empty(max(a.nnz for a in mats) + 1, dtype=odt, device=dev),
                    t_payload=torch.empty(max(a.payload_bytes for a in mats), dtype=torch.uint8,
                                          device=dev), perm=None)

        def view(k):
            a = mats[k]
            return dict(t_row_ptr=flat["t_row_ptr"][:a.n_cols + 1], t_col=flat["t_col"][:a.nnz],
                        t_payload_off=flat["t_payload_off"][:a.nnz + 1],
                        t_payload=flat["t_payload"][:a.payload_bytes], perm=None)
        views = [view(k) for k in range(len(mats))]
        for a, p, o in zip(mats, plans, views):
            mgt.transpose(a, plan=p, workspace=ws1, out=o)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            for a, p, o in zip(mats, plans, views):
                mgt.transpose(a, plan=p, workspace=ws1, out=o)
        ev1.record()
        torch.cuda.synchronize()
        ms_p = ev0.elapsed_time(ev1) / args.steps
        # bit-exactness: each matrix alone against its slot of the batch
        same = ok_status
        for a, p, o, ob in zip(mats, plans, views, outs):
            mgt.transpose(a, plan=p, workspace=ws1, out=o)
            same = same and all(torch.equal(o[k], ob[k]) for k in
                                ("t_row_ptr", "t_col", "t_payload_off", "t_payload"))
        torch.cuda.synchronize()
        # every batched output against the oracle: each matrix regenerated on
        # the host from its seed and transposed there, in parallel threads
        ok_oracle = _oracle_check(
            [(lambda i=i: gen.batch_item(args.seed, i, 1e3, args.batch_n_hi)) for i in idx], outs)
        oracle_all = oracle_all and ok_oracle
        log(f"[batch] wave {wi}: batched {ms_b:.1f} ms tuned ({ms_d:.1f} ms by the rule; graph "
            f"replay {ms_g:.1f} ms), one by one {ms_p:.1f} ms, batched = one by one {same}, "
            f"batched = oracle {ok_oracle}")
        tot_cells += cells
        ms_b_tot += ms_b
        ms_d_tot += ms_d
        ms_g_tot += ms_g
        ms_p_tot += ms_p
        same_all = same_all and same
        del mats, outs, status, plan, plan_t, st_t, ws, plans, ws1, flat, views, g, gst
        torch.cuda.empty_cache()
    res = {"metric": "cells/s, batched vs per-matrix plain launches", "mode": "batch",
           "matrices": n_items, "waves": len(waves), "cells": tot_cells,
           "ms_batched": ms_b_tot, "ms_batched_rule": ms_d_tot, "tuning": tune_report,
           "ms_batched_graph": ms_g_tot, "ms_per_matrix_plain": ms_p_tot,
           "cells_per_s_batched": tot_cells / (ms_b_tot * 1e-3),
           "cells_per_s_plain": tot_cells / (ms_p_tot * 1e-3), "speedup": ms_p_tot / ms_b_tot,
           "algorithmic_bytes": tot_bytes,
           "hbm_frac_batched": tot_bytes / (ms_b_tot * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "hbm_frac_plain": tot_bytes / (ms_p_tot * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "bit_exact_batched_vs_plain": bool(same_all),
           "bit_exact": bool(oracle_all),
           "bit_exact_check": "every matrix of every wave compared in full with the oracle",
           "config": {"workload": f"batch of matrices, n log-uniform 1e3-{args.batch_n_hi:.0e}, "
                                  "mean degree U{8..64}, payload U{0..16} bytes per matrix",
                      "seed": args.seed, "wave_budget_bytes": args.batch_budget}}
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
    pool_n = args.serve_pool
    host = []
    for i in range(pool_n):
        cells, n, deg, width, r = gen.served_request_params(args.seed, i, 1e4, args.serve_c_hi)
        host.append(gen.generate(n, n, seed=(args.seed << 24) + i + 11, deg_law=gen.DEG_POISSON,
                                 deg_mean=float(deg), pay_law=gen.PAY_BYTES, w_lo=width,
                                 w_hi=width, offset_width=8, bounds=gen.equal_bounds(n, min(r, n))))
    pool = [_device(a, dev) for a in host]
    pool_cells = sum(a.nnz for a in host)
    pool_bytes = [a.algorithmic_bytes(partitioned=a.n_parts > 1) for a in host]
    log(f"[serve] pool of {pool_n} inputs, {pool_cells} cells, {time.time() - t0:.1f}s")
    # References for the parity check: each pool input transposed alone by the
    # plain path, every array compared in full with the oracle's on the host.
    # Served outputs are compared with these on the device, so a served output
    # equal to its reference equals the oracle's.
    refs = []
    from paper_2012_06012_amd import mgt
    for a in pool:
        o, st_ = mgt.transpose(a, partitioned=a.n_parts > 1)
        refs.append(o)
    torch.cuda.synchronize()
    refs_ok = _oracle_check([(lambda h=h: h) for h in host], refs, threads=16, partition=True)
    ref_bytes = sum(sum(v.numel() * v.element_size() for v in o.values() if v is not None)
                    for o in refs)
    # kept on the host while the timed runs use the whole budget
    refs = [{k: v.cpu() for k, v in o.items() if v is not None} for o in refs]
    torch.cuda.empty_cache()
    del host
    log(f"[serve] references: {ref_bytes / 1e9:.1f} GB, equal to the oracle: {refs_ok}")
    n_req = args.serve_requests

    def make(rate):
        arr = gen.poisson_arrivals(n_req, rate, args.seed + 3)
        return [Request(rid=i, mat=pool[i % pool_n], arrival=t, partitioned=pool[i % pool_n].n_parts > 1)
                for i, t in enumerate(arr)]

    budget = 200 << 30

    def release(r):  # a served request's outputs go back to the caller at completion
        r.outputs = None
    # capacity of the plain path: back-to-back, no arrivals gaps
    plain = Server(serve.PlainExecutor(), budget, max_batch=1, n_slots=1, on_done=release)
    cap_n = 2 * pool_n  # every pool input twice, back to back
    st = plain.run([Request(rid=i, mat=pool[i % pool_n], arrival=0.0,
                            partitioned=pool[i % pool_n].n_parts > 1) for i in range(cap_n)])
    mu = cap_n / st.last_done
    log(f"[serve] plain capacity {mu:.1f} req/s")
    out = {}
    # at most 2^26 cells (a few ms of device work) per batch: large requests
    # run alone instead of holding a batch of small ones back
    bex = serve.GpuExecutor(n_slots=2, max_items=64, batch_cells=1 << 26)
    pex = serve.PlainExecutor()
    warm = args.serve_warmup  # per rate: device allocations are made and cached there
    bytes_per_cell = (sum(pool_bytes[i % pool_n] for i in range(n_req)) /
                      max(1, sum(pool[i % pool_n].nnz for i in range(n_req))))
    for frac in (0.5, 0.7, 0.9, 1.2):
        rate = frac * mu
        Server(bex, budget, max_batch=32, n_slots=2, on_done=release).run(make(rate)[:warm])
        sb = Server(bex, budget, max_batch=32, n_slots=2, on_done=release).run(make(rate))
        Server(pex, budget, max_batch=1, n_slots=1, on_done=release).run(make(rate)[:warm])
        sp = Server(pex, budget, max_batch=1, n_slots=1, on_done=release).run(make(rate))
        out[f"{frac}mu"] = {"batched": sb.summary(), "plain": sp.summary()}
        for v in out[f"{frac}mu"].values():  # algorithmic bytes per cell of this request stream
            v["hbm_frac"] = v["cells_per_s"] * bytes_per_cell / 1e9 / HBM_PEAK_GBS
        # parity: the same request stream replayed through the same batching
        # server, every completed request's outputs compared on the device with
        # its input's reference (the replay's budget leaves room for them)
        chk = {"checked": 0, "equal": 0}
        refs_dev = [{k: v.to(dev) for k, v in o.items()} for o in refs]

        def check(r):
            if r.status == 0 and r.outputs is not None:
                ref = refs_dev[r.rid % pool_n]
                chk["checked"] += 1
                chk["equal"] += int(all(torch.equal(r.outputs[k], ref[k]) for k in ref))
            r.outputs = None
        sc = Server(bex, budget - ref_bytes, max_batch=32, n_slots=2, on_done=check).run(make(rate))
        del refs_dev
        torch.cuda.empty_cache()
        out[f"{frac}mu"]["parity"] = {
            "bit_exact": bool(refs_ok and chk["checked"] == sc.completed == n_req and
                              chk["equal"] == chk["checked"]),
            "requests_checked": chk["checked"], "requests_equal": chk["equal"],
            "how": "replay of the same stream through the batching server; every completed "
                   "request compared on the device with its input transposed alone, which "
                   "was compared in full with the oracle"}
        log(f"[serve] rate {rate:.1f}/s: batched {sb.summary()} plain {sp.summary()} "
            f"parity {out[f'{frac}mu']['parity']}")
    res = {"metric": "served p50/p99 latency and sustained cells/s, batched vs plain",
           "mode": "serve", "requests": n_req, "warmup_requests": warm,
           "plain_capacity_req_s": mu, "results": out,
           "config": {"workload": f"requests of log-uniform 1e4-{args.serve_c_hi:.0e} cells from a "
                                  f"pool of {pool_n} device-resident inputs, widths U{{0..32}}, "
                                  "R U{1..64}, Poisson arrivals", "budget_bytes": budget}}
    print(json.dumps(res), flush=True)


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def bench_tiny(args):
    """1,000 x 1,000, ~20K cells, R = 4: latency of one call (launch bound)."""
    import torch
    import oracle
    from workloads import gen
    from paper_2012_06012_amd import mgt
    dev = torch.device("cuda:0")
    a = gen.tiny(seed=args.seed)
    d = _device(a, dev)
    res = {"metric": "latency of one transpose call (tiny multigraph)", "mode": "tiny",
           "cells": a.nnz, "payload_bytes": a.payload_bytes}
    for part in (False, True):
        plan = mgt.plan_for(d)
        ws = mgt.workspace_for(plan, dev)
        out = mgt.alloc_outputs(d, partitioned=part)
        ms = _timed(lambda: mgt.transpose(d, plan=plan, workspace=ws, partitioned=part, out=out),
                    max(args.steps, 50), 5)
        # the same call recorded once as a graph and replayed (one launch per call)
        gout = mgt.alloc_outputs(d, partitioned=part)
        g, gout, _ = mgt.transpose_graph(d, plan=plan, workspace=ws, partitioned=part, out=gout)
        ms_g = _timed(g.launch, max(args.steps, 50), 5)
        ref = oracle.transpose(a)

        def exact(o):
            h = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
            return bool(all(np.array_equal(h[k], getattr(ref, k)) for k in
                            ("t_row_ptr", "t_col", "t_payload_off", "t_payload")))
        res["partitioned" if part else "plain"] = {
            "us_per_call": ms * 1e3, "cells_per_s": a.nnz / (ms * 1e-3), "bit_exact": exact(out),
            "graph_us_per_call": ms_g * 1e3, "graph_bit_exact": exact(gout)}
        g.close()
    print(json.dumps(res), flush=True)


def bench_tune(args):
    """The autotuner on the two full-size workloads: the default schedule's time
    against the fastest candidate's (outputs bit-identical for every one)."""
    import torch
    from workloads import gen
    from paper_2012_06012_amd import autotune
    dev = torch.device("cuda:0")
    res = {"metric": "autotuned schedule vs the default rule (ms per transpose)", "mode": "tune",
           "results": {}}
    for name, mk, part in (("large plain", lambda: gen.large(seed=args.seed, scale=args.scale), False),
                           ("hetero partitioned", lambda: gen.hetero(seed=args.seed, scale=args.scale),
                            True)):
        t0 = time.time()
        a = mk()
        d = _device(a, dev)
        del a
        log(f"[tune] {name}: ready in {time.time() - t0:.1f}s")
        plan, r = autotune.autotune(d, partitioned=part, reps=3, use_cache=False)
        res["results"][name] = {"default_ms": r.default_ms, "default_schedule": r.default_schedule,
                                "best": r.best, "candidates": len(r.trials),
                                "all_bit_exact": all(t["bit_exact"] for t in r.trials)}
        log(f"[tune] {name}: default {r.default_ms:.2f} ms {r.default_schedule}; best "
            f"{r.best['ms']:.2f} ms {r.best['schedule']} of {len(r.trials)} candidates")
        del d, plan
        torch.cuda.empty_cache()
    print(json.dumps(res), flush=True)


def stage_times(call, tplan, reps: int) -> dict:
    """Mean device time of each stage of `reps` calls made with a timing plan
    (the library records events around its launches on the call's stream);
    keys are the stage name and its index within one call."""
    acc = {}
    for _ in range(reps):
        call()
        pi = {}
        for name, v in tplan.stage_times():
            k = pi.get(name, 0)
            pi[name] = k + 1
            acc.setdefault((name, k), []).append(v)
    return {f"{n}{k}": float(np.mean(v)) for (n, k), v in acc.items()}


def bench_hetero(args):
    """Heterogeneously balanced multigraph, partitioned (R = 256): 2^21 x 2^21,
    2^30 cells, 28-byte payload; every output array checked against the oracle."""
    import torch
    import oracle
    from workloads import gen
    from paper_2012_06012_amd import mgt
    dev = torch.device("cuda:0")
    t0 = time.time()
    a = gen.hetero(seed=args.seed, scale=args.scale)
    log(f"[hetero] generated nnz={a.nnz} payload={a.payload_bytes} in {time.time() - t0:.1f}s")
    fixed = args.fixed_width
    d = _device(a, dev, fixed_width=fixed)
    plan = mgt.plan_for(d)
    ws = mgt.workspace_for(plan, dev)
    out = mgt.alloc_outputs(d, partitioned=True, payload_off=not fixed)
    ms = _timed(lambda: mgt.transpose(d, plan=plan, workspace=ws, partitioned=True, out=out),
                args.steps, args.warmup)
    tplan = mgt.plan_for(d, mgt.DEBUG_TIMING)
    tws = ws if tplan.workspace_bytes <= ws.numel() else mgt.workspace_for(tplan, dev)
    stages = stage_times(lambda: mgt.transpose(d, plan=tplan, workspace=tws, partitioned=True,
                                               out=out), tplan, 3)
    del tws
    log(f"[hetero] stages (ms): {json.dumps({k: round(v, 3) for k, v in stages.items()})}")
    # every output array against the oracle's whole-matrix transpose (its
    # column-range mode over disjoint ranges in host threads) and partition counts
    torch.cuda.synchronize()
    ref = oracle.transpose_sliced(a, slices=2 * oracle.host_threads())
    ok = True
    for k in ("t_row_ptr", "t_col", "t_payload_off", "t_payload"):
        if out.get(k) is not None:
            ok = ok and bool(np.array_equal(out[k].cpu().numpy(), getattr(ref, k)))
    del ref
    pc = oracle.partition_counts(a)
    for k in ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls", "rdispls"):
        ok = ok and bool(np.array_equal(out[k].cpu().numpy(), getattr(pc, k)))
    log(f"[hetero] full parity against the oracle: {ok}")
    b_alg = a.algorithmic_bytes(partitioned=True)
    if fixed:  # no payload offsets read or written
        b_alg -= 2 * (a.nnz + 1) * a.offset_width
    res = {"metric": "cells/s (partitioned transpose, bit-exact)",
           "mode": "hetero" + (" fixed-width" if fixed else ""),
           "value": a.nnz / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms,
           "hbm_frac_step": b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bit_exact": ok,
           "stages_ms": {k: round(v, 4) for k, v in stages.items()},
           "config": {"workload": "heterogeneous multigraph 2^21 x 2^21, 2^30 cells, 28-byte "
                                  "payload, R=256", "scale_shift": args.scale,
                      "nnz": a.nnz, "payload_bytes": a.payload_bytes}}
    print(json.dumps(res), flush=True)


def bench_involution(args):
    """The paper's check (Section 4): 12 composed transposes of one dataset on
    device-resident ping-pong buffers; T^12(A) must equal T^2(A), which is A
    itself when A's rows are column ordered (the generator's default)."""
    import torch
    from workloads import gen
    from paper_2012_06012_amd import mgt
    dev = torch.device("cuda:0")
    a = gen.large(seed=args.seed, scale=args.scale)
    d = _device(a, dev)
    plan = mgt.plan_for(d)
    ws = mgt.workspace_for(plan, dev)
    bufs = [mgt.alloc_outputs(d), mgt.alloc_outputs(d)]
    orig = {k: v.clone() for k, v in (("row_ptr", d.row_ptr), ("col", d.col),
                                      ("payload_off", d.payload_off), ("payload", d.payload))}

    def twelve():
        x = d
        for i in range(12):
            o = bufs[i & 1]
            mgt.transpose(x, plan=plan, workspace=ws, out=o)
            x = mgt.DeviceCsr(x.n_cols, x.n_rows, o["t_row_ptr"], o["t_col"], o["t_payload_off"],
                              o["t_payload"], x.bounds, x.offset_width)
        return x
    def same(x, ref):
        return bool(torch.equal(x.row_ptr, ref["row_ptr"]) and torch.equal(x.col, ref["col"]) and
                    torch.equal(x.payload_off, ref["payload_off"]) and
                    torch.equal(x.payload, ref["payload"]))

    # T(T(A)) is A with each row's cells ordered by column (ties keep their
    # order); every later even power must reproduce it exactly
    o1 = mgt.alloc_outputs(d)
    mgt.transpose(d, plan=plan, workspace=ws, out=o1)
    t1 = mgt.DeviceCsr(d.n_cols, d.n_rows, o1["t_row_ptr"], o1["t_col"], o1["t_payload_off"],
                       o1["t_payload"], d.bounds, d.offset_width)
    o2 = mgt.alloc_outputs(d)
    mgt.transpose(t1, plan=plan, workspace=ws, out=o2)
    torch.cuda.synchronize()
    t2 = {"row_ptr": o2["t_row_ptr"], "col": o2["t_col"], "payload_off": o2["t_payload_off"],
          "payload": o2["t_payload"]}
    x = twelve()
    torch.cuda.synchronize()
    ok12 = same(x, t2)
    ok2 = same(mgt.DeviceCsr(d.n_rows, d.n_cols, t2["row_ptr"], t2["col"], t2["payload_off"],
                             t2["payload"], d.bounds, d.offset_width), orig)
    ms = _timed(twelve, max(1, args.steps // 3), 1)
    res = {"metric": "12 composed transposes (paper's involution check)", "mode": "involution",
           "ms_for_12": ms, "cells_per_s": 12 * a.nnz / (ms * 1e-3), "T12_equals_T2": ok12,
           "T2_equals_A": ok2,
           "config": {"workload": "large multigraph 2^23 x 2^23, 2^29 cells" if not args.scale
                      else f"large multigraph at 1/2^{args.scale}", "scale_shift": args.scale}}
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
    ap.add_argument("--mode", choices=["plain", "batch", "serve", "tiny", "hetero", "involution",
                                       "tune"],
                    default="plain",
                    help="plain: the headline line; batch: many matrices in one mgt_batch_submit "
                         "vs per-matrix launches; serve: the continuous-batching request loop vs "
                         "per-request plain launches")
    ap.add_argument("--serve-requests", type=int, default=2000, help="serve: requests per rate")
    ap.add_argument("--serve-warmup", type=int, default=100, help="serve: warm-up requests per rate")
    ap.add_argument("--serve-pool", type=int, default=128, help="serve: distinct resident inputs")
    ap.add_argument("--serve-c-hi", type=float, default=1e8,
                    help="serve: largest request size (cells) of the log-uniform range")
    ap.add_argument("--batch-items", type=int, default=4096, help="batch: matrices")
    ap.add_argument("--batch-budget", type=float, default=200e9,
                    help="batch: estimated device bytes per wave of matrices")
    ap.add_argument("--batch-n-hi", type=float, default=1e6,
                    help="batch: largest matrix size of the log-uniform range")
    ap.add_argument("--fixed-width", action="store_true",
                    help="hetero: run the fixed-width mode (no payload offsets on the device)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the library has no "
              "multi-GPU exchange; partitions are logical partitions of one device.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "tiny":
        return bench_tiny(args)
    if args.mode == "hetero":
        return bench_hetero(args)
    if args.mode == "involution":
        return bench_involution(args)
    if args.mode == "tune":
        return bench_tune(args)

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
    status = torch.empty(1, dtype=torch.int32, device=dev)

    def step(p=plan):
        mgt.transpose(d, plan=p, workspace=ws, partitioned=part, out=out, stream=stream,
                      status=status)

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
    if int(status.cpu()[0]) != mgt.OK:
        raise SystemExit(f"device status {int(status.cpu()[0])}")
    # spread across steps: the same number of steps again, each between its own events
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    spread = {"p50": float(np.percentile(per_step, 50)), "p99": float(np.percentile(per_step, 99)),
              "min": float(per_step.min()), "max": float(per_step.max())}

    # per-stage device times (events recorded by the library on the same stream)
    tplan = mgt.plan_for(d, mgt.DEBUG_TIMING)
    stages = stage_times(lambda: step(tplan), tplan, max(3, min(args.steps, 5)))
    log(f"[bench] stages (ms): {json.dumps({k: round(v, 3) for k, v in stages.items()})}")
    n_passes = sum(1 for k in stages if k.rstrip("0123456789") == "scatter")
    packed = packs_records(a, False, n_passes) and not os.environ.get("MGT_NO_PACK")
    # the dominant kernel: the stage with the most device time per step, named
    # as the profiler names it; its own-bytes model is a diagnostic only
    kernels = {}
    for key, v in stages.items():
        st = key.rstrip("0123456789")
        if st not in ("scatter", "finish", "finishb", "finishs", "hist"):
            continue
        pidx = int(key[len(st):] or 0)
        name = profiler_kernel_name(st, pidx, n_passes, part, packed)
        e = kernels.setdefault(name, [0.0, 0, 0])
        e[0] += v
        # the first whole-bucket launch takes the buckets (all of them on this
        # workload); a later one and k_finish take what it left (none here),
        # and k_finish writes the tails
        first_b = "finishs0" if "finishs0" in stages else "finishb0"
        bytes_st = st
        if st in ("finishs", "finishb"):
            bytes_st = "finish" if key == first_b else "tails"
        if st == "finish" and first_b in stages:
            bytes_st = "tails"
        e[1] += kernel_bytes(a, bytes_st, pidx, False, n_passes, packed)
        e[2] += 1
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms = kernels[dom][0] / kernels[dom][2]
    dom_bytes = kernels[dom][1] // kernels[dom][2]

    b_alg = a.algorithmic_bytes(partitioned=part)
    value = a.nnz / (ms * 1e-3)
    # the achievable rate on this part, beside the 8 TB/s peak
    copy_gbs = copy_rate(4096)["GBps_read_plus_write"]
    achieved_step = b_alg / (ms * 1e-3) / 1e9
    traffic = measured_traffic("step", args)

    # bit-exactness: every output array against the oracle's whole-matrix
    # transpose, whose single-threaded run is also the CPU baseline (timed
    # around the oracle call alone, outputs allocated and touched before)
    exact = None
    cpu = cpu_mt = None
    if not (args.no_check and args.no_cpu):
        import oracle
        torch.cuda.synchronize()
        host_out = {k: out[k].cpu().numpy() for k in ("t_row_ptr", "t_col", "t_payload_off",
                                                      "t_payload")}
        if part:
            host_out.update({k: out[k].cpu().numpy() for k in
                             ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off",
                              "sdispls", "rdispls")})
        ref = oracle.alloc_transposed(a)
        c0 = time.perf_counter()
        oracle.transpose(a, out=ref)
        cs = time.perf_counter() - c0
        cpu = {"value": a.nnz / cs, "unit": "cells/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole matrix ({a.nnz} cells, {a.payload_bytes} payload bytes); "
                         f"{cs:.1f} s single-threaded, timed around the oracle call alone",
               "host": host_info()}
        log(f"[bench] cpu oracle: {cpu['value']:.3e} cells/s ({cs:.1f} s)")
        ok = all(np.array_equal(host_out[k], getattr(ref, k)) for k in
                 ("t_row_ptr", "t_col", "t_payload_off", "t_payload"))
        if part:
            pc = oracle.partition_counts(a)
            ok = ok and all(np.array_equal(host_out[k], getattr(pc, k)) for k in
                            ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off",
                             "sdispls", "rdispls"))
        exact = bool(ok)
        log(f"[bench] full parity against the oracle: {exact}")
        del host_out, ref
        if args.no_cpu:
            cpu = None
        else:
            # the multi-threaded scan-based baseline on the same matrix
            nt = oracle.host_threads()
            c0 = time.perf_counter()
            oracle.transpose_mt(a, nt, perm=False)
            cm = time.perf_counter() - c0
            cpu_mt = {"value": a.nnz / cm, "unit": "cells/s", "cores": nt,
                      "kind": "multi-threaded scan-based transpose (per-thread column counts)",
                      "sample": f"the same {a.nnz} cells; {cm:.2f} s on {nt} threads, "
                                "including its output allocation",
                      "host": host_info()}
            log(f"[bench] cpu multi-threaded: {cpu_mt['value']:.3e} cells/s on {nt} threads")

    res = {
        "metric": "cells/s (plain transpose, bit-exact) and % of HBM peak",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step_ms_spread": spread,
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
        "copy_GBps": copy_gbs,
        "copy_frac_step": achieved_step / copy_gbs,
        "algorithmic_GBps_step": achieved_step,
        "algorithmic_bytes_step": b_alg,
        "bit_exact": exact,
        "bit_exact_check": "every output array compared in full with the oracle's transpose "
                           "of the whole matrix",
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        # algorithmic bytes of the whole step (every input read once, every output
        # written once) over the step time; the dominant kernel is named as the
        # profiler names it, with its live per-launch time
        "roofline": {"bound": "hbm", "achieved": achieved_step, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_step / HBM_PEAK_GBS,
                     "frac_of_copy": achieved_step / copy_gbs, "traffic": traffic,
                     "algorithmic_bytes": b_alg, "ms_per_step": ms,
                     "kernel": dom, "kernel_ms_per_launch": dom_ms,
                     "kernel_launches_per_step": kernels[dom][2],
                     "kernel_own_bytes_model": {
                         "bytes_per_launch": dom_bytes,
                         "GBps": dom_bytes / (dom_ms * 1e-3) / 1e9,
                         "frac": dom_bytes / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "note": "the kernel's own arrays, level buffers included, each "
                                 "read or written once: a diagnostic, not the roofline"}},
        "cpu_baseline": cpu,
        "cpu_baseline_mt": cpu_mt,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
