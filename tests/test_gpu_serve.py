"""Serving loop on the GPU: requests that arrive over time are batched
continuously over two streams; every request's result must equal the
oracle's and the result of transposing it alone, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

from .common import assert_matches_oracle, host, to_device

pytestmark = pytest.mark.gpu


def _pool(seed, n):
    mats = []
    for i in range(n):
        cells, n_rows, deg, width, r = gen.served_request_params(seed, i, 1e3, 2e5)
        a = gen.generate(n_rows, n_rows, seed=(seed << 24) + i + 7, deg_law=gen.DEG_POISSON,
                         deg_mean=float(deg), pay_law=gen.PAY_BYTES, w_lo=width, w_hi=width,
                         offset_width=8, bounds=gen.equal_bounds(n_rows, min(r, n_rows)))
        mats.append(a)
    return mats


def _serve(executor, host_mats, dev_mats, arrivals, n_slots=2, budget=40 << 30):
    from paper_2012_06012_amd.serve import Request, Server
    reqs = [Request(rid=i, mat=dev_mats[i % len(dev_mats)], arrival=t,
                    partitioned=dev_mats[i % len(dev_mats)].n_parts > 1)
            for i, t in enumerate(arrivals)]
    st = Server(executor, budget_bytes=budget, max_batch=16, n_slots=n_slots).run(reqs)
    torch.cuda.synchronize()
    return reqs, st


def test_served_results_equal_alone_and_oracle():
    from paper_2012_06012_amd import mgt, serve
    host_mats = _pool(3, 10)
    dev_mats = [to_device(a) for a in host_mats]
    arrivals = gen.poisson_arrivals(30, rate=4000.0, seed=1)
    reqs, st = _serve(serve.GpuExecutor(n_slots=2, max_items=64), host_mats, dev_mats, arrivals)
    assert st.completed == 30 and st.failed == 0 and st.rejected == 0
    assert st.batches < 30  # requests were batched
    for r in reqs:
        a = host_mats[r.rid % len(host_mats)]
        h = host(r.outputs)
        assert_matches_oracle(a, h, partitioned=r.partitioned)
        alone, s = mgt.transpose(dev_mats[r.rid % len(dev_mats)], partitioned=r.partitioned)
        ha = host(alone)
        for k, v in ha.items():
            if v is not None:
                assert np.array_equal(v, h[k]), (r.rid, k)


def test_plain_comparator_matches():
    from paper_2012_06012_amd import serve
    host_mats = _pool(4, 6)
    dev_mats = [to_device(a) for a in host_mats]
    arrivals = gen.poisson_arrivals(12, rate=2000.0, seed=2)
    reqs, st = _serve(serve.PlainExecutor(), host_mats, dev_mats, arrivals, n_slots=1)
    assert st.completed == 12
    for r in reqs:
        assert_matches_oracle(host_mats[r.rid % len(host_mats)], host(r.outputs),
                              partitioned=r.partitioned)


def test_serve_isolates_invalid_request():
    from paper_2012_06012_amd import serve
    host_mats = _pool(5, 5)
    bad = host_mats[2]
    bad.col = bad.col.copy()
    bad.col[bad.nnz // 2] = bad.n_cols + 1
    dev_mats = [to_device(a) for a in host_mats]
    arrivals = [0.0] * 5
    reqs, st = _serve(serve.GpuExecutor(n_slots=1, validate=True, max_items=16), host_mats,
                      dev_mats, arrivals, n_slots=1)
    assert reqs[2].status == -2 and st.failed == 1 and st.completed == 4
    for r in reqs:
        if r.rid != 2:
            assert_matches_oracle(host_mats[r.rid], host(r.outputs), partitioned=r.partitioned)
