"""GPU parity of the fixed-width mode (MGT_FIXED_WIDTH): the homogeneous-value
variant of Section 2, where every cell carries the same number of payload
bytes. The payload offsets then never reach the device. The results must
equal the oracle's transpose of the same matrix with explicit offsets, and
t_payload_off, when asked for, must be p * width."""
import numpy as np
import pytest
import torch

from workloads import gen

from .common import assert_matches_oracle, host, to_device

pytestmark = pytest.mark.gpu


def _fixed(seed, n, width, deg=6.0, ow=8, parts=1, sort_rows=True):
    return gen.random_small(seed, n_rows=n, n_cols=n, deg_mean=deg, w_lo=width, w_hi=width,
                            offset_width=ow, parts=parts, sort_rows=sort_rows)


def _run(a, partitioned=False, with_poff=True, validate=False):
    from paper_2012_06012_amd import mgt
    d = to_device(a, fixed_width=True)
    out = mgt.alloc_outputs(d, perm=True, partitioned=partitioned, payload_off=with_poff)
    out, status = mgt.transpose(d, perm=True, partitioned=partitioned, validate=validate,
                                out=out)
    return host(out), int(status.cpu()[0])


def _check(a, h, partitioned=False):
    if h["t_payload_off"] is None:
        w = a.payload_bytes // max(a.nnz, 1)
        h = dict(h, t_payload_off=np.arange(a.nnz + 1, dtype=a.payload_off.dtype) * w)
    assert_matches_oracle(a, h, partitioned=partitioned)


@pytest.mark.parametrize("width", [0, 1, 3, 4, 8, 28, 36])
@pytest.mark.parametrize("ow", [4, 8])
def test_fixed_width_matches_oracle(width, ow):
    a = _fixed(width, 5000, width, ow=ow, parts=7)
    for part in (False, True):
        for with_poff in (True, False):
            h, st = _run(a, partitioned=part, with_poff=with_poff)
            assert st == 0
            _check(a, h, partitioned=part)


def test_fixed_width_hetero_recipe():
    # the heterogeneous recipe's cells are all 28 bytes: partitioned, R = 256
    a = gen.hetero(seed=2, scale=8)
    assert (np.diff(a.payload_off) == 28).all()
    h, st = _run(a, partitioned=True, with_poff=False)
    assert st == 0
    _check(a, h, partitioned=True)


def test_fixed_width_unsorted_rows_and_validate():
    a = _fixed(3, 3000, 12, sort_rows=False)
    h, st = _run(a, validate=True)
    assert st == 0
    _check(a, h)


def test_fixed_width_validate_flags_bad_column():
    a = _fixed(4, 2000, 8)
    col = a.col.copy()
    col[17] = a.n_cols + 5
    b = gen.from_arrays(a.n_rows, a.n_cols, a.row_ptr, col, np.diff(a.payload_off), a.payload)
    h, st = _run(b, validate=True)
    assert st == -2


def test_fixed_width_long_schedule(monkeypatch):
    monkeypatch.setenv("MGT_MAX_PASS_BITS", "4")
    monkeypatch.setenv("MGT_MAX_FINISH_BITS", "4")
    a = _fixed(5, 30000, 20, deg=5.0)
    h, st = _run(a, with_poff=False)
    assert st == 0
    _check(a, h)


def test_batch_mixes_fixed_and_variable_widths():
    from paper_2012_06012_amd import mgt
    items = [_fixed(6, 4000, 16), gen.random_small(7, n_rows=3000, n_cols=3000, w_lo=0, w_hi=9),
             _fixed(8, 100, 0), _fixed(9, 20000, 5, parts=4)]
    mats = [to_device(a, fixed_width=(i != 1)) for i, a in enumerate(items)]
    outs = [mgt.alloc_outputs(m, perm=True, partitioned=m.n_parts > 1, payload_off=(i % 2 == 1))
            for i, m in enumerate(mats)]
    outs, status, plan, ws = mgt.batch_transpose(mats, perm=True, outs=outs)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    for a, o in zip(items, outs):
        _check(a, host(o), partitioned=a.n_parts > 1)
