"""GPU parity on two-, three- and four-pass schedules.

The library picks one or two partition passes for most shapes. Capping the
bits per pass and per finish bucket (MGT_MAX_PASS_BITS, MGT_MAX_FINISH_BITS)
forces longer schedules on small inputs. The paths that only long schedules
take then run here against the oracle: the payload moving through both level
buffers, the last pass carrying records only, and the finish reading each
payload through its stored offset. The schedule lengths noted per case come
from the library's schedule rule for those caps.
"""
import numpy as np
import pytest
import torch

from workloads import gen

from .common import assert_matches_oracle, gpu_transpose, host, to_device

pytestmark = pytest.mark.gpu


def _caps(monkeypatch, pass_bits, finish_bits):
    monkeypatch.setenv("MGT_MAX_PASS_BITS", str(pass_bits))
    monkeypatch.setenv("MGT_MAX_FINISH_BITS", str(finish_bits))


def _both(a, partitioned_too=True):
    h, st = gpu_transpose(a, partitioned=False, perm=True)
    assert st == 0
    assert_matches_oracle(a, h)
    if partitioned_too and a.n_rows == a.n_cols and a.n_parts > 1:
        h, st = gpu_transpose(a, partitioned=True, perm=True)
        assert st == 0
        assert_matches_oracle(a, h, partitioned=True)


@pytest.mark.parametrize("caps", [(4, 4), (3, 3), (2, 2)])  # plain 3, 4, -; partitioned 2, 2, 4 passes
def test_large_recipe_long_schedules(monkeypatch, caps):
    _caps(monkeypatch, *caps)
    _both(gen.large(seed=3, scale=8))


@pytest.mark.parametrize("caps", [(4, 4), (3, 3)])  # 2 and 3 passes
def test_hetero_recipe_long_schedules(monkeypatch, caps):
    _caps(monkeypatch, *caps)
    _both(gen.hetero(seed=4, scale=9))


@pytest.mark.parametrize("caps,seed,n,deg,wlo,whi,ow,parts", [
    ((3, 3), 0, 3000, 8.0, 0, 13, 4, 1),     # 3 passes; unaligned byte payloads, 4-byte offsets
    ((2, 4), 0, 3000, 8.0, 0, 13, 4, 1),     # 4 passes
    ((4, 4), 1, 5000, 4.0, 0, 40, 8, 12),    # 3 | 2 passes; cells wider than 32 bytes
    ((2, 4), 1, 5000, 4.0, 0, 40, 8, 12),    # partitioned 3 passes
    ((2, 2), 2, 20000, 6.0, 1, 1, 8, 64),    # partitioned 4 passes
    ((4, 4), 3, 70000, 3.0, 0, 9, 8, 1),     # 4 passes
])
def test_random_long_schedules(monkeypatch, caps, seed, n, deg, wlo, whi, ow, parts):
    _caps(monkeypatch, *caps)
    a = gen.random_small(seed, n_rows=n, n_cols=n, deg_mean=deg, w_lo=wlo, w_hi=whi,
                         offset_width=ow, parts=parts)
    _both(a)


def test_hot_column_long_schedule(monkeypatch):
    # 3 passes; one column holds a third of the cells: a multi-chunk finish
    # bucket whose payloads are read through stored offsets
    _caps(monkeypatch, 4, 4)
    a = gen.random_small(9, n_rows=30000, n_cols=30000, deg_mean=5.0, w_lo=0, w_hi=17)
    col = a.col.copy()
    col[::3] = 12345
    a = gen.from_arrays(a.n_rows, a.n_cols, a.row_ptr, col, np.diff(a.payload_off), a.payload)
    _both(a, partitioned_too=False)


def test_batch_mixed_schedule_lengths(monkeypatch):
    # items needing 1 to 4 passes share one launch sequence (shorter schedules
    # are padded with zero-bit passes)
    from paper_2012_06012_amd import mgt
    _caps(monkeypatch, 3, 3)
    items = [gen.tiny(seed=5), gen.large(seed=6, scale=9),
             gen.random_small(7, n_rows=40000, n_cols=40000, deg_mean=4.0, w_lo=0, w_hi=11),
             gen.random_small(8, n_rows=20, n_cols=30, deg_mean=2.0, w_lo=0, w_hi=3)]
    items = [it if it.offset_width == 8 else
             gen.from_arrays(it.n_rows, it.n_cols, it.row_ptr, it.col, np.diff(it.payload_off),
                             it.payload)
             for it in items]
    mats = [to_device(a) for a in items]
    outs, status, plan, ws = mgt.batch_transpose(mats, perm=True)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    for a, o in zip(items, outs):
        assert_matches_oracle(a, host(o))


@pytest.mark.parametrize("caps", [(8, 7), (5, 5)])  # 2 and 3 passes
def test_wide_records_pass(monkeypatch, caps):
    # 8 M cells: 8,192-cell tiles, so the records-only last pass runs with
    # 512-thread workgroups and 4,096-cell sub-chunks
    _caps(monkeypatch, *caps)
    _both(gen.large(seed=5, scale=6))
