"""GPU parity of mgt_symmetrize (unordered multigraphs stored as one triangle,
paper Section 2) against the oracle's symmetrize, element by element."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import symmetric
from workloads import gen
from workloads.gen import from_arrays

from .common import to_device

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _compare(a, lower, validate=False, schedule=None):
    from paper_2012_06012_amd import mgt
    ref = symmetric.symmetrize(a, lower=lower)
    d = to_device(a)
    if schedule is None:
        out, status = mgt.symmetrize(d, lower=lower, validate=validate)
    else:  # a forced transpose schedule for the stored triangle
        plan = mgt.plan_for(d, mgt.VALIDATE if validate else 0)
        plan.set_schedule(*schedule)
        ws = torch.empty(mgt.mgt_symmetrize_workspace(plan), dtype=torch.uint8, device=d.col.device)
        odt = torch.int32 if a.offset_width == 4 else torch.int64
        out = dict(row_ptr=torch.empty(a.n_rows + 1, dtype=odt, device="cuda"),
                   col=torch.empty(max(2 * a.nnz, 1), dtype=torch.int32, device="cuda"),
                   payload_off=torch.empty(2 * a.nnz + 1, dtype=odt, device="cuda"),
                   payload=torch.empty(max(2 * a.payload_bytes, 1), dtype=torch.uint8,
                                       device="cuda"))
        sizes = torch.empty(2, dtype=torch.int64, device="cuda")
        status = torch.empty(1, dtype=torch.int32, device="cuda")
        mgt.mgt_symmetrize(plan, mgt.LOWER if lower else mgt.UPPER, d.row_ptr, d.col,
                           d.payload_off, d.payload, out["row_ptr"], out["col"],
                           out["payload_off"], out["payload"], sizes, ws, status)
        torch.cuda.synchronize()
        m, b = (int(x) for x in sizes.cpu().tolist())
        out = {"row_ptr": out["row_ptr"], "col": out["col"][:m],
               "payload_off": out["payload_off"][:m + 1], "payload": out["payload"][:b]}
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == mgt.OK
    assert np.array_equal(out["row_ptr"].cpu().numpy(), ref.row_ptr)
    assert np.array_equal(out["col"].cpu().numpy(), ref.col)
    assert np.array_equal(out["payload_off"].cpu().numpy(), ref.payload_off)
    assert np.array_equal(out["payload"].cpu().numpy(), ref.payload)


@pytest.mark.parametrize("lower", [True, False], ids=["lower", "upper"])
def test_hand_worked_example(lower):
    with open(os.path.join(HERE, "golden", "symmetric_5v.json")) as f:
        g = json.load(f)
    part = g["lower" if lower else "upper"]
    vals = [v.encode() for v in part["values"]]
    a = from_arrays(g["n"], g["n"], part["row_ptr"], part["col"], [len(v) for v in vals],
                    np.frombuffer(b"".join(vals), np.uint8), 8)
    _compare(a, lower)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("lower", [True, False], ids=["lower", "upper"])
@pytest.mark.parametrize("ow", [4, 8])
def test_random_triangles(seed, lower, ow):
    base = gen.random_small(100 + seed, n_rows=300 + 50 * seed, n_cols=300 + 50 * seed,
                            deg_mean=6.0, w_lo=0, w_hi=11, offset_width=ow,
                            sort_rows=seed % 2 == 0)
    a = symmetric.triangle(base, lower=lower)
    _compare(a, lower)


@pytest.mark.parametrize("lower", [True, False], ids=["lower", "upper"])
def test_large_triangle_two_passes(lower):
    # a 2^15 x 2^15 matrix with 2^21 cells; its triangle through the
    # benchmark's two-pass transpose (packed records), then symmetrized
    a = symmetric.triangle(gen.large(seed=4, scale=8), lower=lower)
    _compare(a, lower, schedule=(8, 4, 0))


def test_edge_cases():
    # empty, diagonal only, a single off-diagonal cell, empty rows
    _compare(from_arrays(4, 4, [0, 0, 0, 0, 0], [], None, None, 8), True)
    _compare(from_arrays(4, 4, [0, 1, 3, 3, 4], [0, 1, 1, 3], [2, 1, 0, 3],
                         np.arange(6, dtype=np.uint8), 8), True)
    _compare(from_arrays(3, 3, [0, 0, 0, 1], [1], [3], np.array([7, 8, 9], np.uint8), 4), True)
    _compare(from_arrays(3, 3, [0, 1, 1, 1], [2], [5], np.arange(5, dtype=np.uint8), 8), False)


def test_validate_flags_cell_outside_the_triangle():
    from paper_2012_06012_amd import mgt
    a = from_arrays(3, 3, [0, 1, 1, 2], [2, 0], [1, 2], np.arange(3, dtype=np.uint8), 8)
    out, status = mgt.symmetrize(to_device(a), lower=True, validate=True)
    assert int(status.cpu()[0]) == mgt.ERANGE
    out, status = mgt.symmetrize(to_device(a), lower=False, validate=True)
    assert int(status.cpu()[0]) == mgt.ERANGE  # row 2 holds column 0
    ok = from_arrays(3, 3, [0, 1, 1, 2], [0, 1], [1, 2], np.arange(3, dtype=np.uint8), 8)
    out, status = mgt.symmetrize(to_device(ok), lower=True, validate=True)
    assert int(status.cpu()[0]) == mgt.OK
