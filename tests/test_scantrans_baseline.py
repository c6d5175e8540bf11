"""Pins for the multi-threaded CPU baseline (oracle/scantrans.c).

The benchmark reports this baseline beside the single-threaded oracle. Its
result must be the oracle's, bit for bit, whatever the thread count: chunk
boundaries inside runs of one column, threads with empty chunks (more threads
than rows), empty rows and columns, zero-width payloads, and both offset
widths. The oracle is pinned on its own (tests/test_oracle.py); brute force on
a tiny case pins this one independently of it.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import gen
from workloads.gen import from_arrays


def _same(a, threads, perm=True):
    ref = oracle.transpose(a)
    got = oracle.transpose_mt(a, threads, perm=perm)
    assert np.array_equal(got.t_row_ptr, ref.t_row_ptr)
    assert np.array_equal(got.t_col, ref.t_col)
    assert np.array_equal(got.t_payload_off, ref.t_payload_off)
    assert np.array_equal(got.t_payload, ref.t_payload)
    if perm:
        assert np.array_equal(got.perm, ref.perm)


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
@pytest.mark.parametrize("ow", [4, 8])
def test_random_against_oracle(threads, ow):
    a = gen.random_small(threads * 7 + ow, n_rows=900, n_cols=700, deg_mean=6.0, w_lo=0, w_hi=13,
                         offset_width=ow)
    _same(a, threads)
    _same(a, threads, perm=False)


@pytest.mark.parametrize("threads", [2, 5])
def test_unsorted_rows_and_recipes(threads):
    _same(gen.random_small(3, n_rows=500, n_cols=400, deg_mean=5.0, sort_rows=False), threads)
    _same(gen.tiny(seed=1), threads)
    _same(gen.large(seed=2, scale=12), threads)
    _same(gen.hetero(seed=3, scale=14, parts=4), threads)


def test_one_hot_column_split_across_threads():
    # every cell in column 3: each thread's cursor must follow the ones before
    n = 40
    rp = np.arange(n + 1) * 3
    col = np.full(3 * n, 3)
    a = from_arrays(n, 8, rp, col, widths=np.arange(3 * n) % 5)
    _same(a, 7)


def test_more_threads_than_rows_and_empty():
    a = from_arrays(3, 5, [0, 2, 2, 5], [4, 0, 1, 1, 0], widths=[1, 0, 2, 3, 4])
    _same(a, 16)
    e = from_arrays(4, 6, [0, 0, 0, 0, 0], [], widths=[])
    _same(e, 3)
    z = from_arrays(0, 0, [0], [], widths=[])
    _same(z, 2)


def test_brute_force_pin():
    # pinned independently of the oracle: sort every cell by (column, input position)
    a = gen.random_small(11, n_rows=60, n_cols=50, deg_mean=3.0, w_lo=0, w_hi=5, sort_rows=False)
    got = oracle.transpose_mt(a, 4)
    t_row_ptr, t_col, t_poff, t_payload, perm = brute.transpose(a)
    assert np.array_equal(got.t_row_ptr, t_row_ptr)
    assert np.array_equal(got.t_col, t_col)
    assert np.array_equal(got.t_payload_off, t_poff)
    assert np.array_equal(got.t_payload, t_payload)
    assert np.array_equal(got.perm, perm)


def test_host_threads_bounds():
    assert 1 <= oracle.host_threads() <= 16
    assert oracle.host_threads(cap=1) == 1
