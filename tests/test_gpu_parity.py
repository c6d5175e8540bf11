"""GPU parity: libmgt (through its C ABI) against the CPU oracle, bit for bit.

Every output of the transpose is integer or byte data, so the bar is exact
equality: transposed row offsets, original row ids, payload offsets, payload
bytes, the permutation, and for the partitioned form the transfer matrices,
partition offsets and Alltoallv displacements.
"""
import numpy as np
import pytest

from workloads import gen
from workloads.gen import from_arrays

from .common import assert_matches_oracle, gpu_transpose

pytestmark = pytest.mark.gpu


def _both(a, partitioned_too=True):
    h, st = gpu_transpose(a, partitioned=False, perm=True)
    assert st == 0
    assert_matches_oracle(a, h)
    # without perm: two-pass schedules carry packed records
    h, st = gpu_transpose(a, partitioned=False, perm=False)
    assert st == 0
    assert_matches_oracle(a, h)
    if partitioned_too and a.n_rows == a.n_cols:
        h, st = gpu_transpose(a, partitioned=True, perm=True)
        assert st == 0
        assert_matches_oracle(a, h, partitioned=True)


def test_tiny_recipe_plain_and_partitioned():
    _both(gen.tiny(seed=0))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tiny_recipe_seeds(seed):
    _both(gen.tiny(seed=seed))


@pytest.mark.parametrize("scale", [8, 7])
def test_large_recipe_scaled(scale):
    _both(gen.large(seed=0, scale=scale))


@pytest.mark.parametrize("scale", [9, 8])
def test_hetero_recipe_scaled(scale):
    _both(gen.hetero(seed=0, scale=scale))


@pytest.mark.parametrize("seed,n_rows,n_cols,deg,wlo,whi,ow,sort_rows,parts", [
    (0, 50, 40, 3.0, 0, 7, 8, True, 1),
    (1, 200, 200, 6.0, 0, 13, 4, False, 3),
    (2, 1000, 1000, 2.0, 1, 1, 8, True, 7),
    (3, 3000, 5000, 10.0, 0, 33, 8, False, 1),
    (4, 4096, 4096, 30.0, 4, 4, 4, True, 16),
    (5, 777, 777, 50.0, 0, 5, 8, True, 5),
    (6, 20000, 20000, 4.0, 0, 9, 8, True, 64),
    # four rows per partition: every wave of a sub-chunk holds many
    # (source, destination) partition pairs of the transfer matrices
    (7, 4096, 4096, 8.0, 0, 9, 8, False, 1024),
])
def test_random_shapes(seed, n_rows, n_cols, deg, wlo, whi, ow, sort_rows, parts):
    a = gen.random_small(seed, n_rows=n_rows, n_cols=n_cols, deg_mean=deg, w_lo=wlo, w_hi=whi,
                         sort_rows=sort_rows, offset_width=ow,
                         parts=parts if n_rows == n_cols else 1)
    _both(a)


def test_many_columns_two_passes_and_ragged_tiles():
    # 2^21 columns and ~300K cells: two partition passes, tiles with ragged tails
    a = gen.random_small(11, n_rows=100000, n_cols=1 << 21, deg_mean=3.0, w_lo=0, w_hi=11)
    _both(a, partitioned_too=False)


def test_hot_columns_multi_chunk_buckets():
    # few columns with many cells each: finish buckets span several LDS sub-chunks
    n = 300
    rng = np.random.default_rng(5)
    deg = rng.poisson(200, size=n)
    rp = np.concatenate([[0], np.cumsum(deg)])
    col = np.sort(rng.integers(0, 7, size=rp[-1]).reshape(-1))  # sorted globally -> rows sorted too
    col = np.concatenate([np.sort(col[rp[i]:rp[i + 1]]) for i in range(n)])
    w = rng.integers(0, 9, size=rp[-1])
    a = from_arrays(n, n, rp, col, w, None, 8, gen.equal_bounds(n, 3))
    _both(a)


def test_single_column_everything():
    n = 5000
    rp = np.arange(n + 1) * 3
    a = from_arrays(n, n, rp, np.full(rp[-1], 17), np.full(rp[-1], 5), None, 8,
                    gen.equal_bounds(n, 4))
    _both(a)


def test_empty_and_degenerate():
    _both(from_arrays(0, 0, [0], [], [], None, 8), partitioned_too=False)
    _both(from_arrays(5, 5, [0] * 6, [], [], None, 8, [0, 2, 2, 5, 5, 5]))
    _both(from_arrays(1, 1, [0, 3], [0, 0, 0], [0, 1, 2], None, 4))
    _both(from_arrays(3, 9, [0, 0, 4, 4], [8, 0, 8, 3], [1, 0, 2, 9], None, 8),
          partitioned_too=False)


def test_empty_partitions_and_uneven_bounds():
    a = gen.random_small(9, n_rows=500, n_cols=500, deg_mean=5.0, w_lo=0, w_hi=6)
    a.bounds = np.array([0, 0, 3, 3, 250, 251, 500, 500], np.int64)
    _both(a)


def test_determinism_repeated_runs():
    a = gen.large(seed=3, scale=9)
    h1, _ = gpu_transpose(a, partitioned=True)
    h2, _ = gpu_transpose(a, partitioned=True)
    for k in h1:
        if h1[k] is not None:
            assert np.array_equal(h1[k], h2[k]), k


def test_involution_on_device():
    a = gen.tiny(seed=4)
    h, _ = gpu_transpose(a, perm=False)
    b = gen.Csr(a.n_cols, a.n_rows, h["t_row_ptr"], h["t_col"], h["t_payload_off"], h["t_payload"],
                a.bounds, a.offset_width)
    h2, _ = gpu_transpose(b, perm=False)
    assert np.array_equal(h2["t_row_ptr"], a.row_ptr)
    assert np.array_equal(h2["t_col"], a.col)
    assert np.array_equal(h2["t_payload_off"], a.payload_off)
    assert np.array_equal(h2["t_payload"], a.payload)


def test_validate_mode_flags_bad_columns():
    a = gen.random_small(2, n_rows=100, n_cols=100, deg_mean=4.0, w_lo=0, w_hi=3)
    a.col = a.col.copy()
    a.col[a.nnz // 2] = a.n_cols  # out of range
    _, st = gpu_transpose(a, validate=True)
    assert st == -2


def test_validate_mode_flags_bad_offsets():
    a = gen.random_small(3, n_rows=100, n_cols=100, deg_mean=4.0, w_lo=1, w_hi=3)
    a.payload_off = a.payload_off.copy()
    k = a.nnz // 3
    a.payload_off[k] = a.payload_off[k + 1] + 1  # a negative size
    _, st = gpu_transpose(a, validate=True)
    assert st == -2
    b = gen.random_small(4, n_rows=100, n_cols=100, deg_mean=4.0, w_lo=1, w_hi=3)
    b.row_ptr = b.row_ptr.copy()
    b.row_ptr[50] = b.row_ptr[51] + 1
    _, st = gpu_transpose(b, validate=True)
    assert st == -2


def test_validate_mode_passes_good_input():
    a = gen.tiny(seed=6)
    h, st = gpu_transpose(a, validate=True, partitioned=True)
    assert st == 0
    assert_matches_oracle(a, h, partitioned=True)
