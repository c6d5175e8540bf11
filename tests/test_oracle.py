"""Pins for the CPU oracle: everything here runs without a GPU.

The oracle (oracle/oracle.c) is checked against things other than itself:
hand-worked examples of the paper's definition (tests/golden), brute-force
sorting of tiny inputs, scipy's CSR->CSC conversion, closed forms, the
involution / degree / payload invariants the paper states (Section 3: the
transpose is involutory; Section 4 composes 12 transposes as a check), and a
rank-by-rank simulation of the paper's staged algorithm (oracle/staged.py).
A final group plants specific mistakes in the oracle and checks that these
pins catch each one.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from oracle import brute, staged
from workloads import gen
from workloads.gen import Csr, from_arrays

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- helpers

def as_csr(a: Csr, t) -> Csr:
    """The transposed result as an input matrix (rows = a's columns)."""
    return Csr(a.n_cols, a.n_rows, t.t_row_ptr, t.t_col, t.t_payload_off, t.t_payload,
               a.bounds if a.n_rows == a.n_cols else np.array([0, a.n_cols]), a.offset_width)


def canon(a: Csr) -> Csr:
    """Rows stably sorted by column, each cell's payload moved with it."""
    rp = np.asarray(a.row_ptr, np.int64)
    po = np.asarray(a.payload_off, np.int64)
    order = []
    for i in range(a.n_rows):
        ks = np.arange(rp[i], rp[i + 1])
        order.extend(ks[np.argsort(a.col[ks], kind="stable")].tolist())
    order = np.array(order, dtype=np.int64)
    widths = (po[1:] - po[:-1])[order] if len(order) else np.zeros(0, np.int64)
    blob = b"".join(bytes(a.payload[po[k]:po[k + 1]]) for k in order)
    return from_arrays(a.n_rows, a.n_cols, rp, a.col[order] if len(order) else a.col, widths,
                       np.frombuffer(blob, np.uint8), a.offset_width, a.bounds)


def same_matrix(a: Csr, b: Csr) -> bool:
    return (a.n_rows == b.n_rows and a.n_cols == b.n_cols
            and np.array_equal(np.asarray(a.row_ptr, np.int64), np.asarray(b.row_ptr, np.int64))
            and np.array_equal(a.col, b.col)
            and np.array_equal(np.asarray(a.payload_off, np.int64), np.asarray(b.payload_off, np.int64))
            and np.array_equal(a.payload, b.payload))


def check_against_brute(a: Csr):
    t = oracle.transpose(a)
    b_rp, b_col, b_poff, b_pay, b_perm = brute.transpose(a)
    assert np.array_equal(np.asarray(t.t_row_ptr, np.int64), b_rp)
    assert np.array_equal(t.t_col, b_col)
    assert np.array_equal(t.perm, b_perm)
    assert np.array_equal(np.asarray(t.t_payload_off, np.int64), b_poff)
    assert np.array_equal(t.t_payload, b_pay)


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------------------- golden

def test_golden_xcsr_multigraph():
    g = load_golden("xcsr_6v_3ranks.json")
    vals = [v.encode() for v in g["values"]]
    a = from_arrays(g["n_rows"], g["n_cols"], g["row_ptr"], g["col"], [len(v) for v in vals],
                    np.frombuffer(b"".join(vals), np.uint8), 8, g["bounds"])
    e = g["expected"]
    t = oracle.transpose(a)
    assert t.t_row_ptr.tolist() == e["t_row_ptr"]
    assert t.t_col.tolist() == e["t_col"]
    assert t.perm.tolist() == e["perm"]
    assert t.t_payload_off.tolist() == e["t_payload_off"]
    assert bytes(t.t_payload) == "".join(e["t_values"]).encode()
    pc = oracle.partition_counts(a)
    for key in ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls", "rdispls"):
        assert getattr(pc, key).tolist() == e[key], key


@pytest.mark.parametrize("ow", [4, 8])
def test_golden_simple_csr(ow):
    g = load_golden("csr_simple_4v.json")
    vals = np.array(g["int32_values"], dtype="<i4")
    a = from_arrays(g["n_rows"], g["n_cols"], g["row_ptr"], g["col"], [4] * len(vals),
                    vals.view(np.uint8), ow, g["bounds"])
    e = g["expected"]
    t = oracle.transpose(a)
    assert t.t_row_ptr.tolist() == e["t_row_ptr"]
    assert t.t_col.tolist() == e["t_col"]
    assert t.perm.tolist() == e["perm"]
    assert t.t_payload.view("<i4").tolist() == e["t_int32_values"]
    pc = oracle.partition_counts(a)
    assert pc.xfer_cells.tolist() == e["xfer_cells"]
    assert pc.xfer_bytes.tolist() == e["xfer_bytes"]
    assert pc.part_cell_off.tolist() == e["part_cell_off"]


# ----------------------------------------------------------------------------- brute force

@st.composite
def tiny_csr(draw):
    n_rows = draw(st.integers(0, 8))
    n_cols = draw(st.integers(1, 8))
    ow = draw(st.sampled_from([4, 8]))
    sort_rows = draw(st.booleans())
    rows = []
    for _ in range(n_rows):
        if draw(st.booleans()):
            cols = draw(st.lists(st.integers(0, n_cols - 1), max_size=8))
        else:  # many repeats of few columns
            c = draw(st.integers(0, n_cols - 1))
            cols = [c] * draw(st.integers(0, 6))
        if sort_rows:
            cols = sorted(cols)
        rows.append(cols)
    col = [c for r in rows for c in r]
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    widths = draw(st.lists(st.integers(0, 7), min_size=len(col), max_size=len(col)))
    seed = draw(st.integers(0, 2**31))
    return from_arrays(n_rows, n_cols, row_ptr, col, widths, None, ow, None, seed)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_csr())
def test_brute_force_tiny(a):
    check_against_brute(a)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_generated(seed):
    a = gen.random_small(seed, n_rows=40, n_cols=30, deg_mean=5.0, w_lo=0, w_hi=9,
                         sort_rows=bool(seed % 2), offset_width=4 if seed % 3 == 0 else 8)
    check_against_brute(a)


def test_brute_force_tiny_recipe_scaled():
    check_against_brute(gen.tiny(seed=3, scale=4))


# ----------------------------------------------------------------------------- scipy pin

@pytest.mark.parametrize("seed,sort_rows", [(0, True), (1, False), (2, True)])
def test_scipy_csr_to_csc(seed, sort_rows):
    """scipy's CSR->CSC keeps duplicates and orders each column by (row, position);
    carrying k+1 as the value recovers the permutation (exact in float64)."""
    a = gen.random_small(seed, n_rows=3000, n_cols=2500, deg_mean=12.0, w_lo=0, w_hi=5,
                         sort_rows=sort_rows)
    t = oracle.transpose(a)
    m = sp.csr_matrix((np.arange(a.nnz, dtype=np.float64) + 1.0, a.col,
                       np.asarray(a.row_ptr, np.int64)), shape=(a.n_rows, a.n_cols))
    c = m.tocsc()
    assert np.array_equal(c.indptr, np.asarray(t.t_row_ptr, np.int64))
    assert np.array_equal(c.indices, t.t_col)
    assert np.array_equal((c.data - 1.0).astype(np.int64), t.perm.astype(np.int64))


# ----------------------------------------------------------------------------- invariants

def test_involution_and_degrees_tiny_recipe():
    a = gen.tiny(seed=0)
    t = oracle.transpose(a)
    rp = np.asarray(a.row_ptr, np.int64)
    # nnz and payload bytes preserved
    assert t.t_col.shape[0] == a.nnz and t.t_payload.shape[0] == a.payload_bytes
    # column degrees of A are the row degrees of T(A), and vice versa
    assert np.array_equal(np.diff(np.asarray(t.t_row_ptr, np.int64)),
                          np.bincount(a.col, minlength=a.n_cols))
    assert np.array_equal(np.bincount(t.t_col, minlength=a.n_rows), np.diff(rp))
    # each cell's payload ends with its original index (tag): payload moved with its cell
    po = np.asarray(t.t_payload_off, np.int64)
    tags = np.array([t.t_payload[po[p + 1] - 4:po[p + 1]].view("<i4")[0] for p in range(a.nnz)])
    assert np.array_equal(tags, t.perm.astype(np.int64))
    # rows of T(A) are canonical (sorted by column)
    tp = np.asarray(t.t_row_ptr, np.int64)
    for c in range(a.n_cols):
        assert np.all(np.diff(t.t_col[tp[c]:tp[c + 1]]) >= 0)
    # T(T(A)) = A for canonical A
    tt = oracle.transpose(as_csr(a, t))
    assert same_matrix(as_csr(as_csr(a, t), tt), a)


@pytest.mark.parametrize("seed", range(4))
def test_involution_unsorted_rows(seed):
    """Any within-row order: T(T(A)) = canon(A), and T^3 = T."""
    a = gen.random_small(seed + 10, n_rows=200, n_cols=150, deg_mean=6.0, w_lo=0, w_hi=6,
                         sort_rows=False)
    t1 = as_csr(a, oracle.transpose(a))
    t2 = as_csr(t1, oracle.transpose(t1))
    t3 = as_csr(t2, oracle.transpose(t2))
    assert same_matrix(t2, canon(a))
    assert same_matrix(t3, t1)


def test_twelve_fold_composition():
    """Section 4 composes 12 transposes of one dataset to check involution."""
    a = gen.tiny(seed=5, scale=1)
    x = a
    for _ in range(12):
        x = as_csr(x, oracle.transpose(x))
    assert same_matrix(x, a)


def test_payload_multiset_swapped_roles():
    a = gen.random_small(21, n_rows=120, n_cols=90, deg_mean=5.0, w_lo=1, w_hi=9)
    t = oracle.transpose(a)
    ed = sorted((i, j, bytes(p)) for (i, j, _, p) in brute.edges(a))
    tt = as_csr(a, t)
    ed_t = sorted((j, i, bytes(p)) for (i, j, _, p) in brute.edges(tt))
    assert ed == ed_t


# ----------------------------------------------------------------------------- closed forms

def test_identity():
    n = 17
    a = from_arrays(n, n, np.arange(n + 1), np.arange(n), [3] * n, None, 8)
    t = oracle.transpose(a)
    assert np.array_equal(t.t_row_ptr, np.arange(n + 1))
    assert np.array_equal(t.t_col, np.arange(n))
    assert np.array_equal(t.t_payload, a.payload)


def test_permutation_matrix_inverse():
    n = 64
    p = np.random.default_rng(4).permutation(n)
    a = from_arrays(n, n, np.arange(n + 1), p, [1] * n, None, 4)
    t = oracle.transpose(a)
    inv = np.empty(n, np.int64)
    inv[p] = np.arange(n)
    assert np.array_equal(t.t_col, inv)  # P^T = P^-1


def test_single_row_becomes_column():
    n = 9
    a = from_arrays(1, n, [0, n], np.arange(n), [2] * n, None, 8)
    t = oracle.transpose(a)
    assert np.array_equal(t.t_row_ptr, np.arange(n + 1))
    assert np.array_equal(t.t_col, np.zeros(n, np.int32))
    assert np.array_equal(t.t_payload, a.payload)


def test_all_cells_in_one_column():
    n, c = 30, 7
    deg = np.arange(n) % 4
    rp = np.concatenate([[0], np.cumsum(deg)])
    a = from_arrays(n, n, rp, np.full(rp[-1], c), np.ones(rp[-1], int), None, 8)
    t = oracle.transpose(a)
    expect = np.zeros(n + 1, np.int64)
    expect[c + 1:] = rp[-1]
    assert np.array_equal(np.asarray(t.t_row_ptr, np.int64), expect)
    assert np.array_equal(t.t_col, np.repeat(np.arange(n), deg))
    assert np.array_equal(t.perm, np.arange(rp[-1]))


def test_symmetric_pattern_fixed_point():
    rng = np.random.default_rng(8)
    n = 40
    m = rng.integers(0, 3, size=(n, n))
    m = m + m.T  # symmetric multiplicities
    rows, cols = [], []
    for i in range(n):
        for j in range(n):
            rows += [i] * int(m[i, j])
            cols += [j] * int(m[i, j])
    rp = np.concatenate([[0], np.cumsum(m.sum(axis=1))])
    a = from_arrays(n, n, rp, cols, np.zeros(len(cols), int), None, 8)
    t = oracle.transpose(a)
    assert np.array_equal(np.asarray(t.t_row_ptr, np.int64), rp)
    assert np.array_equal(t.t_col, np.asarray(cols, np.int32))


def test_diagonal_blocks_give_diagonal_transfer():
    R, w = 5, 6
    n = R * w
    rng = np.random.default_rng(2)
    rows, cols = [], []
    for i in range(n):
        blk = i // w
        cs = sorted(rng.integers(blk * w, blk * w + w, size=rng.integers(0, 5)).tolist())
        cols.append(cs)
    rp = np.concatenate([[0], np.cumsum([len(c) for c in cols])])
    flat = [c for cs in cols for c in cs]
    a = from_arrays(n, n, rp, flat, np.ones(len(flat), int) * 3, None, 8,
                    np.arange(0, n + 1, w))
    pc = oracle.partition_counts(a)
    assert np.array_equal(pc.xfer_cells, np.diag(np.diag(pc.xfer_cells)))
    assert np.array_equal(np.diag(pc.xfer_cells), np.diff(rp[::w]))


def test_empty_inputs():
    a = from_arrays(0, 5, [0], [], [], None, 8)
    t = oracle.transpose(a)
    assert t.t_row_ptr.tolist() == [0] * 6 and t.t_col.size == 0
    b = from_arrays(4, 4, [0, 0, 0, 0, 0], [], [], None, 4, [0, 0, 2, 2, 4])
    pc = oracle.partition_counts(b)
    assert pc.xfer_cells.sum() == 0 and pc.part_cell_off.tolist() == [0] * 5


# ----------------------------------------------------------------------------- partitions

@pytest.mark.parametrize("R,seed", [(1, 0), (3, 1), (4, 2), (7, 3)])
def test_staged_simulation_matches(R, seed):
    a = gen.random_small(seed, n_rows=70, n_cols=70, deg_mean=6.0, w_lo=0, w_hi=8, parts=R,
                         sort_rows=bool(seed % 2))
    s = staged.run(a)
    t = oracle.transpose(a)
    pc = oracle.partition_counts(a)
    assert np.array_equal(s["t_row_ptr"], np.asarray(t.t_row_ptr, np.int64))
    assert np.array_equal(s["t_col"], t.t_col)
    assert np.array_equal(s["perm"], t.perm)
    assert np.array_equal(s["t_payload_off"], np.asarray(t.t_payload_off, np.int64))
    assert np.array_equal(s["t_payload"], t.t_payload)
    for key in ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls", "rdispls"):
        assert np.array_equal(s[key], getattr(pc, key)), key


def test_staged_with_empty_partitions():
    a = gen.random_small(5, n_rows=40, n_cols=40, deg_mean=4.0, w_lo=0, w_hi=4)
    a.bounds = np.array([0, 0, 10, 10, 25, 40, 40], np.int64)
    s = staged.run(a)
    pc = oracle.partition_counts(a)
    t = oracle.transpose(a)
    for key in ("xfer_cells", "xfer_bytes", "part_cell_off", "part_byte_off", "sdispls", "rdispls"):
        assert np.array_equal(s[key], getattr(pc, key)), key
    assert np.array_equal(s["t_payload"], t.t_payload)


def test_partition_invariants_tiny_recipe():
    a = gen.tiny(seed=1)
    pc = oracle.partition_counts(a)
    t = oracle.transpose(a)
    rp = np.asarray(a.row_ptr, np.int64)
    b = a.bounds
    assert pc.xfer_cells.sum() == a.nnz
    assert np.array_equal(pc.xfer_cells.sum(axis=1), rp[b[1:]] - rp[b[:-1]])
    tp = np.asarray(t.t_row_ptr, np.int64)
    assert np.array_equal(pc.xfer_cells.sum(axis=0), tp[b[1:]] - tp[b[:-1]])
    assert np.array_equal(pc.part_cell_off, tp[b])
    assert np.array_equal(pc.part_byte_off, np.asarray(t.t_payload_off, np.int64)[tp[b]])
    assert pc.xfer_bytes.sum() == a.payload_bytes


# ----------------------------------------------------------------------------- slices

def test_column_slices_match_full():
    a = gen.random_small(33, n_rows=500, n_cols=400, deg_mean=7.0, w_lo=0, w_hi=12)
    t = oracle.transpose(a)
    tp = np.asarray(t.t_row_ptr, np.int64)
    po = np.asarray(t.t_payload_off, np.int64)
    for lo, hi in [(0, 400), (0, 1), (37, 38), (100, 250), (399, 400), (5, 5)]:
        s = oracle.transpose_columns(a, lo, hi)
        assert np.array_equal(s.t_row_ptr, tp[lo:hi + 1] - tp[lo])
        assert np.array_equal(s.t_col, t.t_col[tp[lo]:tp[hi]])
        assert np.array_equal(s.perm, t.perm[tp[lo]:tp[hi]])
        assert np.array_equal(s.t_payload_off, po[tp[lo]:tp[hi] + 1] - po[tp[lo]])
        assert np.array_equal(s.t_payload, t.t_payload[po[tp[lo]]:po[tp[hi]]])


@pytest.mark.parametrize("slices", [1, 3, 7, 64])
@pytest.mark.parametrize("ow", [4, 8])
def test_sliced_transpose_equals_whole(slices, ow):
    """Slices assembled by column range give every array of the whole transpose."""
    for seed in range(3):
        a = gen.random_small(40 + seed, n_rows=300, n_cols=50 + 40 * seed, deg_mean=6.0,
                             w_lo=0, w_hi=9, offset_width=ow)
        t = oracle.transpose(a)
        s = oracle.transpose_sliced(a, slices=slices, threads=4)
        for k in ("t_row_ptr", "t_col", "t_payload_off", "t_payload", "perm"):
            x, y = getattr(s, k), getattr(t, k)
            assert x.dtype == y.dtype and np.array_equal(x, y), k
    empty = from_arrays(3, 4, [0, 0, 0, 0], [], None, None, 8)
    s = oracle.transpose_sliced(empty, slices=4, threads=2)
    assert s.t_row_ptr.tolist() == [0] * 5 and s.t_payload_off.tolist() == [0]


# ----------------------------------------------------------------------------- validation

def test_validation_rejects_bad_inputs():
    good = gen.random_small(1, n_rows=10, n_cols=10, deg_mean=3.0, parts=2)
    assert oracle.validate(good, 2) == oracle.OK
    bad = from_arrays(3, 3, [0, 2, 1, 3], [0, 1, 2], None, None, 8)
    assert oracle.validate(bad) == oracle.ERANGE
    bad = from_arrays(2, 3, [0, 1, 2], [0, 3], None, None, 8)
    assert oracle.validate(bad) == oracle.ERANGE
    bad = from_arrays(2, 3, [0, 1, 2], [0, -1], None, None, 8)
    assert oracle.validate(bad) == oracle.ERANGE
    rect = from_arrays(2, 3, [0, 1, 2], [0, 2], None, None, 8, [0, 1, 2])
    assert oracle.validate(rect, 2) == oracle.EINVAL
    nb = from_arrays(3, 3, [0, 1, 2, 3], [0, 1, 2], None, None, 8, [0, 2, 1, 3])
    assert oracle.validate(nb, 3) == oracle.EINVAL
    with pytest.raises(oracle.OracleError):
        oracle.transpose(from_arrays(2, 3, [0, 1, 2], [0, 5], None, None, 8))


# ----------------------------------------------------------------------------- planted faults

# Each planted mistake is a plausible bug of a counting-sort transpose, applied
# to the oracle's own results on the CPU (the oracle's C code carries none of
# them): the pins must reject every one.

def _col_ranges(t_row_ptr):
    rp = np.asarray(t_row_ptr, np.int64)
    return [(int(rp[c]), int(rp[c + 1])) for c in range(len(rp) - 1)]


def _reorder(t, order):
    """The same transposed cells in another order (payload moved with them)."""
    sz = np.diff(np.asarray(t.t_payload_off, np.int64))
    pieces = [t.t_payload[int(t.t_payload_off[p]):int(t.t_payload_off[p + 1])] for p in order]
    poff = np.zeros_like(t.t_payload_off)
    poff[1:] = np.cumsum(sz[order]).astype(poff.dtype)
    pay = np.concatenate(pieces) if pieces else t.t_payload[:0]
    return oracle.Transposed(t.t_row_ptr, t.t_col[order], poff, pay.astype(np.uint8), t.perm[order])


def _plant(kind, transpose, partition_counts):
    def faulty_transpose(a):
        t = transpose(a)
        if kind == "unstable":          # equal-column cells in reverse order
            order = np.concatenate([np.arange(lo, hi)[::-1] for lo, hi in _col_ranges(t.t_row_ptr)]
                                   or [np.zeros(0, np.int64)]).astype(np.int64)
            return _reorder(t, order)
        if kind == "short_copy":        # last payload byte of every cell not copied
            pay = t.t_payload.copy()
            ends = np.asarray(t.t_payload_off[1:], np.int64)
            starts = np.asarray(t.t_payload_off[:-1], np.int64)
            pay[ends[ends > starts] - 1] = 0
            return oracle.Transposed(t.t_row_ptr, t.t_col, t.t_payload_off, pay, t.perm)
        if kind == "index_for_row":     # cell index written where the row goes
            return oracle.Transposed(t.t_row_ptr, t.perm.astype(np.int32), t.t_payload_off,
                                     t.t_payload, t.perm)
        if kind == "inclusive_rowptr":  # inclusive instead of exclusive column offsets
            rp = t.t_row_ptr.copy()
            rp[:-1] = rp[1:]
            return oracle.Transposed(rp, t.t_col, t.t_payload_off, t.t_payload, t.perm)
        return t

    def faulty_counts(a):
        pc = partition_counts(a)
        if kind == "swap_xfer":         # X and B built [dst][src]
            return oracle.PartitionCounts(pc.xfer_cells.T.copy(), pc.xfer_bytes.T.copy(),
                                          pc.part_cell_off, pc.part_byte_off, pc.sdispls,
                                          pc.rdispls)
        return pc
    return faulty_transpose, faulty_counts


def _pins_pass(a_list):
    try:
        for a in a_list:
            check_against_brute(a)
            s = staged.run(a)
            pc = oracle.partition_counts(a)
            for key in ("xfer_cells", "xfer_bytes"):
                assert np.array_equal(s[key], getattr(pc, key))
        g = load_golden("xcsr_6v_3ranks.json")
        vals = [v.encode() for v in g["values"]]
        ga = from_arrays(6, 6, g["row_ptr"], g["col"], [len(v) for v in vals],
                         np.frombuffer(b"".join(vals), np.uint8), 8, g["bounds"])
        assert oracle.transpose(ga).t_col.tolist() == g["expected"]["t_col"]
        assert oracle.partition_counts(ga).xfer_cells.tolist() == g["expected"]["xfer_cells"]
        return True
    except AssertionError:
        return False


@pytest.mark.parametrize("fault", ["unstable", "short_copy", "index_for_row", "swap_xfer",
                                   "inclusive_rowptr"])
def test_planted_faults_are_caught(fault, monkeypatch):
    cases = [gen.random_small(s, n_rows=30, n_cols=30, deg_mean=4.0, w_lo=1, w_hi=5, parts=3)
             for s in range(3)]
    assert _pins_pass(cases)
    ft, fc = _plant(fault, oracle.transpose, oracle.partition_counts)
    with monkeypatch.context() as m:
        m.setattr(oracle, "transpose", ft)
        m.setattr(oracle, "partition_counts", fc)
        assert not _pins_pass(cases)
    assert _pins_pass(cases)
