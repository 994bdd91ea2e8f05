"""Input generators: structure and determinism (no GPU)."""
import numpy as np

import synth


def _check_csr(A):
    assert A.rowptr[0] == 0 and np.all(np.diff(A.rowptr) >= 0)
    assert len(A.col) == A.nnz
    for i in range(A.nrows):
        c, _ = A.row(i)
        assert np.all(np.diff(c) > 0), "row not sorted/unique"
    if A.nnz:
        assert A.col.min() >= 0 and A.col.max() < A.ncols


def test_er_exact_degree_sorted_unique():
    A = synth.er(4096, 4096, 8, 1)
    assert A.nnz == 4096 * 8
    d = np.diff(A.col.reshape(4096, 8), axis=1)
    assert np.all(d > 0)
    assert A.col.min() >= 0 and A.col.max() < 4096
    # roughly uniform columns
    counts = np.bincount(A.col, minlength=4096)
    assert abs(counts.mean() - 8) < 1e-9 and counts.max() < 30


def test_er_edge_cases():
    A = synth.er(3, 5, 5, 7)  # full rows
    assert np.array_equal(A.col, np.tile(np.arange(5), 3))
    Z = synth.er(4, 9, 0, 7)
    assert Z.nnz == 0


def test_rmat_shape_and_dedup():
    A = synth.rmat(12, 16, seed=1)
    _check_csr(A)
    m = 16 << 12
    assert 0.8 * m < A.nnz <= m
    deg = np.diff(A.rowptr)
    # skew: low ids are hubs under (0.57, 0.19, 0.19, 0.05) without relabelling
    assert deg[:64].mean() > 10 * deg[-2048:].mean()


def test_rmat_deterministic_across_threads(monkeypatch):
    a = synth.rmat(11, 8, seed=9)
    b = synth.rmat(11, 8, seed=9)
    assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.col, b.col)
    c = synth.rmat(11, 8, seed=10)
    assert not (len(c.col) == len(a.col) and np.array_equal(c.col, a.col))


def test_values_ranges():
    v = synth.values(synth.VAL_F32_UNIFORM, 100000, 1.0, 100.0, 3)
    assert v.dtype == np.float32 and v.min() >= 1.0 and v.max() < 100.0
    v = synth.values(synth.VAL_I64_UNIFORM, 100000, 1, 9, 3)
    assert set(np.unique(v)) == set(range(1, 10))
    v = synth.values(synth.VAL_F64_NORMAL, 200000, 0, 1, 3)
    assert abs(v.mean()) < 0.01 and abs(v.std() - 1) < 0.01
    v32 = synth.values(synth.VAL_F32_NORMAL, 200000, 0, 1, 3)
    assert np.array_equal(v32, v.astype(np.float32))


def test_block_split_roundtrip():
    A = synth.rmat(9, 8, seed=4)
    A = A.with_values(synth.values(synth.VAL_F64_UNIFORM, A.nnz, 0, 1, 5))
    g = 3
    blocks = synth.block_split(A, g)
    rb = -(-A.nrows // g)
    rows, cols, vals = [], [], []
    for I in range(g):
        for J in range(g):
            b = blocks[I][J]
            _check_csr(b)
            r = np.repeat(np.arange(b.nrows), np.diff(b.rowptr)) + I * rb
            rows.append(r)
            cols.append(b.col.astype(np.int64) + J * rb)
            vals.append(b.val)
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    order = np.lexsort((cols, rows))
    ar = np.repeat(np.arange(A.nrows), np.diff(A.rowptr))
    assert np.array_equal(rows[order], ar)
    assert np.array_equal(cols[order], A.col)
    assert np.array_equal(vals[order], A.val)


def test_select_and_take_rows():
    s = synth.select(1000, 100, 5)
    assert len(np.unique(s)) == 100 and s.min() >= 0 and s.max() < 1000
    A = synth.rmat(8, 8, seed=2)
    S = synth.take_rows(A, s[s < A.nrows][:10])
    _check_csr(S)


def test_transpose_involution():
    A = synth.rmat(8, 4, seed=3)
    A = A.with_values(np.arange(A.nnz, dtype=np.float64))
    T = synth.transpose(synth.transpose(A))
    assert np.array_equal(T.rowptr, A.rowptr) and np.array_equal(T.col, A.col) and np.array_equal(T.val, A.val)
