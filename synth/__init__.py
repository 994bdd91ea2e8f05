"""Seeded synthetic inputs for the semiring SpGEMM library and its oracle.

This module only draws sparsity patterns and values (Erdos-Renyi rows,
R-MAT graphs, value fills, block-grid splits, row selections).  It holds none
of the semiring product's arithmetic, so the CPU oracle and the GPU path can
both be fed from it without sharing any of the method's code.

The native part (``libsynth.so``) is plain C++/OpenMP built with g++; call
:func:`synth.build.build` (done by ``__graft_entry__.build()``) before use.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run synth.build.build() first")
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.synth_er.argtypes = [i64, i64, i32, u64, P, P]
        lib.synth_er.restype = ctypes.c_int
        lib.synth_rmat_edges.argtypes = [i32, i64, f64, f64, f64, u64, P, P]
        lib.synth_rmat_edges.restype = None
        lib.synth_edges_to_csr.argtypes = [i64, i64, P, P, P, P]
        lib.synth_edges_to_csr.restype = i64
        lib.synth_values.argtypes = [i32, i64, f64, f64, u64, P]
        lib.synth_values.restype = ctypes.c_int
        lib.synth_select.argtypes = [i64, i64, u64, P]
        lib.synth_select.restype = ctypes.c_int
        lib.synth_batch_params.argtypes = [i32, f64, f64, i32, i32, u64, P, P]
        lib.synth_batch_params.restype = None
        lib.synth_block_split.argtypes = [i64, i64, P, P, P, i32, i32, i32, i64, i64, P, P, P, P]
        lib.synth_block_split.restype = None
        lib.synth_num_threads.argtypes = []
        lib.synth_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Host CSR matrix: int64 row offsets, int32 sorted unique columns."""

    nrows: int
    ncols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1]) if len(self.rowptr) else 0

    def with_values(self, val: np.ndarray) -> "CSR":
        assert len(val) == self.nnz
        return CSR(self.nrows, self.ncols, self.rowptr, self.col, val, dict(self.meta))

    def row(self, i: int):
        a, b = int(self.rowptr[i]), int(self.rowptr[i + 1])
        return self.col[a:b], (None if self.val is None else self.val[a:b])

    def to_dense(self, fill=0):
        """Dense copy (tests on tiny matrices only)."""
        dt = self.val.dtype if self.val is not None else np.uint8
        d = np.full((self.nrows, self.ncols), fill, dtype=dt)
        present = np.zeros((self.nrows, self.ncols), dtype=bool)
        for i in range(self.nrows):
            c, v = self.row(i)
            d[i, c] = 1 if v is None else v
            present[i, c] = True
        return d, present


# value kinds understood by synth_values
VAL_F64_UNIFORM, VAL_F32_UNIFORM, VAL_I64_UNIFORM, VAL_F64_NORMAL, VAL_F32_NORMAL, VAL_ONES, VAL_BERNOULLI = range(7)
_VAL_DTYPE = {0: np.float64, 1: np.float32, 2: np.int64, 3: np.float64, 4: np.float32, 5: np.uint8, 6: np.uint8}


def values(kind: int, n: int, lo: float = 0.0, hi: float = 1.0, seed: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=_VAL_DTYPE[kind])
    if n:
        rc = _load().synth_values(kind, n, float(lo), float(hi), seed & 0xFFFFFFFFFFFFFFFF, _ptr(out))
        if rc != 0:
            raise ValueError(f"bad value kind {kind}")
    return out


def er(nrows: int, ncols: int, d: int, seed: int) -> CSR:
    """Erdos-Renyi pattern with exactly d distinct uniform columns per row."""
    rowptr = np.empty(nrows + 1, dtype=np.int64)
    col = np.empty(nrows * d, dtype=np.int32)
    rc = _load().synth_er(nrows, ncols, d, seed & 0xFFFFFFFFFFFFFFFF, _ptr(rowptr), _ptr(col))
    if rc != 0:
        raise ValueError("bad ER arguments")
    return CSR(nrows, ncols, rowptr, col, meta={"kind": "er", "d": d, "seed": seed})


def rmat(scale: int, edge_factor: int = 16, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 1) -> CSR:
    """R-MAT pattern of 2^scale vertices and edge_factor*2^scale drawn edges,
    duplicates removed, no relabelling, self loops kept."""
    n = 1 << scale
    m = edge_factor * n
    rows = np.empty(m, dtype=np.int32)
    cols = np.empty(m, dtype=np.int32)
    a, b, c, _ = abcd
    lib = _load()
    lib.synth_rmat_edges(scale, m, a, b, c, seed & 0xFFFFFFFFFFFFFFFF, _ptr(rows), _ptr(cols))
    rowptr = np.empty(n + 1, dtype=np.int64)
    nnz = lib.synth_edges_to_csr(n, m, _ptr(rows), _ptr(cols), _ptr(rowptr), None)
    col = np.empty(nnz, dtype=np.int32)
    lib.synth_edges_to_csr(n, m, _ptr(rows), _ptr(cols), _ptr(rowptr), _ptr(col))
    return CSR(n, n, rowptr, col, meta={"kind": "rmat", "scale": scale, "ef": edge_factor, "seed": seed})


def edges_to_csr(nrows: int, rows: np.ndarray, cols: np.ndarray) -> CSR:
    rows = np.ascontiguousarray(rows, dtype=np.int32).copy()
    cols = np.ascontiguousarray(cols, dtype=np.int32).copy()
    m = len(rows)
    rowptr = np.empty(nrows + 1, dtype=np.int64)
    lib = _load()
    nnz = lib.synth_edges_to_csr(nrows, m, _ptr(rows), _ptr(cols), _ptr(rowptr), None)
    col = np.empty(nnz, dtype=np.int32)
    lib.synth_edges_to_csr(nrows, m, _ptr(rows), _ptr(cols), _ptr(rowptr), _ptr(col))
    return CSR(nrows, int(cols.max()) + 1 if m else 0, rowptr, col)


def select(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices from [0, n), uniform, sorted."""
    out = np.empty(k, dtype=np.int64)
    if _load().synth_select(n, k, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out)) != 0:
        raise ValueError("bad selection size")
    return out


def take_rows(A: CSR, rows: np.ndarray) -> CSR:
    """The sub-matrix A[rows, :] (rows in the given order)."""
    rows = np.asarray(rows, dtype=np.int64)
    lens = A.rowptr[rows + 1] - A.rowptr[rows]
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    idx = np.concatenate([np.arange(A.rowptr[r], A.rowptr[r + 1]) for r in rows]) if len(rows) else np.zeros(0, np.int64)
    idx = idx.astype(np.int64)
    return CSR(len(rows), A.ncols, rowptr, A.col[idx].copy(), None if A.val is None else A.val[idx].copy())


def block_split(A: CSR, grid: int) -> list:
    """Cut square A into a grid x grid array of blocks (block-local columns).
    Returns blocks[I][J] as CSR."""
    lib = _load()
    rb = -(-A.nrows // grid)
    cb = -(-A.ncols // grid)
    nb = grid * grid
    blk_rowptr = np.empty(nb * (rb + 1), dtype=np.int64)
    lib.synth_block_split(A.nrows, A.ncols, _ptr(A.rowptr), _ptr(A.col), None, 0, grid, grid, rb, cb,
                          _ptr(blk_rowptr), None, None, None)
    blk_rowptr = blk_rowptr.reshape(nb, rb + 1)
    nnzs = blk_rowptr[:, -1].copy()
    base = np.zeros(nb, dtype=np.int64)
    np.cumsum(nnzs[:-1], out=base[1:])
    out_col = np.empty(int(nnzs.sum()), dtype=np.int32)
    vb = 0 if A.val is None else A.val.dtype.itemsize
    out_val = None if A.val is None else np.empty(int(nnzs.sum()), dtype=A.val.dtype)
    lib.synth_block_split(A.nrows, A.ncols, _ptr(A.rowptr), _ptr(A.col), _ptr(A.val), vb, grid, grid, rb, cb,
                          _ptr(blk_rowptr), _ptr(base), _ptr(out_col), _ptr(out_val))
    blocks = []
    for I in range(grid):
        row = []
        for J in range(grid):
            b = I * grid + J
            nr = min(rb, A.nrows - I * rb)
            nc = min(cb, A.ncols - J * cb)
            s, e = int(base[b]), int(base[b] + nnzs[b])
            rp = blk_rowptr[b, : nr + 1].copy()
            row.append(CSR(nr, nc, rp, out_col[s:e], None if out_val is None else out_val[s:e]))
        blocks.append(row)
    return blocks


def batch_params(count: int, nlo: float, nhi: float, dlo: int, dhi: int, seed: int):
    n = np.empty(count, dtype=np.int64)
    d = np.empty(count, dtype=np.int32)
    _load().synth_batch_params(count, nlo, nhi, dlo, dhi, seed & 0xFFFFFFFFFFFFFFFF, _ptr(n), _ptr(d))
    return n, d


def num_threads() -> int:
    return int(_load().synth_num_threads())


def identity(n: int, val_dtype=None, one=1) -> CSR:
    rowptr = np.arange(n + 1, dtype=np.int64)
    col = np.arange(n, dtype=np.int32)
    val = None if val_dtype is None else np.full(n, one, dtype=val_dtype)
    return CSR(n, n, rowptr, col, val)


def random_small(nrows: int, ncols: int, density: float, seed: int) -> CSR:
    """Tiny Bernoulli(density) pattern for brute-force tests (uses the value
    stream as a coin per cell)."""
    coins = values(VAL_BERNOULLI, nrows * ncols, density, 0.0, seed).reshape(nrows, ncols).astype(bool)
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(coins.sum(axis=1), out=rowptr[1:])
    col = np.nonzero(coins)[1].astype(np.int32)
    return CSR(nrows, ncols, rowptr, col)


def transpose(A: CSR) -> CSR:
    """Structural transpose (a relabelling of stored entries, no arithmetic)."""
    order = np.lexsort((np.repeat(np.arange(A.nrows), np.diff(A.rowptr)), A.col))
    rows_of = np.repeat(np.arange(A.nrows, dtype=np.int32), np.diff(A.rowptr))
    tcol = rows_of[order]
    counts = np.bincount(A.col, minlength=A.ncols)
    rowptr = np.zeros(A.ncols + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(A.ncols, A.nrows, rowptr, tcol.astype(np.int32), None if A.val is None else A.val[order].copy())
