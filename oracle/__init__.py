"""CPU oracle for the semiring sparse product and merge.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package; the GPU
library never does.  It shares no code with the GPU path: both are fed from
the ``synth`` input generators only.

What it computes: rows of C = A (x).(+) B over one of five semirings, or
one of three semirings a user would define at run time (paper, Section
2.2), and the entry-wise (+) merge of partial products (paper, Section
4.4), by plain row-by-row Gustavson with a ``std::map``
accumulator (``oracle.cpp`` has the definitions).  Results come back as numpy
CSR arrays.
"""
from __future__ import annotations

import ctypes
import os
import time
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, "liboracle.so")

# semiring ids (the oracle's own numbering; it mirrors the library's public
# enum by value only)
PLUS_TIMES_I64, PLUS_TIMES_F32, PLUS_TIMES_F64, OR_AND_BOOL, MIN_PLUS_F32 = 1, 2, 3, 4, 5
SEMIRINGS = (PLUS_TIMES_I64, PLUS_TIMES_F32, PLUS_TIMES_F64, OR_AND_BOOL, MIN_PLUS_F32)
# semirings a user of the library would define at run time (the oracle's own
# definitions of three of them)
MAX_PLUS_F32, MAX_TIMES_F64, MIN_MAX_I64 = 6, 7, 8
USER_SEMIRINGS = (MAX_PLUS_F32, MAX_TIMES_F64, MIN_MAX_I64)
IN_DTYPE = {1: np.int64, 2: np.float32, 3: np.float64, 4: np.uint8, 5: np.float32, 6: np.float32, 7: np.float64,
            8: np.int64}
OUT_DTYPE = {1: np.int64, 2: np.float64, 3: np.float64, 4: np.uint8, 5: np.float32, 6: np.float32, 7: np.float64,
             8: np.int64}
NAMES = {1: "plus_times_i64", 2: "plus_times_f32", 3: "plus_times_f64", 4: "or_and_bool", 5: "min_plus_f32",
         6: "max_plus_f32", 7: "max_times_f64", 8: "min_max_i64"}


@dataclass
class OracleResult:
    """Rows of an oracle result: CSR over the selected rows."""

    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    mag: Optional[np.ndarray]  # sum of |products| per entry (float sums only)
    seconds: float = 0.0

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    def __init__(self, path: str = DEFAULT_LIB):
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run oracle.build.build() first")
        lib = ctypes.CDLL(path)
        P, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_spgemm.argtypes = [ci, i64, i64, P, P, P, i64, i64, P, P, P, P, i64, ci]
        lib.oracle_spgemm.restype = P
        lib.oracle_merge.argtypes = [ci, ci, i64, i64, P, P, P, P, i64, ci]
        lib.oracle_merge.restype = P
        lib.oracle_result_nnz.argtypes = [P]
        lib.oracle_result_nnz.restype = i64
        lib.oracle_result_has_mag.argtypes = [P]
        lib.oracle_result_has_mag.restype = ci
        lib.oracle_result_copy.argtypes = [P, P, P, P, P]
        lib.oracle_result_copy.restype = None
        lib.oracle_result_free.argtypes = [P]
        lib.oracle_result_free.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ci
        self.lib = lib
        self.path = path

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def _collect(self, handle, sr: int, nsel: int, t0: float) -> OracleResult:
        if not handle:
            raise ValueError("oracle rejected the arguments (semiring id or shape)")
        try:
            nnz = self.lib.oracle_result_nnz(handle)
            rowptr = np.empty(nsel + 1, dtype=np.int64)
            col = np.empty(nnz, dtype=np.int32)
            val = np.empty(nnz, dtype=OUT_DTYPE[sr])
            mag = np.empty(nnz, dtype=np.float64) if self.lib.oracle_result_has_mag(handle) else None
            if sr in (PLUS_TIMES_F32, PLUS_TIMES_F64) and mag is None:
                mag = np.zeros(nnz, dtype=np.float64)
            self.lib.oracle_result_copy(handle, _p(rowptr), _p(col), _p(val), _p(mag))
        finally:
            self.lib.oracle_result_free(handle)
        return OracleResult(rowptr, col, val, mag, time.perf_counter() - t0)

    def spgemm(self, sr: int, A, B, rows: Optional[np.ndarray] = None, nthreads: int = 0) -> OracleResult:
        """Rows `rows` (default: all) of A (x).(+) B.  A, B are synth.CSR with
        values of the semiring's input dtype."""
        av = np.ascontiguousarray(A.val, dtype=IN_DTYPE[sr])
        bv = np.ascontiguousarray(B.val, dtype=IN_DTYPE[sr])
        sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
        nsel = A.nrows if sel is None else len(sel)
        t0 = time.perf_counter()
        h = self.lib.oracle_spgemm(sr, A.nrows, A.ncols, _p(A.rowptr), _p(A.col), _p(av), B.nrows, B.ncols,
                                   _p(B.rowptr), _p(B.col), _p(bv), _p(sel), nsel, nthreads)
        return self._collect(h, sr, nsel, t0)

    def merge(self, sr: int, parts: Sequence, rows: Optional[np.ndarray] = None, nthreads: int = 0) -> OracleResult:
        """Rows of parts[0] (+) ... (+) parts[-1] (same shape)."""
        nparts = len(parts)
        nrows, ncols = parts[0].nrows, parts[0].ncols
        vals = [np.ascontiguousarray(p.val, dtype=IN_DTYPE[sr]) for p in parts]
        rp = (ctypes.c_void_p * nparts)(*[p.rowptr.ctypes.data for p in parts])
        cl = (ctypes.c_void_p * nparts)(*[p.col.ctypes.data for p in parts])
        vl = (ctypes.c_void_p * nparts)(*[v.ctypes.data for v in vals])
        sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
        nsel = nrows if sel is None else len(sel)
        t0 = time.perf_counter()
        h = self.lib.oracle_merge(sr, nparts, nrows, ncols, ctypes.cast(rp, ctypes.c_void_p),
                                  ctypes.cast(cl, ctypes.c_void_p), ctypes.cast(vl, ctypes.c_void_p), _p(sel), nsel,
                                  nthreads)
        return self._collect(h, sr, nsel, t0)


_default: Optional[Oracle] = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
