"""Column-major formats and the transposition identity, on the CPU.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``).

What it computes (paper, Section 4.1, Algorithm 1):
  * DCSC stores only the non-empty columns: their ids jc (ascending), the
    offsets cp of their entries (cp[nzc] = nnz), row ids and values.  CSC
    keeps a pointer for every column.  Decompression rebuilds the full
    pointer array, giving every empty column an empty segment:
    colptr[j] = number of entries in the columns before j = cp[#{i : jc[i] < j}].
    Compression keeps the columns whose segment is non-empty.
  * A matrix in CSC is the CSR of its transpose (same arrays), and
    C = A B equals (B^T A^T)^T, so a product of CSC operands is a product of
    CSR operands in swapped order whose CSR result is C in CSC.  Here the
    product itself is done the plain way: both operands are transposed to
    CSR by sorting their entries, the oracle multiplies A by B, and the CSR
    result is transposed back to CSC.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import IN_DTYPE, Oracle

# test-only planted mistakes (tests/test_oracle_mutants.py): 0 = none
MUTANT = 0


@dataclass
class Csc:
    nrows: int
    ncols: int
    colptr: np.ndarray
    row: np.ndarray
    val: np.ndarray


@dataclass
class Csr:
    nrows: int
    ncols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


def decompress(ncols: int, jc: np.ndarray, cp: np.ndarray) -> np.ndarray:
    """Full column pointers (ncols + 1) of a DCSC matrix."""
    jc = np.asarray(jc, dtype=np.int64)
    cp = np.asarray(cp, dtype=np.int64)
    side = "right" if MUTANT == 4 else "left"
    before = np.searchsorted(jc, np.arange(ncols + 1, dtype=np.int64), side=side)
    return cp[before]


def compress(colptr: np.ndarray):
    """(jc, cp) of the non-empty columns of a CSC pointer array."""
    colptr = np.asarray(colptr, dtype=np.int64)
    ncols = len(colptr) - 1
    keep = np.nonzero(colptr[1:] > colptr[:-1])[0]
    if MUTANT == 5 and len(keep):
        keep = keep[:-1]
    jc = keep.astype(np.int32)
    cp = np.append(colptr[keep], colptr[ncols]).astype(np.int64)
    return jc, cp


def _transpose(nrows: int, ncols: int, ptr: np.ndarray, idx: np.ndarray, val: np.ndarray):
    """Compressed arrays of the transpose: entries sorted by (idx, owner)."""
    owner = np.repeat(np.arange(nrows, dtype=np.int64), np.diff(ptr))
    order = np.lexsort((owner, idx))
    tptr = np.zeros(ncols + 1, dtype=np.int64)
    np.cumsum(np.bincount(idx, minlength=ncols), out=tptr[1:])
    return tptr, owner[order].astype(np.int32), val[order]


def csc_to_csr(A: Csc) -> Csr:
    rp, c, v = _transpose(A.ncols, A.nrows, A.colptr, A.row, A.val)
    return Csr(A.nrows, A.ncols, rp, c, v)


def csr_to_csc(A) -> Csc:
    cp, r, v = _transpose(A.nrows, A.ncols, np.asarray(A.rowptr), np.asarray(A.col), np.asarray(A.val))
    return Csc(A.nrows, A.ncols, cp, r, v)


def csc_spgemm(orc: Oracle, sr: int, A: Csc, B: Csc) -> Csc:
    """C = A (x).(+) B for CSC operands, C in CSC (values as the oracle gives
    them: float64 for float sums)."""
    if A.ncols != B.nrows:
        raise ValueError("A.ncols != B.nrows")
    Ar, Br = csc_to_csr(A), csc_to_csr(B)
    Ar.val = np.asarray(Ar.val, dtype=IN_DTYPE[sr])
    Br.val = np.asarray(Br.val, dtype=IN_DTYPE[sr])
    C = orc.spgemm(sr, Br, Ar) if MUTANT == 6 and A.nrows == B.ncols else orc.spgemm(sr, Ar, Br)
    return csr_to_csc(Csr(A.nrows, B.ncols, C.rowptr, C.col, C.val))
