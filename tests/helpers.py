"""Test-side helpers: input recipes per semiring, a dense brute-force product
written directly from the semiring definition (paper, Section 2.2), and
comparison utilities.  Shared by the oracle pins and the GPU parity tests; it
contains no code of either implementation under test."""
from __future__ import annotations

import numpy as np

import synth

I64, F32, F64, BOOL, MINPLUS = 1, 2, 3, 4, 5
ALL = (I64, F32, F64, BOOL, MINPLUS)
EXACT = (I64, BOOL, MINPLUS)
NAME = {I64: "plus_times_i64", F32: "plus_times_f32", F64: "plus_times_f64", BOOL: "or_and_bool",
        MINPLUS: "min_plus_f32"}
IN_DTYPE = {I64: np.int64, F32: np.float32, F64: np.float64, BOOL: np.uint8, MINPLUS: np.float32}


def rand_values(sr: int, n: int, seed: int, style: str = "wide") -> np.ndarray:
    """Values for semiring sr.  style 'wide' exercises signs, wrap-around and
    explicit false entries; 'positive' avoids cancellation; 'int' keeps
    (min,+) weights integral so every sum is exact."""
    if sr == I64:
        if style == "wide":
            return synth.values(synth.VAL_I64_UNIFORM, n, -(2 ** 40), 2 ** 40, seed)
        return synth.values(synth.VAL_I64_UNIFORM, n, 1, 9, seed)
    if sr == F32:
        if style == "wide":
            return synth.values(synth.VAL_F32_NORMAL, n, 0, 1, seed)
        return synth.values(synth.VAL_F32_UNIFORM, n, 0.5, 2.0, seed)
    if sr == F64:
        if style == "wide":
            return synth.values(synth.VAL_F64_UNIFORM, n, -1.0, 1.0, seed)
        return synth.values(synth.VAL_F64_UNIFORM, n, 0.5, 2.0, seed)
    if sr == BOOL:
        if style == "wide":
            return synth.values(synth.VAL_BERNOULLI, n, 0.7, 0, seed)
        return synth.values(synth.VAL_ONES, n, 0, 0, seed)
    if sr == MINPLUS:
        if style == "wide":
            return synth.values(synth.VAL_F32_UNIFORM, n, -50.0, 100.0, seed)
        if style == "int":
            return synth.values(synth.VAL_I64_UNIFORM, n, 1, 20, seed).astype(np.float32)
        return synth.values(synth.VAL_F32_UNIFORM, n, 1.0, 100.0, seed)
    raise ValueError(sr)


def with_vals(A: synth.CSR, sr: int, seed: int, style: str = "wide") -> synth.CSR:
    return A.with_values(rand_values(sr, A.nnz, seed, style))


def one_value(sr: int):
    """The semiring's multiplicative identity."""
    return {I64: 1, F32: 1.0, F64: 1.0, BOOL: 1, MINPLUS: 0.0}[sr]


def identity(n: int, sr: int) -> synth.CSR:
    return synth.identity(n, IN_DTYPE[sr], one_value(sr))


# ---- dense brute force -------------------------------------------------------

def _mul(sr, a, b):
    if sr == I64:
        return a.astype(np.uint64) * b.astype(np.uint64)
    if sr == F32:
        return a.astype(np.float64) * b.astype(np.float64)
    if sr == F64:
        return a * b
    if sr == BOOL:
        return ((a != 0) & (b != 0)).astype(np.uint8)
    if sr == MINPLUS:
        return (a.astype(np.float32) + b.astype(np.float32)).astype(np.float32)
    raise ValueError(sr)


def _add(sr, x, y):
    if sr in (I64, F32, F64):
        return x + y
    if sr == BOOL:
        return ((x != 0) | (y != 0)).astype(np.uint8)
    if sr == MINPLUS:
        return np.where(y < x, y, x)
    raise ValueError(sr)


ACC_DTYPE = {I64: np.uint64, F32: np.float64, F64: np.float64, BOOL: np.uint8, MINPLUS: np.float32}


def brute(sr: int, A: synth.CSR, B: synth.CSR):
    """Dense C = A (x).(+) B with the ascending-k order; returns
    (values, present, magnitude sum)."""
    assert A.ncols == B.nrows
    Ad, Ap = A.to_dense()
    Bd, Bp = B.to_dense()
    C = np.zeros((A.nrows, B.ncols), dtype=ACC_DTYPE[sr])
    P = np.zeros((A.nrows, B.ncols), dtype=bool)
    M = np.zeros((A.nrows, B.ncols), dtype=np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        for k in range(A.ncols):
            mask = Ap[:, k][:, None] & Bp[k, :][None, :]
            if not mask.any():
                continue
            v = _mul(sr, np.broadcast_to(Ad[:, k][:, None], mask.shape), np.broadcast_to(Bd[k, :][None, :], mask.shape))
            new = mask & ~P
            upd = mask & P
            C[new] = v[new]
            C[upd] = _add(sr, C[upd], v[upd])
            P |= mask
            if sr in (F32, F64):
                M[mask] += np.abs(v[mask])
    if sr == I64:
        C = C.view(np.int64)
    return C, P, M


def brute_merge(sr: int, parts):
    C = np.zeros((parts[0].nrows, parts[0].ncols), dtype=ACC_DTYPE[sr])
    P = np.zeros(C.shape, dtype=bool)
    for part in parts:
        d, p = part.to_dense()
        if sr == I64:
            d = d.astype(np.int64).view(np.uint64)
        elif sr == F32:
            d = d.astype(np.float64)
        elif sr == BOOL:
            d = (d != 0).astype(np.uint8)
        new = p & ~P
        upd = p & P
        C[new] = d[new]
        with np.errstate(over="ignore"):
            C[upd] = _add(sr, C[upd], d[upd])
        P |= p
    if sr == I64:
        C = C.view(np.int64)
    return C, P


def dense_to_rows(C, P):
    rowptr = np.zeros(C.shape[0] + 1, dtype=np.int64)
    np.cumsum(P.sum(axis=1), out=rowptr[1:])
    r, c = np.nonzero(P)
    return rowptr, c.astype(np.int32), C[r, c]


# ---- comparisons ---------------------------------------------------------------

def bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view({1: np.uint8, 4: np.uint32, 8: np.uint64}[a.dtype.itemsize])


def assert_same_pattern(rowptr_a, col_a, rowptr_b, col_b, what=""):
    rowptr_a = np.asarray(rowptr_a, dtype=np.int64)
    rowptr_b = np.asarray(rowptr_b, dtype=np.int64)
    assert len(rowptr_a) == len(rowptr_b), f"{what}: row count {len(rowptr_a)} vs {len(rowptr_b)}"
    if not np.array_equal(rowptr_a - rowptr_a[0], rowptr_b - rowptr_b[0]):
        bad = np.nonzero(np.diff(rowptr_a) != np.diff(rowptr_b))[0][:5]
        raise AssertionError(f"{what}: row lengths differ at rows {bad}: "
                             f"{np.diff(rowptr_a)[bad]} vs {np.diff(rowptr_b)[bad]}")
    if not np.array_equal(col_a, col_b):
        bad = np.nonzero(np.asarray(col_a) != np.asarray(col_b))[0][:5]
        raise AssertionError(f"{what}: column ids differ at entries {bad}")


def assert_exact(a, b, what=""):
    """Bit-exact equality, except that +0 and -0 count as equal."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, f"{what}: shape {a.shape} vs {b.shape}"
    if a.dtype.kind == "f":
        same = (bits(a) == bits(b)) | ((a == 0) & (b == 0))
    else:
        same = bits(a) == bits(b)
    if not same.all():
        bad = np.nonzero(~same)[0][:5]
        raise AssertionError(f"{what}: {int((~same).sum())} values differ, e.g. at {bad}: {a[bad]} vs {b[bad]}")


def assert_close_gated(got, ref, mag, tol, what=""):
    """|got - ref| <= tol * max(|ref|, sum|products|) per entry (the
    condition-aware tolerance for float sums under cancellation)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), np.asarray(mag, dtype=np.float64))
    err = np.abs(got - ref)
    ok = err <= tol * scale
    if not ok.all():
        bad = np.nonzero(~ok)[0][:5]
        raise AssertionError(f"{what}: {int((~ok).sum())} entries beyond tol {tol}; e.g. {got[bad]} vs {ref[bad]} "
                             f"(scale {scale[bad]})")


def rel_error_stats(got, ref):
    """Plain per-entry relative error over entries with ref != 0:
    (max, median)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nz = ref != 0
    if not nz.any():
        return 0.0, 0.0
    r = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    return float(r.max()), float(np.median(r))
