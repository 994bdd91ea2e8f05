"""Helpers for the GPU parity tests: run the library through its C ABI (the
ctypes binding) and compare with the CPU oracle."""
from __future__ import annotations

import numpy as np

import oracle
import synth
from helpers import (BOOL, F32, F64, I64, MINPLUS, assert_close_gated, assert_exact, assert_same_pattern,
                     rel_error_stats)

TOL = {F64: 1e-12, F32: 1e-5}


def to_dev(M):
    import paper_2504_06408_amd as sg
    return sg.DeviceCSR.from_host(M, "cuda")


def gpu_product(h, sr: int, A, B, acc: int = 0):
    import torch
    import paper_2504_06408_amd as sg
    dA, dB = to_dev(A), (to_dev(B) if B is not A else None)
    dB = dA if dB is None else dB
    C = h.spgemm(sg.semiring(sr, acc), dA, dB)
    torch.cuda.synchronize()
    h.check()
    return C


def rows_of(C, rows):
    """Host copy of selected rows of a DeviceCSR: (rowptr, col, val)."""
    import torch
    rp = C.rowptr.cpu().numpy()
    rows = np.asarray(rows, dtype=np.int64)
    lens = rp[rows + 1] - rp[rows]
    out_rp = np.zeros(len(rows) + 1, np.int64)
    np.cumsum(lens, out=out_rp[1:])
    if len(rows) == 0 or out_rp[-1] == 0:
        return out_rp, np.zeros(0, np.int32), np.zeros(0, C.val.cpu().numpy().dtype if C.nnz else np.float32)
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    ti = torch.from_numpy(idx).to(C.col.device)
    return out_rp, C.col[ti].cpu().numpy(), C.val[ti].cpu().numpy()


def compare(sr: int, got_rp, got_col, got_val, ref, what: str = ""):
    """Pattern exact; values bit-exact for int64/bool/(min,+), within the
    gated relative tolerance for float sums.  Returns (max, median) plain
    relative error for float sums, else None."""
    assert_same_pattern(got_rp, got_col, ref.rowptr, ref.col, what)
    if sr in (I64, BOOL, MINPLUS):
        assert_exact(got_val, ref.val, what)
        return None
    assert_close_gated(got_val, ref.val, ref.mag, TOL[sr], what)
    return rel_error_stats(got_val, ref.val)


def check_product(h, sr: int, A, B, acc: int = 0, rows=None, what: str = ""):
    C = gpu_product(h, sr, A, B, acc)
    if rows is None:
        rp, cl, vl = C.to_numpy()
        ref = oracle.get().spgemm(sr, A, B)
    else:
        rp, cl, vl = rows_of(C, rows)
        ref = oracle.get().spgemm(sr, A, B, rows=np.asarray(rows, np.int64))
    return compare(sr, rp, cl, vl, ref, what), C


def hcat(mats):
    """Column concatenation [M_1 .. M_n] of equal-height CSRs."""
    n = mats[0].nrows
    rows = []
    off = 0
    for M in mats:
        rows.append((M, off))
        off += M.ncols
    rowptr = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for r in range(n):
        for M, o in rows:
            s, e = M.rowptr[r], M.rowptr[r + 1]
            cols.append(np.asarray(M.col[s:e], np.int64) + o)
            vals.append(np.asarray(M.val[s:e]))
        rowptr[r + 1] = rowptr[r] + sum(M.rowptr[r + 1] - M.rowptr[r] for M, _ in rows)
    return synth.CSR(n, off, rowptr, np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def vcat(mats):
    """Row concatenation of equal-width CSRs."""
    rowptr = [np.zeros(1, np.int64)]
    base = 0
    for M in mats:
        rowptr.append(np.asarray(M.rowptr[1:], np.int64) + base)
        base += int(M.rowptr[-1])
    return synth.CSR(sum(M.nrows for M in mats), mats[0].ncols, np.concatenate(rowptr),
                     np.concatenate([np.asarray(M.col) for M in mats]),
                     np.concatenate([np.asarray(M.val) for M in mats]))
