"""Semiring sparse x sparse product C = A (x).(+) B and the semiring merge of
partial products on an AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libsgspgemm.so`` (C ABI in ``include/spgemm.h``):
it only marshals arguments.  Device memory comes from PyTorch (ROCm build);
every step of the computation runs in the library's HIP kernels.  Importing
this package does not need a GPU; creating a :class:`Handle` does, and any
call raises :class:`SgError` when the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgspgemm.so")

# semiring ids (include/spgemm.h)
PLUS_TIMES_I64, PLUS_TIMES_F32, PLUS_TIMES_F64, OR_AND_BOOL, MIN_PLUS_F32 = 1, 2, 3, 4, 5
SEMIRING_NAMES = {1: "plus_times_i64", 2: "plus_times_f32", 3: "plus_times_f64", 4: "or_and_bool",
                  5: "min_plus_f32"}
ACC_DEFAULT, ACC_COMPENSATED, ACC_PLAIN = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20  # SG_NOALLOC_SCRATCH_BYTES
NP_DTYPE = {1: np.int64, 2: np.float32, 3: np.float64, 4: np.uint8, 5: np.float32}

STATUS = {0: "SG_OK", -1: "SG_ERR_INVALID", -2: "SG_ERR_SHAPE", -3: "SG_ERR_SEMIRING", -4: "SG_ERR_NOMEM",
          -5: "SG_ERR_OVERFLOW", -6: "SG_ERR_UNSORTED", -7: "SG_ERR_HIP"}

# every function include/spgemm.h declares
EXPORTS = ("sg_semiring_make", "sg_handle_create", "sg_handle_destroy", "sg_handle_set_option",
           "sg_spgemm_symbolic", "sg_spgemm_numeric", "sg_spgemm_numeric_noalloc", "sg_spgemm_merge_symbolic",
           "sg_spgemm_merge_numeric",
           "sg_batch_plan", "sg_batch_execute", "sg_batch_results", "sg_plan_destroy", "sg_tune", "sg_tune_load",
           "sg_handle_check", "sg_handle_timings", "sg_handle_stats", "sg_status_string", "sg_last_error",
           "sg_dcsc_decompress", "sg_dcsc_compress", "sg_spgemm_csc_symbolic", "sg_spgemm_csc_numeric",
           "sg_power_run", "sg_power_result", "sg_power_destroy", "sg_waves_plan", "sg_waves_info", "sg_waves_run",
           "sg_waves_results", "sg_waves_destroy", "sg_semiring_define")
POWER_SELF_LOOPS, POWER_SQUARING, POWER_FIXPOINT = 1, 2, 4

PHASES = ("sym_analyze", "sym_bounds", "sym_small", "sym_hash", "sym_dense", "sym_scan", "num_analyze", "num_small",
          "num_hash", "num_dense", "sym_dense_bitmap", "num_dense_slab", "num_dense_tiles", "num_dense_ranges")
STATS = ("dense_rows", "slab_tasks", "tile_tasks", "range_tasks", "slab_entries", "tile_entries", "range_entries")


class SgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class sg_semiring(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int32), ("value_bytes", ctypes.c_int32), ("acc_flags", ctypes.c_uint32),
                ("comp_min_terms", ctypes.c_int32), ("comp_min_products", ctypes.c_int64)]


class sg_csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class sg_csc(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("row", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class sg_dcsc(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nzc", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("jc", ctypes.c_void_p), ("cp", ctypes.c_void_p), ("row", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class sg_semiring_def(ctypes.Structure):
    _fields_ = [("value_type", ctypes.c_char_p), ("add", ctypes.c_char_p), ("mul", ctypes.c_char_p),
                ("zero", ctypes.c_char_p), ("one", ctypes.c_char_p), ("flags", ctypes.c_uint32)]


SR_IDEMPOTENT = 1
USER_VALUE_DTYPES = {"float": np.float32, "double": np.float64, "int32_t": np.int32, "uint32_t": np.uint32,
                     "int64_t": np.int64, "uint64_t": np.uint64}

_lib = None


def lib():
    """The loaded C library; raises SgError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SgError(-7, f"{LIB_PATH} is not built (run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime with the same soname as the
        # system one; load it first so the library binds to that one copy
        # and the process has a single HIP runtime.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, ci = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
        SR, CSR = ctypes.POINTER(sg_semiring), ctypes.POINTER(sg_csr)
        sig = {
            "sg_semiring_make": ([ci, ctypes.c_uint32, SR], ci),
            "sg_handle_create": ([ci, ctypes.c_char_p, ctypes.POINTER(P)], ci),
            "sg_handle_destroy": ([P], ci),
            "sg_handle_set_option": ([P, ctypes.c_char_p, ctypes.c_char_p], ci),
            "sg_spgemm_symbolic": ([P, CSR, CSR, P, ctypes.POINTER(i64), P], ci),
            "sg_spgemm_numeric": ([P, SR, CSR, CSR, CSR, P], ci),
            "sg_spgemm_numeric_noalloc": ([P, SR, CSR, CSR, CSR, P], ci),
            "sg_spgemm_merge_symbolic": ([P, ci, CSR, P, ctypes.POINTER(i64), P], ci),
            "sg_spgemm_merge_numeric": ([P, SR, ci, CSR, CSR, P], ci),
            "sg_batch_plan": ([P, SR, ci, CSR, CSR, ci, ctypes.POINTER(i32), ctypes.c_size_t, ctypes.POINTER(P)], ci),
            "sg_batch_execute": ([P, P], ci),
            "sg_batch_results": ([P, CSR], ci),
            "sg_plan_destroy": ([P], ci),
            "sg_tune": ([P, SR, CSR, CSR, ctypes.c_char_p], ci),
            "sg_tune_load": ([P, SR, ctypes.c_char_p], ci),
            "sg_handle_check": ([P], ci),
            "sg_handle_timings": ([P, ctypes.POINTER(ctypes.c_double), ci], ci),
            "sg_handle_stats": ([P, ctypes.POINTER(i64), ci], ci),
            "sg_dcsc_decompress": ([P, ctypes.POINTER(sg_dcsc), P, P], ci),
            "sg_dcsc_compress": ([P, i64, P, P, P, ctypes.POINTER(i64), P], ci),
            "sg_spgemm_csc_symbolic": ([P, ctypes.POINTER(sg_csc), ctypes.POINTER(sg_csc), P, ctypes.POINTER(i64), P],
                                       ci),
            "sg_spgemm_csc_numeric": ([P, SR, ctypes.POINTER(sg_csc), ctypes.POINTER(sg_csc), ctypes.POINTER(sg_csc),
                                       P], ci),
            "sg_power_run": ([P, SR, CSR, i32, ctypes.c_uint32, P, ctypes.POINTER(P)], ci),
            "sg_power_result": ([P, CSR, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], ci),
            "sg_power_destroy": ([P], ci),
            "sg_waves_plan": ([P, SR, ci, CSR, CSR, ci, ctypes.POINTER(i32), ctypes.c_size_t, ctypes.POINTER(P)], ci),
            "sg_waves_info": ([P, ctypes.POINTER(ci), ctypes.POINTER(i64), ctypes.POINTER(i32),
                               ctypes.POINTER(ctypes.c_size_t)], ci),
            "sg_waves_run": ([P, ci, P], ci),
            "sg_waves_results": ([P, CSR], ci),
            "sg_waves_destroy": ([P], ci),
            "sg_semiring_define": ([P, ctypes.POINTER(sg_semiring_def), SR], ci),
            "sg_status_string": ([ci], ctypes.c_char_p),
            "sg_last_error": ([P], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def semiring(sid: int, acc: int = ACC_DEFAULT, comp_min_terms: int = 64, comp_min_products: int = 0) -> sg_semiring:
    s = sg_semiring()
    rc = lib().sg_semiring_make(sid, acc, ctypes.byref(s))
    if rc != 0:
        raise SgError(rc, f"bad semiring {sid} / accumulation {acc}")
    s.comp_min_terms = comp_min_terms
    s.comp_min_products = comp_min_products
    return s


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class DeviceCSR:
    """CSR matrix in device memory (torch tensors): rowptr int64[nrows+1],
    col int32[nnz], val[nnz] of the semiring's value type."""

    def __init__(self, nrows: int, ncols: int, rowptr, col, val=None):
        self.nrows, self.ncols = int(nrows), int(ncols)
        self.rowptr, self.col, self.val = rowptr, col, val
        self.nnz = int(col.numel())

    @classmethod
    def from_numpy(cls, nrows, ncols, rowptr, col, val=None, device="cuda"):
        torch = _torch()
        rp = torch.from_numpy(np.ascontiguousarray(rowptr, dtype=np.int64)).to(device)
        cl = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device)
        vl = None if val is None else torch.from_numpy(np.ascontiguousarray(val)).to(device)
        return cls(nrows, ncols, rp, cl, vl)

    @classmethod
    def from_host(cls, M, device="cuda"):
        """From any object with nrows, ncols, rowptr, col, val (numpy)."""
        return cls.from_numpy(M.nrows, M.ncols, M.rowptr, M.col, M.val, device)

    def desc(self) -> sg_csr:
        d = sg_csr()
        d.nrows, d.ncols, d.nnz = self.nrows, self.ncols, self.nnz
        d.rowptr = self.rowptr.data_ptr()
        d.col = self.col.data_ptr() if self.nnz else 0
        d.val = self.val.data_ptr() if (self.val is not None and self.nnz) else 0
        return d

    def to_numpy(self):
        rp = self.rowptr.cpu().numpy()
        cl = self.col.cpu().numpy()
        vl = None if self.val is None else self.val.cpu().numpy()
        return rp, cl, vl


class DeviceCSC:
    """CSC matrix in device memory: colptr int64[ncols+1], row int32[nnz]
    (ascending within a column), val[nnz]."""

    def __init__(self, nrows: int, ncols: int, colptr, row, val=None):
        self.nrows, self.ncols = int(nrows), int(ncols)
        self.colptr, self.row, self.val = colptr, row, val
        self.nnz = int(row.numel())

    def desc(self) -> sg_csc:
        d = sg_csc()
        d.nrows, d.ncols, d.nnz = self.nrows, self.ncols, self.nnz
        d.colptr = self.colptr.data_ptr()
        d.row = self.row.data_ptr() if self.nnz else 0
        d.val = self.val.data_ptr() if (self.val is not None and self.nnz) else 0
        return d

    def to_numpy(self):
        return self.colptr.cpu().numpy(), self.row.cpu().numpy(), (None if self.val is None else self.val.cpu().numpy())


def _torch_dtype(sid: int):
    torch = _torch()
    if sid in (1, 2, 3, 4, 5):
        return {1: torch.int64, 2: torch.float32, 3: torch.float64, 4: torch.uint8, 5: torch.float32}[sid]
    return {np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64, np.dtype(np.int32): torch.int32,
            np.dtype(np.uint32): torch.uint32, np.dtype(np.int64): torch.int64,
            np.dtype(np.uint64): torch.uint64}[np.dtype(NP_DTYPE[sid])]


class Plan:
    """A recorded batched execution (sg_batch_plan)."""

    def __init__(self, handle: "Handle", ptr, nprob: int, ngroups: int, keep):
        self.handle, self.ptr, self.nprob, self.ngroups, self._keep = handle, ptr, nprob, ngroups, keep

    def execute(self, stream=None):
        self.handle._rc(lib().sg_batch_execute(self.ptr, _stream_ptr(stream)))

    def results(self) -> List[sg_csr]:
        n = self.nprob + self.ngroups
        arr = (sg_csr * n)()
        self.handle._rc(lib().sg_batch_results(self.ptr, arr))
        return list(arr)

    def results_numpy(self):
        """Host copies (rowptr, col, val) of every result: the nprob products,
        then the ngroups merges."""
        sid = self._keep[2].id
        out = []
        for r in self.results():
            rp = _to_numpy(r.rowptr, r.nrows + 1, np.int64)
            cl = _to_numpy(r.col, r.nnz, np.int32)
            vl = _to_numpy(r.val, r.nnz, NP_DTYPE[sid])
            out.append((rp, cl, vl))
        return out

    def destroy(self):
        if self.ptr:
            lib().sg_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Waves:
    """Memory-budgeted waves of a batch (sg_waves_*)."""

    def __init__(self, handle: "Handle", ptr, nprob: int, group_offsets, keep):
        self.handle, self.ptr, self.nprob, self._keep = handle, ptr, nprob, keep
        self.group_offsets = list(group_offsets)
        n = ctypes.c_int()
        handle._rc(lib().sg_waves_info(ptr, ctypes.byref(n), None, None, None))
        self.count = int(n.value)
        nnz = (ctypes.c_int64 * nprob)()
        wg = (ctypes.c_int32 * (self.count + 1))()
        wb = (ctypes.c_size_t * self.count)()
        handle._rc(lib().sg_waves_info(ptr, ctypes.byref(n), nnz, wg, wb))
        self.product_nnz = list(nnz)
        self.wave_groups = list(wg)
        self.wave_bytes = list(wb)
        self.current = -1

    def run(self, wave: int, stream=None):
        self.handle._rc(lib().sg_waves_run(self.ptr, wave, _stream_ptr(stream)))
        self.current = wave

    def results(self) -> List[sg_csr]:
        """The current wave's products, then its merges (views into its pool)."""
        g0, g1 = self.wave_groups[self.current], self.wave_groups[self.current + 1]
        n = (self.group_offsets[g1] - self.group_offsets[g0]) + (g1 - g0)
        arr = (sg_csr * n)()
        self.handle._rc(lib().sg_waves_results(self.ptr, arr))
        return list(arr)

    def destroy(self):
        if self.ptr:
            lib().sg_waves_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Handle:
    def __init__(self, device: int = 0, tuning: Optional[str] = None):
        p = ctypes.c_void_p()
        rc = lib().sg_handle_create(device, tuning.encode() if tuning else None, ctypes.byref(p))
        if rc != 0:
            raise SgError(rc, "sg_handle_create failed")
        self.ptr = p
        self.device = device

    def close(self):
        if self.ptr:
            lib().sg_handle_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc: int):
        if rc != 0:
            msg = lib().sg_last_error(self.ptr)
            raise SgError(rc, msg.decode() if msg else "")

    def set_option(self, name: str, value) -> None:
        self._rc(lib().sg_handle_set_option(self.ptr, name.encode(), str(value).encode()))

    def check(self) -> None:
        self._rc(lib().sg_handle_check(self.ptr))

    def timings(self) -> dict:
        """Per-phase device milliseconds of the last symbolic and numeric
        calls (needs set_option("timing", 1))."""
        arr = (ctypes.c_double * len(PHASES))()
        self._rc(lib().sg_handle_timings(self.ptr, arr, len(PHASES)))
        return dict(zip(PHASES, list(arr)))

    def stats(self) -> dict:
        """Dense-row task split of the last numeric call (waits for the device)."""
        arr = (ctypes.c_int64 * len(STATS))()
        self._rc(lib().sg_handle_stats(self.ptr, arr, len(STATS)))
        return dict(zip(STATS, list(arr)))

    # ---- product -------------------------------------------------------------
    def symbolic(self, A: DeviceCSR, B: DeviceCSR, stream=None):
        torch = _torch()
        rowptr = torch.empty(A.nrows + 1, dtype=torch.int64, device=A.rowptr.device)
        nnz = ctypes.c_int64()
        a, b = A.desc(), B.desc()
        self._rc(lib().sg_spgemm_symbolic(self.ptr, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.c_void_p(rowptr.data_ptr()), ctypes.byref(nnz), _stream_ptr(stream)))
        return rowptr, int(nnz.value)

    def numeric(self, sr: sg_semiring, A: DeviceCSR, B: DeviceCSR, C: DeviceCSR, stream=None) -> None:
        a, b, c = A.desc(), B.desc(), C.desc()
        self._rc(lib().sg_spgemm_numeric(self.ptr, ctypes.byref(sr), ctypes.byref(a), ctypes.byref(b),
                                         ctypes.byref(c), _stream_ptr(stream)))

    def numeric_noalloc(self, sr: sg_semiring, A: DeviceCSR, B: DeviceCSR, C: DeviceCSR, stream=None) -> None:
        """Pass 2 with all scratch taken from the library's fixed device array
        (no device allocation; SG_ERR_NOMEM beyond NOALLOC_SCRATCH_BYTES)."""
        a, b, c = A.desc(), B.desc(), C.desc()
        self._rc(lib().sg_spgemm_numeric_noalloc(self.ptr, ctypes.byref(sr), ctypes.byref(a), ctypes.byref(b),
                                                 ctypes.byref(c), _stream_ptr(stream)))

    def spgemm(self, sr, A: DeviceCSR, B: DeviceCSR, stream=None) -> DeviceCSR:
        """C = A (x).(+) B (both passes); sr: semiring id or descriptor."""
        torch = _torch()
        if isinstance(sr, int):
            sr = semiring(sr)
        rowptr, nnz = self.symbolic(A, B, stream)
        dev = A.rowptr.device
        C = DeviceCSR(A.nrows, B.ncols, rowptr, torch.empty(nnz, dtype=torch.int32, device=dev),
                      torch.empty(nnz, dtype=_torch_dtype(sr.id), device=dev))
        self.numeric(sr, A, B, C, stream)
        return C

    # ---- merge ----------------------------------------------------------------
    def merge_symbolic(self, parts: Sequence[DeviceCSR], stream=None):
        torch = _torch()
        arr = (sg_csr * len(parts))(*[p.desc() for p in parts])
        rowptr = torch.empty(parts[0].nrows + 1, dtype=torch.int64, device=parts[0].rowptr.device)
        nnz = ctypes.c_int64()
        self._rc(lib().sg_spgemm_merge_symbolic(self.ptr, len(parts), arr, ctypes.c_void_p(rowptr.data_ptr()),
                                                ctypes.byref(nnz), _stream_ptr(stream)))
        return rowptr, int(nnz.value)

    def merge_numeric(self, sr: sg_semiring, parts: Sequence[DeviceCSR], C: DeviceCSR, stream=None) -> None:
        arr = (sg_csr * len(parts))(*[p.desc() for p in parts])
        c = C.desc()
        self._rc(lib().sg_spgemm_merge_numeric(self.ptr, ctypes.byref(sr), len(parts), arr, ctypes.byref(c),
                                               _stream_ptr(stream)))

    def merge(self, sr, parts: Sequence[DeviceCSR], stream=None) -> DeviceCSR:
        torch = _torch()
        if isinstance(sr, int):
            sr = semiring(sr)
        rowptr, nnz = self.merge_symbolic(parts, stream)
        dev = parts[0].rowptr.device
        C = DeviceCSR(parts[0].nrows, parts[0].ncols, rowptr, torch.empty(nnz, dtype=torch.int32, device=dev),
                      torch.empty(nnz, dtype=_torch_dtype(sr.id), device=dev))
        self.merge_numeric(sr, parts, C, stream)
        return C

    # ---- batched ----------------------------------------------------------------
    def batch_plan(self, sr, As: Sequence[DeviceCSR], Bs: Sequence[DeviceCSR], group_offsets=None,
                   pool_bytes: int = 0) -> Plan:
        if isinstance(sr, int):
            sr = semiring(sr)
        n = len(As)
        a = (sg_csr * n)(*[x.desc() for x in As])
        b = (sg_csr * n)(*[x.desc() for x in Bs])
        ng = 0 if group_offsets is None else len(group_offsets) - 1
        go = None if group_offsets is None else (ctypes.c_int32 * len(group_offsets))(*group_offsets)
        p = ctypes.c_void_p()
        self._rc(lib().sg_batch_plan(self.ptr, ctypes.byref(sr), n, a, b, ng, go, pool_bytes, ctypes.byref(p)))
        return Plan(self, p, n, ng, (As, Bs, sr))

    def waves(self, sr, As: Sequence[DeviceCSR], Bs: Sequence[DeviceCSR], group_offsets, budget_bytes: int) -> Waves:
        if isinstance(sr, int):
            sr = semiring(sr)
        n = len(As)
        a = (sg_csr * n)(*[x.desc() for x in As])
        b = (sg_csr * n)(*[x.desc() for x in Bs])
        go = (ctypes.c_int32 * len(group_offsets))(*group_offsets)
        p = ctypes.c_void_p()
        self._rc(lib().sg_waves_plan(self.ptr, ctypes.byref(sr), n, a, b, len(group_offsets) - 1, go,
                                     int(budget_bytes), ctypes.byref(p)))
        return Waves(self, p, n, group_offsets, (As, Bs, sr))

    def tune(self, sr, A: DeviceCSR, B: DeviceCSR, out_json: str) -> None:
        if isinstance(sr, int):
            sr = semiring(sr)
        a, b = A.desc(), B.desc()
        self._rc(lib().sg_tune(self.ptr, ctypes.byref(sr), ctypes.byref(a), ctypes.byref(b), out_json.encode()))

    # ---- column-major operands -----------------------------------------------------
    def dcsc_decompress(self, nrows: int, ncols: int, jc, cp, row, val=None, stream=None) -> "DeviceCSC":
        """CSC view of a DCSC matrix (device tensors jc int32[nzc], cp
        int64[nzc+1], row, val): new column pointers, the same row and value
        tensors."""
        torch = _torch()
        colptr = torch.empty(ncols + 1, dtype=torch.int64, device=cp.device)
        d = sg_dcsc()
        d.nrows, d.ncols, d.nzc, d.nnz = nrows, ncols, int(jc.numel()), int(row.numel())
        d.jc = jc.data_ptr() if jc.numel() else 0
        d.cp = cp.data_ptr()
        d.row = row.data_ptr() if row.numel() else 0
        d.val = val.data_ptr() if (val is not None and val.numel()) else 0
        self._rc(lib().sg_dcsc_decompress(self.ptr, ctypes.byref(d), ctypes.c_void_p(colptr.data_ptr()),
                                          _stream_ptr(stream)))
        return DeviceCSC(nrows, ncols, colptr, row, val)

    def dcsc_compress(self, colptr, stream=None):
        """(jc, cp) device tensors of the non-empty columns of colptr."""
        torch = _torch()
        ncols = int(colptr.numel()) - 1
        jc = torch.empty(max(ncols, 1), dtype=torch.int32, device=colptr.device)
        cp = torch.empty(ncols + 1, dtype=torch.int64, device=colptr.device)
        nzc = ctypes.c_int64()
        self._rc(lib().sg_dcsc_compress(self.ptr, ncols, ctypes.c_void_p(colptr.data_ptr()),
                                        ctypes.c_void_p(jc.data_ptr()), ctypes.c_void_p(cp.data_ptr()),
                                        ctypes.byref(nzc), _stream_ptr(stream)))
        k = int(nzc.value)
        return jc[:k], cp[:k + 1]

    def spgemm_csc(self, sr, A: "DeviceCSC", B: "DeviceCSC", stream=None) -> "DeviceCSC":
        """C = A (x).(+) B for CSC operands, C in CSC (both passes)."""
        torch = _torch()
        if isinstance(sr, int):
            sr = semiring(sr)
        a, b = A.desc(), B.desc()
        colptr = torch.empty(B.ncols + 1, dtype=torch.int64, device=A.colptr.device)
        nnz = ctypes.c_int64()
        self._rc(lib().sg_spgemm_csc_symbolic(self.ptr, ctypes.byref(a), ctypes.byref(b),
                                              ctypes.c_void_p(colptr.data_ptr()), ctypes.byref(nnz),
                                              _stream_ptr(stream)))
        dev = A.colptr.device
        C = DeviceCSC(A.nrows, B.ncols, colptr, torch.empty(nnz.value, dtype=torch.int32, device=dev),
                      torch.empty(nnz.value, dtype=_torch_dtype(sr.id), device=dev))
        c = C.desc()
        self._rc(lib().sg_spgemm_csc_numeric(self.ptr, ctypes.byref(sr), ctypes.byref(a), ctypes.byref(b),
                                             ctypes.byref(c), _stream_ptr(stream)))
        return C

    # ---- powers -------------------------------------------------------------------
    def power(self, sr, W: DeviceCSR, max_hops: int, self_loops: bool = False, squaring: bool = False,
              fixpoint: bool = False, stream=None):
        """(D, hops, products, converged): D = W'^hops (W' = I (+) W with
        self loops) as a DeviceCSR of fresh tensors (sg_power_run)."""
        torch = _torch()
        if isinstance(sr, int):
            sr = semiring(sr)
        flags = (POWER_SELF_LOOPS if self_loops else 0) | (POWER_SQUARING if squaring else 0) | \
                (POWER_FIXPOINT if fixpoint else 0)
        w = W.desc()
        p = ctypes.c_void_p()
        self._rc(lib().sg_power_run(self.ptr, ctypes.byref(sr), ctypes.byref(w), int(max_hops), flags,
                                    _stream_ptr(stream), ctypes.byref(p)))
        try:
            d = sg_csr()
            hops, prods, conv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            self._rc(lib().sg_power_result(p, ctypes.byref(d), ctypes.byref(hops), ctypes.byref(prods),
                                           ctypes.byref(conv)))
            dev = W.rowptr.device
            D = DeviceCSR(d.nrows, d.ncols, _wrap(d.rowptr, d.nrows + 1, np.int64, dev).clone(),
                          _wrap(d.col, d.nnz, np.int32, dev).clone(),
                          _wrap(d.val, d.nnz, NP_DTYPE[sr.id], dev).clone())
            torch.cuda.synchronize(dev)
        finally:
            lib().sg_power_destroy(p)
        return D, int(hops.value), int(prods.value), bool(conv.value)

    def define_semiring(self, value_type: str, add: str, mul: str, zero: str, one: str,
                        idempotent: bool = False) -> sg_semiring:
        """A semiring defined at run time (sg_semiring_define): add and mul
        are device expressions in a and b, zero and one expressions."""
        d = sg_semiring_def(value_type.encode(), add.encode(), mul.encode(), zero.encode(), one.encode(),
                            SR_IDEMPOTENT if idempotent else 0)
        s = sg_semiring()
        self._rc(lib().sg_semiring_define(self.ptr, ctypes.byref(d), ctypes.byref(s)))
        NP_DTYPE[s.id] = USER_VALUE_DTYPES[value_type]
        return s

    def tune_load(self, sr, path: str) -> None:
        """Adopt a tuning table; sr (id or descriptor, or None) must match the
        table's semiring."""
        if isinstance(sr, int):
            sr = semiring(sr)
        self._rc(lib().sg_tune_load(self.ptr, None if sr is None else ctypes.byref(sr), path.encode()))


class _DevArray:
    """A raw device range exposed through __cuda_array_interface__ so that
    torch can wrap it without a copy."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 3}


_TYPESTR = {np.dtype(np.int64): "<i8", np.dtype(np.int32): "<i4", np.dtype(np.float32): "<f4",
            np.dtype(np.float64): "<f8", np.dtype(np.uint8): "|u1"}


def _wrap(ptr, n: int, dtype, device="cuda"):
    torch = _torch()
    if n == 0 or not ptr:
        return torch.empty(0, dtype={np.dtype(np.int64): torch.int64, np.dtype(np.int32): torch.int32,
                                     np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64,
                                     np.dtype(np.uint8): torch.uint8}[np.dtype(dtype)], device=device)
    return torch.as_tensor(_DevArray(int(ptr), int(n), _TYPESTR[np.dtype(dtype)]), device=device)


def _to_numpy(ptr, n: int, dtype) -> np.ndarray:
    """Host copy of n elements at device address ptr."""
    if n == 0 or not ptr:
        return np.empty(0, dtype=dtype)
    return _wrap(ptr, n, dtype).cpu().numpy()


def view_results(res: sg_csr, sid: int, device="cuda") -> DeviceCSR:
    """Wrap a result descriptor returned by Plan.results() as torch tensors
    (views of the plan's pool, no copy; valid until the plan is executed
    again or destroyed)."""
    return DeviceCSR(res.nrows, res.ncols, _wrap(res.rowptr, res.nrows + 1, np.int64, device),
                     _wrap(res.col, res.nnz, np.int32, device), _wrap(res.val, res.nnz, NP_DTYPE[sid], device))
