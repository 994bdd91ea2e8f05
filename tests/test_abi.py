"""The C-ABI library loads and exports every function include/spgemm.h
declares; host-only calls (no device work) behave as documented.  No GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_]+)\s*\(", src)))


def _lib():
    import paper_2504_06408_amd as sg
    if not os.path.exists(sg.LIB_PATH):
        pytest.skip("HIP library not built")
    return sg, sg.lib()


def test_header_lists_the_binding_exports():
    import paper_2504_06408_amd as sg
    assert sorted(sg.EXPORTS) == _declared()


def test_every_declared_symbol_is_exported():
    _, L = _lib()
    for name in _declared():
        assert hasattr(L, name), f"{name} not exported"


def test_semiring_make_host_only():
    sg, L = _lib()
    s = sg.sg_semiring()
    for sid, vb in [(1, 8), (2, 4), (3, 8), (4, 1), (5, 4)]:
        assert L.sg_semiring_make(sid, 0, ctypes.byref(s)) == 0
        assert s.id == sid and s.value_bytes == vb and s.comp_min_terms == 64
    assert L.sg_semiring_make(0, 0, ctypes.byref(s)) == -3
    assert L.sg_semiring_make(6, 0, ctypes.byref(s)) == -3
    assert L.sg_semiring_make(2, 7, ctypes.byref(s)) == -3
    assert L.sg_semiring_make(2, 0, None) == -1


def test_status_strings():
    _, L = _lib()
    for code, name in [(0, b"SG_OK"), (-2, b"SG_ERR_SHAPE"), (-6, b"SG_ERR_UNSORTED"), (-7, b"SG_ERR_HIP")]:
        assert L.sg_status_string(code) == name


def test_null_handle_rejected():
    _, L = _lib()
    assert L.sg_handle_destroy(None) == -1
    assert L.sg_handle_check(None) == -1
    assert L.sg_handle_set_option(None, b"validate", b"1") == -1


def test_missing_library_fails_loudly(monkeypatch):
    import paper_2504_06408_amd as sg
    monkeypatch.setattr(sg, "_lib", None)
    monkeypatch.setattr(sg, "LIB_PATH", "/nonexistent/libsgspgemm.so")
    with pytest.raises(sg.SgError):
        sg.lib()
