"""The C-ABI library loads and exports every declared entry point (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("wtd.h", "wtd_debug.h"))
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wtd_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("wtd_apply_liouville", "wtd_apply_liouville_bwd", "wtd_davidson", "wtd_create",
              "wtd_destroy", "wtd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2309_03513_amd import load_library
    lib = load_library()
    for n in _declared():
        assert hasattr(lib, n), n


def test_argument_errors_without_device():
    from paper_2309_03513_amd import load_library
    from paper_2309_03513_amd.wtd import _System
    lib = load_library()
    h = ctypes.c_void_p()
    assert lib.wtd_create(None, 4, None, ctypes.byref(h)) == -1
    assert b"null" in lib.wtd_last_error()
    s = _System()
    assert lib.wtd_create(ctypes.byref(s), 4, None, ctypes.byref(h)) == -1   # null arrays
    assert h.value is None
    assert lib.wtd_apply_liouville(None, 1, None, None) == -1
    assert lib.wtd_destroy(None) == 0
    sz = ctypes.c_size_t()
    assert lib.wtd_workspace_bytes(None, ctypes.byref(sz)) == -1
