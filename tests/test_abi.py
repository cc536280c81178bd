"""The C-ABI library builds, loads without a GPU and exports every symbol
that include/caps.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "caps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(caps_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("caps_build", "caps_search", "caps_search_probes", "caps_free", "caps_last_error",
              "caps_index_info", "caps_index_export"):
        assert n in names


def test_library_exports_declared_symbols():
    from paper_2308_15014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcaps.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n
    # the binding declares exactly the header's entry points
    assert sorted(_lib.SIGNATURES) == _declared()


def test_binding_loads():
    from paper_2308_15014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcaps.so not built")
    L = _lib.lib()
    assert L.caps_last_error() is not None or True


def test_load_refuses_missing_and_foreign_files(tmp_path):
    """caps_load checks the file before touching the device."""
    import ctypes
    from paper_2308_15014_amd import _lib
    L = _lib.lib()
    out = ctypes.c_void_p()
    assert L.caps_load(str(tmp_path / "missing.caps").encode(), None, ctypes.byref(out)) == -6
    p = tmp_path / "foreign.caps"
    p.write_bytes(b"NOTCAPS!" + bytes(64))
    assert L.caps_load(str(p).encode(), None, ctypes.byref(out)) == -6
    assert not out.value
