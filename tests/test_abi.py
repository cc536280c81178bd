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


def test_bliss_assign_host_call_matches_oracle(orc):
    """caps_bliss_assign is a host computation: callable without a GPU, and
    equal to the oracle's re-partitioning rule item for item."""
    from paper_2308_15014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcaps.so not built")
    import numpy as np
    import paper_2308_15014_amd as caps
    rng = np.random.default_rng(11)
    for n, k, b in ((1, 1, 1), (1000, 4, 37), (20000, 8, 1024), (5000, 3, 2)):
        cand = rng.integers(0, b, size=(n, k)).astype(np.int32)
        assert np.array_equal(caps.bliss_assign(cand, b), orc.bliss_assign(cand, b))
    with pytest.raises(caps.CapsError):
        caps.bliss_assign(np.array([[0, 3]], np.int32), 3)
    assert caps.bliss_assign(np.zeros((0, 2), np.int32), 3).shape == (0,)
