"""The C-ABI library loads and exports every symbol include/gvote.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gvote.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gv_[a-z_]+)\s*\(", src)))


def test_header_declares_the_interface():
    names = declared_symbols()
    for n in ["gv_create", "gv_destroy", "gv_solve", "gv_parametrize", "gv_submit", "gv_poll", "gv_cancel",
              "gv_status_str", "gv_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2107_11810_amd import gvote
    path = gvote.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libgvote.so not built")
    lib = ctypes.CDLL(path)
    for n in declared_symbols():
        assert hasattr(lib, n), n
    # status text needs no device
    lib.gv_status_str.restype = ctypes.c_char_p
    assert lib.gv_status_str(0) == b"ok"
    assert lib.gv_status_str(-4) == b"inlier buffer too small"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2107_11810_amd import gvote
    monkeypatch.setattr(gvote, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gvote, "_lib", None)
    with pytest.raises(ImportError):
        gvote.lib()
