"""The C-ABI library loads and exports every function include/gks.h declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gks.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gks_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_step_api():
    names = declared()
    for must in ("gks_init", "gks_step", "gks_state", "gks_free", "gks_last_error", "gks_init_device",
                 "gks_state_device"):
        assert must in names


def test_library_exports_every_declared_function():
    from paper_1901_00261_amd import gks
    if not os.path.exists(gks.LIB_PATH):
        pytest.fail("libgks.so is not built (run python paper_1901_00261_amd/build.py)")
    lib = ctypes.CDLL(gks.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding wraps exactly the declared set
    assert sorted(gks.EXPORTED) == declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1901_00261_amd import gks
    monkeypatch.setattr(gks, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gks, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        gks.lib()
