"""The C-ABI library: it loads and exports every symbol include/sfem.h
declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfem.h")
LIB = os.path.join(ROOT, "paper_2001_08849_amd", "libsfem.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfem_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("sfem_create", "sfem_set_mesh", "sfem_assemble", "sfem_get_csr", "sfem_solve"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsfem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2001_08849_amd import sfem
    assert sorted(sfem.EXPORTS) == declared_symbols()


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    from paper_2001_08849_amd import sfem
    monkeypatch.setattr(sfem, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(sfem, "_LIB", None)
    with pytest.raises(ImportError):
        sfem.lib()
