"""The C-ABI library loads and exports every symbol include/gdm.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gdm.h")
LIB = os.path.join(ROOT, "paper_2505_09545_amd", "libgdm.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gdm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    syms = declared_symbols()
    for s in ("gdm_create", "gdm_set_structure", "gdm_assemble", "gdm_factorize", "gdm_solve", "gdm_fields",
              "gdm_cross_sections", "gdm_getrf", "gdm_getrs"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdm.so not built")
def test_binding_covers_the_header():
    from paper_2505_09545_amd import gdm
    assert sorted(gdm.EXPORTED) == declared_symbols()
    gdm.load_library()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2505_09545_amd import gdm
    saved = gdm._lib
    gdm._lib = None
    try:
        with pytest.raises(ImportError):
            gdm.load_library(str(tmp_path / "missing.so"))
    finally:
        gdm._lib = saved
