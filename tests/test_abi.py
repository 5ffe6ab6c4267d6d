"""The C-ABI library loads and exports every entry point that include/pcloth.h
declares (no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "pcloth.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^(?:pc_status|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("pc_create", "pc_destroy", "cloth_assemble", "cloth_pcg_solve", "cloth_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2008_00409_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libpcloth.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(binding.ABI_SYMBOLS) == declared_symbols()
