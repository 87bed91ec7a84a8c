"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parac.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(parac_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("parac_factor", "parac_apply", "parac_pcg", "parac_serve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2505_02977_amd import parac
    if not os.path.exists(parac.LIB_PATH):
        pytest.fail("libparac.so is not built")
    L = parac.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert parac.status_str(parac.EPOOL) == "fill pool exhausted"
