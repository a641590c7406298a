"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/prcg.h declares, and the binding declares
the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prcg.h")
LIB = os.path.join(ROOT, "paper_1905_01549_amd", "libprcg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(prcg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("prcg_create_csr", "prcg_solve", "prcg_solve_batched", "prcg_adjoint"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libprcg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1905_01549_amd import prcg
    assert sorted(prcg.EXPORTED) == declared_functions()
    for name in prcg.EXPORTED:
        assert callable(getattr(prcg, name))


def test_binding_refuses_missing_library(tmp_path):
    from paper_1905_01549_amd import prcg
    saved = prcg._LIB
    prcg._LIB = None
    try:
        with pytest.raises(ImportError):
            prcg.load_library(str(tmp_path / "nope.so"))
    finally:
        prcg._LIB = saved
