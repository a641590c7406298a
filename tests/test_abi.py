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


def header_enum(name):
    """{constant: value} of a typedef'd enum of include/prcg.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef enum \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    return {k: int(v) for k, v in re.findall(r"(PRCG_[A-Z_]+)\s*=\s*(-?\d+)", body)}


def test_binding_constants_match_the_header():
    from paper_1905_01549_amd import prcg
    variants = header_enum("prcg_variant")
    assert sorted(variants.values()) == sorted(prcg.VARIANTS.values())
    for key, code in prcg.VARIANTS.items():
        assert variants["PRCG_" + key.upper()] == code, key
    assert header_enum("prcg_precond") == {"PRCG_PRECOND_" + k.upper(): v for k, v in prcg.PRECONDS.items()}
    assert header_enum("prcg_batch_mode_t") == {"PRCG_BATCH_" + k.upper(): v for k, v in prcg.BATCH_MODES.items()}
    assert header_enum("prcg_batch_fusion_t") == {"PRCG_BATCH_FUSION_" + k.upper(): v
                                                  for k, v in prcg.BATCH_FUSION.items()}


def header_struct(name):
    """[(field, C type)] of a typedef'd struct of include/prcg.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    return re.findall(r"(int32_t|int64_t|double)\s+(\w+)\s*;", body)


@pytest.mark.parametrize("name", ["prcg_matrix_props", "prcg_info", "prcg_batch_props"])
def test_binding_structs_match_the_header(name):
    """Field order, names and widths of the structs passed across the ABI."""
    from paper_1905_01549_amd import prcg
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    fields = getattr(prcg, name)._fields_
    assert [(f, ctype[t]) for t, f in header_struct(name)] == [(f, t) for f, t in fields]


def test_noalloc_limit_matches_the_header():
    from paper_1905_01549_amd import prcg
    m = re.search(r"#define\s+PRCG_NOALLOC_MAX_ITERS\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == prcg.NOALLOC_MAX_ITERS
