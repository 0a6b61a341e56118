"""The C-ABI library loads and exports every entry point include/xls.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xls.h")
LIB = os.path.join(ROOT, "paper_2609_13115_amd", "libxls.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(xls_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("xls_subdomain_create", "xls_chefsi_step", "xls_subdomain_density"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libxls.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2609_13115_amd import xls
    assert sorted(set(xls.EXPORTED)) == declared_functions()


def test_binding_struct_layout_matches_header_order():
    from paper_2609_13115_amd import xls
    names = [f[0] for f in xls.xls_subdomain_desc_t._fields_]
    src = open(HEADER).read()
    body = src[src.index("typedef struct {\n  int32_t n[3];"):src.index("} xls_subdomain_desc_t;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";")[:-1]:
        decl = decl.replace("typedef struct {", "")
        for part in decl.split(","):
            m = re.findall(r"\**\s*([a-z_0-9]+)\s*(?:\[\d\])?\s*$", part.strip())
            if m:
                fields.append(m[-1])
    assert names == fields
