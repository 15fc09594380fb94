"""The C-ABI library loads and exports every function that include/*.h
declares (no GPU needed: nothing is called)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1204_5463_amd", "libdwsap.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "sizeof", "return") and not text[m.start():m.end()].lstrip().startswith("typedef"):
                names.add(name)
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dw_apply", "sap_precondition", "fgmresdr_solve", "dw_ctx_create", "dw_field_create", "dw_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libdwsap.so is not built (run python -m paper_1204_5463_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1204_5463_amd as P
    with pytest.raises(RuntimeError):
        P._lib = None
        P.load(str(tmp_path / "nope.so"))
    P._lib = None
