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


def test_request_footprint_host_logic():
    """dw_request_footprint is host arithmetic: links + per-RHS solver memory, linear in nrhs."""
    import ctypes

    import paper_1204_5463_amd as P

    def fp(L=(8, 8, 8, 8), block=(4, 4, 4, 4), nrhs=1, m=20, k=5, prec=P.DW_PREC_F16):
        r = P._Request()
        for i in range(4):
            r.L[i], r.block[i] = L[i], block[i]
        r.nrhs = nrhs
        r.params = P.SolverParams(m=m, k=k, sap=P.SapParams(block=block, storage=prec))._c()
        return int(P.lib().dw_request_footprint(ctypes.byref(r)))

    V = 8 ** 4
    f1, f2, f3 = fp(nrhs=1), fp(nrhs=2), fp(nrhs=3)
    per = f2 - f1
    assert per > 0 and f3 - f2 == per
    links = f1 - per
    assert links == V * 36 * (16 + 8 + 4 + 4)
    # the Krylov bases dominate the per-RHS part: (m+1) V and m Z columns in FP64
    assert per >= V * 12 * 16 * (21 + 20)
    assert fp(m=30, k=5) > f1
    assert fp(block=(3, 4, 4, 4)) == 0 and fp(nrhs=0) == 0 and fp(m=49) == 0


def test_tune_cache_roundtrip(tmp_path):
    import paper_1204_5463_amd as P

    c = P.TuneCache(str(tmp_path / "t.json"))
    base = P.SolverParams(m=30, k=12, tol=1e-10, sap=P.SapParams(block=(4, 4, 4, 4), storage=P.DW_PREC_F16))
    k1 = P.TuneCache.key("gfx950", (32, 32, 32, 64), -1.137, base, 1)
    k2 = P.TuneCache.key("gfx950", (32, 32, 32, 64), -1.138, base, 1)
    k3 = P.TuneCache.key("gfx950", (32, 32, 32, 64), -1.137, base, 12)
    assert len({k1, k2, k3}) == 3
    assert c.get(k1) is None
    tuned = P.SolverParams(m=24, k=8, tol=1e-10, sap=P.SapParams(block=(8, 4, 4, 4), ncycles=2, nmr=5,
                                                                  storage=P.DW_PREC_F16, mr_reduction=0.1))
    c.put(k1, tuned, [{"block": [8, 4, 4, 4], "seconds": 1.0}])
    c.put(k3, base)
    assert c.get(k1) == tuned and c.get(k3) == base and c.get(k2) is None
    # the C struct carries every field of the space
    s = P.TuneSpace(blocks=((4, 4, 4, 4), (8, 4, 4, 4)), nmr=(3, 6), s=(1, 3), mk=((20, 5),), repeats=2)._c()
    assert s.nblocks == 2 and list(s.blocks[1]) == [8, 4, 4, 4] and (s.nmr_min, s.nmr_max) == (3, 6)
    assert s.nmk == 1 and list(s.mk[0]) == [20, 5] and s.repeats == 2


def test_sap_params_layout():
    """sap_params: four int32 extents, four int32 fields, then the double
    mr_reduction at byte 32; it is embedded in fgmresdr_params."""
    import ctypes

    import paper_1204_5463_amd as P

    assert ctypes.sizeof(P._SapParams) == 40 and P._SapParams.mr_reduction.offset == 32
    p = P.SapParams(block=(4, 2, 2, 2), ncycles=3, nmr=7, mr_reduction=0.25)._c()
    assert (p.ncycles, p.nmr, p.mr_reduction) == (3, 7, 0.25)
    q = P._params_from_c(P.SolverParams(sap=P.SapParams(mr_reduction=0.1))._c())
    assert q.sap.mr_reduction == 0.1
