"""Autotuner (dw_autotune): coordinate search scored by time to solution."""
import numpy as np
import pytest

import paper_1204_5463_amd as P
import synth
from oracle import wilson as W

pytestmark = pytest.mark.gpu

L, EPS, M0 = (8, 8, 8, 8), 0.3, -0.1


def test_autotune_picks_fastest_converged_and_caches(dwctx, tmp_path):
    U = synth.gauge_field(L, EPS, 0)
    b = synth.gaussian_spinors(L, 2, seed0=1000)
    Ud, bd = P.to_device(U), P.to_device(b)
    base = P.SolverParams(m=20, k=5, max_iter=3000, tol=1e-10,
                          sap=P.SapParams(block=(4, 4, 4, 4), ncycles=1, nmr=4, storage=P.DW_PREC_F16))
    space = P.TuneSpace(nmr=(3, 5), s=(1, 2), mk=((16, 4), (24, 8)), repeats=2)
    cache = P.TuneCache(str(tmp_path / "tune.json"))
    best, trials = P.autotune(dwctx, L, Ud, M0, base, bd, space=space, cache=cache)
    # base + 5 valid block shapes of 8^4 (extents 2 and 4, volume 128..512) + nmr + s + (m, k), minus repeats
    blocks = {tuple(t["block"]) for t in trials}
    assert blocks == {(4, 4, 4, 4), (2, 4, 4, 4), (4, 2, 4, 4), (4, 4, 2, 4), (4, 4, 4, 2)}
    assert len(trials) >= 8
    conv = [t for t in trials if t["converged"]]
    fastest = min(conv, key=lambda t: t["seconds"])
    assert list(best.sap.block) == fastest["block"]
    assert (best.sap.nmr, best.sap.ncycles, best.m, best.k) == (fastest["nmr"], fastest["ncycles"], fastest["m"],
                                                                fastest["k"])
    assert best.max_iter == base.max_iter and best.sap.storage == base.sap.storage
    # the tuned parameters solve the system
    f = P.Field(dwctx, L, best.sap.block, Ud)
    x, st = f.solve(M0, best, bd)
    x = x.cpu().numpy()
    for r in range(2):
        assert st[r].converged
        assert np.linalg.norm(b[r] - W.apply_D(U, M0, x[r])) <= 1e-10 * np.linalg.norm(b[r]) * 1.01
    # second call is served from the cache
    best2, trials2 = P.autotune(dwctx, L, Ud, M0, base, bd, space=space, cache=cache)
    assert trials2 == [] and best2 == best


def test_autotune_rejects_bad_space(dwctx):
    U = P.to_device(synth.unit_gauge_field(L))
    b = P.to_device(synth.gaussian_spinors(L, 1, seed0=3))
    base = P.SolverParams(sap=P.SapParams(block=(4, 4, 4, 4)))
    with pytest.raises(P.DwError):
        P.autotune(dwctx, L, U, 0.1, base, b, space=P.TuneSpace(blocks=((8, 4, 4, 4),)))
    with pytest.raises(P.DwError):
        P.autotune(dwctx, L, U, 0.1, base, b, space=P.TuneSpace(mk=((10, 10),)))
