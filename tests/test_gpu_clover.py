"""Clover-improved operator on the GPU against the oracle (``oracle/clover.py``).

* D_sw: FP64 to 1e-13 and every storage precision within its rounding;
  sampled sites of the 32^3 x 64 lattice;
* SAP with the clover term in every block operator: FP64 to 1e-12, FP16
  within its rounding;
* the solve reaches the 1e-10 true residual of D_sw (oracle operator) and,
  all in FP64, follows the oracle's FGMRES-DR iteration;
* c_sw = 0 removes the term exactly; a server request with c_sw gives the
  result of the same solve made directly.
"""
import numpy as np
import pytest
import torch

import paper_1204_5463_amd as P
import synth
from oracle import clover as Cl
from oracle import fgmresdr as F
from oracle import sap as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu

L, B, EPS, M0, CSW = (8, 8, 8, 8), (4, 4, 4, 4), 0.5, -0.3, 1.7
TOL = {P.DW_PREC_F64: 1e-13, P.DW_PREC_F32: 2e-6, P.DW_PREC_F16: 3e-3, P.DW_PREC_BF16: 2.5e-2}


@pytest.fixture(scope="module")
def cf(dwctx):
    U = synth.gauge_field(L, EPS, 11)
    C = Cl.clover_term(U, CSW)
    f = P.Field(dwctx, L, B, P.to_device(U))
    f.set_clover(CSW)
    return U, C, f


def test_apply_fp64_matches_oracle(cf):
    U, C, f = cf
    x = synth.gaussian_spinor(L, 21)
    y = f.apply(M0, P.to_device(x)).cpu().numpy()
    ref = W.apply_D(U, M0, x, C)
    assert np.max(np.abs(y - ref)) < 1e-13 * np.max(np.abs(ref))
    # the term is really there
    assert np.linalg.norm(ref - W.apply_D(U, M0, x)) > 1e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", [P.DW_PREC_F64, P.DW_PREC_F32, P.DW_PREC_F16, P.DW_PREC_BF16])
def test_apply_ex_each_precision(cf, prec):
    U, C, f = cf
    x = synth.gaussian_spinor(L, 22)
    xi = f.pack(prec, P.to_device(x))
    yi = torch.empty_like(xi)
    f.apply_ex(M0, prec, xi, yi)
    y = f.unpack(prec, yi).cpu().numpy()[0]
    ref = W.apply_D(U, M0, x, C)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < TOL[prec]


@pytest.mark.parametrize("prec,tol", [(P.DW_PREC_F64, 1e-12), (P.DW_PREC_F16, 2e-2)])
def test_sap_matches_oracle(cf, prec, tol):
    U, C, f = cf
    v = synth.gaussian_spinor(L, 23)
    z = f.sap(M0, P.SapParams(block=B, ncycles=2, nmr=4, storage=prec), P.to_device(v)).cpu().numpy()
    zo = S.sap(U, M0, L, B, 2, 4, v, C=C)
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) < tol


def test_adaptive_sap_and_standalone_sap_with_clover(cf):
    """The adaptive block solves and the stand-alone SAP iteration with the
    clover term in every block operator, FP64 storage against the oracle."""
    U, C, f = cf
    v = synth.gaussian_spinor(L, 25)
    sp = P.SapParams(block=B, ncycles=2, nmr=12, storage=P.DW_PREC_F64, mr_reduction=0.1)
    z = f.sap(M0, sp, P.to_device(v)).cpu().numpy()
    zo = S.sap(U, M0, L, B, 2, 12, v, C=C, reduction=0.1)
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) < 1e-12
    x, hist = f.sap_solve(M0, P.SapParams(block=B, ncycles=1, nmr=4, storage=P.DW_PREC_F64), P.to_device(v), 6)
    xo, ho = S.sap_solve(U, M0, L, B, 1, 4, v, 6, C=C)
    assert np.max(np.abs(np.array(hist) - ho) / np.array(ho)) < 1e-10
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) < 1e-10


def test_solve_fp64_follows_oracle_and_mixed_reaches_residual(cf):
    U, C, f = cf
    b = synth.gaussian_spinor(L, 24)
    shp = b.shape
    A = lambda v: W.apply_D(U, M0, v.reshape(shp), C).reshape(-1)
    M = lambda v: S.sap(U, M0, L, B, 1, 4, v.reshape(shp), C=C).reshape(-1)
    xo, info = F.fgmresdr(A, M, b.reshape(-1), 16, 4, tol=1e-10, max_iter=2000)
    for prec in (P.DW_PREC_F64, P.DW_PREC_F16):
        prm = P.SolverParams(m=16, k=4, max_iter=2000, tol=1e-10,
                             sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=prec))
        x, st = f.solve(M0, prm, P.to_device(b))
        x = x.cpu().numpy()
        assert st[0].converged
        r = b - W.apply_D(U, M0, x, C)
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
        assert np.linalg.norm(x - xo.reshape(shp)) <= 1e-8 * np.linalg.norm(xo)
        if prec == P.DW_PREC_F64:
            assert abs(st[0].iterations - info.iterations) <= 1


def test_zero_csw_removes_the_term(dwctx):
    U = synth.gauge_field(L, EPS, 12)
    x = P.to_device(synth.gaussian_spinor(L, 25))
    f = P.Field(dwctx, L, B, P.to_device(U))
    y0 = f.apply(M0, x).cpu().numpy()
    f.set_clover(1.3)
    y1 = f.apply(M0, x).cpu().numpy()
    f.set_clover(0.0)
    y2 = f.apply(M0, x).cpu().numpy()
    assert not np.array_equal(y0, y1) and np.array_equal(y0, y2)
    with pytest.raises(P.DwError):
        f.set_clover(float("nan"))


def test_full_size_sampled_sites(dwctx):
    Lb = (32, 32, 32, 64)
    U = synth.gauge_field(Lb, 0.7, 0)
    f = P.Field(dwctx, Lb, B, P.to_device(U))
    f.set_clover(1.9)
    x = synth.gaussian_spinor(Lb, 1000)
    y = f.apply(-1.0, P.to_device(x)).cpu().numpy().reshape(-1, 4, 3)
    V = synth.volume(Lb)
    rng = np.random.default_rng(1)
    sites = list(rng.integers(0, V, 60)) + [0, V - 1, 31, 32 * 32 * 32 * 63]
    Cs = Cl.clover_at_sites(U, 1.9, sites)
    ref = W.apply_D_at_sites(U, -1.0, x, sites, Cs)
    assert np.max(np.abs(y[sites] - ref)) < 1e-13 * np.max(np.abs(ref))


def test_server_request_with_clover(dwctx, cf):
    U, C, f = cf
    b = synth.gaussian_spinors(L, 1, seed0=26)
    prm = P.SolverParams(m=16, k=4, max_iter=2000, tol=1e-10,
                         sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=P.DW_PREC_F16))
    xa, _ = f.solve(M0, prm, P.to_device(b))
    srv = P.Server(dwctx, slots=1, queue_capacity=2)
    try:
        t = srv.submit(L, B, M0, P.to_device(U), P.to_device(b), prm, csw=CSW)
        x, st, _ = srv.wait(t)
    finally:
        srv.close()
    assert st[0].converged
    assert np.array_equal(x.cpu().numpy(), xa.cpu().numpy())
