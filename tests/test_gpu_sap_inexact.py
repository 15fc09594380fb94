"""GPU parity of the adaptive inexact SAP (block solves stopped at a 0.1
residual reduction, Section 3) and of SAP as a stand-alone solver
(Section 3, Fig. 5) against the FP64 oracle."""
import numpy as np
import pytest

import paper_1204_5463_amd as P
import synth
from oracle import sap as S

pytestmark = pytest.mark.gpu

CASES = [
    # L, block, ncycles, nmr (cap), eps, m0, reduction
    ((8, 8, 8, 8), (4, 4, 4, 4), 2, 12, 0.6, -0.4, 0.1),
    ((8, 4, 4, 8), (2, 2, 2, 2), 2, 8, 0.6, 0.0, 0.1),
    ((4, 2, 6, 10), (2, 1, 3, 5), 2, 10, 0.5, -0.2, 0.2),   # 30-site blocks (partial wavefront)
    ((16, 8, 8, 8), (8, 4, 4, 4), 1, 16, 0.7, -0.3, 0.1),   # 512-site blocks
]


@pytest.mark.parametrize("L,block,ncyc,nmr,eps,m0,red", CASES)
def test_adaptive_sap_fp64_matches_oracle(dwctx, L, block, ncyc, nmr, eps, m0, red):
    U = synth.gauge_field(L, eps, 1)
    f = P.Field(dwctx, L, block, P.to_device(U))
    v = synth.gaussian_spinor(L, 5)
    sp = P.SapParams(block=block, ncycles=ncyc, nmr=nmr, storage=P.DW_PREC_F64, mr_reduction=red)
    z = f.sap(m0, sp, P.to_device(v)).cpu().numpy()
    ref = S.sap(U, m0, L, block, ncyc, nmr, v, reduction=red)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    assert err < 1e-12, err
    # the rule changed the result: the fixed-step sweep differs
    fixed = S.sap(U, m0, L, block, ncyc, nmr, v)
    assert np.max(np.abs(fixed - ref)) > 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec,tol", [(P.DW_PREC_F32, 1e-5), (P.DW_PREC_F16, 2e-2)])
def test_adaptive_sap_low_precision_close_to_oracle(dwctx, prec, tol):
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.6, 2)
    f = P.Field(dwctx, L, block, P.to_device(U))
    v = synth.gaussian_spinor(L, 6)
    m0 = -0.3
    sp = P.SapParams(block=block, ncycles=2, nmr=12, storage=prec, mr_reduction=0.1)
    z = f.sap(m0, sp, P.to_device(v)).cpu().numpy()
    ref = S.sap(U, m0, L, block, 2, 12, v, reduction=0.1)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    assert err < tol, err


def test_adaptive_sap_rejects_bad_reduction(dwctx):
    L, block = (8, 4, 4, 8), (2, 2, 2, 2)
    f = P.Field(dwctx, L, block, P.to_device(synth.gauge_field(L, 0.5, 3)))
    v = P.to_device(synth.gaussian_spinor(L, 7))
    for bad in (-0.1, 1.0, float("nan")):
        with pytest.raises(P.DwError):
            f.sap(0.1, P.SapParams(block=block, ncycles=1, nmr=3, mr_reduction=bad), v)


@pytest.mark.parametrize("m0", [0.2, -0.26])   # heavy: converges; past m_c = -0.226: diverges
def test_standalone_sap_fp64_matches_oracle(dwctx, m0):
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.3, 0)
    f = P.Field(dwctx, L, block, P.to_device(U))
    b = synth.gaussian_spinor(L, 7)
    niter = 12
    sp = P.SapParams(block=block, ncycles=1, nmr=4, storage=P.DW_PREC_F64)
    x, hist = f.sap_solve(m0, sp, P.to_device(b), niter)
    xr, hr = S.sap_solve(U, m0, L, block, 1, 4, b, niter)
    assert np.max(np.abs(np.array(hist) - hr) / np.array(hr)) < 1e-10
    assert np.max(np.abs(x.cpu().numpy() - xr)) < 1e-10 * np.max(np.abs(xr))
    assert (hist[-1] < hist[6]) == (m0 > 0)


def test_standalone_sap_fp16_outer_fp64(dwctx):
    """FP16 preconditioner inside the FP64 iteration: the history follows the
    FP64 one and the residual falls well below FP16's unit roundoff."""
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.3, 0)
    f = P.Field(dwctx, L, block, P.to_device(U))
    b = synth.gaussian_spinor(L, 7)
    niter, m0 = 12, 0.2
    sp = P.SapParams(block=block, ncycles=1, nmr=4, storage=P.DW_PREC_F16)
    _, hist = f.sap_solve(m0, sp, P.to_device(b), niter)
    _, hr = S.sap_solve(U, m0, L, block, 1, 4, b, niter)
    assert np.max(np.abs(np.array(hist) - hr) / np.array(hr)) < 5e-2
    assert hist[-1] < 1e-4


def test_standalone_sap_edge_cases(dwctx):
    L, block = (8, 4, 4, 8), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.5, 3)
    f = P.Field(dwctx, L, block, P.to_device(U))
    b = P.to_device(synth.gaussian_spinor(L, 8))
    sp = P.SapParams(block=block, ncycles=1, nmr=3, storage=P.DW_PREC_F64)
    x, hist = f.sap_solve(0.1, sp, b, 0)
    assert hist == [1.0] and np.count_nonzero(x.cpu().numpy()) == 0
    x, hist = f.sap_solve(0.1, P.SapParams(block=block, ncycles=0, nmr=3), b, 2)
    assert hist == [1.0, 1.0, 1.0]
    with pytest.raises(P.DwError):
        f.sap_solve(0.1, sp, b * 0, 3)


def test_solve_with_adaptive_sap_converges(dwctx):
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.3, 0)
    f = P.Field(dwctx, L, block, P.to_device(U))
    b = synth.gaussian_spinor(L, 9)
    m0 = -0.2
    prm = P.SolverParams(m=20, k=5, tol=1e-10, sap=P.SapParams(block=block, ncycles=2, nmr=10,
                                                                  storage=P.DW_PREC_F16, mr_reduction=0.1))
    x, st = f.solve(m0, prm, P.to_device(b))
    assert st[0].converged and st[0].true_relres < 1e-10
    r = b - f.apply(m0, x).cpu().numpy()
    assert np.linalg.norm(r) < 1.01e-10 * np.linalg.norm(b)
