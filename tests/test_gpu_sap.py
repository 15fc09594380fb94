"""GPU parity of the SAP preconditioner (Alg. 2 with MR block solves)
against the FP64 oracle, at FP64 (to rounding) and at each low storage
precision (within the precision's unit roundoff times a conditioning factor).
"""
import numpy as np
import pytest

import paper_1204_5463_amd as P
import synth
from oracle import sap as S

pytestmark = pytest.mark.gpu

CASES = [
    # L, block, ncycles, nmr, eps, m0
    ((8, 8, 8, 8), (4, 4, 4, 4), 1, 4, 0.3, -0.1),
    ((8, 8, 8, 8), (4, 4, 4, 4), 2, 5, 0.6, -0.4),
    ((8, 4, 4, 8), (2, 2, 2, 2), 3, 2, 0.6, 0.0),
    ((4, 2, 6, 10), (2, 1, 3, 5), 2, 3, 0.5, -0.2),   # 30-site blocks (partial wavefront)
    ((16, 8, 8, 8), (8, 4, 4, 4), 1, 5, 0.7, -0.3),   # 512-site blocks
]


@pytest.mark.parametrize("L,block,ncyc,nmr,eps,m0", CASES)
def test_sap_fp64_matches_oracle(dwctx, L, block, ncyc, nmr, eps, m0):
    U = synth.gauge_field(L, eps, 1)
    f = P.Field(dwctx, L, block, P.to_device(U))
    v = synth.gaussian_spinor(L, 5)
    sp = P.SapParams(block=block, ncycles=ncyc, nmr=nmr, storage=P.DW_PREC_F64)
    z = f.sap(m0, sp, P.to_device(v)).cpu().numpy()
    ref = S.sap(U, m0, L, block, ncyc, nmr, v)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    assert err < 1e-12, err


@pytest.mark.parametrize("prec,tol", [(P.DW_PREC_F32, 1e-5), (P.DW_PREC_F16, 2e-2), (P.DW_PREC_BF16, 1e-1)])
def test_sap_low_precision_close_to_oracle(dwctx, prec, tol):
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.6, 2)
    f = P.Field(dwctx, L, block, P.to_device(U))
    v = 1e-3 * synth.gaussian_spinor(L, 6)      # tiny entries: the scaling keeps FP16 in range
    m0 = -0.3
    sp = P.SapParams(block=block, ncycles=2, nmr=5, storage=prec)
    z = f.sap(m0, sp, P.to_device(v)).cpu().numpy()
    ref = S.sap(U, m0, L, block, 2, 5, v)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    assert err < tol, err


def test_sap_multi_rhs_and_zero_cycles(dwctx):
    L, block = (8, 4, 4, 8), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.5, 3)
    f = P.Field(dwctx, L, block, P.to_device(U))
    v = synth.gaussian_spinors(L, 3)
    sp = P.SapParams(block=block, ncycles=1, nmr=3, storage=P.DW_PREC_F64)
    z = f.sap(0.1, sp, P.to_device(v)).cpu().numpy()
    for r in range(3):
        ref = S.sap(U, 0.1, L, block, 1, 3, v[r])
        assert np.max(np.abs(z[r] - ref)) < 1e-12 * np.max(np.abs(ref))
    z0 = f.sap(0.1, P.SapParams(block=block, ncycles=0, nmr=3), P.to_device(v)).cpu().numpy()
    assert np.count_nonzero(z0) == 0
    with pytest.raises(P.DwError):
        f.sap(0.1, P.SapParams(block=(4, 2, 2, 2), ncycles=1, nmr=3), P.to_device(v))
