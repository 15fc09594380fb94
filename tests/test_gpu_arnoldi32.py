"""The single-precision Arnoldi of Section 4.7 (DW_SOLVE_A32): V and Z in
FP32, w = D z_j with FP32 links and arithmetic, Gram-Schmidt in FP32; the
explicit FP64 residual of every restart enters c, G_{k+1} and v_{k+1}
(DW_SOLVE_INJECT), and a drifting cycle is caught by the clean restart.

  * it reaches the 1e-10 true residual measured by the oracle's FP64
    operator, and the oracle's FP64 solution within the conditioning bound;
  * its iteration count stays near that of the oracle's own
    single-precision Arnoldi (a different FP32 rounding order, so not equal);
  * replayed from captured cycles it gives bit for bit the eager solve.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_1204_5463_amd as P
import synth
from oracle import fgmresdr as F
from oracle import sap as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
MC6 = json.load(open(os.path.join(HERE, "golden", "critical_mass.json")))["8^4_eps0.6"]["m_c"]
L, B = (8, 8, 8, 8), (4, 4, 4, 4)
# (eps, m0, m, k, |lambda_min| estimate for the conditioning bound)
CASES = [(0.3, -0.1, 20, 5, 0.1), (0.6, MC6 + 0.02, 30, 12, 0.02)]


def _low_op(U, m0, shp):
    U32 = U.astype(np.complex64)
    return lambda v: W.apply_D(U32, m0, np.asarray(v, dtype=np.complex64).reshape(shp)).reshape(-1).astype(
        np.complex64)


@pytest.mark.parametrize("eps,m0,m,k,lam", CASES)
@pytest.mark.parametrize("prec", [P.DW_PREC_F16, P.DW_PREC_F64])
def test_single_precision_arnoldi_reaches_fp64_residual(dwctx, eps, m0, m, k, lam, prec):
    U = synth.gauge_field(L, eps, 0)
    b = synth.gaussian_spinor(L, 1000)
    shp = b.shape
    f = P.Field(dwctx, L, B, P.to_device(U))
    A = lambda v: W.apply_D(U, m0, v.reshape(shp)).reshape(-1)
    M = lambda v: S.sap(U, m0, L, B, 1, 4, v.reshape(shp)).reshape(-1)
    xo, io = F.fgmresdr(A, M, b.reshape(-1), m, k, tol=1e-10, max_iter=3000)
    xl, il = F.fgmresdr(A, M, b.reshape(-1), m, k, tol=1e-10, max_iter=3000, inject=True, A_low=_low_op(U, m0, shp))
    prm = P.SolverParams(m=m, k=k, max_iter=3000, tol=1e-10, flags=P.SOLVE_A32 | P.SOLVE_INJECT,
                         sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=prec))
    x, st = f.solve(m0, prm, P.to_device(b))
    st = st[0]
    print(f"A32 eps={eps} ({m},{k}) prec {prec}: GPU {st.iterations} it / {st.cycles} cycles / "
          f"{st.clean_restarts} clean; oracle single {il.iterations} / {il.cycles} / {il.clean_restarts}; "
          f"oracle double {io.iterations}", flush=True)
    x = x.cpu().numpy().reshape(-1)
    assert st.converged and il.converged
    r = b.reshape(-1) - A(x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    # |x - x*| <= cond (relres + relres*), cond ~ 8 / |lambda_min|
    cond = 8.0 / lam
    assert np.linalg.norm(x - xo) <= cond * 2.02e-10 * np.linalg.norm(xo)
    assert abs(st.iterations - il.iterations) <= max(3, 0.15 * il.iterations), (st.iterations, il.iterations)
    f.close()


def test_single_precision_arnoldi_graphs_equal_eager(dwctx):
    U = synth.gauge_field(L, 0.6, 0)
    b = synth.gaussian_spinor(L, 1000)
    f = P.Field(dwctx, L, B, P.to_device(U))
    m0 = MC6 + 0.02
    st_ = torch.cuda.Stream()
    flags = P.SOLVE_A32 | P.SOLVE_INJECT
    prm = lambda fl: P.SolverParams(m=30, k=12, max_iter=3000, tol=1e-10, flags=fl,
                                    sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=P.DW_PREC_F16))
    with torch.cuda.stream(st_):
        bd = P.to_device(b)
        xe, se = f.solve(m0, prm(flags), bd, stream=st_)
        for _ in range(2):
            xg, sg = f.solve(m0, prm(flags | P.SOLVE_GRAPHS), bd, stream=st_)
            st_.synchronize()
            assert se[0].iterations == sg[0].iterations and se[0].cycles == sg[0].cycles
            assert np.array_equal(xe.cpu().numpy(), xg.cpu().numpy())
    f.close()
