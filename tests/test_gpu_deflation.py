"""Deflated restarts (Alg. 4, Sections 4.4-4.5) at the benchmark's solver
shapes, against the FP64 oracle.

  * whole solves with FP64 SAP at FGMRES-DR(30, 12) and (30, 10) on a
    near-critical 8^4 system that needs four deflated restarts: the GPU
    follows the oracle's cycles (equal count), iterations (within one) and
    solution (1e-8);
  * the small dense restart step itself (harmonic Ritz values of Lemma 1,
    G_{k+1} = [[G_k; 0], c - H^ eta], its QR factor Q_{k+1} and
    H^_k = Q_{k+1}^H H^ Q_k), run by the solver's one-wavefront kernel on an
    H^ taken from an oracle Arnoldi cycle, against SciPy's eigensolver and
    NumPy's QR: Ritz values element by element, Q_{k+1} up to the phase of
    each column (the only freedom of a QR factor), H^_k likewise, and the
    restart relation H^ Q_k = Q_{k+1} H^_k;
  * the small least-squares problem (Section 4.2) against NumPy's lstsq.
"""
import json
import os

import numpy as np
import pytest

import paper_1204_5463_amd as P
import synth
from oracle import fgmresdr as F
from oracle import sap as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
L, B, EPS = (8, 8, 8, 8), (4, 4, 4, 4), 0.6
MC = json.load(open(os.path.join(HERE, "golden", "critical_mass.json")))["8^4_eps0.6"]["m_c"]
M0 = MC + 0.02


@pytest.fixture(scope="module")
def system(dwctx):
    U = synth.gauge_field(L, EPS, 0)
    b = synth.gaussian_spinor(L, 1000)
    f = P.Field(dwctx, L, B, P.to_device(U))
    shp = b.shape
    A = lambda v: W.apply_D(U, M0, v.reshape(shp)).reshape(-1)
    M = lambda v: S.sap(U, M0, L, B, 1, 4, v.reshape(shp)).reshape(-1)
    yield U, b, f, A, M
    f.close()


@pytest.mark.parametrize("m,k", [(30, 12), (30, 10)])
def test_deflated_restarts_follow_oracle(system, m, k):
    U, b, f, A, M = system
    print(f"deflation solve 8^4 m0={M0:.6f} FGMRES-DR({m},{k})", flush=True)
    xo, info = F.fgmresdr(A, M, b.reshape(-1), m, k, tol=1e-10, max_iter=3000)
    assert info.converged and info.cycles >= 4 and info.clean_restarts == 0, info.cycles
    params = P.SolverParams(m=m, k=k, max_iter=3000, tol=1e-10,
                            sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=P.DW_PREC_F64))
    x, st = f.solve(M0, params, P.to_device(b))
    st = st[0]
    x = x.cpu().numpy().reshape(-1)
    assert st.converged and st.clean_restarts == 0
    assert st.cycles == info.cycles, (st.cycles, info.cycles)
    assert abs(st.iterations - info.iterations) <= 1, (st.iterations, info.iterations)
    r = b.reshape(-1) - A(x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.fixture(scope="module")
def arnoldi_cycle(system):
    """H^ (31 x 30), c = beta e_1 and eta of one oracle FGMRES cycle."""
    U, b, f, A, M = system
    V, Z, H = F.flexible_arnoldi(A, M, b.reshape(-1), 30)
    c = np.zeros(31, dtype=np.complex128)
    c[0] = np.linalg.norm(b)
    return H, c


def _phase_match(Qg, Qo):
    """Column phases d with Qg ~ Qo diag(d) (QR factors agree up to them)."""
    d = np.einsum("ij,ij->j", Qo.conj(), Qg)
    return d / np.abs(d)


@pytest.mark.parametrize("mm,k", [(30, 12), (30, 10), (17, 12), (30, 5)])
def test_dense_restart_matches_scipy(dwctx, arnoldi_cycle, mm, k):
    H, c = arnoldi_cycle
    Hh = np.ascontiguousarray(H[:mm + 1, :mm])
    cc = c[:mm + 1].copy()
    eta = np.linalg.lstsq(Hh, cc, rcond=None)[0]
    ritz, Qg, Hkg, status = P.dense_restart(dwctx, Hh, cc, eta, k)
    assert status == 0
    lam, G = F.harmonic_ritz(Hh)
    assert np.max(np.abs(ritz - lam)) <= 1e-10 * np.max(np.abs(lam)), np.max(np.abs(ritz - lam))
    # the oracle's restart basis: G_{k+1} = [[G_k; 0], c - H^ eta], Q R = G_{k+1}
    Gk1 = np.zeros((mm + 1, k + 1), dtype=np.complex128)
    Gk1[:mm, :k] = G[:, :k]
    Gk1[:, k] = cc - Hh @ eta
    Qo, _ = np.linalg.qr(Gk1)
    d = _phase_match(Qg, Qo)
    assert np.max(np.abs(Qg - Qo * d)) <= 1e-9
    Hko = Qo.conj().T @ Hh @ Qo[:mm, :k]
    assert np.max(np.abs(Hkg - (d.conj()[:, None] * Hko * d[None, :k]))) <= 1e-9 * np.max(np.abs(Hko))
    # restart relation with the GPU's own factors
    assert np.linalg.norm(Hh @ Qg[:mm, :k] - Qg @ Hkg) <= 1e-12 * np.linalg.norm(Hh)
    assert np.linalg.norm(Qg.conj().T @ Qg - np.eye(k + 1)) <= 1e-13


@pytest.mark.parametrize("cols", [1, 7, 30])
def test_dense_lsq_matches_numpy(dwctx, arnoldi_cycle, cols):
    H, c = arnoldi_cycle
    Hh = np.ascontiguousarray(H[:cols + 1, :cols])
    cc = c[:cols + 1].copy()
    eta_g, res_g = P.dense_lsq(dwctx, Hh, cc)
    eta_o = np.linalg.lstsq(Hh, cc, rcond=None)[0]
    res_o = np.linalg.norm(cc - Hh @ eta_o)
    assert np.linalg.norm(eta_g - eta_o) <= 1e-12 * np.linalg.norm(eta_o)
    assert abs(res_g - res_o) <= 1e-12 * np.linalg.norm(cc)
