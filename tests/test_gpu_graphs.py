"""Whole restart cycles captured as HIP graphs (DW_SOLVE_GRAPHS), and the
asynchronous operator and preconditioner entry points.

A captured cycle holds every launch of the cycle: the Arnoldi steps (Alg. 3),
the cycle end with the explicit residual and the restart of Alg. 4, each
kernel gated by the right-hand side's control record on the device. Replays
must give bit for bit the eager solve, also when a later solve on the same
field replays the graphs with another mass and right-hand side, with the
program's own eager work and synchronisations in between, for one and for
several right-hand sides, with the FP32 basis and residual injection, and
with the shared deflation space.

dw_apply and sap_precondition enqueue their work without synchronising the
stream: right after they return, work queued before them is still running.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_1204_5463_amd as P
import synth
from oracle import sap as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
L, B, EPS = (8, 8, 8, 8), (4, 4, 4, 4), 0.6
MC = json.load(open(os.path.join(HERE, "golden", "critical_mass.json")))["8^4_eps0.6"]["m_c"]


@pytest.fixture(scope="module")
def field(dwctx):
    U = synth.gauge_field(L, EPS, 0)
    f = P.Field(dwctx, L, B, P.to_device(U))
    yield U, f
    f.close()


def _prm(prec=P.DW_PREC_F16, m=12, k=4, flags=0, shared=0):
    return P.SolverParams(m=m, k=k, max_iter=4000, tol=1e-10, flags=flags, shared_defl=shared,
                          sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=prec))


def _busy(n=64):
    a = torch.randn(n * 16, n * 16, device="cuda")
    return float((a @ a).sum())


@pytest.mark.parametrize("flags,nrhs,shared", [(0, 1, 0), (P.SOLVE_V32 | P.SOLVE_INJECT, 1, 0), (0, 3, 0),
                                               (0, 3, 1)])
def test_cycle_graphs_equal_eager(field, flags, nrhs, shared):
    U, f = field
    st = torch.cuda.Stream()
    cases = [(MC + 0.02, 1000), (MC + 0.05, 1003), (MC + 0.02, 1000)]
    for i, (m0, seed) in enumerate(cases):
        b = synth.gaussian_spinors(L, nrhs, seed0=seed) if nrhs > 1 else synth.gaussian_spinor(L, seed)
        print(f"graph case flags={flags} nrhs={nrhs} shared={shared} solve {i} m0={m0:.4f}", flush=True)
        with torch.cuda.stream(st):
            bd = P.to_device(b)
            xe, se = f.solve(m0, _prm(flags=flags, shared=shared), bd, stream=st)
            _busy()
            st.synchronize()
            xg, sg = f.solve(m0, _prm(flags=flags | P.SOLVE_GRAPHS, shared=shared), bd, stream=st)
        st.synchronize()
        assert all(s.converged for s in se) and min(s.cycles for s in se) >= 3
        assert [s.iterations for s in se] == [s.iterations for s in sg]
        assert [s.cycles for s in se] == [s.cycles for s in sg]
        assert [s.clean_restarts for s in se] == [s.clean_restarts for s in sg]
        assert np.array_equal(xe.cpu().numpy(), xg.cpu().numpy()), i


def test_kept_workspace_serves_a_timed_solve(field):
    """A solve with per-kernel timing on (so without graphs) after a captured
    solve of the same shape runs in the workspace the captured solve kept:
    one lock-step batch for the three right-hand sides, the same iterations
    and the same iterate bit for bit; the captured cycles then replay again."""
    U, f = field
    st = torch.cuda.Stream()
    nrhs, m0 = 3, MC + 0.03
    b = synth.gaussian_spinors(L, nrhs, seed0=1010)
    prm = _prm(flags=P.SOLVE_GRAPHS)
    with torch.cuda.stream(st):
        bd = P.to_device(b)
        xg, sg = f.solve(m0, prm, bd, stream=st)
        st.synchronize()
        f.ctx.profile_reset()
        f.ctx.profile(True)
        xp, sp = f.solve(m0, prm, bd, stream=st)
        f.ctx.profile(False)
        sap = f.ctx.profile_stats()["sap"]["launches"]
        xg2, sg2 = f.solve(m0, prm, bd, stream=st)
    st.synchronize()
    its = [s.iterations for s in sg]
    assert all(s.converged for s in sg) and [s.iterations for s in sp] == its == [s.iterations for s in sg2]
    assert np.array_equal(xg.cpu().numpy(), xp.cpu().numpy())
    assert np.array_equal(xg.cpu().numpy(), xg2.cpu().numpy())
    # SAP (one cycle: two colour launches per Arnoldi step) covered all three
    # right-hand sides per launch, not one batch after another
    print(f"timed solve after a captured one: iterations {its}, {sap} SAP launches", flush=True)
    assert 2 * max(its) <= sap < 2 * sum(its)


def test_solution_of_graph_solve_is_right(field):
    """The replayed solve reaches the 1e-10 true residual by the oracle's D."""
    U, f = field
    st = torch.cuda.Stream()
    b = synth.gaussian_spinor(L, 1007)
    m0 = MC + 0.03
    with torch.cuda.stream(st):
        for _ in range(2):
            x, s = f.solve(m0, _prm(flags=P.SOLVE_GRAPHS), P.to_device(b), stream=st)
    st.synchronize()
    x = x.cpu().numpy()
    r = b - W.apply_D(U, m0, x)
    assert s[0].converged and np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_apply_and_sap_do_not_synchronise(field):
    U, f = field
    x = synth.gaussian_spinor(L, 1011)
    m0 = -0.3
    sp = P.SapParams(block=B, ncycles=2, nmr=4, storage=P.DW_PREC_F16)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        xd = P.to_device(x)
        y = torch.empty_like(xd)
        z = torch.empty_like(xd)
        f.apply(m0, xd, y, stream=st)  # warm the allocator's cache for the temporaries
        f.sap(m0, sp, xd, z, stream=st)
        st.synchronize()
        torch.cuda._sleep(200_000_000)  # a bounded spin kernel queued ahead of the calls
        f.apply(m0, xd, y, stream=st)
        f.sap(m0, sp, xd, z, stream=st)
        pending = not st.query()
    st.synchronize()
    assert pending, "the calls waited for work queued before them"
    assert np.max(np.abs(y.cpu().numpy() - W.apply_D(U, m0, x))) <= 1e-13 * np.max(np.abs(x)) * 8
    zr = S.sap(U, m0, L, B, 2, 4, x)
    assert np.linalg.norm(z.cpu().numpy() - zr) <= 2e-2 * np.linalg.norm(zr)
