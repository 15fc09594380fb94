"""Serving loop (continuous batching of solve requests) on the GPU.

Requests run concurrently on the server's slots, each on its own stream,
with footprint admission. The kernels reduce in a fixed order, so a
request's result in the concurrent mix is bitwise the result of the same
solve made alone through fgmresdr_solve; every solution is also checked
with the oracle's operator.
"""
import time

import numpy as np
import pytest
import torch

import paper_1204_5463_amd as P
import synth
from oracle import wilson as W

pytestmark = pytest.mark.gpu

L, B = (8, 8, 8, 8), (4, 4, 4, 4)


def _params(prec=P.DW_PREC_F16, m=16, k=4):
    return P.SolverParams(m=m, k=k, max_iter=2000, tol=1e-10,
                          sap=P.SapParams(block=B, ncycles=1, nmr=4, storage=prec))


@pytest.fixture(scope="module")
def reqs():
    """Three requests: different gauge fields, masses and RHS counts."""
    out = []
    for i, (eps, m0, nrhs) in enumerate([(0.3, -0.1, 1), (0.3, -0.15, 2), (0.2, 0.0, 1)]):
        U = synth.gauge_field(L, eps, 10 + i)
        b = synth.gaussian_spinors(L, nrhs, seed0=2000 + 10 * i)
        out.append((U, b, m0))
    return out


def _alone(dwctx, U, b, m0, prm):
    f = P.Field(dwctx, L, B, P.to_device(U))
    x, st = f.solve(m0, prm, P.to_device(b))
    torch.cuda.synchronize()
    f.close()
    return x.cpu().numpy(), st


def test_mixed_requests_match_alone(dwctx, reqs):
    prm = _params()
    alone = [_alone(dwctx, U, b, m0, prm) for U, b, m0 in reqs]
    srv = P.Server(dwctx, slots=2, queue_capacity=8)
    try:
        dev = [(P.to_device(U), P.to_device(b), m0) for U, b, m0 in reqs]
        tickets = [srv.submit(L, B, m0, Ud, bd, prm) for Ud, bd, m0 in dev]
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for (U, b, m0), (xa, sa), (x, st, tm) in zip(reqs, alone, res):
        x = x.cpu().numpy()
        assert np.array_equal(x, xa)
        assert [s.iterations for s in st] == [s.iterations for s in sa]
        assert tm["latency"] >= tm["running"] >= 0 and tm["queued"] >= 0
        for r in range(b.shape[0]):
            assert st[r].converged
            res_r = b[r] - W.apply_D(U, m0, x[r])
            assert np.linalg.norm(res_r) <= 1e-10 * np.linalg.norm(b[r]) * 1.01


def test_admission_one_at_a_time_and_ticket_release(dwctx, reqs):
    """A budget that fits one request serialises them; results are unchanged."""
    prm = _params()
    U, b, m0 = reqs[0]
    Ud, bd = P.to_device(U), P.to_device(b)
    fp = P.Server.footprint(L, B, m0, Ud, bd, prm)
    assert fp > 0
    srv = P.Server(dwctx, slots=3, queue_capacity=8, budget_bytes=fp * 1.5)
    try:
        t = [srv.submit(L, B, m0, Ud, bd, prm) for _ in range(3)]
        out = [srv.wait(ti) for ti in t]
        xs = [o[0].cpu().numpy() for o in out]
        assert all(np.array_equal(xs[0], xi) for xi in xs[1:])
        with pytest.raises(KeyError):
            srv.poll(t[0])
        # the C entry point forgets a released ticket
        import ctypes
        state = ctypes.c_int32()
        rc = P.lib().solve_poll(srv.handle, ctypes.c_uint64(t[0]), ctypes.byref(state), None, None)
        assert rc == P.DW_ENOTFOUND
        # a request above the budget is rejected at submit
        b2 = P.to_device(synth.gaussian_spinors(L, 2, seed0=7))
        with pytest.raises(P.DwError) as e:
            srv.submit(L, B, m0, Ud, b2, prm)
        assert e.value.status == P.DW_EINVAL
    finally:
        srv.close()


def test_queue_full_and_bad_requests(dwctx, reqs):
    prm = _params()
    U, b, m0 = reqs[0]
    Ud, bd = P.to_device(U), P.to_device(b)
    srv = P.Server(dwctx, slots=1, queue_capacity=1)
    try:
        busy, tickets = 0, []
        for _ in range(3):
            try:
                tickets.append(srv.submit(L, B, m0, Ud, bd, prm))
            except P.DwError as e:
                assert e.status == P.DW_EBUSY
                busy += 1
        assert busy >= 1 and len(tickets) >= 1
        for t in tickets:
            x, st, _ = srv.wait(t)
            assert st[0].converged
        # geometry and parameter errors
        with pytest.raises(P.DwError):
            srv.submit(L, (3, 4, 4, 4), m0, Ud, bd, _params())
        with pytest.raises(P.DwError):
            srv.submit(L, B, m0, Ud, bd, _params(m=60))
        with pytest.raises(P.DwError):
            srv.submit(L, B, m0, Ud, bd, P.SolverParams(sap=P.SapParams(block=(2, 2, 2, 2))))
    finally:
        srv.close()


def test_destroy_drains_queue(dwctx, reqs):
    prm = _params()
    U, b, m0 = reqs[1]
    Ud, bd = P.to_device(U), P.to_device(b)
    x = torch.zeros_like(bd)
    srv = P.Server(dwctx, slots=1, queue_capacity=4)
    srv.submit(L, B, m0, Ud, bd, prm, x=x)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 60
    xa, _ = _alone(dwctx, U, b, m0, prm)
    assert np.array_equal(x.cpu().numpy(), xa)


def test_slot_reuses_field_and_captured_cycles(dwctx):
    """One slot, back-to-back requests of one lattice and parameter set with
    new links, masses and right-hand sides each time: the slot loads the
    links into the field it holds and replays the restart cycles captured
    for the first request. Every result equals the same solve made alone,
    bit for bit, and a request of another lattice in between changes
    nothing."""
    prm = _params()
    cases = [(0.3, -0.1, 11, 1), (0.35, -0.2, 12, 1), (0.3, -0.05, 13, 1)]
    data = []
    for eps, m0, seed, nrhs in cases:
        U = synth.gauge_field(L, eps, seed)
        b = synth.gaussian_spinors(L, nrhs, seed0=3000 + seed)
        data.append((U, b, m0))
    L2 = (8, 8, 8, 16)
    U2 = synth.gauge_field(L2, 0.3, 5)
    b2 = synth.gaussian_spinor(L2, 3100)[None]
    alone = [_alone(dwctx, U, b, m0, prm) for U, b, m0 in data]
    f2 = P.Field(dwctx, L2, B, P.to_device(U2))
    x2a, _ = f2.solve(-0.1, prm, P.to_device(b2))
    x2a = x2a.cpu().numpy()
    f2.close()
    srv = P.Server(dwctx, slots=1, queue_capacity=8)
    try:
        dev = [(P.to_device(U), P.to_device(b), m0) for U, b, m0 in data]
        t = [srv.submit(L, B, m0, Ud, bd, prm) for Ud, bd, m0 in dev[:2]]
        t.append(srv.submit(L2, B, -0.1, P.to_device(U2), P.to_device(b2), prm))
        t.append(srv.submit(L, B, dev[2][2], dev[2][0], dev[2][1], prm))
        res = [srv.wait(q) for q in t]
    finally:
        srv.close()
    order = [0, 1, None, 2]
    for i, (x, st, tm) in zip(order, res):
        if i is None:
            assert np.array_equal(x.cpu().numpy(), x2a)
            continue
        xa, sa = alone[i]
        assert np.array_equal(x.cpu().numpy(), xa), i
        assert [s.iterations for s in st] == [s.iterations for s in sa]
