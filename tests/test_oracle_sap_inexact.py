"""Pins of the oracle's adaptive inexact SAP and stand-alone SAP iteration
(Section 3; Fig. 5).

  * Adaptive MR: on every block the result equals fixed-step MR with that
    block's own step count n_b, the first n at which the explicit block
    residual ||r - D^l y_n|| is at most delta ||r||, found by brute force
    block by block (capped at n_MR); the step count is minimal.
  * delta = 0 is the fixed-step method; a tiny delta changes nothing.
  * Stand-alone SAP with exact block solves: the residual after k
    iterations is (I - D M_s)^k b, assembled from the dense splitting series
    of Section 4; its asymptotic rate is the spectral radius of I - M_s D,
    below one for a heavy mass and above one well past the critical mass.
  * Stand-alone SAP with MR block solves: x_k equals k * s cycles of Alg. 2
    applied to D x = b from zero (the iteration continues the sweep).
"""
import numpy as np
import pytest

import synth
from oracle import sap as S
from oracle import wilson as W


def test_adaptive_mr_equals_per_block_fixed_steps():
    L = (8, 4, 4, 4)
    block = (4, 2, 2, 2)
    U = synth.gauge_field(L, 0.7, 11)
    m0 = -0.4
    delta, nmr = 0.1, 12
    r = synth.gaussian_spinor(L, 12) * S.colour_mask(L, block, 0)[..., None, None]
    y, rho = S.mr_blocks(U, m0, L, block, r, nmr, reduction=delta)
    assert np.max(np.abs(r - W.apply_D_blocks(U, m0, y, block) - rho)) < 1e-12
    steps = []
    for colour, origin in S.block_list(L, block):
        if colour != 0:
            continue
        mask = S.single_block_mask(L, block, origin)[..., None, None]
        rb = r * mask
        rn = np.linalg.norm(rb)
        nb = nmr
        for n in range(nmr + 1):
            yn, _ = S.mr_blocks(U, m0, L, block, rb, n)
            if np.linalg.norm(rb - W.apply_D_blocks(U, m0, yn, block)) <= delta * rn:
                nb = n
                break
        yb, _ = S.mr_blocks(U, m0, L, block, rb, nb)
        assert np.max(np.abs(y * mask - yb)) <= 1e-13 * np.max(np.abs(yb))
        steps.append(nb)
    # the rule is active: blocks stop before the cap, not all at once
    assert max(steps) < nmr and min(steps) >= 1
    # every block meets the criterion
    assert np.all(S.block_norm(rho, L, block) <= delta * S.block_norm(r, L, block) + 1e-300)


def test_adaptive_mr_limits():
    L = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.5, 13)
    m0 = -0.2
    r = synth.gaussian_spinor(L, 14) * S.colour_mask(L, block, 1)[..., None, None]
    y0, _ = S.mr_blocks(U, m0, L, block, r, 6)
    y1, _ = S.mr_blocks(U, m0, L, block, r, 6, reduction=1e-30)
    assert np.array_equal(y0, y1)
    # a reduction reached at step 0 by no block: never before step 1
    y2, _ = S.mr_blocks(U, m0, L, block, r, 6, reduction=0.999)
    y3, _ = S.mr_blocks(U, m0, L, block, r, 1)
    assert np.max(np.abs(y2 - y3)) == 0.0
    # the adaptive SAP cycle equals fixed SAP when no block stops early
    v = synth.gaussian_spinor(L, 15)
    assert np.array_equal(S.sap(U, m0, L, block, 2, 4, v), S.sap(U, m0, L, block, 2, 4, v, reduction=1e-30))


def _colour_perm(L, block):
    c0 = np.repeat(S.colour_mask(L, block, 0).reshape(-1), 12)
    return np.concatenate([np.flatnonzero(c0), np.flatnonzero(~c0)]), int(c0.sum())


def _exact_solver(U, m0, L, block):
    Dl = W.dense_D(U, m0, block=block)

    def solve(r, colour):
        y = np.zeros(r.size, complex)
        idx = np.flatnonzero(np.repeat(S.colour_mask(L, block, colour).reshape(-1), 12))
        y[idx] = np.linalg.solve(Dl[np.ix_(idx, idx)], r.reshape(-1)[idx])
        return y.reshape(r.shape)
    return solve


@pytest.mark.parametrize("m0,converges", [(0.2, True), (-1.6, False)])
def test_standalone_exact_sap_residual_powers(m0, converges):
    L = (4, 2, 2, 4)
    block = (2, 1, 1, 2)
    U = synth.gauge_field(L, 0.6, 16)
    b = synth.gaussian_spinor(L, 17)
    s, niter = 1, 40
    _, hist = S.sap_solve(U, m0, L, block, s, 0, b, niter, block_solver=_exact_solver(U, m0, L, block))
    D = W.dense_D(U, m0)
    perm, n0 = _colour_perm(L, block)
    inv = np.argsort(perm)
    M = S.splitting_series(D[np.ix_(perm, perm)], n0, s)[np.ix_(inv, inv)]
    E = np.eye(D.shape[0]) - D @ M
    r = b.reshape(-1).copy()
    for k in range(8):
        assert abs(hist[k] - np.linalg.norm(r) / np.linalg.norm(b)) < 1e-11 * max(1.0, hist[k])
        r = E @ r
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(D.shape[0]) - M @ D)))
    assert (rho < 1) == converges
    rate = (hist[niter] / hist[niter - 15]) ** (1 / 15)
    assert abs(rate - rho) < 0.03 * rho
    assert (hist[niter] < hist[0]) == converges


def test_standalone_mr_sap_continues_the_sweep():
    L = (8, 4, 4, 4)
    block = (4, 2, 2, 2)
    U = synth.gauge_field(L, 0.7, 18)
    m0 = -0.3
    b = synth.gaussian_spinor(L, 19)
    for s, k, red in [(1, 3, 0.0), (2, 2, 0.0), (1, 3, 0.2)]:
        x, hist = S.sap_solve(U, m0, L, block, s, 4, b, k, reduction=red)
        z = S.sap(U, m0, L, block, s * k, 4, b, reduction=red)
        assert np.max(np.abs(x - z)) < 1e-12 * np.max(np.abs(z))
        assert abs(hist[k] - np.linalg.norm(b - W.apply_D(U, m0, z)) / np.linalg.norm(b)) < 1e-12
        assert hist[0] == 1.0
