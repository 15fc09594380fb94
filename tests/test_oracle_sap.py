"""Pins of the oracle's MR block solver and SAP sweep.

  * MR: the residual norm never grows; the returned residual is r - D^l y;
    one step is exact when D^l is a multiple of the identity (1^4 blocks);
    many steps reach the dense block solve.
  * SAP with exact block solves equals the truncated series
    M_s = sum_{j<s} (A_L^{-1} A_U)^j A_L^{-1} of the red/black block
    splitting (Section 4), assembled densely.
  * 1^4 blocks, one cycle: the closed form of a two-colour block
    Gauss-Seidel step.
  * Alg. 1 (sequential, any block order within a colour) equals Alg. 2.
  * M(alpha v) = alpha M(v) and gauge covariance of M.
"""
import numpy as np
import pytest

import synth
from oracle import sap as S
from oracle import wilson as W


def _system(L, eps=0.5, seed=0):
    return synth.gauge_field(L, eps, seed)


def test_blocking_checks():
    with pytest.raises(ValueError):
        S.check_blocking((8, 8, 8, 8), (4, 4, 4, 3))
    with pytest.raises(ValueError):
        S.check_blocking((12, 8, 8, 8), (4, 4, 4, 4))   # 3 blocks in x
    S.check_blocking((8, 8, 8, 8), (4, 4, 4, 4))


def test_mr_monotone_and_residual():
    L = (8, 4, 4, 4)
    block = (4, 2, 2, 2)
    U = _system(L, 0.7, 1)
    m0 = -0.3
    r = synth.gaussian_spinor(L, 3) * S.colour_mask(L, block, 0)[..., None, None]
    prev = None
    for nmr in range(0, 7):
        y, rho = S.mr_blocks(U, m0, L, block, r, nmr)
        rr = r - W.apply_D_blocks(U, m0, y, block)
        assert np.max(np.abs(rr - rho)) < 1e-12
        # per-block residual norms never increase
        nb = S.block_sum(np.abs(rho) ** 2, L, block)
        if prev is not None:
            assert np.all(nb <= prev * (1 + 1e-12))
        prev = nb
        # y stays on the solved blocks
        assert np.max(np.abs(y * S.colour_mask(L, block, 1)[..., None, None])) == 0.0


def test_mr_one_step_exact_on_unit_blocks():
    L = (4, 4, 2, 2)
    block = (1, 1, 1, 1)
    U = _system(L, 0.9, 2)
    m0 = 0.25
    r = synth.gaussian_spinor(L, 4) * S.colour_mask(L, block, 1)[..., None, None]
    y, rho = S.mr_blocks(U, m0, L, block, r, 1)
    assert np.max(np.abs(y - r / (4 + m0))) < 1e-15
    assert np.max(np.abs(rho)) < 1e-15


def test_mr_converges_to_dense_block_solve():
    L = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = _system(L, 0.3, 3)
    m0 = 0.5            # field of values of D^l well away from 0
    mask = S.single_block_mask(L, block, (2, 0, 2, 0))
    r = synth.gaussian_spinor(L, 5) * mask[..., None, None]
    y, _ = S.mr_blocks(U, m0, L, block, r, 80)
    Dl = W.dense_D(U, m0, block=block)
    idx = np.flatnonzero(np.repeat(mask.reshape(-1), 12))
    ys = np.linalg.solve(Dl[np.ix_(idx, idx)], r.reshape(-1)[idx])
    assert np.max(np.abs(y.reshape(-1)[idx] - ys)) < 1e-12 * np.max(np.abs(ys))


def _colour_perm(L, block):
    c0 = np.repeat(S.colour_mask(L, block, 0).reshape(-1), 12)
    return np.concatenate([np.flatnonzero(c0), np.flatnonzero(~c0)]), int(c0.sum())


@pytest.mark.parametrize("s", [1, 2, 3])
def test_sap_exact_equals_splitting_series(s):
    L = (4, 4, 2, 4)
    block = (2, 2, 1, 2)
    U = _system(L, 0.5, 4)
    m0 = -0.2
    D = W.dense_D(U, m0)
    Dl = W.dense_D(U, m0, block=block)      # block diagonal part, for exact solves
    perm, n0 = _colour_perm(L, block)
    Dp = D[np.ix_(perm, perm)]
    M = S.splitting_series(Dp, n0, s)
    v = synth.gaussian_spinor(L, 8)

    def exact(r, colour):
        y = np.zeros(r.size, complex)
        mask = np.repeat(S.colour_mask(L, block, colour).reshape(-1), 12)
        idx = np.flatnonzero(mask)
        y[idx] = np.linalg.solve(Dl[np.ix_(idx, idx)], r.reshape(-1)[idx])
        return y.reshape(r.shape)

    z = S.sap(U, m0, L, block, s, 0, v, block_solver=exact)
    zp = M @ v.reshape(-1)[perm]
    assert np.max(np.abs(z.reshape(-1)[perm] - zp)) < 1e-12 * np.max(np.abs(zp))
    # more cycles of exact SAP converge to D^{-1} v when SAP converges here
    if s == 3:
        xs = np.linalg.solve(D, v.reshape(-1))
        e3 = np.linalg.norm(z.reshape(-1) - xs)
        z1 = S.sap(U, m0, L, block, 1, 0, v, block_solver=exact)
        assert e3 < np.linalg.norm(z1.reshape(-1) - xs)


def test_unit_blocks_closed_form():
    L = (4, 2, 2, 4)
    block = (1, 1, 1, 1)
    U = _system(L, 0.8, 5)
    m0 = 0.1
    v = synth.gaussian_spinor(L, 9)
    z = S.sap(U, m0, L, block, 1, 1, v)
    e = S.colour_mask(L, block, 0)[..., None, None]
    o = ~e
    ze = v * e / (4 + m0)
    zo = (v - W.apply_D(U, m0, ze)) * o / (4 + m0)
    assert np.max(np.abs(z - (ze + zo))) < 1e-14


def test_alg1_any_order_equals_alg2():
    L = (8, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = _system(L, 0.6, 6)
    m0 = -0.1
    v = synth.gaussian_spinor(L, 10)
    z2 = S.sap(U, m0, L, block, 2, 3, v)
    blocks = S.block_list(L, block)
    rng = np.random.default_rng(0)
    c0 = [o for c, o in blocks if c == 0]
    c1 = [o for c, o in blocks if c == 1]
    for _ in range(2):
        order = list(rng.permutation(len(c0)))
        order1 = list(rng.permutation(len(c1)))
        seq = [c0[i] for i in order] + [c1[i] for i in order1]
        z1 = S.multiplicative_schwarz(U, m0, L, block, 2, 3, v, seq)
        assert np.max(np.abs(z1 - z2)) < 1e-13 * np.max(np.abs(z2))
    # an order that interleaves colours is a different method
    inter = [o for pair in zip(c1, c0) for o in pair]
    z3 = S.multiplicative_schwarz(U, m0, L, block, 2, 3, v, inter)
    assert np.max(np.abs(z3 - z2)) > 1e-6


def test_sap_scale_equivariance_and_gauge_covariance():
    L = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = _system(L, 0.6, 7)
    m0 = -0.05
    v = synth.gaussian_spinor(L, 11)
    z = S.sap(U, m0, L, block, 2, 4, v)
    a = 0.3 - 1.7j
    za = S.sap(U, m0, L, block, 2, 4, a * v)
    assert np.max(np.abs(za - a * z)) < 1e-13 * np.max(np.abs(za))
    Om = synth.haar_su3_field(L, seed=7)
    UO = np.empty_like(U)
    for mu in range(4):
        Omf = np.roll(Om, -1, axis=W.AXIS[mu])
        UO[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Omf, -1, -2))
    rot = lambda f: np.einsum("...ab,...sb->...sa", Om, f)
    zO = S.sap(UO, m0, L, block, 2, 4, rot(v))
    assert np.max(np.abs(zO - rot(z))) < 1e-13 * np.max(np.abs(zO)) * 10
