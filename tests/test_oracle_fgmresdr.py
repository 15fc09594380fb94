"""Pins of the oracle's FGMRES-DR (Alg. 3, Alg. 4) against properties the
paper and the mathematics fix:

  * the flexible Arnoldi relation A Z = V H^ and orthonormal V (eq. for the
    flexible Arnoldi relation), also for a preconditioner that changes at
    every call;
  * the minimal-residual property of an FGMRES cycle, checked by brute
    force (explicit A Z and a dense least-squares solve; for M = I, the
    explicit Krylov matrix [b, Ab, ...]);
  * Definition 1 of harmonic Ritz pairs, checked directly with explicit A
    products, and Lemma 1b (all harmonic Ritz residuals are parallel to
    the GMRES residual);
  * after deflated restarts, A Z = V H^ still holds with the dense leading
    (k+1) x k block (eq. for H^_k);
  * GMRES-DR (M = I) harmonic Ritz values converge to the smallest-modulus
    eigenvalues of a dense D;
  * clean restarts at every cycle reduce FGMRES-DR to FGMRES(m);
  * a happy breakdown for an eigenvector right-hand side;
  * the converged solution against dense LU, gauge covariance of the whole
    solve, and non-convergence reporting;
  * the injected v_{k+1} (Section 4.7): unit, orthogonal to V_k, r in
    span(V_k, v_{k+1}), phase of the replaced vector; with an exact Arnoldi
    the injected solve follows the plain one to rounding.
"""
import numpy as np
import pytest

import synth
from oracle import fgmresdr as F
from oracle import sap as S
from oracle import wilson as W


def _ops(L, eps, seed, m0, block=(2, 2, 2, 2), ncyc=1, nmr=4):
    U = synth.gauge_field(L, eps, seed)
    shp = synth.lattice_shape(L) + (4, 3)
    A = lambda v: W.apply_D(U, m0, v.reshape(shp)).reshape(-1)
    M = lambda v: S.sap(U, m0, L, block, ncyc, nmr, v.reshape(shp)).reshape(-1)
    return U, A, M


def test_flexible_arnoldi_relation():
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.1)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    V, Z, H = F.flexible_arnoldi(A, M, b, 10)
    AZ = np.stack([A(Z[:, j]) for j in range(10)], axis=1)
    assert np.linalg.norm(AZ - V @ H) < 1e-13 * np.linalg.norm(H)
    assert np.linalg.norm(V.conj().T @ V - np.eye(11)) < 1e-11  # two projection passes keep V orthonormal
    assert np.all(np.tril(H, -2) == 0)


def test_flexible_arnoldi_varying_preconditioner():
    L = (4, 4, 2, 4)
    U, A, _ = _ops(L, 0.3, 0, 0.0, block=(2, 2, 1, 2))
    rng = np.random.default_rng(1)
    n = 12 * synth.volume(L)

    def M(v):  # a different diagonal preconditioner at every call
        return v * (0.5 + rng.random(n))

    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    V, Z, H = F.flexible_arnoldi(A, M, b, 8)
    AZ = np.stack([A(Z[:, j]) for j in range(8)], axis=1)
    assert np.linalg.norm(AZ - V @ H) < 1e-13 * np.linalg.norm(H)
    x, info = F.fgmresdr(A, M, b, 8, 3, tol=1e-10, max_iter=2000)
    assert info.converged and info.true_relres <= 1e-10
    assert np.linalg.norm(b - A(x)) <= 1e-10 * np.linalg.norm(b)


def test_cycle_minimal_residual_brute_force():
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.1)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    m = 8
    x, info, (V, Z, H) = F.fgmresdr(A, M, b, m, 0, tol=1e-30, max_iter=m, keep_basis=True)
    AZ = np.stack([A(Z[:, j]) for j in range(m)], axis=1)
    eta = np.linalg.lstsq(AZ, b, rcond=None)[0]
    assert np.linalg.norm(x - Z @ eta) < 1e-10 * np.linalg.norm(x)
    # M = I: the search space is the Krylov space span{b, Ab, ..., A^{m-1} b}
    ident = lambda v: v.copy()
    x1, _ = F.fgmresdr(A, ident, b, m, 0, tol=1e-30, max_iter=m)
    K = [b / np.linalg.norm(b)]
    for _ in range(m - 1):
        w = A(K[-1])
        K.append(w / np.linalg.norm(w))
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    AQ = np.stack([A(Q[:, j]) for j in range(m)], axis=1)
    y = np.linalg.lstsq(AQ, b, rcond=None)[0]
    assert np.linalg.norm(x1 - Q @ y) < 1e-9 * np.linalg.norm(x1)


def test_harmonic_ritz_definition_and_lemma1b():
    L = (4, 4, 2, 4)
    U, A, M = _ops(L, 0.4, 2, -0.1, block=(2, 2, 1, 2))
    b = synth.gaussian_spinor(L, 1001).reshape(-1)
    m = 12
    # M = I: Definition 1 directly, A u - lam u orthogonal to A K_m
    ident = lambda v: v.copy()
    V, Z, H = F.flexible_arnoldi(A, ident, b, m)
    lam, G = F.harmonic_ritz(H)
    AV = np.stack([A(V[:, j]) for j in range(m)], axis=1)
    for i in range(m):
        u = V[:, :m] @ G[:, i]
        res = A(u) - lam[i] * u
        assert np.linalg.norm(AV.conj().T @ res) < 1e-10 * np.linalg.norm(AV) * np.linalg.norm(u)
    assert np.all(np.diff(np.abs(lam)) >= 0)
    # flexible case, Lemma 1b: V_{m+1}(H^ g - lam [g; 0]) is parallel to the
    # GMRES residual V_{m+1}(c - H^ eta)
    V, Z, H = F.flexible_arnoldi(A, M, b, m)
    lam, G = F.harmonic_ritz(H)
    c = np.zeros(m + 1, complex)
    c[0] = np.linalg.norm(b)
    eta = np.linalg.lstsq(H, c, rcond=None)[0]
    rs = c - H @ eta
    for i in range(m):
        d = H @ G[:, i] - lam[i] * np.concatenate([G[:, i], [0]])
        cos = abs(np.vdot(rs, d)) / (np.linalg.norm(rs) * np.linalg.norm(d))
        assert abs(cos - 1) < 1e-9


def test_deflated_restart_keeps_arnoldi_relation():
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.21)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    m, k = 20, 5
    # stop after several deflated cycles
    x, info, (V, Z, H) = F.fgmresdr(A, M, b, m, k, tol=1e-30, max_iter=20 + 3 * 15, keep_basis=True)
    assert info.cycles == 4 and info.clean_restarts == 0
    AZ = np.stack([A(Z[:, j]) for j in range(Z.shape[1])], axis=1)
    assert np.linalg.norm(AZ - V @ H) < 1e-12 * np.linalg.norm(H)
    assert np.linalg.norm(V.conj().T @ V - np.eye(V.shape[1])) < 1e-10
    # the leading (k+1) x k block is dense, the rest is Hessenberg
    assert np.count_nonzero(np.abs(H[:k + 1, :k]) > 1e-14) > (k + 1) * k // 2
    assert np.all(H[k + 1:, :k] == 0)
    assert np.all(np.tril(H[:, k:], -(k + 2)) == 0)
    # explicit residuals are non-increasing from cycle to cycle
    res = [r for _, r in info.cycle_ends]
    assert all(res[i + 1] <= res[i] * (1 + 1e-10) for i in range(len(res) - 1))
    # implicit residuals are non-increasing within the run
    h = [r for _, r in info.history]
    assert all(h[i + 1] <= h[i] * (1 + 1e-8) for i in range(len(h) - 1))


def test_gmres_dr_ritz_values_match_dense_eigenvalues():
    L = (2, 2, 2, 4)
    U = synth.gauge_field(L, 0.5, 3)
    m0 = -0.49            # leftmost eigenvalue of D(0) is 0.609 - 0.062i here
    D = W.dense_D(U, m0)
    ev = np.linalg.eigvals(D)
    ev = ev[np.argsort(np.abs(ev))]
    A = lambda v: D @ v
    ident = lambda v: v.copy()
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    k = 6
    x, info = F.fgmresdr(A, ident, b, 16, k, tol=1e-13, max_iter=3000)
    assert info.converged and info.cycles > 10
    got = info.ritz_values[:k]
    err = [np.min(np.abs(ev[:10] - g)) / np.abs(ev[0]) for g in got]
    # the smallest pair has converged, the others are close
    assert max(err[:2]) < 1e-4
    assert max(err) < 2e-3


def test_clean_restart_every_cycle_is_fgmres():
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.1)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    x0, i0 = F.fgmresdr(A, M, b, 8, 0, tol=1e-8, max_iter=400)
    x1, i1 = F.fgmresdr(A, M, b, 8, 3, tol=1e-8, max_iter=400, t_clean=0.5)
    assert i1.clean_restarts == i1.cycles - 1 and i0.clean_restarts == 0
    assert i0.iterations == i1.iterations
    h0 = np.array([r for _, r in i0.history])
    h1 = np.array([r for _, r in i1.history])
    assert np.max(np.abs(h0 - h1) / h0) < 1e-8
    assert np.linalg.norm(x0 - x1) < 1e-10 * np.linalg.norm(x0)


def test_happy_breakdown_on_eigenvector():
    L = (4, 4, 2, 4)
    U = synth.unit_gauge_field(L)
    m0 = 0.2
    shp = synth.lattice_shape(L) + (4, 3)
    A = lambda v: W.apply_D(U, m0, v.reshape(shp)).reshape(-1)
    ident = lambda v: v.copy()
    # zero momentum: D = m0 on constant spinors
    b = np.ones(shp, complex).reshape(-1)
    x, info = F.fgmresdr(A, ident, b, 10, 3, tol=1e-12)
    assert info.converged and info.iterations == 1
    assert np.allclose(x, b / m0)


def test_solution_matches_dense_lu_and_gauge_covariance():
    L = (4, 4, 2, 4)
    block = (2, 2, 1, 2)
    m0 = -0.15
    U, A, M = _ops(L, 0.4, 5, m0, block=block)
    b = synth.gaussian_spinor(L, 1002)
    x, info = F.fgmresdr(A, M, b.reshape(-1), 12, 4, tol=1e-12, max_iter=2000)
    assert info.converged and info.true_relres <= 1e-12
    xs = np.linalg.solve(W.dense_D(U, m0), b.reshape(-1))
    assert np.linalg.norm(x - xs) < 1e-9 * np.linalg.norm(xs)
    Om = synth.haar_su3_field(L, seed=7)
    UO = np.empty_like(U)
    for mu in range(4):
        Omf = np.roll(Om, -1, axis=W.AXIS[mu])
        UO[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Omf, -1, -2))
    shp = synth.lattice_shape(L) + (4, 3)
    rot = lambda f: np.einsum("...ab,...sb->...sa", Om, f.reshape(shp))
    AO = lambda v: W.apply_D(UO, m0, v.reshape(shp)).reshape(-1)
    MO = lambda v: S.sap(UO, m0, L, block, 1, 4, v.reshape(shp)).reshape(-1)
    xO, infoO = F.fgmresdr(AO, MO, rot(b).reshape(-1), 12, 4, tol=1e-12, max_iter=2000)
    assert np.linalg.norm(xO - rot(x).reshape(-1)) < 1e-9 * np.linalg.norm(xO)
    assert abs(infoO.iterations - info.iterations) <= 1


def test_deflation_beats_plain_restart_near_critical():
    # qualitative claim of the paper (Section 5), on a synthetic field
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.222)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    _, i5 = F.fgmresdr(A, M, b, 20, 5, tol=1e-8, max_iter=3000)
    assert i5.converged
    # without deflation, twice as many iterations do not reach the tolerance
    _, i0 = F.fgmresdr(A, M, b, 20, 0, tol=1e-8, max_iter=2 * i5.iterations)
    assert not i0.converged and i0.true_relres > 10 * i5.true_relres


def test_nonconvergence_is_reported():
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.1)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    x, info = F.fgmresdr(A, M, b, 10, 3, tol=1e-10, max_iter=7)
    assert not info.converged and info.iterations == 7
    assert 1e-10 < info.true_relres < 1.0
    with pytest.raises(ValueError):
        F.fgmresdr(A, M, b, 5, 5)


def test_injected_vector_properties():
    rng = np.random.default_rng(5)
    n, k = 60, 5
    Q, _ = np.linalg.qr(rng.standard_normal((n, k + 1)) + 1j * rng.standard_normal((n, k + 1)))
    Vk, v_old = Q[:, :k], Q[:, k]
    # r in span(V_k, v_old) plus a small perturbation, as after a drift
    r = Vk @ (rng.standard_normal(k) + 1j * rng.standard_normal(k)) + (0.7 - 0.4j) * v_old
    r = r + 1e-3 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    v = F.injected_vector(Vk, v_old, r)
    assert abs(np.linalg.norm(v) - 1) < 1e-14
    assert np.max(np.abs(Vk.conj().T @ v)) < 1e-14
    Vn = np.concatenate([Vk, v[:, None]], axis=1)
    assert np.linalg.norm(r - Vn @ (Vn.conj().T @ r)) < 1e-13 * np.linalg.norm(r)
    p = np.vdot(v, v_old)
    assert abs(p.imag) < 1e-14 and p.real > 0.99
    # r in span(V_k): the rotated vector is kept
    assert np.array_equal(F.injected_vector(Vk, v_old, Vk @ np.ones(k)), v_old)


def test_injection_follows_plain_solve_in_fp64():
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.21)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    x0, i0 = F.fgmresdr(A, M, b, 20, 5, tol=1e-10)
    x1, i1 = F.fgmresdr(A, M, b, 20, 5, tol=1e-10, inject=True)
    assert i0.converged and i1.converged and i0.cycles >= 3
    assert abs(i0.iterations - i1.iterations) <= 1 and i1.clean_restarts == i0.clean_restarts
    h0 = np.array([r for _, r in i0.history])
    h1 = np.array([r for _, r in i1.history])
    nh = min(len(h0), len(h1))
    assert np.max(np.abs(h0[:nh] - h1[:nh]) / h0[:nh]) < 1e-6
    assert np.linalg.norm(x0 - x1) < 1e-9 * np.linalg.norm(x0)



def _low_op(U, m0, shp):
    """The operator on single-precision links and vectors, result rounded to single."""
    U32 = U.astype(np.complex64)
    return lambda v: W.apply_D(U32, m0, np.asarray(v, dtype=np.complex64).reshape(shp)).reshape(-1).astype(
        np.complex64)


def test_low_precision_arnoldi_is_single_precision():
    """With A_low the Arnoldi basis is single precision: V is orthonormal and
    A_low Z = V H^ holds only to single-precision rounding (not to double)."""
    L = (4, 4, 4, 4)
    U, A, M = _ops(L, 0.3, 0, -0.1)
    shp = synth.lattice_shape(L) + (4, 3)
    Al = _low_op(U, -0.1, shp)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    _, info, (V, Z, H) = F.fgmresdr(A, M, b, 12, 0, tol=1e-30, max_iter=12, keep_basis=True, A_low=Al)
    assert V.dtype == np.complex64 and Z.dtype == np.complex64
    V64, Z64 = V.astype(np.complex128), Z.astype(np.complex128)
    orth = np.linalg.norm(V64.conj().T @ V64 - np.eye(V.shape[1]))
    assert 1e-9 < orth < 1e-5, orth
    AZ = np.stack([A(Z64[:, j]) for j in range(Z.shape[1])], axis=1)
    rel = np.linalg.norm(AZ - V64 @ H) / np.linalg.norm(H)
    assert 1e-10 < rel < 1e-5, rel


def test_low_precision_arnoldi_with_injection_reaches_fp64_residual():
    """Section 4.7: a single-precision Arnoldi with the explicit FP64 residual
    entering each restart (c, G_{k+1}, v_{k+1}) still reaches a 1e-10 true
    residual in FP64, in about the iterations of the double-precision solve;
    the solution agrees with dense LU within the conditioning bound."""
    L = (4, 4, 4, 4)
    m0 = -0.1
    U, A, M = _ops(L, 0.3, 0, m0)
    shp = synth.lattice_shape(L) + (4, 3)
    Al = _low_op(U, m0, shp)
    b = synth.gaussian_spinor(L, 1000).reshape(-1)
    x64, i64 = F.fgmresdr(A, M, b, 8, 3, tol=1e-10, max_iter=400)
    x32, i32 = F.fgmresdr(A, M, b, 8, 3, tol=1e-10, max_iter=400, inject=True, A_low=Al)
    assert i64.converged and i32.converged
    assert np.linalg.norm(b - A(x32)) <= 1e-10 * np.linalg.norm(b)
    assert i32.iterations <= 1.5 * i64.iterations + 8, (i32.iterations, i64.iterations)
    Dd = W.dense_D(U, m0)
    xs = np.linalg.solve(Dd, b)
    assert np.linalg.norm(x32 - xs) <= 1e-8 * np.linalg.norm(xs)
