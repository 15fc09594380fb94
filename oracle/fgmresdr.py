"""Flexible GMRES with deflated restarts (FGMRES-DR), FP64 NumPy oracle.

Test infrastructure only. Follows the paper's Section 4:
  * flexible Arnoldi process (Alg. 3), keeping the preconditioned vectors
    z_j = M_j v_j; the new vector A z_j is made orthogonal to v_1..v_j by
    projection, repeated once (the listing orthogonalises one basis vector
    at a time; in exact arithmetic every Gram-Schmidt variant yields the
    same coefficients h_{i,j}, and the repeated projection keeps V
    orthonormal to FP64 rounding);
  * flexible Arnoldi relation A Z_m = V_{m+1} H^_m and the small least
    squares problem for the iterate (Section 4.2);
  * harmonic Ritz pairs from H_m + f_m h_m^H with H_m^H f_m = h_m
    (Lemma 1a) and the deflated restart of Section 4.4: G_{k+1} built from
    the k Ritz vectors of smallest-modulus harmonic Ritz values and the
    small residual c - H^ eta, its QR factorisation, H^_k = Q^H H^ Q_k,
    V_{k+1} = V Q_{k+1}, Z_k = Z Q_k (Alg. 4 and Section 4.5);
  * explicit FP64 residual once per cycle, injected into the right-hand
    side c = [V_{k+1}^H r; 0], and a clean restart (no deflation) when
    ||r_explicit|| / ||r_implicit|| > t (Section 4.7);
  * optionally (``inject``) the explicit residual also enters G_{k+1} in
    place of the small residual c - H^ eta (as V_{m+1}^H r), and becomes the
    last vector v_{k+1} after orthonormalisation against the rotated V_k,
    as Section 4.7 does for its low-precision Arnoldi;
  * optionally (``A_low``) the low-precision Arnoldi of Section 4.7: the
    bases V and Z are stored in single precision, w = A z_j comes from the
    low-precision operator A_low on the stored z_j and is orthogonalised in
    single-precision arithmetic; the iterate, the explicit residual, its
    injection and the small dense problems stay in double precision.

Readings taken where the paper is silent:
  * m is the total basis size including the k deflation vectors; cycles
    after the first perform m - k new Arnoldi steps;
  * one iteration = one flexible Arnoldi step (one M and one A product);
  * x0 = 0; the solve stops when the explicit residual satisfies
    ||b - A x|| <= tol ||b||; a cycle ends early once the implicit residual
    (from the small least-squares problem) reaches tol ||b||;
  * h_{j+1,j} <= 1e-14 ||H^|| is a breakdown that ends the cycle;
  * a singular H_m, a cycle too short to deflate (fewer than k + 1 steps)
    or a non-finite value leads to a clean restart;
  * harmonic Ritz values are ordered by modulus with a stable sort;
  * the injected v_{k+1} takes the phase of the rotated v_{k+1} it replaces
    (the paper leaves the phase open; this choice keeps the coefficients of
    A Z_k = V_{k+1} H^_k), orthogonalised by classical Gram-Schmidt with a
    second pass; a zero or non-finite result keeps the rotated vector.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg


@dataclasses.dataclass
class SolveInfo:
    converged: bool
    iterations: int
    cycles: int
    clean_restarts: int
    true_relres: float
    implicit_relres: float
    history: list            # (iteration, implicit relative residual) per Arnoldi step
    cycle_ends: list         # (iteration, explicit relative residual) per cycle
    ritz_values: np.ndarray  # harmonic Ritz values of the last restart (sorted by modulus)


def _lsq(H, c):
    """eta = argmin ||c - H eta||; returns (eta, ||c - H eta||)."""
    eta = np.linalg.lstsq(H, c, rcond=None)[0]
    return eta, float(np.linalg.norm(c - H @ eta))


def harmonic_ritz(Hhat):
    """Harmonic Ritz pairs from H^ = [H_m; h_m^H] (Lemma 1a).

    Returns (lam, G) sorted by |lam| ascending (stable), eigenvectors in the
    columns of G.
    """
    mm = Hhat.shape[1]
    Hm = Hhat[:mm, :]
    hrow = Hhat[mm, :]                       # this row is h_m^H
    f = np.linalg.solve(Hm.conj().T, hrow.conj())  # H_m^H f = h_m
    lam, G = scipy.linalg.eig(Hm + np.outer(f, hrow))
    order = np.argsort(np.abs(lam), kind="stable")
    return lam[order], G[:, order]


def injected_vector(Vk, v_old, r):
    """The explicit residual r orthonormalised against Vk (classical
    Gram-Schmidt, two passes), with the phase of v_old (Section 4.7).
    Returns v_old when r lies in span(Vk) (||w|| <= 1e-12 ||r||), or w is
    orthogonal to v_old, or a value is not finite."""
    w = r.copy()
    for _ in range(2):
        w = w - Vk @ (Vk.conj().T @ w)
    wn = float(np.linalg.norm(w))
    p = np.vdot(w, v_old)
    if wn > 1e-12 * np.linalg.norm(r) and abs(p) > 0.0 and np.isfinite(wn) and np.isfinite(p):
        return (p / abs(p)) * w / wn
    return v_old


def project_out(Vj, w):
    """Coefficients and remainder of w against the orthonormal columns of Vj.

    Returns (h, w') with w = Vj h + w' and Vj^H w' = 0 (to rounding): the
    projection h = Vj^H w, w' = w - Vj h is applied twice and the two
    coefficient vectors are summed.
    """
    h = np.zeros(Vj.shape[1], dtype=np.complex128)
    for _ in range(2):
        g = Vj.conj().T @ w
        w = w - Vj @ g
        h = h + g
    return h, w


def arnoldi_step(A, M, V, Z, H, j):
    """One flexible Arnoldi step (Alg. 3) on column j (0-based): the
    preconditioned vector z_j = M_j v_j is kept, w = A z_j gives the new
    Hessenberg column H[:j+1, j] by projection onto v_1..v_{j+1} and
    h_{j+2,j+1} = ||w'|| (0-based H[j+1, j]). Returns the remainder w';
    the caller normalises it into v_{j+2} unless the step broke down."""
    Z[:, j] = M(V[:, j])
    h, w = project_out(V[:, :j + 1], A(Z[:, j]))
    H[:j + 1, j] = h
    H[j + 1, j] = np.linalg.norm(w)
    return w


def flexible_arnoldi(A, M, b, m):
    """Alg. 3: m steps from v_1 = b/||b||. Returns (V, Z, H) with
    A Z = V H (the flexible Arnoldi relation of Section 4.2)."""
    n = b.size
    V = np.zeros((n, m + 1), dtype=np.complex128)
    Z = np.zeros((n, m), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        w = arnoldi_step(A, M, V, Z, H, j)
        V[:, j + 1] = w / H[j + 1, j]
    return V, Z, H


def fgmresdr(A, M, b, m, k, tol=1e-10, max_iter=10000, t_clean=5.0,
             breakdown_tol=1e-14, keep_basis=False, inject=False, A_low=None):
    """Solve A x = b by FGMRES-DR(m, k) (Alg. 4) from x0 = 0.

    A, M: callables on flat complex vectors. M may change from call to call
    (flexible preconditioning). A_low (optional): the low-precision
    operator, a callable on complex64 vectors returning complex64; given,
    the Arnoldi process runs in single precision (Section 4.7). Returns
    (x, SolveInfo) and, with ``keep_basis``, also (V, Z, H^) of the last
    cycle, cut to the steps that cycle performed.
    """
    if not (0 <= k < m):
        raise ValueError("need 0 <= k < m")
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n, dtype=np.complex128)
    r = b.copy()
    # basis storage: assignments into single-precision arrays round to them
    basis = np.complex64 if A_low is not None else np.complex128
    A_arnoldi = A_low if A_low is not None else A
    V = np.zeros((n, m + 1), dtype=basis)
    Z = np.zeros((n, m), dtype=basis)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    c = np.zeros(m + 1, dtype=np.complex128)
    iters = cycles = clean = 0
    history, cycle_ends = [], []
    ritz = np.zeros(0, dtype=np.complex128)
    fresh = True
    res_e = bnorm
    res_i = bnorm
    if bnorm == 0.0:
        return x, SolveInfo(True, 0, 0, 0, 0.0, 0.0, [], [], ritz)

    while True:
        if fresh:
            beta = float(np.linalg.norm(r))
            V[:] = 0.0
            Z[:] = 0.0
            H[:] = 0.0
            c[:] = 0.0
            V[:, 0] = r / beta
            c[0] = beta
            j0 = 0
        else:
            j0 = k
        jend = j0
        broke = False
        # flexible Arnoldi steps j0 .. m-1 (0-based column index)
        for j in range(j0, m):
            w = arnoldi_step(A_arnoldi, M, V, Z, H, j)
            iters += 1
            jend = j + 1
            hnorm = np.linalg.norm(H[:j + 2, :j + 1])
            broke = bool(abs(H[j + 1, j]) <= breakdown_tol * hnorm)
            if not broke:
                V[:, j + 1] = w / H[j + 1, j]
            _, ri = _lsq(H[:j + 2, :j + 1], c[:j + 2])
            history.append((iters, ri / bnorm))
            if broke or ri <= tol * bnorm or iters >= max_iter:
                break
        # iterate and explicit residual for this cycle
        Hc = H[:jend + 1, :jend]
        eta, res_i = _lsq(Hc, c[:jend + 1])
        x = x + Z[:, :jend] @ eta
        r = b - A(x)
        res_e = float(np.linalg.norm(r))
        cycles += 1
        cycle_ends.append((iters, res_e / bnorm))
        if res_e <= tol * bnorm:
            return _finish(x, True, iters, cycles, clean, res_e, res_i, bnorm,
                           history, cycle_ends, ritz, keep_basis, V, Z, H, jend)
        if iters >= max_iter:
            return _finish(x, False, iters, cycles, clean, res_e, res_i, bnorm,
                           history, cycle_ends, ritz, keep_basis, V, Z, H, jend)
        if k == 0:
            fresh = True          # plain restarted FGMRES(m)
            continue
        # clean restart when explicit and implicit residual disagree (Section 4.7)
        if broke or jend <= k or res_e > t_clean * max(res_i, 1e-300):
            clean += 1
            fresh = True
            continue
        # deflated restart (Section 4.4/4.5)
        try:
            lam, G = harmonic_ritz(Hc)
        except np.linalg.LinAlgError:
            clean += 1
            fresh = True
            continue
        if not np.all(np.isfinite(lam)) or not np.all(np.isfinite(G)):
            clean += 1
            fresh = True
            continue
        ritz = lam
        Gk1 = np.zeros((jend + 1, k + 1), dtype=np.complex128)
        Gk1[:jend, :k] = G[:, :k]
        if inject:
            Gk1[:, k] = V[:, :jend + 1].conj().T @ r
        else:
            Gk1[:, k] = c[:jend + 1] - Hc @ eta
        Q, _ = np.linalg.qr(Gk1)
        Qk = Q[:jend, :k]
        Hk = Q.conj().T @ Hc @ Qk
        V[:, :k + 1] = V[:, :jend + 1] @ Q
        Z[:, :k] = Z[:, :jend] @ Qk
        if inject:
            V[:, k] = injected_vector(V[:, :k], V[:, k], r)
        V[:, k + 1:] = 0.0
        Z[:, k:] = 0.0
        H[:] = 0.0
        H[:k + 1, :k] = Hk
        c[:] = 0.0
        c[:k + 1] = V[:, :k + 1].conj().T @ r
        fresh = False


def _finish(x, conv, iters, cycles, clean, res_e, res_i, bnorm, history,
            cycle_ends, ritz, keep_basis, V, Z, H, jend):
    info = SolveInfo(conv, iters, cycles, clean, res_e / bnorm, res_i / bnorm,
                     history, cycle_ends, ritz)
    if keep_basis:
        return x, info, (V[:, :jend + 1], Z[:, :jend], H[:jend + 1, :jend])
    return x, info
