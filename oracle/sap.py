"""Schwarz alternating procedure (SAP) and minimal-residual block solves.

FP64 NumPy oracle, test infrastructure only.

Follows the paper:
  * Alg. 1 (Section 2): sequential multiplicative Schwarz over the domains;
  * Alg. 2 (Section 2): SAP, all blocks of one colour, then the other;
  * Section 3: inexact block solves by a fixed number of minimal-residual
    (MR) steps, independent of the accuracy reached (as in the experiments
    of Section 5), or, adaptively, until the block residual has dropped by
    a given factor (the factor 10 of Section 3), block by block;
  * Section 3 and Fig. 5: SAP iterated on its own as a solver, which
    converges for heavy masses and diverges near the critical one;
  * Section 4: with exact block solves, s SAP cycles from a zero start give
    the truncated series M_s = sum_{j<s} (A_L^{-1} A_U)^j A_L^{-1} of the
    block splitting D = A_L - A_U (the printed formula lacks the power j;
    the splitting makes it clear that the j-th power is meant).

Readings of the paper taken here:
  * "replace part x^l in x by y^l" is the additive correction x^l += y^l,
    because y^l solves the block system for the residual r^l = (b - D x)^l;
  * colour 0 is the set of blocks whose block coordinates have an even sum
    (it contains the block at the origin) and is processed first;
  * MR starts from y = 0, uses alpha = (p^H rho)/(p^H p) over the block's
    sites (alpha = 0 if p = 0) and no relaxation;
  * the adaptive inexact solve tests ||rho_n|| <= delta ||r^l|| before each
    step n = 0, 1, ..., stops the block at the first n that passes, and
    never takes more than n_MR steps;
  * the stand-alone SAP solver starts from x = 0 and each iteration applies
    s cycles to the current residual: x_{k+1} = x_k + M_s (b - D x_k);
  * one SAP cycle = both colours once.

``C`` (optional) is a site-local 12x12 term added to the operator, the
clover term of ``oracle/clover.py``; being site-local it belongs to every
block operator D^l whole.
"""
from __future__ import annotations

import itertools

import numpy as np

from .wilson import apply_D, apply_D_blocks


def check_blocking(L, block):
    """The red/black argument needs an even number of blocks per direction."""
    for mu in range(4):
        if block[mu] <= 0 or L[mu] % block[mu] != 0:
            raise ValueError(f"block {block} does not tile lattice {L}")
        if (L[mu] // block[mu]) % 2 != 0:
            raise ValueError(f"odd number of blocks in direction {mu}")


def block_grid(L, block):
    return tuple(L[mu] // block[mu] for mu in range(4))


def colour_mask(L, block, colour):
    """Boolean site mask (t, z, y, x) of the blocks with the given colour."""
    Lx, Ly, Lz, Lt = L
    bx, by, bz, bt = block
    t = np.arange(Lt)[:, None, None, None] // bt
    z = np.arange(Lz)[None, :, None, None] // bz
    y = np.arange(Ly)[None, None, :, None] // by
    x = np.arange(Lx)[None, None, None, :] // bx
    return ((x + y + z + t) % 2) == colour


def block_sum(a, L, block):
    """Sum of a site field over each block: returns array (Nt, Nz, Ny, Nx)."""
    Lx, Ly, Lz, Lt = L
    bx, by, bz, bt = block
    r = a.reshape(Lt // bt, bt, Lz // bz, bz, Ly // by, by, Lx // bx, bx, *a.shape[4:])
    axes = (1, 3, 5, 7) + tuple(range(8, r.ndim))
    return r.sum(axis=axes)


def block_broadcast(s, L, block):
    """Inverse of block_sum's reduction: expand a per-block scalar to sites."""
    bx, by, bz, bt = block
    e = np.repeat(s, bt, axis=0)
    e = np.repeat(e, bz, axis=1)
    e = np.repeat(e, by, axis=2)
    e = np.repeat(e, bx, axis=3)
    return e


def block_norm(a, L, block):
    """Euclidean norm of a spinor field over each block: (Nt, Nz, Ny, Nx)."""
    return np.sqrt(block_sum(np.abs(a) ** 2, L, block))


def mr_blocks(U, m0, L, block, r, nmr, C=None, reduction=0.0):
    """n_MR minimal-residual steps for D^l y^l = r^l on every block at once.

    ``r`` must vanish outside the blocks being solved (the hop cut of D^l
    keeps blocks independent). Returns (y, rho) with rho = r - D^l y.
    ``reduction`` = delta > 0: a block stops before the first step n at
    which ||rho_n|| <= delta ||r^l|| (Section 3); n_MR is then the cap.
    """
    y = np.zeros_like(r)
    rho = r.copy()
    r_norm = block_norm(r, L, block)
    running = np.ones(r_norm.shape, dtype=bool)
    for _ in range(nmr):
        if reduction > 0.0:
            running &= ~(block_norm(rho, L, block) <= reduction * r_norm)
        p = apply_D_blocks(U, m0, rho, block, C)
        num = block_sum(np.conj(p) * rho, L, block)           # p^H rho per block
        den = block_sum(np.abs(p) ** 2, L, block).real          # p^H p per block
        alpha = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 0.0)
        alpha = np.where(running, alpha, 0.0)                   # stopped blocks keep y
        a = block_broadcast(alpha, L, block)[..., None, None]
        y = y + a * rho
        rho = rho - a * p
    return y, rho


def sap(U, m0, L, block, ncycles, nmr, v, block_solver=None, C=None, reduction=0.0):
    """z = M v: ``ncycles`` SAP cycles (Alg. 2) from z = 0.

    Per cycle and colour: r = (v - D z) on the blocks of that colour, block
    solves D^l y^l = r^l (n_MR MR steps, adaptive with ``reduction`` > 0, or
    ``block_solver`` if given), then z += y on those blocks.
    """
    check_blocking(L, block)
    z = np.zeros_like(v)
    masks = [colour_mask(L, block, c)[..., None, None] for c in (0, 1)]
    for _ in range(ncycles):
        for c in (0, 1):
            r = (v - apply_D(U, m0, z, C)) * masks[c]
            if block_solver is None:
                y, _ = mr_blocks(U, m0, L, block, r, nmr, C, reduction)
            else:
                y = block_solver(r, c) * masks[c]
            z = z + y
    return z


def sap_solve(U, m0, L, block, ncycles, nmr, b, niter, C=None, reduction=0.0, block_solver=None):
    """SAP as a stand-alone solver (Section 3, Fig. 5): x_0 = 0,
    x_{k+1} = x_k + M_s (b - D x_k) with M_s = ``ncycles`` SAP cycles.

    Returns (x_niter, [||b - D x_k|| / ||b|| for k = 0..niter]).
    """
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    hist = []
    for k in range(niter + 1):
        r = b - apply_D(U, m0, x, C)
        hist.append(np.linalg.norm(r) / bnorm)
        if k < niter:
            x = x + sap(U, m0, L, block, ncycles, nmr, r, block_solver, C, reduction)
    return x, hist


def block_list(L, block):
    """All blocks as (colour, origin) pairs, lexicographic in (t, z, y, x)."""
    N = block_grid(L, block)
    out = []
    for bt, bz, by, bx in itertools.product(range(N[3]), range(N[2]), range(N[1]), range(N[0])):
        out.append(((bx + by + bz + bt) % 2, (bx * block[0], by * block[1], bz * block[2], bt * block[3])))
    return out


def single_block_mask(L, block, origin):
    Lx, Ly, Lz, Lt = L
    m = np.zeros((Lt, Lz, Ly, Lx), dtype=bool)
    ox, oy, oz, ot = origin
    m[ot:ot + block[3], oz:oz + block[2], oy:oy + block[1], ox:ox + block[0]] = True
    return m


def multiplicative_schwarz(U, m0, L, block, ncycles, nmr, v, order):
    """Alg. 1: sequential sweep over single blocks in the given order
    (a list of block origins), each block using the freshest iterate."""
    check_blocking(L, block)
    z = np.zeros_like(v)
    for _ in range(ncycles):
        for origin in order:
            m = single_block_mask(L, block, origin)[..., None, None]
            r = (v - apply_D(U, m0, z)) * m
            y, _ = mr_blocks(U, m0, L, block, r, nmr)
            z = z + y * m
    return z


def splitting_series(Dperm, n0, s):
    """Dense M_s = sum_{j<s} (A_L^{-1} A_U)^j A_L^{-1} (Section 4).

    ``Dperm`` is D with the colour-0 unknowns first (n0 of them), then the
    colour-1 unknowns. A_L is the block lower-triangular part (with the
    diagonal blocks) and A_U = A_L - D.
    """
    A_L = Dperm.copy()
    A_L[:n0, n0:] = 0.0
    A_U = A_L - Dperm
    A_L_inv = np.linalg.inv(A_L)
    T = A_L_inv @ A_U
    M = np.zeros_like(Dperm)
    P = np.eye(Dperm.shape[0], dtype=Dperm.dtype)
    for _ in range(s):
        M = M + P @ A_L_inv
        P = T @ P
    return M
