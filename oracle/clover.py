"""Sheikholeslami-Wohlert (clover) term, FP64 NumPy oracle (test
infrastructure only).

The paper's experiments use the clover-improved Wilson operator. In the
mass normalisation of ``oracle.wilson`` it reads

    D_sw = D + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(n)
         = D + (i c_sw / 2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(n),

    sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
    F_{mu nu}(n)  = (Q_{mu nu}(n) - Q_{mu nu}(n)^dagger) / 8,

where Q_{mu nu}(n) is the sum of the four plaquettes in the (mu, nu) plane
that start and end at n (the "clover leaves"). F is anti-Hermitian and
sigma Hermitian, so the term is Hermitian; sigma commutes with gamma5 and,
in the chiral basis, is block diagonal in the two chiralities (spins 0, 1
and 2, 3). The term acts site by site, so the block operator D^l keeps it
whole.
"""
from __future__ import annotations

import numpy as np

from .wilson import AXIS, GAMMA


def _shift(A, mu, s):
    """A at n + s * mu (periodic)."""
    return np.roll(A, -s, axis=AXIS[mu])


def _dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def clover_leaves(U, mu, nu):
    """Q_{mu nu}(n): the four plaquettes of the (mu, nu) plane around n."""
    Um, Un = U[mu], U[nu]
    # n -> n+mu -> n+mu+nu -> n+nu -> n
    q = Um @ _shift(Un, mu, 1) @ _dag(_shift(Um, nu, 1)) @ _dag(Un)
    # n -> n+nu -> n+nu-mu -> n-mu -> n
    q = q + Un @ _dag(_shift(_shift(Um, mu, -1), nu, 1)) @ _dag(_shift(Un, mu, -1)) @ _shift(Um, mu, -1)
    # n -> n-mu -> n-mu-nu -> n-nu -> n
    q = q + (_dag(_shift(Um, mu, -1)) @ _dag(_shift(_shift(Un, mu, -1), nu, -1))
             @ _shift(_shift(Um, mu, -1), nu, -1) @ _shift(Un, nu, -1))
    # n -> n-nu -> n-nu+mu -> n+mu -> n
    q = q + _dag(_shift(Un, nu, -1)) @ _shift(Um, nu, -1) @ _shift(_shift(Un, mu, 1), nu, -1) @ _dag(Um)
    return q


def field_strength(U, mu, nu):
    """F_{mu nu}(n) = (Q - Q^dagger) / 8, a 3x3 anti-Hermitian matrix per site."""
    q = clover_leaves(U, mu, nu)
    return (q - _dag(q)) / 8.0


def sigma(mu, nu):
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def clover_term(U, csw):
    """The site-local 12x12 matrix per site, indexed [t, z, y, x, s, a, s', b]
    (spin s, colour a acting on spin s', colour b)."""
    shape = U.shape[1:5]
    C = np.zeros(shape + (4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            F = field_strength(U, mu, nu)
            C += (0.5j * csw) * np.einsum("st,...ab->...satb", sigma(mu, nu), F)
    return C


def apply_clover(C, x):
    """(C x)(n)_{s a} = sum_{t b} C(n)_{s a, t b} x(n)_{t b}."""
    return np.einsum("...satb,...tb->...sa", C, x)


def clover_at_sites(U, csw, sites):
    """The 12x12 clover matrix at a list of lexicographic sites, computed
    site by site from explicit link products (for lattices too large for
    ``clover_term``). Returns [len(sites), 4, 3, 4, 3]."""
    Lt, Lz, Ly, Lx = U.shape[1:5]
    ext = (Lx, Ly, Lz, Lt)

    def link(mu, c):
        x, y, z, t = (c[d] % ext[d] for d in range(4))
        return U[mu, t, z, y, x]

    def step(c, mu, s):
        c = list(c)
        c[mu] += s
        return c

    out = np.zeros((len(sites), 4, 3, 4, 3), dtype=np.complex128)
    for i, s in enumerate(sites):
        s = int(s)
        n = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]
        for mu in range(4):
            for nu in range(mu + 1, 4):
                a, b = step(n, mu, 1), step(n, nu, 1)
                c = step(n, mu, -1)
                d = step(c, nu, 1)
                f = step(c, nu, -1)
                h = step(n, nu, -1)
                k = step(h, mu, 1)
                q = link(mu, n) @ link(nu, a) @ _dag(link(mu, b)) @ _dag(link(nu, n))
                q = q + link(nu, n) @ _dag(link(mu, d)) @ _dag(link(nu, c)) @ link(mu, c)
                q = q + _dag(link(mu, c)) @ _dag(link(nu, f)) @ link(mu, f) @ link(nu, h)
                q = q + _dag(link(nu, h)) @ link(mu, h) @ link(nu, k) @ _dag(link(mu, n))
                F = (q - _dag(q)) / 8.0
                out[i] += (0.5j * csw) * np.einsum("st,ab->satb", sigma(mu, nu), F)
    return out
