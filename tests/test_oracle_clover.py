"""Pins of the oracle's clover term (``oracle/clover.py``) against facts that
do not come from its own formulas:

* free field and pure gauge: every plaquette is the identity, F = 0;
* a constant abelian magnetic field B in the (x, y) plane: every plaquette
  away from the x wrap is exp(iB) in the first two colours, so
  F_xy = i sin(B) diag(1, -1, 0) and all other planes vanish;
* sigma_xy = -diag(s3, s3) in the chiral basis (from gamma_x gamma_y = i diag(s3, s3));
* the term is Hermitian, commutes with gamma5 (no coupling between the
  chiralities), is gauge covariant, and D_sw stays gamma5-Hermitian.
"""
import numpy as np

import synth
from oracle import clover as Cl
from oracle import wilson as W

L = (4, 4, 4, 8)


def test_free_field_and_pure_gauge_vanish():
    U1 = synth.unit_gauge_field(L)
    assert np.count_nonzero(Cl.clover_term(U1, 1.7)) == 0
    Om = synth.haar_su3_field(L, 7)
    Ug = synth.pure_gauge_field(Om)
    assert np.max(np.abs(Cl.clover_term(Ug, 1.7))) < 1e-13


def test_sigma_xy_closed_form():
    s3 = np.diag([1.0, -1.0])
    expect = -np.kron(np.eye(2), s3)
    assert np.allclose(Cl.sigma(0, 1), expect, atol=0, rtol=0)


def test_constant_abelian_field():
    Lx, Ly, Lz, Lt = 8, 4, 4, 4
    B = 0.3
    U = synth.unit_gauge_field((Lx, Ly, Lz, Lt))
    x = np.arange(Lx)
    ph = np.exp(1j * B * x)
    Uy = np.zeros((Lx, 3, 3), dtype=np.complex128)
    Uy[:, 0, 0], Uy[:, 1, 1], Uy[:, 2, 2] = ph, np.conj(ph), 1.0
    U[1] = np.broadcast_to(Uy, (Lt, Lz, Ly, Lx, 3, 3))
    F = Cl.field_strength(U, 0, 1)
    inner = F[:, :, :, 1:Lx - 1]
    assert np.max(np.abs(inner - 1j * np.sin(B) * np.diag([1.0, -1.0, 0.0]))) < 1e-15
    for mu, nu in [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]:
        assert np.max(np.abs(Cl.field_strength(U, mu, nu))) < 1e-15
    # the 12x12 term at an interior site: (i csw / 2) sigma_xy (x) F_xy
    csw = 1.9
    C = Cl.clover_term(U, csw)[0, 0, 0, 3].reshape(12, 12)
    s = np.diag([-1.0, 1.0, -1.0, 1.0])
    expect = (0.5j * csw) * np.kron(s, 1j * np.sin(B) * np.diag([1.0, -1.0, 0.0]))
    assert np.max(np.abs(C - expect)) < 1e-15


def test_hermitian_chiral_and_linear():
    U = synth.gauge_field(L, 0.6, 3)
    C = Cl.clover_term(U, 1.3)
    M = C.reshape(C.shape[:4] + (12, 12))
    assert np.max(np.abs(M - np.conj(np.swapaxes(M, -1, -2)))) < 1e-15
    assert np.max(np.abs(M[..., :6, 6:])) == 0 and np.max(np.abs(M[..., 6:, :6])) == 0
    assert np.allclose(Cl.clover_term(U, 2.6), 2 * C, rtol=1e-15, atol=1e-16)
    assert np.max(np.abs(Cl.clover_term(U, 0.0))) == 0


def test_gauge_covariance():
    U = synth.gauge_field(L, 0.6, 4)
    Om = synth.haar_su3_field(L, 7)
    # U_mu(n) -> Om(n) U_mu(n) Om(n + mu)^dagger
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = Om @ U[mu] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=W.AXIS[mu]), -1, -2))
    C = Cl.clover_term(U, 1.1)
    Cg = Cl.clover_term(Ug, 1.1)
    # C[U^Om](n) = Om(n) C[U](n) Om(n)^dagger on the colour indices
    rot = np.einsum("...ac,...sctd,...bd->...satb", Om, C, np.conj(Om))
    assert np.max(np.abs(Cg - rot)) < 1e-13


def test_dsw_gamma5_hermitian():
    U = synth.gauge_field(L, 0.6, 5)
    C = Cl.clover_term(U, 1.5)
    x = synth.gaussian_spinor(L, 1)
    y = synth.gaussian_spinor(L, 2)
    m0 = -0.3
    lhs = W.inner(y, W.gamma5_apply(W.apply_D(U, m0, W.gamma5_apply(x), C)))
    rhs = W.inner(W.apply_D(U, m0, y, C), x)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    # block operator keeps the (site-local) term
    yb = W.apply_D_blocks(U, m0, x, (2, 2, 2, 2), C) - W.apply_D_blocks(U, m0, x, (2, 2, 2, 2))
    assert np.max(np.abs(yb - Cl.apply_clover(C, x))) < 1e-14


def test_site_by_site_matches_whole_lattice():
    U = synth.gauge_field(L, 0.6, 6)
    C = Cl.clover_term(U, 1.4)
    V = int(np.prod(L))
    sites = [0, 1, 17, V // 2, V - 1]
    Cs = Cl.clover_at_sites(U, 1.4, sites)
    flat = C.reshape((V, 4, 3, 4, 3))
    assert np.max(np.abs(Cs - flat[sites])) < 1e-14


def test_sampled_sites_with_clover_match_whole_lattice():
    """apply_D_at_sites with the site-local term (used to sample D_sw on
    lattices too large for a whole-field comparison) equals the whole-field
    D_sw = D + C, at sites on every face and wrap of a 4x4x4x8 lattice."""
    U = synth.gauge_field(L, 0.7, 2)
    csw, m0 = 1.9, -0.31
    C = Cl.clover_term(U, csw)
    x = synth.gaussian_spinor(L, 1009)
    y = W.apply_D(U, m0, x, C).reshape(-1, 4, 3)
    V = int(np.prod(L))
    rng = np.random.default_rng(5)
    sites = np.unique(np.concatenate([[0, 3, 12, 15, 48, 63, V - 64, V - 1], rng.integers(0, V, 40)]))
    Cs = Cl.clover_at_sites(U, csw, sites)
    ys = W.apply_D_at_sites(U, m0, x, sites, Cs)
    scale = np.max(np.abs(y))
    assert np.max(np.abs(ys - y[sites])) <= 1e-14 * scale
    # the clover part is really present in the sampled values
    ys0 = W.apply_D_at_sites(U, m0, x, sites)
    assert np.max(np.abs(ys0 - ys)) > 1e-2 * scale
