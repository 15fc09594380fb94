"""Pins of the oracle's Wilson-Dirac operator against facts that the paper
and the mathematics fix, independent of the oracle's own code:

  * the gamma algebra of the chosen basis;
  * the free-field (U = 1) momentum-space closed form of eq. (1), by plane
    waves at any size and by the full dense spectrum on 2^4;
  * the same closed form under a pure-gauge field U = Omega Omega(n+mu)^+;
  * gamma5-hermiticity and gauge covariance on random SU(3) fields;
  * a brute-force site-by-site assembly of [D]_{nm} from eq. (1) on 2^4
    (explicit loops, no array shifts), dense LU for the solution;
  * the block operator D^l of eq. (2) as the restriction of D.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import wilson as W


def test_gamma_algebra():
    for mu in range(4):
        assert np.allclose(W.GAMMA[mu], W.GAMMA[mu].conj().T)
        for nu in range(4):
            ac = W.GAMMA[mu] @ W.GAMMA[nu] + W.GAMMA[nu] @ W.GAMMA[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4))
    assert np.allclose(W.GAMMA5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(W.GAMMA5 @ W.GAMMA[mu] @ W.GAMMA5, -W.GAMMA[mu])


def _plane_wave(L, kvec, chi):
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    p = [2 * np.pi * kvec[mu] / L[mu] for mu in range(4)]
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return phase[..., None, None] * chi[None, None, None, None], p


def _free_symbol(m0, p):
    """m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu, a 4x4 spin matrix."""
    S = (m0 + sum(1 - np.cos(pm) for pm in p)) * np.eye(4, dtype=complex)
    for mu in range(4):
        S = S + 1j * np.sin(p[mu]) * W.GAMMA[mu]
    return S


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 2, 8)])
def test_free_field_plane_waves(L):
    rng = np.random.default_rng(3)
    U = synth.unit_gauge_field(L)
    m0 = -0.37
    for _ in range(5):
        kvec = [int(rng.integers(0, L[mu])) for mu in range(4)]
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        x, p = _plane_wave(L, kvec, chi)
        y = W.apply_D(U, m0, x)
        expect = np.einsum("st,...ta->...sa", _free_symbol(m0, p), x)
        assert np.max(np.abs(y - expect)) < 1e-13 * np.max(np.abs(x))


def test_free_field_dense_spectrum_2x4():
    L = (2, 2, 2, 2)
    m0 = 0.3
    D = W.dense_D(synth.unit_gauge_field(L), m0)
    ev = np.sort_complex(np.linalg.eigvals(D))
    expect = []
    for k in itertools.product(range(2), repeat=4):
        p = [np.pi * ki for ki in k]
        s = np.linalg.eigvals(_free_symbol(m0, p))
        expect.extend(list(s) * 3)                 # colour multiplicity
    expect = np.sort_complex(np.array(expect))
    assert np.max(np.abs(ev - expect)) < 1e-12


def test_pure_gauge_plane_waves():
    L = (4, 4, 2, 4)
    Om = synth.haar_su3_field(L, seed=7)
    U = synth.pure_gauge_field(Om)
    m0 = 0.1
    rng = np.random.default_rng(11)
    kvec = [1, 3, 1, 2]
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    x, p = _plane_wave(L, kvec, chi)
    # psi = Omega x is an eigenfunction of D[U] with the free-field symbol
    psi = np.einsum("...ab,...sb->...sa", Om, x)
    y = W.apply_D(U, m0, psi)
    expect = np.einsum("...ab,...sb->...sa", Om, np.einsum("st,...ta->...sa", _free_symbol(m0, p), x))
    assert np.max(np.abs(y - expect)) < 1e-13 * np.max(np.abs(psi)) * 10


@pytest.mark.parametrize("block", [None, (2, 2, 2, 2)])
def test_gamma5_hermiticity(block):
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.7, seed=1)
    x = synth.gaussian_spinor(L, 1)
    y = synth.gaussian_spinor(L, 2)
    m0 = -0.4

    def D(v):
        return W.apply_D(U, m0, v) if block is None else W.apply_D_blocks(U, m0, v, block)

    lhs = W.inner(y, W.gamma5_apply(D(W.gamma5_apply(x))))
    rhs = W.inner(D(y), x)
    assert abs(lhs - rhs) < 1e-13 * abs(rhs) * 10
    # and D itself is not Hermitian (the test would be vacuous otherwise)
    assert abs(W.inner(y, D(x)) - W.inner(D(y), x)) > 1e-3 * abs(rhs)


def test_gauge_covariance():
    L = (4, 4, 4, 6)
    U = synth.gauge_field(L, 0.6, seed=2)
    Om = synth.haar_su3_field(L, seed=7)
    UO = np.empty_like(U)
    for mu in range(4):
        Omf = np.roll(Om, -1, axis=W.AXIS[mu])
        UO[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Omf, -1, -2))
    psi = synth.gaussian_spinor(L, 3)
    m0 = 0.05
    lhs = W.apply_D(UO, m0, np.einsum("...ab,...sb->...sa", Om, psi))
    rhs = np.einsum("...ab,...sb->...sa", Om, W.apply_D(U, m0, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(rhs)) * 10


def _brute_force_dense(U, m0, L):
    """[D]_{nm} assembled site by site from eq. (1) with explicit loops."""
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    D = np.zeros((12 * V, 12 * V), dtype=complex)
    ext = (Lx, Ly, Lz, Lt)
    G = W.GAMMA
    I4 = np.eye(4)
    for n in range(V):
        c = [n % Lx, (n // Lx) % Ly, (n // (Lx * Ly)) % Lz, n // (Lx * Ly * Lz)]
        for s in range(4):
            for a in range(3):
                D[12 * n + 3 * s + a, 12 * n + 3 * s + a] += 4.0 + m0
        for mu in range(4):
            f = list(c)
            f[mu] = (c[mu] + 1) % ext[mu]
            b = list(c)
            b[mu] = (c[mu] - 1) % ext[mu]
            nf = f[0] + Lx * (f[1] + Ly * (f[2] + Lz * f[3]))
            nb = b[0] + Lx * (b[1] + Ly * (b[2] + Lz * b[3]))
            Uf = U[mu, c[3], c[2], c[1], c[0]]
            Ub = U[mu, b[3], b[2], b[1], b[0]]
            for s in range(4):
                for t in range(4):
                    for a in range(3):
                        for bb in range(3):
                            D[12 * n + 3 * s + a, 12 * nf + 3 * t + bb] -= 0.5 * (I4 - G[mu])[s, t] * Uf[a, bb]
                            D[12 * n + 3 * s + a, 12 * nb + 3 * t + bb] -= 0.5 * (I4 + G[mu])[s, t] * np.conj(Ub[bb, a])
    return D


def test_brute_force_dense_2x4_and_lu():
    L = (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.5, seed=0)
    m0 = -0.2
    Dbf = _brute_force_dense(U, m0, L)
    Dor = W.dense_D(U, m0)
    assert np.max(np.abs(Dbf - Dor)) < 1e-13
    b = synth.gaussian_spinor(L, 1000)
    xs = np.linalg.solve(Dbf, b.reshape(-1))
    r = b - W.apply_D(U, m0, xs.reshape(b.shape))
    assert np.linalg.norm(r) < 1e-13 * np.linalg.norm(b) * 10


def test_sampled_sites_match_whole_field():
    L = (4, 4, 2, 6)
    U = synth.gauge_field(L, 0.7, seed=4)
    x = synth.gaussian_spinor(L, 5)
    y = W.apply_D(U, 0.2, x)
    sites = [0, 5, 17, 31, 63, 64, 100, 191]
    ys = W.apply_D_at_sites(U, 0.2, x, sites)
    flat = y.reshape(-1, 4, 3)
    assert np.max(np.abs(ys - flat[sites])) < 1e-13


def test_block_operator_is_restriction():
    L = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, seed=5)
    x = synth.gaussian_spinor(L, 6)
    m0 = 0.1
    Lx, Ly, Lz, Lt = L
    for origin in [(0, 0, 0, 0), (2, 0, 2, 2), (2, 2, 2, 2)]:
        mask = np.zeros((Lt, Lz, Ly, Lx), bool)
        ox, oy, oz, ot = origin
        mask[ot:ot + 2, oz:oz + 2, oy:oy + 2, ox:ox + 2] = True
        xl = x * mask[..., None, None]
        yb = W.apply_D_blocks(U, m0, xl, block)
        yf = W.apply_D(U, m0, xl)
        assert np.max(np.abs((yb - yf)[mask])) < 1e-15 * 10
        assert np.max(np.abs(yb[~mask])) == 0.0
        # the full operator does leak out of the block (nearest neighbours)
        assert np.max(np.abs(yf[~mask])) > 0.1


def test_mass_shift_is_identity_shift():
    L = (4, 2, 2, 4)
    U = synth.gauge_field(L, 0.6, seed=9)
    x = synth.gaussian_spinor(L, 9)
    d = W.apply_D(U, 0.3, x) - W.apply_D(U, -0.2, x)
    assert np.max(np.abs(d - 0.5 * x)) < 1e-14
