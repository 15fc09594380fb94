"""Wilson-Dirac operator, FP64 NumPy oracle (test infrastructure only).

Operator (paper Section 2, eq. 1, written in the mass normalisation used
throughout this project):

    (D x)(n) = (4 + m0) x(n)
               - 1/2 sum_mu [ (1 - gamma_mu) U_mu(n) x(n + mu)
                            + (1 + gamma_mu) U_mu(n - mu)^dagger x(n - mu) ]

with periodic boundaries in all four directions. Relation to the paper's
hopping-parameter form: kappa = 1/(2(4 + m0)) and
D = (4 + m0) gamma5 D_paper(kappa) gamma5 (gamma5 gamma_mu gamma5 = -gamma_mu
swaps the sign of the projectors), so the two have the same spectrum up to
the factor 4 + m0.

The block operator D^l (eq. 2) is the same stencil restricted to a
hyper-rectangular domain: every hop whose target lies outside the domain
is dropped.

Gamma matrices: Euclidean chiral basis,
    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = x, y, z),
    gamma_t = [[0, I], [I, 0]],  gamma5 = gamma_x gamma_y gamma_z gamma_t.
The paper does not fix a basis; any Hermitian basis gives a unitarily
equivalent operator.

Array conventions: U[mu, t, z, y, x, a, b], psi[t, z, y, x, spin, colour];
mu = 0..3 = x, y, z, t.
"""
from __future__ import annotations

import numpy as np

# array axis of each direction mu (arrays are stored t, z, y, x)
AXIS = (3, 2, 1, 0)

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)


def _chiral(A):
    return np.block([[_Z2, A], [A.conj().T, _Z2]])


GAMMA = np.array([
    _chiral(-1j * _s1),
    _chiral(-1j * _s2),
    _chiral(-1j * _s3),
    _chiral(_I2),
])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
I4 = np.eye(4, dtype=np.complex128)
P_MINUS = np.array([I4 - g for g in GAMMA])   # (1 - gamma_mu), forward hop
P_PLUS = np.array([I4 + g for g in GAMMA])    # (1 + gamma_mu), backward hop


def _colour_mul(U, x):
    """(U x)(n)_{s,a} = sum_b U(n)_{ab} x(n)_{s,b}, i.e. x(n) U(n)^T per site."""
    return np.matmul(x, np.swapaxes(U, -1, -2))


def _colour_mul_dag(U, x):
    """(U^dagger x)(n)_{s,a} = sum_b conj(U(n)_{ba}) x(n)_{s,b}, i.e. x(n) conj(U(n))."""
    return np.matmul(x, U.conj())


def _spin_mul(P, x):
    """(P x)(n)_{s,a} = sum_t P_{st} x(n)_{t,a}."""
    return np.matmul(P, x)


def hop_forward(U, x, mu):
    """(1 - gamma_mu) U_mu(n) x(n + mu) for every site n."""
    x_fwd = np.roll(x, -1, axis=AXIS[mu])
    return _spin_mul(P_MINUS[mu], _colour_mul(U[mu], x_fwd))


def hop_backward(U, x, mu):
    """(1 + gamma_mu) U_mu(n - mu)^dagger x(n - mu) for every site n."""
    t = _colour_mul_dag(U[mu], x)            # U_mu(m)^dagger x(m) at m
    t = np.roll(t, 1, axis=AXIS[mu])         # moved to n = m + mu
    return _spin_mul(P_PLUS[mu], t)


def _site_term(C, x):
    """Site-local 12x12 term (the clover term of ``oracle.clover``), or 0."""
    if C is None:
        return 0.0
    return np.einsum("...satb,...tb->...sa", C, x)


def apply_D(U, m0, x, C=None):
    """y = D x, eq. (1), periodic lattice; plus the site-local term C x if given."""
    y = (4.0 + m0) * x + _site_term(C, x)
    for mu in range(4):
        y = y - 0.5 * (hop_forward(U, x, mu) + hop_backward(U, x, mu))
    return y


def block_coords_masks(shape, block):
    """For each mu: boolean arrays (over sites) telling whether the forward /
    backward neighbour lies in the same block. ``block`` = (bx, by, bz, bt)."""
    fwd, bwd = [], []
    for mu in range(4):
        ax = AXIS[mu]
        n = np.arange(shape[ax])
        local = n % block[mu]
        sh = [1, 1, 1, 1]
        sh[ax] = shape[ax]
        fwd.append((local != block[mu] - 1).reshape(sh))
        bwd.append((local != 0).reshape(sh))
    return fwd, bwd


def apply_D_blocks(U, m0, x, block, C=None):
    """Block-diagonal part of D: D^l applied on every block at once (eq. 2).

    A hop n -> n +/- mu is kept only if both sites lie in the same block.
    Requires at least two blocks per direction, so that no periodic wrap
    stays inside a block.
    """
    shape = x.shape[:4]
    fwd, bwd = block_coords_masks(shape, block)
    y = (4.0 + m0) * x + _site_term(C, x)
    for mu in range(4):
        hf = hop_forward(U, x, mu) * fwd[mu][..., None, None]
        hb = hop_backward(U, x, mu) * bwd[mu][..., None, None]
        y = y - 0.5 * (hf + hb)
    return y


def apply_D_at_sites(U, m0, x, sites, C=None):
    """(D x)(n) for a list of lexicographic site indices, one site at a time.

    A direct transcription of eq. (1) per site, used to sample outputs of
    lattices too large for a whole-field comparison. ``C`` (optional) holds
    the site-local 12x12 term at those sites, in the order of ``sites``.
    """
    Lt, Lz, Ly, Lx = x.shape[:4]
    ext = (Lx, Ly, Lz, Lt)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    for i, s in enumerate(sites):
        s = int(s)
        c = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]
        acc = (4.0 + m0) * x[c[3], c[2], c[1], c[0]]
        if C is not None:
            acc = acc + np.einsum("satb,tb->sa", C[i], x[c[3], c[2], c[1], c[0]])
        for mu in range(4):
            f = list(c)
            f[mu] = (f[mu] + 1) % ext[mu]
            b = list(c)
            b[mu] = (b[mu] - 1) % ext[mu]
            Un = U[mu, c[3], c[2], c[1], c[0]]
            Ub = U[mu, b[3], b[2], b[1], b[0]]
            xf = x[f[3], f[2], f[1], f[0]]
            xb = x[b[3], b[2], b[1], b[0]]
            acc = acc - 0.5 * (P_MINUS[mu] @ (xf @ Un.T) + P_PLUS[mu] @ (xb @ Ub.conj()))
        out[i] = acc
    return out


def dense_D(U, m0, block=None, C=None):
    """Assemble D (or the block-diagonal part if ``block`` is given) as a dense
    matrix by applying it to every unit vector. Only for tiny lattices."""
    shape = U.shape[1:5]
    n = int(np.prod(shape)) * 12
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        x = e.reshape(shape + (4, 3))
        y = apply_D(U, m0, x, C) if block is None else apply_D_blocks(U, m0, x, block, C)
        M[:, j] = y.reshape(-1)
        e[j] = 0.0
    return M


def gamma5_apply(x):
    return np.einsum("st,...ta->...sa", GAMMA5, x)


def inner(a, b):
    """<a, b> = sum conj(a) b over all sites, spins and colours."""
    return np.vdot(a.reshape(-1), b.reshape(-1))


def norm(a):
    return float(np.linalg.norm(a.reshape(-1)))
