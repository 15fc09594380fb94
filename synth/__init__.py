"""Seeded synthetic inputs for the Wilson-Dirac solver.

This module only draws random numbers and shapes them into lattice fields.
It holds none of the solver's arithmetic: no Dirac operator, no Schwarz
sweep, no Krylov method. Both the CPU oracle's tests and the GPU path's
tests/benchmarks take their inputs from here, so the two sides see the same
fields without sharing any code of the method.

Conventions (fixed for the whole project):
  * lattice extents ``L = (Lx, Ly, Lz, Lt)``; direction index mu = 0..3 is
    x, y, z, t; the lexicographic site index is
    ``n = x + Lx*(y + Ly*(z + Lz*t))``;
  * numpy arrays are stored in that order, i.e. shaped
    ``(Lt, Lz, Ly, Lx, ...)`` (C order), so a flat view is canonical;
  * gauge field ``U[mu, t, z, y, x, a, b]`` = U_mu(n)_{ab}, complex128;
  * spinor field ``psi[t, z, y, x, spin, colour]``, complex128.

The paper measures on thermalised gauge configurations that are not
available; the fields here are i.i.d. near-unit SU(3) links
``exp(i*eps*H)`` with H a random traceless Hermitian Gaussian matrix.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "lattice_shape",
    "volume",
    "gauge_field",
    "unit_gauge_field",
    "gaussian_spinor",
    "gaussian_spinors",
    "point_source_noise",
    "haar_su3_field",
    "pure_gauge_field",
]


def lattice_shape(L):
    """Array shape (Lt, Lz, Ly, Lx) for extents L = (Lx, Ly, Lz, Lt)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return (Lt, Lz, Ly, Lx)


def volume(L):
    return int(np.prod([int(v) for v in L]))


def _gauss_complex(rng, shape):
    """(N(0,1) + i N(0,1))/sqrt(2), drawn as one real array of shape+(2,)."""
    x = rng.standard_normal(tuple(shape) + (2,))
    return (x[..., 0] + 1j * x[..., 1]) * (1.0 / math.sqrt(2.0))


def _traceless_hermitian(A):
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    return H - tr[..., None, None] * np.eye(3)


def exp_i_eps_h_eigh(A, eps):
    """exp(i eps H) through eigh(H) (reference form, used in tests)."""
    d, W = np.linalg.eigh(_traceless_hermitian(A))
    ph = np.exp(1j * eps * d)
    return np.matmul(W * ph[..., None, :], np.conj(np.swapaxes(W, -1, -2)))


def exp_i_eps_h(A, eps):
    """exp(i eps H), H the traceless Hermitian part of A, by PyTorch's CPU
    matrix exponential (multi-threaded; equals the eigh form to rounding)."""
    import torch

    X = torch.from_numpy(np.ascontiguousarray((1j * eps) * _traceless_hermitian(A)))
    return torch.linalg.matrix_exp(X).numpy()


def gauge_field(L, eps, seed, t_chunk=None):
    """Random SU(3) links U_mu(n) = exp(i*eps*H), H traceless Hermitian Gaussian.

    Stream: ``numpy.random.default_rng(seed)`` draws X of shape
    (4, Lt, Lz, Ly, Lx, 3, 3, 2) in C order (generated in chunks along the
    leading axes, which consumes the same stream). A = (X0 + i X1)/sqrt(2),
    H = (A + A^H)/2 - tr/3, U = exp(i eps H).
    """
    shp = lattice_shape(L)
    Lt = shp[0]
    rng = np.random.default_rng(seed)
    U = np.empty((4,) + shp + (3, 3), dtype=np.complex128)
    if t_chunk is None:
        sites_per_t = int(np.prod(shp[1:]))
        t_chunk = max(1, min(Lt, (1 << 20) // max(1, sites_per_t)))
    for mu in range(4):
        for t0 in range(0, Lt, t_chunk):
            t1 = min(Lt, t0 + t_chunk)
            A = _gauss_complex(rng, (t1 - t0,) + shp[1:] + (3, 3))
            U[mu, t0:t1] = exp_i_eps_h(A, eps)
    return U


def unit_gauge_field(L):
    """Free field: every link is the 3x3 identity."""
    shp = lattice_shape(L)
    U = np.zeros((4,) + shp + (3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_spinor(L, seed):
    """Gaussian complex spinor, each component (N(0,1)+iN(0,1))/sqrt(2)."""
    rng = np.random.default_rng(seed)
    return _gauss_complex(rng, lattice_shape(L) + (4, 3))


def gaussian_spinors(L, nrhs, seed0=1000):
    """nrhs Gaussian spinors, RHS j drawn with seed ``seed0 + j``."""
    return np.stack([gaussian_spinor(L, seed0 + j) for j in range(nrhs)])


def point_source_noise(L, j, seed, noise=None):
    """Point source at the origin in spin j//3, colour j%3, plus Gaussian noise.

    The noise amplitude defaults to 1/sqrt(12 V) per component so that the
    noise and the point source have comparable norms.
    """
    V = volume(L)
    if noise is None:
        noise = 1.0 / math.sqrt(12.0 * V)
    b = noise * gaussian_spinor(L, seed)
    b[0, 0, 0, 0, (j // 3) % 4, j % 3] += 1.0
    return b


def haar_su3_field(L, seed):
    """Haar-random SU(3) matrix per site (QR of a complex Gaussian with the
    diagonal phase fix of Mezzadri 2007, divided by det^(1/3))."""
    rng = np.random.default_rng(seed)
    Z = _gauss_complex(rng, lattice_shape(L) + (3, 3))
    Q, R = np.linalg.qr(Z)
    dR = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (dR / np.abs(dR))[..., None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[..., None, None]


def pure_gauge_field(Omega):
    """Links U_mu(n) = Omega(n) Omega(n+mu)^dagger (a gauge copy of U = 1)."""
    shp = Omega.shape[:4]
    U = np.empty((4,) + shp + (3, 3), dtype=np.complex128)
    axes = (3, 2, 1, 0)  # mu = x, y, z, t -> array axis
    for mu in range(4):
        Om_fwd = np.roll(Omega, -1, axis=axes[mu])
        U[mu] = np.matmul(Omega, np.conj(np.swapaxes(Om_fwd, -1, -2)))
    return U
