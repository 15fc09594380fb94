"""GPU parity of the Wilson-Dirac operator (eq. 1) against the FP64 oracle.

Element by element on whole fields (lattices spanning several blocks and a
ragged last workgroup), at FP64 and at each storage precision; sampled
sites and the free-field closed form on the 32^3 x 64 lattice timed by the
benchmark.
"""
import numpy as np
import pytest
import torch

import paper_1204_5463_amd as P
import synth
from oracle import wilson as W

pytestmark = pytest.mark.gpu

# (L, block): 8^4 with 4^4 blocks; a ragged lattice (480 sites, block 30 sites)
CASES = [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 2, 6, 10), (2, 1, 3, 5)), ((8, 4, 4, 8), (2, 2, 2, 2))]
# relative tolerance per storage precision (unit roundoff times a small factor
# for the 8-hop sum: FP32 2^-24, FP16 2^-11, BF16 2^-8)
TOL = {P.DW_PREC_F64: 1e-14, P.DW_PREC_F32: 2e-6, P.DW_PREC_F16: 3e-3, P.DW_PREC_BF16: 2.5e-2}


def _field(ctx, L, block, eps=0.6, seed=0):
    U = synth.gauge_field(L, eps, seed)
    return U, P.Field(ctx, L, block, P.to_device(U))


@pytest.mark.parametrize("L,block", CASES)
def test_dw_apply_fp64_matches_oracle(dwctx, L, block):
    U, f = _field(dwctx, L, block)
    x = synth.gaussian_spinors(L, 2)
    for m0 in (-0.1, 0.37):
        y = f.apply(m0, P.to_device(x)).cpu().numpy()
        for r in range(2):
            ref = W.apply_D(U, m0, x[r])
            err = np.max(np.abs(y[r] - ref)) / np.max(np.abs(ref))
            assert err < TOL[P.DW_PREC_F64], (L, m0, r, err)


@pytest.mark.parametrize("prec", [P.DW_PREC_F64, P.DW_PREC_F32, P.DW_PREC_F16, P.DW_PREC_BF16])
def test_dw_apply_ex_each_precision(dwctx, prec):
    L, block = (8, 4, 4, 8), (2, 2, 2, 2)
    U, f = _field(dwctx, L, block, eps=0.5, seed=3)
    x = synth.gaussian_spinor(L, 7)
    m0 = -0.2
    xt = P.to_device(x)
    xi = f.pack(prec, xt)
    yi = torch.empty_like(xi)
    f.apply_ex(m0, prec, xi, yi)
    y = f.unpack(prec, yi).cpu().numpy()[0]
    ref = W.apply_D(U, m0, x)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err < TOL[prec], err
    # pack/unpack is a lossless round trip at FP64
    if prec == P.DW_PREC_F64:
        assert np.array_equal(f.unpack(prec, xi).cpu().numpy()[0], x)


def test_zero_rhs_and_linearity(dwctx):
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U, f = _field(dwctx, L, block)
    z = torch.zeros((1,) + synth.lattice_shape(L) + (4, 3), dtype=torch.complex128, device="cuda")
    assert torch.count_nonzero(f.apply(0.1, z)) == 0
    a = synth.gaussian_spinor(L, 1)
    b = synth.gaussian_spinor(L, 2)
    ya = f.apply(0.1, P.to_device(a)).cpu().numpy()
    yb = f.apply(0.1, P.to_device(b)).cpu().numpy()
    yab = f.apply(0.1, P.to_device(2.0 * a - 3.0j * b)).cpu().numpy()
    assert np.max(np.abs(yab - (2.0 * ya - 3.0j * yb))) < 1e-12 * np.max(np.abs(yab))


def test_invalid_geometry_rejected(dwctx):
    U = P.to_device(synth.unit_gauge_field((8, 8, 8, 8)))
    with pytest.raises(P.DwError) as e:
        P.Field(dwctx, (8, 8, 8, 8), (4, 4, 4, 3), U)
    assert e.value.status == P.DW_EINVAL
    with pytest.raises(P.DwError):
        P.Field(dwctx, (8, 8, 8, 8), (8, 4, 4, 4), U)   # one block in x: odd count


def test_full_size_free_field_and_sampled_sites(dwctx):
    """32^3 x 64 (the benchmark lattice): plane-wave eigen-action of the
    free-field operator, and sampled sites of a random field against the
    oracle's per-site formula."""
    L, block = (32, 32, 32, 64), (4, 4, 4, 4)
    m0 = -0.05
    Lx, Ly, Lz, Lt = L
    f = P.Field(dwctx, L, block, P.to_device(synth.unit_gauge_field(L)))
    kvec = (3, 1, 5, 7)
    p = [2 * np.pi * kvec[mu] / L[mu] for mu in range(4)]
    chi = (np.arange(12).reshape(4, 3) + 1j).astype(np.complex128)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = ph[..., None, None] * chi
    out = f.apply(m0, P.to_device(psi)).cpu().numpy()
    S = (m0 + sum(1 - np.cos(q) for q in p)) * np.eye(4, dtype=complex)
    for mu in range(4):
        S = S + 1j * np.sin(p[mu]) * W.GAMMA[mu]
    expect = ph[..., None, None] * (S @ chi)
    assert np.max(np.abs(out - expect)) < 1e-12 * np.max(np.abs(expect))
    del f, psi, out, expect
    # random field: sampled sites
    U = synth.gauge_field(L, 0.7, 0)
    f = P.Field(dwctx, L, block, P.to_device(U))
    b = synth.gaussian_spinor(L, 1000)
    yv = f.apply(m0, P.to_device(b)).cpu().numpy().reshape(-1, 4, 3)
    rng = np.random.default_rng(0)
    V = synth.volume(L)
    sites = list(rng.integers(0, V, 200)) + [0, V - 1, Lx - 1, Lx * Ly * Lz * (Lt - 1)]
    ref = W.apply_D_at_sites(U, m0, b, sites)
    assert np.max(np.abs(yv[sites] - ref)) < 1e-13 * np.max(np.abs(ref))
