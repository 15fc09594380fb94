"""Parity at the benchmark lattice (32^3 x 64, eps = 0.7 links, seed 0) in the
benchmark's launch configuration.

* SAP: one cycle of the preconditioner on the full lattice, compared on
  sampled blocks with the oracle run on a 16^4 window of the lattice. Blocks
  of colour 0 depend only on their own data; blocks of colour 1 also on the
  colour-0 result of their 8 neighbours, so the window's inner 2^4 blocks are
  exact. The window straddles the periodic boundary in x and t.
* Solve: the full FGMRES-DR solve with the benchmark's parameters and mass,
  checked by the oracle's operator (true residual at 1e-10).
"""
import json
import os

import numpy as np
import pytest

import paper_1204_5463_amd as P
import synth
from oracle import sap as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu

L, B = (32, 32, 32, 64), (4, 4, 4, 4)


@pytest.fixture(scope="module")
def big(dwctx):
    U = synth.gauge_field(L, 0.7, 0)
    f = P.Field(dwctx, L, B, P.to_device(U))
    # the benchmark's mass: 0.005 above the critical mass of the 16^3x32 field of the same eps
    with open(os.path.join(os.path.dirname(__file__), "golden", "critical_mass.json")) as fh:
        crit = json.load(fh)
    name = next(n for n in ("32^3x64_eps0.7", "16^3x32_eps0.7", "12^4_eps0.7") if n in crit)
    m0 = crit[name]["m_c"] + 0.005
    return U, f, m0


def _window(a, shift):
    """Rolls a field with axes [..., t, z, y, x, ...] so that lattice site
    `shift` (x, y, z, t) moves to the origin; returns the 16^4 corner."""
    lead = a.ndim - 6  # lattice axes, then two site-local axes (spin, colour or a, b)
    out = a
    for mu, s in enumerate(shift):
        out = np.roll(out, -s, axis=lead + 3 - mu)
    sl = [slice(None)] * out.ndim
    for mu in range(4):
        sl[lead + 3 - mu] = slice(0, 16)
    return out[tuple(sl)]


@pytest.mark.parametrize("prec,tol", [(P.DW_PREC_F64, 1e-12), (P.DW_PREC_F16, 2e-2)])
def test_sap_full_size_sampled_blocks(big, prec, tol):
    U, f, m0 = big
    v = synth.gaussian_spinor(L, 1000)
    nmr = 8
    z = f.sap(m0, P.SapParams(block=B, ncycles=1, nmr=nmr, storage=prec), P.to_device(v)).cpu().numpy()
    # window origin in blocks (7, 3, 1, 15): even coordinate sum keeps the colours; wraps in x and t
    shift = (28, 12, 4, 60)
    Uw = np.stack([_window(U[mu], shift) for mu in range(4)])
    vw = _window(v, shift)
    zo = S.sap(Uw, m0, (16, 16, 16, 16), B, 1, nmr, vw)
    zg = _window(z, shift)
    inner = (slice(4, 12),) * 4
    err = np.linalg.norm(zg[inner] - zo[inner]) / np.linalg.norm(zo[inner])
    assert err < tol, err
    # colour-0 blocks are exact anywhere in the window
    mask0 = S.colour_mask((16, 16, 16, 16), B, 0)
    e0 = np.linalg.norm((zg - zo)[mask0]) / np.linalg.norm(zo[mask0])
    assert e0 < tol, e0
    if prec == P.DW_PREC_F16:
        # element by element against the oracle on the same FP16-rounded links
        # and RMS-scaled input, with the bound 2 u (nmr + 1) (|ref| + rms(ref))
        # of the 8^4 element-wise test, on the window's exact blocks
        def r16(a):
            return a.real.astype(np.float16).astype(np.float64) + 1j * a.imag.astype(np.float16).astype(np.float64)
        sigma = np.sqrt(v.size / np.vdot(v, v).real)
        ref = S.sap(r16(Uw), m0, (16, 16, 16, 16), B, 1, nmr, r16(sigma * vw)) / sigma
        inner_m = np.zeros(mask0.shape, dtype=bool)
        inner_m[inner] = True
        exact = mask0 | (inner_m & S.colour_mask((16, 16, 16, 16), B, 1))
        r = ref[exact]
        bound = 2 * 2.0 ** -11 * (nmr + 1) * (np.abs(r) + np.sqrt(np.mean(np.abs(r) ** 2)))
        ratio = float((np.abs(zg[exact] - r) / bound).max())
        print(f"32^3x64 FP16 SAP element-wise max error / bound = {ratio:.3f}", flush=True)
        assert ratio <= 1.0, ratio


@pytest.mark.parametrize("flags", [0, P.SOLVE_V32, P.SOLVE_A32 | P.SOLVE_INJECT])
def test_solve_full_size_true_residual(big, flags):
    U, f, m0 = big
    b = synth.gaussian_spinor(L, 1000)
    prm = P.SolverParams(m=30, k=12, max_iter=2000, tol=1e-10, flags=flags,
                         sap=P.SapParams(block=B, ncycles=13, nmr=8, storage=P.DW_PREC_F16))
    x, st = f.solve(m0, prm, P.to_device(b))
    print(f"32^3x64 solve flags {flags}: {st[0].iterations} it, {st[0].cycles} cycles, "
          f"{st[0].clean_restarts} clean restarts", flush=True)
    assert st[0].converged and st[0].true_relres <= 1e-10
    if flags == 0:
        assert st[0].cycles >= 2  # the benchmark's solve includes a deflated restart
    x = x.cpu().numpy()
    r = b - W.apply_D(U, m0, x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
