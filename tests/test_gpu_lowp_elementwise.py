"""Low-precision paths against the oracle run on the same rounded inputs,
element by element.

Storage conversion (the rounding reading: to nearest even, from FP64 in one
step for FP32 and FP16, through FP32 for BF16) is checked bit for bit
against NumPy's rounding of the same numbers.

Operator at storage precision (dw_apply_ex): links and spinor are held at
FP32/FP16/BF16, the hops run in FP32 and the result is stored at the
storage precision. The oracle applies eq. 1 in FP64 to the same rounded
links and spinor, so the only differences are the FP32 arithmetic, the
final rounding and, at FP16, the rounding of each projected half-spinor
entry to FP16 (the hops project in packed FP16 arithmetic and multiply by
the links with exact FP16 products accumulated in FP32). Per output
element n the error is then at most
    u |ref_n| + (p + (1 + u) g) Mag_n,
u the storage format's unit roundoff (2^-24, 2^-11, 2^-8), p = 2^-11 for
FP16 (the projection rounding, relative to the projected entry, whose
magnitude the stencil below bounds) and 0 otherwise, g = 32 * 2^-24 for
the FP32 sums of at most 24 products per element (7 terms per hop
product, 8 hops, the diagonal), and Mag_n the same stencil applied to
absolute values (|4 + m0| |x_n| + 1/2 sum over hops of
|1 -/+ gamma_mu| |U| |x|), which bounds every partial sum.

SAP (Alg. 2 with MR) at 16-bit storage: the kernel also rounds the
neighbours' copy of the block residual and each projected half spinor to
16 bits before the link products, then accumulates in FP32. Each MR step's
block operator therefore carries a relative error of about 2u in its
magnitude bound, which reaches z through the (nmr + 1) operator
applications of a block solve (the MR coefficients are scale-invariant
ratios of those results); later sweeps add corrections that shrink with the
block residuals, so their rounding adds little. The element-wise tolerance
is
    |z_n - ref_n| <= 2 u (nmr + 1) (|ref_n| + rms(ref)),
with ref the FP64 oracle SAP on the rounded links and input.
"""
import numpy as np
import pytest
import torch

import paper_1204_5463_amd as P
import synth
from oracle import sap as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu

UNIT = {P.DW_PREC_F32: 2.0 ** -24, P.DW_PREC_F16: 2.0 ** -11, P.DW_PREC_BF16: 2.0 ** -8}
# rounding of the projected half spinor before the link products (operator)
PROJ = {P.DW_PREC_F32: 0.0, P.DW_PREC_F16: 2.0 ** -11, P.DW_PREC_BF16: 0.0}


def _round_real(a, prec):
    """FP64 -> storage format, to nearest even (BF16 through FP32), back to FP64."""
    a = np.asarray(a, dtype=np.float64)
    if prec == P.DW_PREC_F16:
        return a.astype(np.float16).astype(np.float64)
    f = a.astype(np.float32)
    if prec == P.DW_PREC_F32:
        return f.astype(np.float64)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_c(z, prec):
    return _round_real(z.real, prec) + 1j * _round_real(z.imag, prec)


def magnitude_stencil(U, m0, x):
    """|4 + m0| |x_n| + 1/2 sum_mu (|1 - g_mu| |U_mu(n)| |x(n+mu)| + |1 + g_mu| |U_mu(n-mu)|^T |x(n-mu)|)."""
    Ua, xa = np.abs(U), np.abs(x)
    out = abs(4.0 + m0) * xa
    for mu in range(4):
        ax = W.AXIS[mu]
        xf = np.roll(xa, -1, axis=ax)
        t = np.einsum("...ab,...sb->...sa", Ua[mu], xf)
        out = out + 0.5 * np.einsum("st,...ta->...sa", np.abs(W.P_MINUS[mu]), t)
        tb = np.einsum("...ba,...sb->...sa", Ua[mu], xa)
        tb = np.roll(tb, 1, axis=ax)
        out = out + 0.5 * np.einsum("st,...ta->...sa", np.abs(W.P_PLUS[mu]), tb)
    return out


@pytest.mark.parametrize("prec", [P.DW_PREC_F32, P.DW_PREC_F16, P.DW_PREC_BF16])
def test_conversion_is_bitwise_round_to_nearest_even(dwctx, prec):
    L, block = (8, 4, 4, 8), (2, 2, 2, 2)
    f = P.Field(dwctx, L, block, P.to_device(synth.unit_gauge_field(L)))
    rng = np.random.default_rng(11)
    x = synth.gaussian_spinor(L, 21) * np.exp(rng.uniform(-6, 6, size=synth.gaussian_spinor(L, 21).shape))
    xi = f.pack(prec, P.to_device(x))
    back = f.unpack(prec, xi).cpu().numpy()[0]
    ref = round_c(x, prec)
    assert np.array_equal(back.view(np.float64), ref.view(np.float64))
    f.close()


@pytest.mark.parametrize("prec", [P.DW_PREC_F32, P.DW_PREC_F16, P.DW_PREC_BF16])
@pytest.mark.parametrize("L,block", [((8, 4, 4, 8), (2, 2, 2, 2)), ((8, 8, 8, 8), (4, 4, 4, 4))])
def test_operator_elementwise_on_rounded_inputs(dwctx, prec, L, block):
    U = synth.gauge_field(L, 0.6, 3)
    x = synth.gaussian_spinor(L, 7)
    m0 = -0.2
    f = P.Field(dwctx, L, block, P.to_device(U))
    xi = f.pack(prec, P.to_device(x))
    yi = torch.empty_like(xi)
    f.apply_ex(m0, prec, xi, yi)
    y = f.unpack(prec, yi).cpu().numpy()[0]
    Ur, xr = round_c(U, prec), round_c(x, prec)
    ref = W.apply_D(Ur, m0, xr)
    u = UNIT[prec]
    g = 32 * 2.0 ** -24
    bound = u * np.abs(ref) + (PROJ[prec] + (1 + u) * g) * magnitude_stencil(Ur, m0, xr)
    ratio = np.abs(y - ref) / bound
    print(f"operator prec {prec} L={L}: max error / bound = {ratio.max():.3f}", flush=True)
    assert np.all(ratio <= 1.0), ratio.max()
    f.close()


@pytest.mark.parametrize("prec", [P.DW_PREC_F32, P.DW_PREC_F16, P.DW_PREC_BF16])
@pytest.mark.parametrize("ncyc,nmr", [(1, 4), (2, 5)])
def test_sap_elementwise_on_rounded_inputs(dwctx, prec, ncyc, nmr):
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    m0 = -0.4
    U = synth.gauge_field(L, 0.6, 2)
    v = synth.gaussian_spinor(L, 9)
    f = P.Field(dwctx, L, block, P.to_device(U))
    sp = P.SapParams(block=block, ncycles=ncyc, nmr=nmr, storage=prec)
    z = f.sap(m0, sp, P.to_device(v)).cpu().numpy()
    # sap_precondition scales v to unit RMS entries before the cast: the
    # oracle takes the same scaled, rounded input (M is scale-equivariant)
    sigma = np.sqrt(v.size / np.vdot(v, v).real)
    Ur, vr = round_c(U, prec), round_c(sigma * v, prec)
    ref = S.sap(Ur, m0, L, block, ncyc, nmr, vr) / sigma
    u = UNIT[prec]
    tol = 2 * u * (nmr + 1) * (np.abs(ref) + np.sqrt(np.mean(np.abs(ref) ** 2)))
    ratio = np.abs(z - ref) / tol
    print(f"SAP prec {prec} s={ncyc} nmr={nmr}: max error / tolerance = {ratio.max():.3f}", flush=True)
    assert np.all(ratio <= 1.0), ratio.max()
    f.close()
