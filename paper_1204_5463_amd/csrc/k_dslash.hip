// Wilson-Dirac operator on the whole periodic lattice (paper eq. 1).
//
// One thread per site; every thread gathers its 8 neighbours' spinors and
// the 8 links it needs (its own 4 forward links and the 4 backward links
// stored at the neighbours). Fields are in the block-tiled internal layout,
// so each spinor component and link entry is a contiguous run over a
// block's sites and a wavefront's loads are coalesced; neighbour reuse
// across threads goes through L1/L2.
//
// Bandwidth bound: per site and right-hand side the algorithmic traffic is
// one spinor read, 4 links read and one spinor write (FP64: 960 bytes).
#include "dw_internal.hpp"
#include "dw_stencil.hpp"

namespace dw {

namespace {

constexpr int kThreads = 256;
// flops of one site of D: 8 hops x (12 projection + 2 x 66 SU(3) x vector
// + 24 accumulation) - 24 (first accumulation is a copy) + 48 (diagonal)
constexpr double kFlopsPerSite = 1368.0;

// MODE 0: y = scale * D x ; MODE 1: y = b - scale * D x
template <typename T, typename SX, typename SG, typename SY, int MODE>
__global__ void __launch_bounds__(kThreads)
    k_dslash(Geom g, T diag, const SX* __restrict__ x, T scale, const SG* __restrict__ U, SY* __restrict__ y,
             const SY* __restrict__ bsrc, long long xs, long long ys) {
  const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= g.V) return;
  const SX* xr = x + (long long)blockIdx.y * xs;
  SY* yr = y + (long long)blockIdx.y * ys;
  const int b = (int)(s / g.bvol);
  const int l = (int)(s - (long long)b * g.bvol);
  int bc[4], lc[4];
  decode_block(g, b, bc);
  decode_local(g, l, lc);
  cplx<T> acc[12];
  hop_sum_lattice<T>(g, b, l, bc, lc, U,
                     [&](int nb, int nl, int comp) { return ld<T>(xr + spinor_index(g, nb, comp, nl)); }, acc);
  const T half = (T)0.5;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const long long idx = spinor_index(g, b, c, l);
    cplx<T> xo = ld<T>(xr + idx);
    cplx<T> d = scale * (diag * xo - half * acc[c]);
    if constexpr (MODE == 1) {
      const SY* br = bsrc + (long long)blockIdx.y * ys;
      d = ld<T>(br + idx) - d;
    }
    st(yr + idx, d);
  }
}

dim3 grid_for(const Geom& g, int nrhs) { return dim3((unsigned)((g.V + kThreads - 1) / kThreads), (unsigned)nrhs); }

}  // namespace

dw_status launch_dslash_outer(const Geom& g, double m0, int prec_x, const void* x, double scale, const void* U64,
                              double* y, const double* b, int mode, int nrhs, long long xs, long long ys,
                              hipStream_t s) {
  const double diag = 4.0 + m0;
  const s64* Ug = (const s64*)U64;
  s64* yo = (s64*)y;
  const s64* bo = (const s64*)b;
  dim3 grid = grid_for(g, nrhs);
  KTimer kt(DW_K_DSLASH_F64, s);
  if (prec_x == DW_PREC_F64) {
    const s64* xi = (const s64*)x;
    if (mode == 0)
      hipLaunchKernelGGL((k_dslash<double, s64, s64, s64, 0>), grid, kThreads, 0, s, g, diag, xi, scale, Ug, yo, bo, xs, ys);
    else
      hipLaunchKernelGGL((k_dslash<double, s64, s64, s64, 1>), grid, kThreads, 0, s, g, diag, xi, scale, Ug, yo, bo, xs, ys);
  } else if (prec_x == DW_PREC_F32) {
    const s32* xi = (const s32*)x;
    if (mode == 0)
      hipLaunchKernelGGL((k_dslash<double, s32, s64, s64, 0>), grid, kThreads, 0, s, g, diag, xi, scale, Ug, yo, bo, xs, ys);
    else
      hipLaunchKernelGGL((k_dslash<double, s32, s64, s64, 1>), grid, kThreads, 0, s, g, diag, xi, scale, Ug, yo, bo, xs, ys);
  } else {
    set_error("outer dslash input precision must be F64 or F32");
    return DW_EINVAL;
  }
  DW_CHECK_LAUNCH();
  kt.done((double)g.V * nrhs * (12.0 * pair_bytes(prec_x) + 36 * 16 + 12 * 16 + (mode == 1 ? 12 * 16 : 0)),
          (double)g.V * nrhs * kFlopsPerSite);
  return DW_OK;
}

dw_status launch_dslash_lowp(const Geom& g, double m0, int prec, const void* x, const void* U, void* y, int nrhs,
                             hipStream_t s) {
  dim3 grid = grid_for(g, nrhs);
  const long long st = g.V * 12;
  KTimer kt(DW_K_DSLASH_LOWP, s);
  switch (prec) {
    case DW_PREC_F64:
      hipLaunchKernelGGL((k_dslash<double, s64, s64, s64, 0>), grid, kThreads, 0, s, g, 4.0 + m0, (const s64*)x, 1.0,
                         (const s64*)U, (s64*)y, (const s64*)nullptr, st, st);
      break;
    case DW_PREC_F32:
      hipLaunchKernelGGL((k_dslash<float, s32, s32, s32, 0>), grid, kThreads, 0, s, g, (float)(4.0 + m0),
                         (const s32*)x, 1.0f, (const s32*)U, (s32*)y, (const s32*)nullptr, st, st);
      break;
    case DW_PREC_F16:
      hipLaunchKernelGGL((k_dslash<float, s16, s16, s16, 0>), grid, kThreads, 0, s, g, (float)(4.0 + m0),
                         (const s16*)x, 1.0f, (const s16*)U, (s16*)y, (const s16*)nullptr, st, st);
      break;
    case DW_PREC_BF16:
      hipLaunchKernelGGL((k_dslash<float, sbf, sbf, sbf, 0>), grid, kThreads, 0, s, g, (float)(4.0 + m0),
                         (const sbf*)x, 1.0f, (const sbf*)U, (sbf*)y, (const sbf*)nullptr, st, st);
      break;
    default: set_error("unknown precision %d", prec); return DW_EINVAL;
  }
  DW_CHECK_LAUNCH();
  kt.done((double)g.V * nrhs * 60.0 * pair_bytes(prec), (double)g.V * nrhs * kFlopsPerSite);
  return DW_OK;
}

}  // namespace dw
