// Wilson-Dirac operator on the whole periodic lattice (paper eq. 1).
//
// One workgroup per storage block, one thread per site. The block's
// spinor is staged in LDS once, so in-block neighbours are read from LDS;
// only the faces of neighbouring blocks come from L2/HBM. Every link is read
// once: a thread loads its own forward link U_mu(n), uses it for the
// forward hop and also forms U_mu(n)^+ (1 + g_mu) psi(n), the backward-hop
// half spinor that site n + mu needs, and hands it over through LDS
// (sites on a block's lower face compute theirs from the neighbouring
// block). Launch order is XCD-aware so neighbouring blocks share an L2.
// Blocks whose LDS footprint exceeds the CU's 160 KiB fall back to a
// gather kernel that reads all neighbours through the caches.
//
// Bandwidth bound: per site and right-hand side the algorithmic traffic is
// one spinor read, 4 links read and one spinor write (FP64: 960 bytes). The
// result is written with streaming stores (it is not read again by this
// launch), which leaves more of the caches to the block faces.
#include "dw_clover.hpp"
#include "dw_internal.hpp"
#include "dw_stencil.hpp"

namespace dw {

namespace {

constexpr int kThreads = 256;
// flops of one site of D: 8 hops x (12 projection + 2 x 66 SU(3) x vector
// + 24 accumulation) - 24 (first accumulation is a copy) + 48 (diagonal)
constexpr double kFlopsPerSite = 1368.0;

// ---- block-staged kernel ---------------------------------------------------------
template <typename T, typename SX, typename SG>
struct BlkCtx {
  const Geom& g;
  int b, l;
  bool active;
  const int* bc;
  const int* lc;
  const SX* xr;
  const SX* xsh;   // LDS: block spinor [12][bvol], storage type
  cplx<T>* pb;     // LDS: handed-over half spinors [6][bvol]
  const SG* U;
};

template <int MU, typename T, typename SX, typename SG>
__device__ __forceinline__ void blk_dir(const BlkCtx<T, SX, SG>& c, cplx<T> acc[12], const cplx<T> psi[12]) {
  const Geom& g = c.g;
  const int bvol = g.bvol, l = c.l;
  const int st = g.lstride[MU];
  cplx<T> h0[3], h1[3], g0[3], g1[3];
  if (c.active) {
    cplx<T> w[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) w[e] = ld<T>(c.U + gauge_index(g, c.b, MU, e, l));
    auto wl = [&](int e) { return w[e]; };
    // backward-hop half spinor for site n + mu: U_mu(n)^+ (1 + g_mu) psi(n)
    proj<MU, -1, T>([&](int k) { return psi[k]; }, h0, h1);
    su3_mul<true, T>(wl, h0, h1, g0, g1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c.pb[a * bvol + l] = g0[a];
      c.pb[(3 + a) * bvol + l] = g1[a];
    }
    // forward hop: (1 - g_mu) U_mu(n) psi(n + mu)
    if (c.lc[MU] < g.B[MU] - 1) {
      proj<MU, +1, T>([&](int k) { return ld<T>(c.xsh + k * bvol + l + st); }, h0, h1);
    } else {
      int c2[4] = {c.bc[0], c.bc[1], c.bc[2], c.bc[3]};
      c2[MU] = (c.bc[MU] + 1 == g.N[MU]) ? 0 : c.bc[MU] + 1;
      const int nb = encode_block(g, c2), nl = l - (g.B[MU] - 1) * st;
      proj<MU, +1, T>([&](int k) { return ld<T>(c.xr + spinor_index(g, nb, k, nl)); }, h0, h1);
    }
    su3_mul<false, T>(wl, h0, h1, g0, g1);
    recon_acc<MU, +1, T>(acc, g0, g1);
  }
  __syncthreads();
  if (c.active) {
    if (c.lc[MU] > 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        g0[a] = c.pb[a * bvol + l - st];
        g1[a] = c.pb[(3 + a) * bvol + l - st];
      }
    } else {
      int c2[4] = {c.bc[0], c.bc[1], c.bc[2], c.bc[3]};
      c2[MU] = (c.bc[MU] == 0) ? g.N[MU] - 1 : c.bc[MU] - 1;
      const int nb = encode_block(g, c2), nl = l + (g.B[MU] - 1) * st;
      proj<MU, -1, T>([&](int k) { return ld<T>(c.xr + spinor_index(g, nb, k, nl)); }, h0, h1);
      su3_mul<true, T>([&](int e) { return ld<T>(c.U + gauge_index(g, nb, MU, e, nl)); }, h0, h1, g0, g1);
    }
    recon_acc<MU, -1, T>(acc, g0, g1);
  }
  __syncthreads();
}

// FP16 spinors and links: the same scheme with packed FP16 operands. The
// half spinors are projected in packed FP16 arithmetic (one rounding to
// FP16 per entry) and multiplied by the raw link entries with two-term dot
// products accumulated in FP32 (exact products), so a hop is 36 dot
// products, 12 packed adds and the FP32 rebuild. psi16 holds the site's
// own spinor as packed (re, im) pairs.
template <int MU, typename SX, typename SG>
__device__ __forceinline__ void blk_dir16(const BlkCtx<float, SX, SG>& c, cplx<float> acc[12], const h2v psi16[12]) {
  const Geom& g = c.g;
  const int bvol = g.bvol, l = c.l;
  const int st = g.lstride[MU];
  const h2v* xsh = reinterpret_cast<const h2v*>(c.xsh);
  const h2v* xr = reinterpret_cast<const h2v*>(c.xr);
  const h2v* U = reinterpret_cast<const h2v*>(c.U);
  cplx<float> g0[3], g1[3];
  if (c.active) {
    h2v w[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) w[e] = U[gauge_index(g, c.b, MU, e, l)];
    auto wl = [&](int e) { return w[e]; };
    // backward-hop half spinor for site n + mu: U_mu(n)^+ (1 + g_mu) psi(n)
    hop16p_g<MU, -1>([&](int k) { return psi16[k]; }, wl, g0, g1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c.pb[a * bvol + l] = g0[a];
      c.pb[(3 + a) * bvol + l] = g1[a];
    }
    // forward hop: (1 - g_mu) U_mu(n) psi(n + mu)
    if (c.lc[MU] < g.B[MU] - 1) {
      hop16p<MU, +1>(acc, [&](int k) { return xsh[k * bvol + l + st]; }, wl);
    } else {
      int c2[4] = {c.bc[0], c.bc[1], c.bc[2], c.bc[3]};
      c2[MU] = (c.bc[MU] + 1 == g.N[MU]) ? 0 : c.bc[MU] + 1;
      const int nb = encode_block(g, c2), nl = l - (g.B[MU] - 1) * st;
      hop16p<MU, +1>(acc, [&](int k) { return xr[spinor_index(g, nb, k, nl)]; }, wl);
    }
  }
  __syncthreads();
  if (c.active) {
    if (c.lc[MU] > 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        g0[a] = c.pb[a * bvol + l - st];
        g1[a] = c.pb[(3 + a) * bvol + l - st];
      }
      recon_acc<MU, -1, float>(acc, g0, g1);
    } else {
      int c2[4] = {c.bc[0], c.bc[1], c.bc[2], c.bc[3]};
      c2[MU] = (c.bc[MU] == 0) ? g.N[MU] - 1 : c.bc[MU] - 1;
      const int nb = encode_block(g, c2), nl = l + (g.B[MU] - 1) * st;
      hop16p<MU, -1>(acc, [&](int k) { return xr[spinor_index(g, nb, k, nl)]; },
                     [&](int e) { return U[gauge_index(g, nb, MU, e, nl)]; });
    }
  }
  __syncthreads();
}

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// per-right-hand-side gate and device-side mass (both optional)
struct DCtl {
  const int* gate = nullptr;
  int gstride = 0;
  const double* dmass = nullptr;
};

// CLOV: add the clover term (site-local, dw_clover.hpp) from Cl.
template <typename T, typename SX, typename SG, typename SY, int MODE, int MAXT, bool CLOV>
__global__ void __launch_bounds__(MAXT)
    k_dslash_blk(Geom g, T diag, const SX* __restrict__ x, T scale, const SG* __restrict__ U, SY* __restrict__ y,
                 const SY* __restrict__ bsrc, long long xs, long long ys, int nr, const int* __restrict__ rlist,
                 const SG* __restrict__ Cl, DCtl dc) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  SX* xsh = reinterpret_cast<SX*>(smem);
  cplx<T>* pb = reinterpret_cast<cplx<T>*>(smem + align16((size_t)12 * g.bvol * sizeof(SX)));
  // work item -> (block, RHS) with the RHS fastest: workgroups that read the
  // same links run together on one XCD
  const int wi = xcd_remap(blockIdx.x, g.nblk * nr);
  if (wi < 0) return;  // uniform for the workgroup
  const int b = wi / nr;
  const int rhs = rlist ? rlist[wi - b * nr] : wi - b * nr;
  if (dc.gate && dc.gate[(long long)rhs * dc.gstride] == 0) return;  // uniform for the workgroup
  if (dc.dmass) diag = (T)(4.0 + *dc.dmass);
  const int l = threadIdx.x;
  const bool active = l < g.bvol;
  const SX* xr = x + (long long)rhs * xs;
  SY* yr = y + (long long)rhs * ys;
  int bc[4], lc[4] = {0, 0, 0, 0};
  decode_block(g, b, bc);
  cplx<T> psi[12], acc[12];
  // FP16 spinors and links without the clover term: packed FP16 hops
  constexpr bool P16 = std::is_same<SX, s16>::value && std::is_same<SG, s16>::value &&
                       std::is_same<T, float>::value && !CLOV;
  h2v psi16[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    psi[k] = mk<T>(0, 0);
    acc[k] = mk<T>(0, 0);
    psi16[k] = h2v{0, 0};
  }
  if (active) {
    decode_local(g, l, lc);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const SX v = xr[spinor_index(g, b, k, l)];
      xsh[k * g.bvol + l] = v;
      psi[k] = storage_traits<SX>::template load<T>(v);
      if constexpr (P16) psi16[k] = __builtin_bit_cast(h2v, v);
    }
  }
  __syncthreads();
  const BlkCtx<T, SX, SG> c{g, b, l, active, bc, lc, xr, xsh, pb, U};
  if constexpr (P16) {
    blk_dir16<0>(c, acc, psi16);
    blk_dir16<1>(c, acc, psi16);
    blk_dir16<2>(c, acc, psi16);
    blk_dir16<3>(c, acc, psi16);
  } else {
    blk_dir<0>(c, acc, psi);
    blk_dir<1>(c, acc, psi);
    blk_dir<2>(c, acc, psi);
    blk_dir<3>(c, acc, psi);
  }
  if (active) {
    const T half = (T)0.5;
    if constexpr (CLOV) {
      // acc holds the hop sum; -1/2 acc + C psi = -1/2 (acc - 2 C psi)
      cplx<T> cx[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) cx[k] = mk<T>(0, 0);
      clover_acc<T>(Cl + (long long)b * kCloverPairs * g.bvol, g.bvol, l, psi, cx);
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] -= (T)2 * cx[k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const long long idx = spinor_index(g, b, k, l);
      cplx<T> d = scale * (diag * psi[k] - half * acc[k]);
      if constexpr (MODE == 1) d = ld<T>(bsrc + (long long)rhs * ys + idx) - d;
      st_nt(yr + idx, d);
    }
  }
}

template <typename T, typename SX>
size_t blk_lds(const Geom& g) {
  return align16((size_t)12 * g.bvol * sizeof(SX)) + (size_t)6 * g.bvol * sizeof(cplx<T>);
}

// ---- gather kernel (blocks too large for LDS staging) -------------------------------
// MODE 0: y = scale * D x ; MODE 1: y = b - scale * D x
template <typename T, typename SX, typename SG, typename SY, int MODE, bool CLOV>
__global__ void __launch_bounds__(kThreads)
    k_dslash(Geom g, T diag, const SX* __restrict__ x, T scale, const SG* __restrict__ U, SY* __restrict__ y,
             const SY* __restrict__ bsrc, long long xs, long long ys, int nr, const int* __restrict__ rlist,
             const SG* __restrict__ Cl, DCtl dc) {
  const int chunk = xcd_remap(blockIdx.x, (int)((g.V + kThreads - 1) / kThreads));
  if (chunk < 0) return;
  const long long s = (long long)chunk * kThreads + threadIdx.x;
  if (s >= g.V) return;
  const int rhs = rlist ? rlist[blockIdx.y] : blockIdx.y;
  if (dc.gate && dc.gate[(long long)rhs * dc.gstride] == 0) return;
  if (dc.dmass) diag = (T)(4.0 + *dc.dmass);
  const SX* xr = x + (long long)rhs * xs;
  SY* yr = y + (long long)rhs * ys;
  const int b = (int)(s / g.bvol);
  const int l = (int)(s - (long long)b * g.bvol);
  int bc[4], lc[4];
  decode_block(g, b, bc);
  decode_local(g, l, lc);
  cplx<T> acc[12];
  hop_sum_lattice<T>(g, b, l, bc, lc, U,
                     [&](int nb, int nl, int comp) { return ld<T>(xr + spinor_index(g, nb, comp, nl)); }, acc);
  const T half = (T)0.5;
  if constexpr (CLOV) {
    cplx<T> xo[12], cx[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      xo[c] = ld<T>(xr + spinor_index(g, b, c, l));
      cx[c] = mk<T>(0, 0);
    }
    clover_acc<T>(Cl + (long long)b * kCloverPairs * g.bvol, g.bvol, l, xo, cx);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] -= (T)2 * cx[c];
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const long long idx = spinor_index(g, b, c, l);
    cplx<T> xo = ld<T>(xr + idx);
    cplx<T> d = scale * (diag * xo - half * acc[c]);
    if constexpr (MODE == 1) {
      const SY* br = bsrc + (long long)rhs * ys;
      d = ld<T>(br + idx) - d;
    }
    st(yr + idx, d);
  }
}

template <typename T, typename SX, typename SG, typename SY, int MODE, bool CLOV>
dw_status launch_any(const Geom& g, T diag, const SX* x, T scale, const SG* U, SY* y, const SY* b, long long xs,
                     long long ys, int nrhs, const int* rlist, hipStream_t s, const SG* Cl, DCtl dc);

dim3 grid_for(const Geom& g, int nrhs) {
  return dim3((unsigned)xcd_grid((int)((g.V + kThreads - 1) / kThreads)), (unsigned)nrhs);
}

template <typename T, typename SX, typename SG, typename SY, int MODE, bool CLOV>
dw_status launch_any(const Geom& g, T diag, const SX* x, T scale, const SG* U, SY* y, const SY* b, long long xs,
                     long long ys, int nrhs, const int* rlist, hipStream_t s, const SG* Cl, DCtl dc) {
  const size_t lds = blk_lds<T, SX>(g);
  const int threads = ((g.bvol + 63) / 64) * 64;
  if (lds <= 160 * 1024) {
    auto launch_t = [&](auto kernel) -> dw_status {
      if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
          set_error("hipFuncSetAttribute(LDS %zu) failed: %s", lds, hipGetErrorString(e));
          return DW_EHIP;
        }
      }
      dim3 grid((unsigned)xcd_grid(g.nblk * nrhs), 1);
      hipLaunchKernelGGL(kernel, grid, threads, lds, s, g, diag, x, scale, U, y, b, xs, ys, nrhs, rlist, Cl, dc);
      DW_CHECK_LAUNCH();
      return DW_OK;
    };
    if (threads <= 256) return launch_t(k_dslash_blk<T, SX, SG, SY, MODE, 256, CLOV>);
    if (threads <= 512) return launch_t(k_dslash_blk<T, SX, SG, SY, MODE, 512, CLOV>);
    return launch_t(k_dslash_blk<T, SX, SG, SY, MODE, 1024, CLOV>);
  }
  hipLaunchKernelGGL((k_dslash<T, SX, SG, SY, MODE, CLOV>), grid_for(g, nrhs), kThreads, 0, s, g, diag, x, scale, U,
                     y, b, xs, ys, nrhs, rlist, Cl, dc);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

// dispatch on the presence of a clover term
template <typename T, typename SX, typename SG, typename SY, int MODE>
dw_status launch_c(const Geom& g, T diag, const SX* x, T scale, const SG* U, SY* y, const SY* b, long long xs,
                   long long ys, int nrhs, const int* rlist, hipStream_t s, const SG* Cl, DCtl dc = DCtl{}) {
  if (Cl) return launch_any<T, SX, SG, SY, MODE, true>(g, diag, x, scale, U, y, b, xs, ys, nrhs, rlist, s, Cl, dc);
  return launch_any<T, SX, SG, SY, MODE, false>(g, diag, x, scale, U, y, b, xs, ys, nrhs, rlist, s, Cl, dc);
}

}  // namespace

dw_status launch_dslash_outer(const Geom& g, double m0, int prec_x, const void* x, double scale, const void* U64,
                              double* y, const double* b, int mode, int nrhs, long long xs, long long ys,
                              hipStream_t s, const int* rlist, const void* C64, const int* gate, int gstride,
                              const double* dmass) {
  if (nrhs < 1) return DW_OK;
  const double diag = 4.0 + m0;
  DCtl dc;
  dc.gate = gate;
  dc.gstride = gstride;
  dc.dmass = dmass;
  const s64* Ug = (const s64*)U64;
  const s64* Cg = (const s64*)C64;
  s64* yo = (s64*)y;
  const s64* bo = (const s64*)b;
  KTimer kt(DW_K_DSLASH_F64, s);
  dw_status st;
  if (prec_x == DW_PREC_F64) {
    const s64* xi = (const s64*)x;
    st = mode == 0 ? launch_c<double, s64, s64, s64, 0>(g, diag, xi, scale, Ug, yo, bo, xs, ys, nrhs, rlist, s, Cg, dc)
                   : launch_c<double, s64, s64, s64, 1>(g, diag, xi, scale, Ug, yo, bo, xs, ys, nrhs, rlist, s, Cg, dc);
  } else if (prec_x == DW_PREC_F32) {
    const s32* xi = (const s32*)x;
    st = mode == 0 ? launch_c<double, s32, s64, s64, 0>(g, diag, xi, scale, Ug, yo, bo, xs, ys, nrhs, rlist, s, Cg, dc)
                   : launch_c<double, s32, s64, s64, 1>(g, diag, xi, scale, Ug, yo, bo, xs, ys, nrhs, rlist, s, Cg, dc);
  } else {
    set_error("outer dslash input precision must be F64 or F32");
    return DW_EINVAL;
  }
  DW_TRY(st);
  kt.done((double)g.V * nrhs *
              (12.0 * pair_bytes(prec_x) + 36 * 16 + 12 * 16 + (mode == 1 ? 12 * 16 : 0) + (Cg ? kCloverPairs * 16 : 0)),
          (double)g.V * nrhs * (kFlopsPerSite + (Cg ? kCloverFlops : 0.0)));
  return DW_OK;
}

dw_status launch_dslash_a32(const Geom& g, const void* x, const void* U32, void* y, int nrhs, long long xs,
                            long long ys, hipStream_t s, const int* rlist, const void* C32, const int* gate, int gstride,
                            const double* dmass) {
  if (nrhs < 1) return DW_OK;
  DCtl dc;
  dc.gate = gate;
  dc.gstride = gstride;
  dc.dmass = dmass;
  KTimer kt(DW_K_DSLASH_LOWP, s);
  DW_TRY((launch_c<float, s32, s32, s32, 0>(g, 4.0f, (const s32*)x, 1.0f, (const s32*)U32, (s32*)y, nullptr, xs, ys,
                                             nrhs, rlist, s, (const s32*)C32, dc)));
  kt.done((double)g.V * nrhs * (60.0 * 8 + (C32 ? kCloverPairs * 8 : 0)),
          (double)g.V * nrhs * (kFlopsPerSite + (C32 ? kCloverFlops : 0.0)));
  return DW_OK;
}

dw_status launch_dslash_lowp(const Geom& g, double m0, int prec, const void* x, const void* U, void* y, int nrhs,
                             hipStream_t s, const void* C) {
  const long long sd = g.V * 12;
  KTimer kt(DW_K_DSLASH_LOWP, s);
  dw_status st;
  const float df = (float)(4.0 + m0);
  switch (prec) {
    case DW_PREC_F64:
      st = launch_c<double, s64, s64, s64, 0>(g, 4.0 + m0, (const s64*)x, 1.0, (const s64*)U, (s64*)y, nullptr, sd,
                                              sd, nrhs, nullptr, s, (const s64*)C);
      break;
    case DW_PREC_F32:
      st = launch_c<float, s32, s32, s32, 0>(g, df, (const s32*)x, 1.0f, (const s32*)U, (s32*)y, nullptr, sd, sd,
                                             nrhs, nullptr, s, (const s32*)C);
      break;
    case DW_PREC_F16:
      st = launch_c<float, s16, s16, s16, 0>(g, df, (const s16*)x, 1.0f, (const s16*)U, (s16*)y, nullptr, sd, sd,
                                             nrhs, nullptr, s, (const s16*)C);
      break;
    case DW_PREC_BF16:
      st = launch_c<float, sbf, sbf, sbf, 0>(g, df, (const sbf*)x, 1.0f, (const sbf*)U, (sbf*)y, nullptr, sd, sd,
                                             nrhs, nullptr, s, (const sbf*)C);
      break;
    default: set_error("unknown precision %d", prec); return DW_EINVAL;
  }
  DW_TRY(st);
  kt.done((double)g.V * nrhs * (60.0 + (C ? kCloverPairs : 0)) * pair_bytes(prec),
          (double)g.V * nrhs * (kFlopsPerSite + (C ? kCloverFlops : 0.0)));
  return DW_OK;
}

}  // namespace dw
