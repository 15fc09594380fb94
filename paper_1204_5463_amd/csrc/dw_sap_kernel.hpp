// One colour of the Schwarz alternating procedure (paper Section 2, Alg. 2):
// the kernel template and its launch-shape selection, instantiated once per
// storage precision by k_sap_<prec>.hip.
//
// One workgroup per block of the given colour; blocks of one colour do not
// couple (red/black colouring with an even block count per direction), so
// the whole colour is one launch. Per block:
//   1. block residual r = (v - D z) restricted to the block, using z on the
//      block and its one-site halo in blocks of the other colour;
//   2. nmr minimal-residual steps on D^l y = r (eq. 2) starting from y = 0,
//      alpha = (p^H rho) / (p^H p) over the block's sites, with the
//      residual rho kept in LDS so that neighbours can read it and, when
//      they fit (FP32/FP16/BF16 storage), the block's links staged in LDS
//      once so the MR steps touch no global memory;
//   3. z += y on the block.
// With red2 = delta^2 > 0 the block solve is inexact in the adaptive sense
// (Section 3): a block stops at the first step n whose residual satisfies
// ||rho_n||^2 <= delta^2 ||r||^2, nmr being the largest step count. Only
// ||r||^2 takes a reduction of its own; each MR step lowers the squared
// residual norm by |p^H rho|^2 / p^H p (rho - alpha p is orthogonal to p),
// which the step's reductions already give, so the MR loop keeps its
// per-site work and the whole workgroup stops together.
// With z_zero set (first colour of the first cycle) z is not read and is
// initialised here: y on this colour's blocks, zero on the other colour's.
// Same-colour blocks never read each other's z, so updating z in place is
// race-free. Arithmetic is T (float for FP32/FP16/BF16 storage, double for
// FP64 storage); the block inner products are wavefront reductions followed
// by a fixed-order sum over the workgroup's waves (deterministic).
#pragma once

#include <cfloat>

#include <type_traits>

#include "dw_clover.hpp"
#include "dw_internal.hpp"
#include "dw_stencil.hpp"

namespace dw {

namespace sapk {

constexpr int kWave = 64;

// Wavefront sum. FP32: an inclusive scan within each row of 16 lanes by
// DPP row shifts, then the row totals combined by the row broadcasts, so
// that lane 63 holds the sum (no LDS traffic); its value is returned to all
// lanes. FP64 goes through cross-lane shuffles.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false);
  return v + __int_as_float(s);
}
template <typename T>
__device__ __forceinline__ T wave_sum(T a) {
  if constexpr (std::is_same<T, float>::value) {
    a = dpp_add<0x111, 0xf>(a);  // row_shr:1
    a = dpp_add<0x112, 0xf>(a);  // row_shr:2
    a = dpp_add<0x114, 0xf>(a);  // row_shr:4
    a = dpp_add<0x118, 0xf>(a);  // row_shr:8
    a = dpp_add<0x142, 0xa>(a);  // row_bcast:15 into rows 1 and 3
    a = dpp_add<0x143, 0xc>(a);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a), 63));
  } else {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
    return a;
  }
}

// BS > 0: hypercubic BS^4 blocks known at compile time (LDS offsets and
// link strides become immediates, local coordinates bit fields).
// CLOV: the operator includes the clover term Cl (site-local, dw_clover.hpp),
// in the residual and in every MR step.
// FP32 arithmetic without the clover term: ask for four waves per SIMD
// (at most 128 VGPRs), which keeps two 512-thread workgroups per CU; the
// other variants need more registers and take what they need.
template <typename T, bool CLOV>
constexpr int sap_waves_per_simd() {
  return std::is_same<T, float>::value && !CLOV ? 4 : 1;
}

template <typename T, typename SV, typename SZ, typename SG, int MAXT, bool LDSL, int BS, bool CLOV>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(sap_waves_per_simd<T, CLOV>())))
    k_sap_colour(Geom g, int colour, T diag, const SV* __restrict__ v, SZ* __restrict__ z, const SG* __restrict__ U,
                 int nmr, int z_zero, long long vs, long long zs, int nr, const int* __restrict__ rlist,
                 const SG* __restrict__ Cl, T red2, const int* __restrict__ gate, int gstride,
                 const double* __restrict__ dmass) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int bvol = BS > 0 ? BS * BS * BS * BS : g.bvol;
  // LDS: [links 36 x bvol (LDSL)] [rho 12 x bvol] [rho16 (P16)] [reduction 2 x nw x 3] [||r||^2 nw]
  SG* lks = reinterpret_cast<SG*>(smem);
  const size_t lbytes = LDSL ? (((size_t)36 * bvol * sizeof(SG) + 15) & ~(size_t)15) : 0;
  cplx<T>* rho_s = reinterpret_cast<cplx<T>*>(smem + lbytes);
  const int nw = blockDim.x / kWave;
  // FP16 storage: a packed FP16 copy of rho for the neighbours' hops
  constexpr bool P16 = std::is_same<SG, s16>::value && std::is_same<T, float>::value;
  h2v* rho16 = reinterpret_cast<h2v*>(rho_s + 12 * bvol);
  T* red = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(rho_s + 12 * bvol) + (P16 ? 12 * bvol * 4 : 0));
  auto put_rho = [&](int c, int site, cplx<T> r) {
    rho_s[c * bvol + site] = r;
    if constexpr (P16) rho16[c * bvol + site] = link16<s16>::pk(r.re, r.im);
  };
  // work item -> (block, right-hand side) with the RHS index fastest, so that
  // workgroups sharing a block's links run together on one XCD
  const int wi = xcd_remap(blockIdx.x, g.nbc * nr);
  if (wi < 0) return;  // whole workgroup: uniform exit before any barrier
  const int jb = wi / nr;
  const int rhs = rlist ? rlist[wi - jb * nr] : wi - jb * nr;
  if (gate && gate[(long long)rhs * gstride] == 0) return;  // uniform per workgroup, before any barrier
  if (dmass) diag = (T)(4.0 + *dmass);
  const int b = colour_block(g, colour, jb);
  const int l = threadIdx.x;
  const bool active = l < bvol;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const SV* vr = v + (long long)rhs * vs;
  SZ* zr = z + (long long)rhs * zs;
  const T half = (T)0.5;
  const T diag2 = diag + diag;

  // this block's spinors and links (contiguous chunks of the tiled layout)
  const SV* vb = vr + (long long)b * 12 * bvol;
  SZ* zb = zr + (long long)b * 12 * bvol;
  const SG* Ub = U + (long long)b * 36 * bvol;
  int bc[4], lc[4] = {0, 0, 0, 0};
  decode_block(g, b, bc);
  if (active) decode_local(g, l, lc);
  // the block's links, read once per launch
  if constexpr (LDSL) {
    if (active)
      for (int q = 0; q < 36; ++q) lks[q * bvol + l] = Ub[q * bvol + l];
  }
  // 16-bit links: hops take the raw packed entries (dot-product form)
  constexpr bool L16 = is_link16<SG> && std::is_same<T, float>::value;
  using LK = std::conditional_t<L16, SG, void>;
  auto load_link = [&](const SG* p) {
    if constexpr (L16) return link16<SG>::raw(p);
    else return ld<T>(p);
  };
  // links from memory: buffer loads with the block's links as the resource,
  // the entry's offset in a scalar register and the lane's site in one vector
  // register (no per-entry 64-bit address arithmetic)
  [[maybe_unused]] const __amdgpu_buffer_rsrc_t ub_rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)Ub, (short)0, 36 * bvol * (int)sizeof(SG), 0x00020000);
  auto u_blk = [&](int mu, int e, int ls) {
    constexpr int sz = (int)sizeof(SG);
    const int vo = ls * sz, so = (mu * 9 + e) * bvol * sz;
    if constexpr (LDSL) {
      return load_link(lks + (mu * 9 + e) * bvol + ls);
    } else if constexpr (L16 && sz == 4) {
      return __builtin_bit_cast(decltype(load_link(Ub)), __builtin_amdgcn_raw_buffer_load_b32(ub_rsrc, vo, so, 0));
    } else if constexpr (std::is_same<SG, s32>::value && std::is_same<T, float>::value) {
      typedef float f2 __attribute__((ext_vector_type(2)));
      const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(ub_rsrc, vo, so, 0));
      return mk<T>(v.x, v.y);
    } else if constexpr (std::is_same<SG, s64>::value && std::is_same<T, double>::value) {
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 v = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(ub_rsrc, vo, so, 0));
      return mk<T>(v.x, v.y);
    } else {
      return load_link(Ub + (mu * 9 + e) * bvol + ls);
    }
  };
  auto u_halo = [&](int nb, int mu, int e, int nl) {
    return load_link(U + ((long long)nb * 36 + mu * 9 + e) * bvol + nl);
  };

  // The MR residual rho lives in LDS only (neighbours read it there and
  // each thread re-reads its own site), which keeps the register footprint
  // low enough for four waves per SIMD.
  cplx<T> y[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) y[c] = mk<T>(0, 0);
  if (!z_zero) {
    // block residual r = v - D z: z of this block staged in LDS, the one-site
    // halo of z read from the neighbouring blocks of the other colour
    if (active) {
#pragma unroll
      for (int c = 0; c < 12; ++c) rho_s[c * bvol + l] = ld<T>(zb + c * bvol + l);
    }
    __syncthreads();
    cplx<T> acc[12];
    if (active) {
      if constexpr (BS > 0 && std::is_same<T, float>::value)
        hop_sum_halo_ahead<T, LK, BS>(
            g, b, l, bc, [&](int nl, int k) { return rho_s[k * bvol + nl]; },
            [&](int nb, int nl, int k) { return ld<T>(zr + ((long long)nb * 12 + k) * bvol + nl); },
            [&](int nb, int mu, int e, int nl) { return u_halo(nb, mu, e, nl); }, acc);
      else
        hop_sum_staged<T, true, LK, BS>(
            g, b, l, bc, lc, [&](int nl, int k) { return rho_s[k * bvol + nl]; }, u_blk,
            [&](int nb, int nl, int k) { return ld<T>(zr + ((long long)nb * 12 + k) * bvol + nl); }, u_halo, acc);
      if constexpr (CLOV) {
        // -1/2 hops + C z = -1/2 (hops - 2 C z)
        clover_acc_f<T>(Cl + (long long)b * kCloverPairs * bvol, bvol, l,
                        [&](int c) { return rho_s[c * bvol + l]; }, (T)-2, acc);
      }
#pragma unroll
      for (int c = 0; c < 12; ++c)
        acc[c] = ld<T>(vb + c * bvol + l) - diag * rho_s[c * bvol + l] + half * acc[c];
    }
    __syncthreads();  // z reads from LDS done before rho overwrites it
    if (active) {
#pragma unroll
      for (int c = 0; c < 12; ++c) put_rho(c, l, acc[c]);
    }
  } else if (active) {
#pragma unroll
    for (int c = 0; c < 12; ++c) put_rho(c, l, ld<T>(vb + c * bvol + l));
  }

  // adaptive stop: rr0 = ||r||^2 over the block, rr = ||rho_it||^2
  const bool adapt = red2 > (T)0;
  T rr0 = 0, rr = 0;
  if (adapt) {
    __syncthreads();  // rho written
    T sq = 0;
    if (active) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sq += norm2(rho_s[c * bvol + l]);
    }
    sq = wave_sum(sq);
    if (lane == 0) red[6 * nw + wave] = sq;
    __syncthreads();
    for (int w = 0; w < nw; ++w) rr0 += red[6 * nw + w];
    rr = rr0;
  }
  // FP16 links without the clover term on 4^4 blocks: the lane's own x, y and
  // z links stay in registers through the MR steps; the backward hops read the
  // neighbour's links from the lane 1, 4 or 16 below (a wave holds one t slice
  // of the block, x fastest), so an MR step loads only the t links. This cuts
  // the step's link traffic, which would otherwise come from beyond the L2
  // (the links of the blocks in flight exceed it), to a quarter.
  constexpr int NREG = (BS == 4 && L16 && !CLOV && !LDSL) ? 4 : 0;
  using XW = std::conditional_t<(NREG > 0), decltype(u_blk(0, 0, 0)), int>;
  XW ux[NREG > 0 ? NREG : 1][9];
  if constexpr (NREG > 0) {
#pragma unroll
    for (int d = 0; d < NREG; ++d)
#pragma unroll
      for (int e = 0; e < 9; ++e) ux[d][e] = u_blk(d, e, l);
  }
  for (int it = 0; it < nmr; ++it) {
    if (adapt && rr <= red2 * rr0) break;  // uniform over the workgroup
    __syncthreads();  // rho (and staged links) visible to the whole block
    cplx<T> p[12];
    T nre = 0, nim = 0, den = 0;
    if (active) {
      // links loaded one hop ahead where the registers allow it without
      // losing occupancy (16-bit links, no clover term)
      constexpr bool AHEAD = BS > 0 && !CLOV;
      if constexpr (AHEAD && P16)
        hop_sum_block_unrolled<T, h2v, BS, NREG>(l, [&](int nl, int k) { return rho16[k * bvol + nl]; }, u_blk,
                                                 p, reinterpret_cast<const XW(*)[9]>(ux));
      else if constexpr (AHEAD && NREG > 0)
        hop_sum_block_unrolled<T, LK, BS, NREG>(l, [&](int nl, int k) { return rho_s[k * bvol + nl]; }, u_blk, p,
                                                reinterpret_cast<const XW(*)[9]>(ux));
      else if constexpr (AHEAD)
        hop_sum_block_unrolled<T, LK, BS>(l, [&](int nl, int k) { return rho_s[k * bvol + nl]; }, u_blk, p);
      else if constexpr (P16)
        hop_sum_staged<T, false, h2v, BS>(
            g, b, l, bc, lc, [&](int nl, int k) { return rho16[k * bvol + nl]; }, u_blk,
            [&](int, int, int) { return h2v{0, 0}; }, u_halo, p);
      else
        hop_sum_staged<T, false, LK, BS>(
            g, b, l, bc, lc, [&](int nl, int k) { return rho_s[k * bvol + nl]; }, u_blk,
            [&](int, int, int) { return mk<T>(0, 0); }, u_halo, p);
      if constexpr (CLOV) {
        // the clover entries are re-read every MR step: an offset the
        // compiler cannot see through keeps their loads inside the loop
        // (hoisted, they would hold 72 registers)
        int cofs = 0;
        asm volatile("" : "+v"(cofs));
        clover_acc_f<T>(Cl + (long long)b * kCloverPairs * bvol + cofs, bvol, l,
                        [&](int c) { return rho_s[c * bvol + l]; }, (T)-2, p);
      }
      // p2 = 2 D^l rho = 2 diag rho - hops: the factor 2 cancels in the
      // residual update (alpha p = alpha2 p2 with alpha2 = (p2^H rho)/(p2^H p2))
      // and is restored in the iterate update, which saves the 1/2 scaling
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const cplx<T> r = rho_s[c * bvol + l];
        p[c] = mk<T>(fma(diag2, r.re, -p[c].re), fma(diag2, r.im, -p[c].im));
        nre = fma(p[c].re, r.re, nre);
        nre = fma(p[c].im, r.im, nre);
        nim = fma(p[c].re, r.im, nim);
        nim = fma(-p[c].im, r.re, nim);
        den = fma(p[c].re, p[c].re, den);
        den = fma(p[c].im, p[c].im, den);
      }
    }
    nre = wave_sum(nre);
    nim = wave_sum(nim);
    den = wave_sum(den);
    T* rb = red + (it & 1) * 3 * nw;
    if (lane == 0) {
      rb[wave * 3 + 0] = nre;
      rb[wave * 3 + 1] = nim;
      rb[wave * 3 + 2] = den;
    }
    __syncthreads();  // also: every hop sum of this step has read rho
    nre = nim = den = 0;
    for (int w = 0; w < nw; ++w) {
      nre += rb[w * 3 + 0];
      nim += rb[w * 3 + 1];
      den += rb[w * 3 + 2];
    }
    // alpha = (p2^H rho) / (p2^H p2); in FP32 one hardware reciprocal
    // (1 ulp) replaces the two IEEE divisions
    cplx<T> alpha = mk<T>(0, 0);
    if constexpr (std::is_same<T, float>::value) {
      const float inv = den > FLT_MIN ? __builtin_amdgcn_rcpf(den) : 0.f;
      alpha = mk<T>(nre * inv, nim * inv);
      if (adapt) rr -= (nre * nre + nim * nim) * inv;
    } else if (den > (T)0) {
      alpha = mk<T>(nre / den, nim / den);
      if (adapt) rr -= (nre * nre + nim * nim) / den;
    }
    const cplx<T> alpha_y = mk<T>(alpha.re + alpha.re, alpha.im + alpha.im);
    if (active) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        cplx<T> r = rho_s[c * bvol + l];
        cmac(y[c], alpha_y, r);
        cmsub(r, alpha, p[c]);
        put_rho(c, l, r);
      }
    }
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      SZ* zp = zb + c * bvol + l;
      st(zp, z_zero ? y[c] : ld<T>(zp) + y[c]);
    }
    // z starts at zero: this workgroup also clears one block of the other
    // colour (same count per colour), which this launch never reads
    if (z_zero) {
      const int bo = colour_block(g, 1 - colour, jb);
#pragma unroll
      for (int c = 0; c < 12; ++c) st(zr + ((long long)bo * 12 + c) * bvol + l, mk<T>(0, 0));
    }
  }
}

template <typename T, typename SV, typename SZ, typename SG, int MAXT, bool LDSL, int BS, bool CLOV>
dw_status launch_t(const Geom& g, double m0, const void* v, void* z, const void* U, int colour, int nmr, int z_zero,
                   int nrhs, long long vs, long long zs, const int* rlist, hipStream_t s, const void* C, double red2, const int* gate, int gs, const double* dmass) {
  const int threads = ((g.bvol + kWave - 1) / kWave) * kWave;
  const size_t lbytes = LDSL ? (((size_t)36 * g.bvol * sizeof(SG) + 15) & ~(size_t)15) : 0;
  constexpr bool P16 = std::is_same<SG, s16>::value && std::is_same<T, float>::value;
  const size_t shmem = lbytes + (size_t)12 * g.bvol * sizeof(cplx<T>) + (P16 ? (size_t)12 * g.bvol * 4 : 0) +
                       (size_t)(2 * 3 + 1) * (threads / kWave) * sizeof(T);
  if (shmem > 160 * 1024) {
    set_error("SAP block of %d sites needs %zu bytes of LDS", g.bvol, shmem);
    return DW_EINVAL;
  }
  if (shmem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sap_colour<T, SV, SZ, SG, MAXT, LDSL, BS, CLOV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) {
      set_error("hipFuncSetAttribute(LDS %zu bytes) failed: %s", shmem, hipGetErrorString(e));
      return DW_EHIP;
    }
  }
  dim3 grid((unsigned)xcd_grid(g.nbc * nrhs), 1);
  KTimer kt(DW_K_SAP, s);
  hipLaunchKernelGGL((k_sap_colour<T, SV, SZ, SG, MAXT, LDSL, BS, CLOV>), grid, threads, shmem, s, g, colour,
                     (T)(4.0 + m0), (const SV*)v, (SZ*)z, (const SG*)U, nmr, z_zero, vs, zs, nrhs, rlist,
                     (const SG*)C, (T)red2, gate, gs, dmass);
  DW_CHECK_LAUNCH();
  // algorithmic traffic per site of this colour: v, 4 links, z read (or the
  // other colour's z cleared) and z written; flops: block residual stencil
  // plus nmr MR steps (block stencil over the kept hops + 4 block vector ops);
  // with the adaptive stop nmr is only the cap and the flops an upper bound
  double kept = 0;
  for (int mu = 0; mu < 4; ++mu) kept += 2.0 * (g.B[mu] - 1) / g.B[mu];
  const double sites = (double)g.nbc * g.bvol * nrhs;
  const double sv = sizeof(SV), sz = sizeof(SZ), sg = sizeof(SG);
  const double csteps = CLOV ? nmr + (z_zero ? 0 : 1) : 0;
  kt.done(sites * (12 * sv + 36 * sg + 24 * sz + (CLOV ? kCloverPairs * sg : 0)),
          sites * ((z_zero ? 0.0 : 1368.0) + nmr * (48.0 + 168.0 * kept + 336.0) + csteps * kCloverFlops));
  return DW_OK;
}

template <typename T, typename SV, typename SZ, typename SG, int MAXT, bool CLOV>
dw_status launch_m(const Geom& g, double m0, const void* v, void* z, const void* U, int colour, int nmr, int z_zero,
                   int nrhs, long long vs, long long zs, const int* rlist, hipStream_t s, const void* C,
                   double red2, const int* gate, int gs, const double* dmass) {
  // Stage the block's links in LDS only when that keeps several workgroups
  // per CU: the MR steps are VALU bound and lose more to lower occupancy
  // than they gain from fewer cached link reads (measured on 4^4 blocks
  // with FP16 links: 380 us with links from L1/L2, 517 us staged).
  const size_t need = (size_t)36 * g.bvol * sizeof(SG) + (size_t)12 * g.bvol * sizeof(cplx<T>) + 512;
  const bool hyper4 = g.B[0] == 4 && g.B[1] == 4 && g.B[2] == 4 && g.B[3] == 4;
  if constexpr (MAXT == 256)
    if (hyper4 && need > 40 * 1024)
      return launch_t<T, SV, SZ, SG, 256, false, 4, CLOV>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s,
                                                          C, red2, gate, gs, dmass);
  if (need <= 40 * 1024)
    return launch_t<T, SV, SZ, SG, MAXT, true, 0, CLOV>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s,
                                                        C, red2, gate, gs, dmass);
  return launch_t<T, SV, SZ, SG, MAXT, false, 0, CLOV>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s,
                                                       C, red2, gate, gs, dmass);
}

template <typename T, typename SV, typename SZ, typename SG, bool CLOV>
dw_status launch_b(const Geom& g, double m0, const void* v, void* z, const void* U, int colour, int nmr, int z_zero,
                   int nrhs, long long vs, long long zs, const int* rlist, hipStream_t s, const void* C,
                   double red2, const int* gate, int gs, const double* dmass) {
  if (g.bvol <= 256)
    return launch_m<T, SV, SZ, SG, 256, CLOV>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s, C, red2, gate, gs, dmass);
  if (g.bvol <= 512)
    return launch_m<T, SV, SZ, SG, 512, CLOV>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s, C, red2, gate, gs, dmass);
  return launch_m<T, SV, SZ, SG, 1024, CLOV>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s, C, red2, gate, gs, dmass);
}

template <typename T, typename SV, typename SZ, typename SG>
dw_status launch(const Geom& g, double m0, const void* v, void* z, const void* U, int colour, int nmr, int z_zero,
                 int nrhs, long long vs, long long zs, const int* rlist, hipStream_t s, const void* C,
                   double red2, const int* gate, int gs, const double* dmass) {
  if (C) return launch_b<T, SV, SZ, SG, true>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s, C, red2, gate, gs, dmass);
  return launch_b<T, SV, SZ, SG, false>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s, C, red2, gate, gs, dmass);
}

}  // namespace sapk

}  // namespace dw
