// The Wilson-Dirac hopping term, site by site (paper Section 2, eq. 1).
//
//   (D x)(n) = (4 + m0) x(n)
//              - 1/2 sum_mu [ (1 - g_mu) U_mu(n) x(n+mu) + (1 + g_mu) U_mu(n-mu)^+ x(n-mu) ]
//
// Each of the 8 hops projects the neighbour spinor onto a half spinor
// (two spin components), multiplies both by the SU(3) link and rebuilds
// the lower two spin components from the upper two. The gamma matrices
// are in the Euclidean chiral basis
//   g_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z),  g_t = [[0, 1], [1, 0]],
// for which (1 -/+ g_mu) psi = [h; c h] with h = psi_up -/+ A_mu psi_dn.
//
// Per direction and sign the projection is h0 = psi0 + a*psi_pa,
// h1 = psi1 + b*psi_pb and the reconstruction r2 = c*h_qc, r3 = d*h_qd,
// with a, b, c, d in {+1, -1, +i, -i}.
#pragma once

#include <type_traits>
#include <utility>

#include "dw_geom.hpp"
#include "dw_types.hpp"

namespace dw {

enum { CP1 = 0, CM1 = 1, CPI = 2, CMI = 3 };

template <int K, typename T>
__device__ __forceinline__ cplx<T> coef(cplx<T> z) {
  if constexpr (K == CP1) return z;
  else if constexpr (K == CM1) return -z;
  else if constexpr (K == CPI) return mul_i(z);
  else return mul_mi(z);
}

// flip the sign of a coefficient (backward hops use 1 + g instead of 1 - g)
constexpr int neg(int k) { return k == CP1 ? CM1 : k == CM1 ? CP1 : k == CPI ? CMI : CPI; }

template <int MU>
struct proj_table;
// forward hop (1 - g_mu)
template <> struct proj_table<0> { static constexpr int pa = 3, a = CPI, pb = 2, b = CPI, qc = 1, c = CMI, qd = 0, d = CMI; };
template <> struct proj_table<1> { static constexpr int pa = 3, a = CP1, pb = 2, b = CM1, qc = 1, c = CM1, qd = 0, d = CP1; };
template <> struct proj_table<2> { static constexpr int pa = 2, a = CPI, pb = 3, b = CMI, qc = 0, c = CMI, qd = 1, d = CPI; };
template <> struct proj_table<3> { static constexpr int pa = 2, a = CM1, pb = 3, b = CM1, qc = 0, c = CM1, qd = 1, d = CM1; };

// acc += (1 -/+ g_mu) W psi, where W = U (DIR > 0) or U^+ (DIR < 0).
// psi(comp) returns the neighbour spinor component comp = spin*3 + colour,
// u(e) returns link entry e = a*3 + b.
template <int MU, int DIR, typename T, typename PsiF, typename UF>
__device__ __forceinline__ void hop(cplx<T> acc[12], PsiF&& psi, UF&& u) {
  using P = proj_table<MU>;
  constexpr int A = DIR > 0 ? P::a : neg(P::a);
  constexpr int B = DIR > 0 ? P::b : neg(P::b);
  constexpr int C = DIR > 0 ? P::c : neg(P::c);
  constexpr int D = DIR > 0 ? P::d : neg(P::d);
  cplx<T> h0[3], h1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h0[a] = psi(a) + coef<A>(psi(P::pa * 3 + a));
    h1[a] = psi(3 + a) + coef<B>(psi(P::pb * 3 + a));
  }
  cplx<T> w[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) w[e] = u(e);
  cplx<T> g0[3], g1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if constexpr (DIR > 0) {
        s0 += w[a * 3 + b] * h0[b];
        s1 += w[a * 3 + b] * h1[b];
      } else {
        s0 += cdot(w[b * 3 + a], h0[b]);
        s1 += cdot(w[b * 3 + a], h1[b]);
      }
    }
    g0[a] = s0;
    g1[a] = s1;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] += g0[a];
    acc[3 + a] += g1[a];
    acc[6 + a] += coef<C>(P::qc == 0 ? g0[a] : g1[a]);
    acc[9 + a] += coef<D>(P::qd == 0 ? g0[a] : g1[a]);
  }
}

// The three parts of one hop, for kernels that move half spinors around.
// proj: h = upper two spin components of (1 -/+ g_mu) psi.
template <int MU, int DIR, typename T, typename PsiF>
__device__ __forceinline__ void proj(PsiF&& psi, cplx<T> h0[3], cplx<T> h1[3]) {
  using P = proj_table<MU>;
  constexpr int A = DIR > 0 ? P::a : neg(P::a);
  constexpr int B = DIR > 0 ? P::b : neg(P::b);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h0[a] = psi(a) + coef<A>(psi(P::pa * 3 + a));
    h1[a] = psi(3 + a) + coef<B>(psi(P::pb * 3 + a));
  }
}
// g = W h with W = U (DAG false) or U^+ (DAG true), for both spin rows
template <bool DAG, typename T, typename UF>
__device__ __forceinline__ void su3_mul(UF&& u, const cplx<T> h0[3], const cplx<T> h1[3], cplx<T> g0[3],
                                        cplx<T> g1[3]) {
  cplx<T> w[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) w[e] = u(e);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if constexpr (!DAG) {
        s0 += w[a * 3 + b] * h0[b];
        s1 += w[a * 3 + b] * h1[b];
      } else {
        s0 += cdot(w[b * 3 + a], h0[b]);
        s1 += cdot(w[b * 3 + a], h1[b]);
      }
    }
    g0[a] = s0;
    g1[a] = s1;
  }
}
// acc += the full spinor rebuilt from the half spinor g of hop (MU, DIR)
template <int MU, int DIR, typename T>
__device__ __forceinline__ void recon_acc(cplx<T> acc[12], const cplx<T> g0[3], const cplx<T> g1[3]) {
  using P = proj_table<MU>;
  constexpr int C = DIR > 0 ? P::c : neg(P::c);
  constexpr int D = DIR > 0 ? P::d : neg(P::d);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] += g0[a];
    acc[3 + a] += g1[a];
    acc[6 + a] += coef<C>(P::qc == 0 ? g0[a] : g1[a]);
    acc[9 + a] += coef<D>(P::qd == 0 ? g0[a] : g1[a]);
  }
}

// Dispatch hop h = 2*mu + (0: forward, 1: backward). h is uniform across the
// wave, so the switch is a scalar branch to code with compile-time
// projection coefficients.
template <typename T, typename PsiF, typename UF>
__device__ __forceinline__ void hop_dispatch(int h, cplx<T> acc[12], PsiF&& psi, UF&& u) {
  switch (h) {
    case 0: hop<0, +1, T>(acc, psi, u); break;
    case 1: hop<0, -1, T>(acc, psi, u); break;
    case 2: hop<1, +1, T>(acc, psi, u); break;
    case 3: hop<1, -1, T>(acc, psi, u); break;
    case 4: hop<2, +1, T>(acc, psi, u); break;
    case 5: hop<2, -1, T>(acc, psi, u); break;
    case 6: hop<3, +1, T>(acc, psi, u); break;
    default: hop<3, -1, T>(acc, psi, u); break;
  }
}

// ---- FP16 / BF16 links --------------------------------------------------
// With 16-bit links the two half-spinor rows are rounded to the link format
// (round to nearest even) and every complex product is a pair of two-term
// dot products of 16-bit operands accumulated in FP32 (v_dot2 on gfx950):
//   (w h).re = dot((w.re, w.im), (h.re, -h.im)),  (w h).im = dot(w, (h.im, h.re)),
//   (w* h).re = dot(w, (h.re, h.im)),             (w* h).im = dot(w, (h.im, -h.re)).
// The products of 16-bit numbers are exact in FP32, so the only extra
// rounding is that of the half spinor.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));

// First term of a dot-product chain, a.x b.x + a.y b.y in FP32. Written as
// the three-operand form with an inline zero addend: the builtin with a zero
// addend becomes a register copy of 0 plus the two-operand accumulate form,
// one extra VALU instruction per chain (12 per hop).
__device__ __forceinline__ float dot2_first(h2v a, h2v b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float dot2_first(b2v a, b2v b) {
  float r;
  asm("v_dot2_f32_bf16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

template <typename SG>
struct link16;
template <>
struct link16<s16> {
  using V = h2v;
  static __device__ __forceinline__ V pk(float a, float b) {
    V r;
    r.x = (_Float16)a;
    r.y = (_Float16)b;
    return r;
  }
  static __device__ __forceinline__ V raw(const s16* p) { return *reinterpret_cast<const V*>(p); }
  static __device__ __forceinline__ float dot(V a, V b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }
  static __device__ __forceinline__ float dot0(V a, V b) { return dot2_first(a, b); }
};
template <>
struct link16<sbf> {
  using V = b2v;
  static __device__ __forceinline__ V pk(float a, float b) {
    V r;
    r.x = (__bf16)a;
    r.y = (__bf16)b;
    return r;
  }
  static __device__ __forceinline__ V raw(const sbf* p) { return *reinterpret_cast<const V*>(p); }
  static __device__ __forceinline__ float dot(V a, V b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(a, b, c, false);
  }
  static __device__ __forceinline__ float dot0(V a, V b) { return dot2_first(a, b); }
};

template <typename SG>
constexpr bool is_link16 = std::is_same<SG, s16>::value || std::is_same<SG, sbf>::value;

// acc += (1 -/+ g_mu) W psi with 16-bit links; u(e) returns the raw packed entry e.
template <int MU, int DIR, typename SG, typename PsiF, typename UF>
__device__ __forceinline__ void hop16(cplx<float> acc[12], PsiF&& psi, UF&& u) {
  using L = link16<SG>;
  using V = typename L::V;
  cplx<float> h0[3], h1[3];
  proj<MU, DIR, float>(psi, h0, h1);
  V a0[3], b0[3], a1[3], b1[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if constexpr (DIR > 0) {
      a0[b] = L::pk(h0[b].re, -h0[b].im);
      b0[b] = L::pk(h0[b].im, h0[b].re);
      a1[b] = L::pk(h1[b].re, -h1[b].im);
      b1[b] = L::pk(h1[b].im, h1[b].re);
    } else {
      a0[b] = L::pk(h0[b].re, h0[b].im);
      b0[b] = L::pk(h0[b].im, -h0[b].re);
      a1[b] = L::pk(h1[b].re, h1[b].im);
      b1[b] = L::pk(h1[b].im, -h1[b].re);
    }
  }
  cplx<float> g0[3], g1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const V w0 = u(DIR > 0 ? a * 3 : a);
    float r0 = L::dot0(w0, a0[0]), i0 = L::dot0(w0, b0[0]), r1 = L::dot0(w0, a1[0]), i1 = L::dot0(w0, b1[0]);
#pragma unroll
    for (int b = 1; b < 3; ++b) {
      const V w = u(DIR > 0 ? a * 3 + b : b * 3 + a);
      r0 = L::dot(w, a0[b], r0);
      i0 = L::dot(w, b0[b], i0);
      r1 = L::dot(w, a1[b], r1);
      i1 = L::dot(w, b1[b], i1);
    }
    g0[a] = mk(r0, i0);
    g1[a] = mk(r1, i1);
  }
  recon_acc<MU, DIR, float>(acc, g0, g1);
}

// Fully packed FP16 variant: the neighbour spinor is already FP16 (packed
// (re, im) pairs) and the projection is done in packed FP16 arithmetic,
// producing the two dot-product operands of each half-spinor entry directly
// (the lane swaps and sign flips fold into the packed adds' operand
// modifiers). Accumulation stays FP32.
template <int K>
__device__ __forceinline__ h2v cmul16(h2v b) {
  if constexpr (K == CP1) return b;
  else if constexpr (K == CM1) return h2v{-b.x, -b.y};
  else if constexpr (K == CPI) return h2v{-b.y, b.x};
  else return h2v{b.y, -b.x};
}
__device__ __forceinline__ h2v cj16(h2v v) { return h2v{v.x, -v.y}; }
__device__ __forceinline__ h2v sw16(h2v v) { return h2v{v.y, v.x}; }
__device__ __forceinline__ h2v swn16(h2v v) { return h2v{v.y, -v.x}; }

// g = W h for the half spinor h of hop (MU, DIR), packed FP16 operands:
// the projection and the two SU(3) products of hop16p without the rebuild.
template <int MU, int DIR, typename PsiF, typename UF>
__device__ __forceinline__ void hop16p_g(PsiF&& psi, UF&& u, cplx<float> g0[3], cplx<float> g1[3]) {
  using P = proj_table<MU>;
  constexpr int A = DIR > 0 ? P::a : neg(P::a);
  constexpr int B = DIR > 0 ? P::b : neg(P::b);
  h2v a0[3], b0[3], a1[3], b1[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const h2v p0 = psi(b), q0 = cmul16<A>(psi(P::pa * 3 + b));
    const h2v p1 = psi(3 + b), q1 = cmul16<B>(psi(P::pb * 3 + b));
    if constexpr (DIR > 0) {
      a0[b] = cj16(p0) + cj16(q0);
      b0[b] = sw16(p0) + sw16(q0);
      a1[b] = cj16(p1) + cj16(q1);
      b1[b] = sw16(p1) + sw16(q1);
    } else {
      a0[b] = p0 + q0;
      b0[b] = swn16(p0) + swn16(q0);
      a1[b] = p1 + q1;
      b1[b] = swn16(p1) + swn16(q1);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const h2v w0 = u(DIR > 0 ? a * 3 : a);
    float r0 = dot2_first(w0, a0[0]), i0 = dot2_first(w0, b0[0]), r1 = dot2_first(w0, a1[0]),
          i1 = dot2_first(w0, b1[0]);
#pragma unroll
    for (int b = 1; b < 3; ++b) {
      const h2v w = u(DIR > 0 ? a * 3 + b : b * 3 + a);
      r0 = __builtin_amdgcn_fdot2(w, a0[b], r0, false);
      i0 = __builtin_amdgcn_fdot2(w, b0[b], i0, false);
      r1 = __builtin_amdgcn_fdot2(w, a1[b], r1, false);
      i1 = __builtin_amdgcn_fdot2(w, b1[b], i1, false);
    }
    g0[a] = mk(r0, i0);
    g1[a] = mk(r1, i1);
  }
}

template <int MU, int DIR, typename PsiF, typename UF>
__device__ __forceinline__ void hop16p(cplx<float> acc[12], PsiF&& psi, UF&& u) {
  cplx<float> g0[3], g1[3];
  hop16p_g<MU, DIR>(psi, u, g0, g1);
  recon_acc<MU, DIR, float>(acc, g0, g1);
}

template <typename PsiF, typename UF>
__device__ __forceinline__ void hop16p_dispatch(int h, cplx<float> acc[12], PsiF&& psi, UF&& u) {
  switch (h) {
    case 0: hop16p<0, +1>(acc, psi, u); break;
    case 1: hop16p<0, -1>(acc, psi, u); break;
    case 2: hop16p<1, +1>(acc, psi, u); break;
    case 3: hop16p<1, -1>(acc, psi, u); break;
    case 4: hop16p<2, +1>(acc, psi, u); break;
    case 5: hop16p<2, -1>(acc, psi, u); break;
    case 6: hop16p<3, +1>(acc, psi, u); break;
    default: hop16p<3, -1>(acc, psi, u); break;
  }
}

template <typename SG, typename PsiF, typename UF>
__device__ __forceinline__ void hop16_dispatch(int h, cplx<float> acc[12], PsiF&& psi, UF&& u) {
  switch (h) {
    case 0: hop16<0, +1, SG>(acc, psi, u); break;
    case 1: hop16<0, -1, SG>(acc, psi, u); break;
    case 2: hop16<1, +1, SG>(acc, psi, u); break;
    case 3: hop16<1, -1, SG>(acc, psi, u); break;
    case 4: hop16<2, +1, SG>(acc, psi, u); break;
    case 5: hop16<2, -1, SG>(acc, psi, u); break;
    case 6: hop16<3, +1, SG>(acc, psi, u); break;
    default: hop16<3, -1, SG>(acc, psi, u); break;
  }
}

// Hopping sum over all 8 neighbours on the periodic lattice, reading the
// spinor through xin(block, local, comp) and links from U (internal layout).
// The hop loop is deliberately not unrolled: unrolling lets the compiler
// hoist all 8 hops' loads and spill; one hop's loads in flight per wave
// plus other resident waves hide the latency.
template <typename T, typename SG, typename XF>
__device__ __forceinline__ void hop_sum_lattice(const Geom& g, int b, int l, const int bc[4], const int lc[4],
                                                const SG* __restrict__ U, XF&& xin, cplx<T> acc[12]) {
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    const int mu = h >> 1;
    int nb, nl;
    long long ub;
    if ((h & 1) == 0) {
      neighbour<+1>(g, b, l, bc, lc, mu, &nb, &nl);
      ub = gauge_index(g, b, mu, 0, l);
    } else {
      neighbour<-1>(g, b, l, bc, lc, mu, &nb, &nl);
      ub = gauge_index(g, nb, mu, 0, nl);
    }
    hop_dispatch<T>(h, acc, [&](int comp) { return xin(nb, nl, comp); },
                    [&](int e) { return ld<T>(U + ub + (long long)e * g.bvol); });
  }
}

// Hopping sum restricted to one block (eq. 2): hops that leave the block
// are dropped. The block's spinor is read through xin(local, comp).
template <typename T, typename SG, typename XF>
__device__ __forceinline__ void hop_sum_block(const Geom& g, int b, int l, const int lc[4], const SG* __restrict__ U,
                                              XF&& xin, cplx<T> acc[12]) {
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    const int mu = h >> 1;
    const bool fwd = (h & 1) == 0;
    if (fwd ? lc[mu] >= g.B[mu] - 1 : lc[mu] <= 0) continue;
    const int nl = fwd ? l + g.lstride[mu] : l - g.lstride[mu];
    const long long ub = gauge_index(g, b, mu, 0, fwd ? l : nl);
    hop_dispatch<T>(h, acc, [&](int comp) { return xin(nl, comp); },
                    [&](int e) { return ld<T>(U + ub + (long long)e * g.bvol); });
  }
}

// Hopping sum of site (b, l) for kernels that stage a block in LDS:
// in-block neighbours through xin_blk(nl, comp) and in-block links through
// u_blk(mu, e, local site); with HALO, neighbours in other blocks through
// xin_halo(nb, nl, comp) and their links through u_halo(nb, mu, e, nl)
// (hops leaving the block are dropped without HALO, eq. 2).
// With SG = s16 / sbf the link functors return raw packed 16-bit entries
// and the hops use the dot-product form above (T must be float); with
// SG = h2v the block spinor functor also returns packed FP16 pairs and the
// projection is packed too (in-block hops only).
// BS > 0 (a power of two): the block is BS^4, known at compile time, and
// local coordinates are bit fields of the local index.
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <typename T, bool HALO, typename SG = void, int BS = 0, typename XB, typename UB, typename XH, typename UH>
__device__ __forceinline__ void hop_sum_staged(const Geom& g, int b, int l, const int bc[4], const int lc[4],
                                               XB&& xin_blk, UB&& u_blk, XH&& xin_halo, UH&& u_halo,
                                               cplx<T> acc[12]) {
  static_assert(BS == 0 || (BS & (BS - 1)) == 0, "compile-time block side must be a power of two");
  constexpr int LB = ilog2(BS);
  auto dispatch = [&](int h, auto&& psi, auto&& u) {
    if constexpr (std::is_same<SG, h2v>::value) hop16p_dispatch(h, acc, psi, u);
    else if constexpr (is_link16<SG>) hop16_dispatch<SG>(h, acc, psi, u);
    else hop_dispatch<T>(h, acc, psi, u);
  };
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    const int mu = h >> 1;
    const bool fwd = (h & 1) == 0;
    const int st = BS > 0 ? 1 << (LB * mu) : g.lstride[mu];
    const int bm = BS > 0 ? BS : g.B[mu];
    const int lcm = BS > 0 ? (l >> (LB * mu)) & (BS - 1) : lc[mu];
    const bool inb = fwd ? lcm < bm - 1 : lcm > 0;
    if (inb) {
      const int nl = fwd ? l + st : l - st;
      const int ul = fwd ? l : nl;
      dispatch(h, [&](int k) { return xin_blk(nl, k); }, [&](int e) { return u_blk(mu, e, ul); });
    } else if constexpr (HALO) {
      int c2[4] = {bc[0], bc[1], bc[2], bc[3]};
      int nl;
      if (fwd) {
        c2[mu] = (bc[mu] + 1 == g.N[mu]) ? 0 : bc[mu] + 1;
        nl = l - (bm - 1) * st;
      } else {
        c2[mu] = (bc[mu] == 0) ? g.N[mu] - 1 : bc[mu] - 1;
        nl = l + (bm - 1) * st;
      }
      const int nb = encode_block(g, c2);
      if (fwd)
        dispatch(h, [&](int k) { return xin_halo(nb, nl, k); }, [&](int e) { return u_blk(mu, e, l); });
      else
        dispatch(h, [&](int k) { return xin_halo(nb, nl, k); }, [&](int e) { return u_halo(nb, mu, e, nl); });
    }
  }
}

// The value of a 32-bit register in the lane S below (S = 1, 2, 4 or 8),
// within rows of 16 lanes (DPP row shift; the first S lanes of a row get 0).
template <int S, typename W>
__device__ __forceinline__ W lane_below(W v) {
  static_assert(sizeof(W) == 4, "one register");
  if constexpr (S <= 15) {
    return __builtin_bit_cast(W, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 + S, 0xF, 0xF, false));
  } else {
    // across rows: the LDS crossbar's backward permute (no LDS memory used)
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return __builtin_bit_cast(W, __builtin_amdgcn_ds_bpermute(((lane - S) & 63) * 4, __builtin_bit_cast(int, v)));
  }
}

// One direction of hop_sum_block_unrolled (below). Directions MU < NREG take
// their links from registers (ux[MU], the lane's own site's links, held across
// calls): the forward hop uses them directly and the backward hop those of the
// lane st below (the site n - mu, in the same 16-lane row for x and y of 4^4
// blocks).
template <int MU, int BS, int NREG, typename T, typename SG, typename XB, typename UB, typename W>
__device__ __forceinline__ void block_dir_unrolled(int l, XB& xin_blk, UB& u_blk, cplx<T> acc[12], W wf[9],
                                                   const W (*ux)[9]) {
  constexpr int LB = ilog2(BS);
  constexpr int st = 1 << (LB * MU);
  const int lcm = (l >> (LB * MU)) & (BS - 1);
  const int ub = lcm > 0 ? l - st : l;
  W wb[9];
  // keep each direction's loads inside its own stretch of code (hoisted,
  // the next directions' links would not fit the register budget)
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (MU < NREG && MU < 3) {
#pragma unroll
    for (int e = 0; e < 9; ++e) wb[e] = lane_below<st>(ux[MU][e]);
  } else {
#pragma unroll
    for (int e = 0; e < 9; ++e) wb[e] = u_blk(MU, e, ub);
  }
  auto do_hop = [&](auto dirc, auto&& psi, auto&& u) {
    constexpr int DIR = decltype(dirc)::value;
    if constexpr (std::is_same<SG, h2v>::value) hop16p<MU, DIR>(acc, psi, u);
    else if constexpr (is_link16<SG>) hop16<MU, DIR, SG>(acc, psi, u);
    else hop<MU, DIR, T>(acc, psi, u);
  };
  if (lcm < BS - 1)
    do_hop(std::integral_constant<int, 1>{}, [&](int k) { return xin_blk(l + st, k); }, [&](int e) { return wf[e]; });
  if constexpr (MU < 3) {
#pragma unroll
    for (int e = 0; e < 9; ++e) wf[e] = MU + 1 < NREG ? ux[MU + 1][e] : u_blk(MU + 1, e, l);
  }
  if (lcm > 0)
    do_hop(std::integral_constant<int, -1>{}, [&](int k) { return xin_blk(l - st, k); }, [&](int e) { return wb[e]; });
}

// In-block hopping sum of D^l (eq. 2) for compile-time BS^4 blocks, with
// the link loads one hop ahead: per direction the backward hop's links are
// loaded before the forward hop's arithmetic and the next direction's
// forward links before the backward hop's, so each hop's L1/L2 latency
// overlaps the previous hop's work. Sites on the lower face load their own
// link in place of the (skipped) backward one, which keeps every load inside
// the block. u_blk(mu, e, local site) returns a link entry as the hop takes it.
// Directions are unrolled at compile time: every hop is a straight-line
// body under its lane mask (no switch over the hop index), so the
// accumulator stays in the same registers from hop to hop.
template <typename T, typename SG, int BS, int NREG = 0, typename XB, typename UB,
          typename W = std::remove_cv_t<std::remove_reference_t<decltype(std::declval<UB>()(0, 0, 0))>>>
__device__ __forceinline__ void hop_sum_block_unrolled(int l, XB&& xin_blk, UB&& u_blk, cplx<T> acc[12],
                                                       const W (*ux)[9] = nullptr) {
  static_assert(BS > 0 && (BS & (BS - 1)) == 0, "compile-time block side must be a power of two");
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
  W wf[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) wf[e] = NREG > 0 ? ux[0][e] : u_blk(0, e, l);
  block_dir_unrolled<0, BS, NREG, T, SG>(l, xin_blk, u_blk, acc, wf, ux);
  block_dir_unrolled<1, BS, NREG, T, SG>(l, xin_blk, u_blk, acc, wf, ux);
  block_dir_unrolled<2, BS, NREG, T, SG>(l, xin_blk, u_blk, acc, wf, ux);
  block_dir_unrolled<3, BS, NREG, T, SG>(l, xin_blk, u_blk, acc, wf, ux);
}

// Full hopping sum (faces included) for compile-time BS^4 blocks: each hop's
// neighbour spinor is read into registers first, from the block (xin_blk,
// in-block sites) or from the neighbouring block (xin_halo, face sites), so
// that the hop arithmetic runs once per hop for all lanes (a branch per
// source around the whole hop would run it twice on the faces of x, y, z).
// Links: u_at(block, mu, e, local site); the backward hop's link comes from
// this block or from the neighbouring block per lane, loaded one hop ahead
// as in hop_sum_block_unrolled.
template <typename T, typename SG, int BS, typename XB, typename XH, typename UA>
__device__ __forceinline__ void hop_sum_halo_ahead(const Geom& g, int b, int l, const int bc[4], XB&& xin_blk,
                                                   XH&& xin_halo, UA&& u_at, cplx<T> acc[12]) {
  static_assert(BS > 0 && (BS & (BS - 1)) == 0, "compile-time block side must be a power of two");
  constexpr int LB = ilog2(BS);
  using W = decltype(u_at(0, 0, 0, 0));
  auto dispatch = [&](int h, auto&& psi, auto&& u) {
    if constexpr (is_link16<SG>) hop16_dispatch<SG>(h, acc, psi, u);
    else hop_dispatch<T>(h, acc, psi, u);
  };
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
  W wf[9], wb[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) wf[e] = u_at(b, 0, e, l);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    const int st = 1 << (LB * mu);
    const int lcm = (l >> (LB * mu)) & (BS - 1);
    // neighbouring blocks in +mu and -mu (uniform over the workgroup)
    int cf[4] = {bc[0], bc[1], bc[2], bc[3]}, cb[4] = {bc[0], bc[1], bc[2], bc[3]};
    cf[mu] = (bc[mu] + 1 == g.N[mu]) ? 0 : bc[mu] + 1;
    cb[mu] = (bc[mu] == 0) ? g.N[mu] - 1 : bc[mu] - 1;
    const int nbf = encode_block(g, cf), nbb = encode_block(g, cb);
    const bool inf = lcm < BS - 1, inbk = lcm > 0;
    const int nlb = inbk ? l - st : l + (BS - 1) * st;
#pragma unroll
    for (int e = 0; e < 9; ++e) wb[e] = u_at(inbk ? b : nbb, mu, e, nlb);
    cplx<T> q[12];
    if (inf) {
#pragma unroll
      for (int k = 0; k < 12; ++k) q[k] = xin_blk(l + st, k);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) q[k] = xin_halo(nbf, l - (BS - 1) * st, k);
    }
    dispatch(2 * mu, [&](int k) { return q[k]; }, [&](int e) { return wf[e]; });
    if (mu < 3) {
#pragma unroll
      for (int e = 0; e < 9; ++e) wf[e] = u_at(b, mu + 1, e, l);
    }
    if (inbk) {
#pragma unroll
      for (int k = 0; k < 12; ++k) q[k] = xin_blk(l - st, k);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) q[k] = xin_halo(nbb, nlb, k);
    }
    dispatch(2 * mu + 1, [&](int k) { return q[k]; }, [&](int e) { return wb[e]; });
  }
}

}  // namespace dw
