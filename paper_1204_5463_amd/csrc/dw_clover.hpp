// The clover (Sheikholeslami-Wohlert) term, site by site.
//
//   D_sw = D + (i c_sw / 2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(n),
//   sigma_{mu nu} = (i/2) [g_mu, g_nu],  F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^+) / 8,
//
// with Q_{mu nu}(n) the four plaquettes of the (mu, nu) plane around n. In
// the chiral basis sigma is block diagonal in the chiralities (spins 0, 1
// and 2, 3), so the term is two Hermitian 6x6 matrices per site (spin x
// colour within a chirality).
//
// Storage, per chirality: 18 complex pairs, the first three holding the six
// real diagonal entries (d0, d1), (d2, d3), (d4, d5), then the 15 entries
// above the diagonal in row-major order (0,1)..(0,5), (1,2)..(4,5). Site
// (b, l), pair q (0..35, chirality q / 18) sits at (b * 36 + q) * bvol + l.
#pragma once

#include "dw_types.hpp"

namespace dw {

constexpr int kCloverPairs = 36;

// y += C x for one site; Cb points at the site's block, x and y are the 12
// spinor components (spin * 3 + colour).
template <typename T, typename SC>
__device__ __forceinline__ void clover_acc(const SC* __restrict__ Cb, int bvol, int l, const cplx<T> x[12],
                                           cplx<T> y[12]) {
#pragma unroll
  for (int chi = 0; chi < 2; ++chi) {
    const SC* c = Cb + (long long)chi * 18 * bvol + l;
    const cplx<T>* v = x + 6 * chi;
    cplx<T> w[6];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const cplx<T> d = ld<T>(c + q * bvol);
      w[2 * q] = d.re * v[2 * q];
      w[2 * q + 1] = d.im * v[2 * q + 1];
    }
    int q = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j) {
        const cplx<T> o = ld<T>(c + (q++) * bvol);
        w[i] += o * v[j];
        w[j] += cdot(o, v[i]);
      }
#pragma unroll
    for (int i = 0; i < 6; ++i) y[6 * chi + i] += w[i];
  }
}

// y += s * C x for one site, with x read through xin(comp) one chirality at
// a time (fewer live registers than clover_acc).
template <typename T, typename SC, typename XF>
__device__ __forceinline__ void clover_acc_f(const SC* __restrict__ Cb, int bvol, int l, XF&& xin, T s,
                                             cplx<T> y[12]) {
#pragma unroll
  for (int chi = 0; chi < 2; ++chi) {
    const SC* c = Cb + (long long)chi * 18 * bvol + l;
    cplx<T> v[6], w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = xin(6 * chi + i);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const cplx<T> d = ld<T>(c + q * bvol);
      w[2 * q] = d.re * v[2 * q];
      w[2 * q + 1] = d.im * v[2 * q + 1];
    }
    int q = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j) {
        const cplx<T> o = ld<T>(c + (q++) * bvol);
        w[i] += o * v[j];
        w[j] += cdot(o, v[i]);
      }
#pragma unroll
    for (int i = 0; i < 6; ++i) y[6 * chi + i] += s * w[i];
  }
}

// flops of clover_acc per site: 2 x (6 x 2 + 15 x 2 x 8)
constexpr double kCloverFlops = 504.0;

}  // namespace dw
