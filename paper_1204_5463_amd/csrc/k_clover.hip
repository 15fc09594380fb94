// Builds the clover term of a field from its FP64 links (see dw_clover.hpp).
// One thread per site: the four leaves of each of the six planes from links
// around the site (periodic), F = (Q - Q^+)/8, then the two chirality
// blocks (i c_sw / 2) sum sigma^chi_{mu nu} (x) F_{mu nu}, stored packed.
#include "dw_clover.hpp"
#include "dw_internal.hpp"

namespace dw {

namespace {

constexpr int kThreads = 128;
using C = cplx<double>;

struct M3 {
  C e[9];
};

__device__ __forceinline__ M3 mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C s = a.e[i * 3] * b.e[j];
      s += a.e[i * 3 + 1] * b.e[3 + j];
      s += a.e[i * 3 + 2] * b.e[6 + j];
      r.e[i * 3 + j] = s;
    }
  return r;
}
__device__ __forceinline__ M3 dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i * 3 + j] = conj(a.e[j * 3 + i]);
  return r;
}

// U_mu at lattice coordinates c (wrapped periodically)
__device__ M3 link(const Geom& g, const s64* __restrict__ U, int mu, const int c[4]) {
  int bc[4], lc[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    int v = c[d] % g.L[d];
    if (v < 0) v += g.L[d];
    bc[d] = v / g.B[d];
    lc[d] = v - bc[d] * g.B[d];
  }
  const int b = encode_block(g, bc);
  const int l = lc[0] + g.B[0] * (lc[1] + g.B[1] * (lc[2] + g.B[2] * lc[3]));
  M3 r;
#pragma unroll
  for (int e = 0; e < 9; ++e) r.e[e] = ld<double>(U + gauge_index(g, b, mu, e, l));
  return r;
}

__device__ __forceinline__ void shift(int c[4], const int o[4], int mu, int s) {
#pragma unroll
  for (int d = 0; d < 4; ++d) c[d] = o[d];
  c[mu] += s;
}

// sum of the four leaves of plane (mu, nu) at coordinates n
__device__ M3 leaves(const Geom& g, const s64* __restrict__ U, int mu, int nu, const int n[4]) {
  int a[4], b[4];
  // n -> n+mu -> n+mu+nu -> n+nu -> n
  shift(a, n, mu, 1);
  shift(b, n, nu, 1);
  M3 q = mul(mul(link(g, U, mu, n), link(g, U, nu, a)), mul(dag(link(g, U, mu, b)), dag(link(g, U, nu, n))));
  // n -> n+nu -> n+nu-mu -> n-mu -> n
  int c[4];
  shift(c, n, mu, -1);
  int d[4];
  shift(d, c, nu, 1);
  M3 t = mul(mul(link(g, U, nu, n), dag(link(g, U, mu, d))), mul(dag(link(g, U, nu, c)), link(g, U, mu, c)));
#pragma unroll
  for (int e = 0; e < 9; ++e) q.e[e] += t.e[e];
  // n -> n-mu -> n-mu-nu -> n-nu -> n
  int f[4];
  shift(f, c, nu, -1);
  int h[4];
  shift(h, n, nu, -1);
  t = mul(mul(dag(link(g, U, mu, c)), dag(link(g, U, nu, f))), mul(link(g, U, mu, f), link(g, U, nu, h)));
#pragma unroll
  for (int e = 0; e < 9; ++e) q.e[e] += t.e[e];
  // n -> n-nu -> n-nu+mu -> n+mu -> n
  int k[4];
  shift(k, h, mu, 1);
  t = mul(mul(dag(link(g, U, nu, h)), link(g, U, mu, h)), mul(link(g, U, nu, k), dag(link(g, U, mu, n))));
#pragma unroll
  for (int e = 0; e < 9; ++e) q.e[e] += t.e[e];
  return q;
}

__global__ void __launch_bounds__(kThreads)
    k_clover_build(Geom g, const s64* __restrict__ U, SigmaBlocks sb, double csw, s64* __restrict__ out) {
  const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= g.V) return;
  const int b = (int)(s / g.bvol);
  const int l = (int)(s - (long long)b * g.bvol);
  int bc[4], lc[4], n[4];
  decode_block(g, b, bc);
  decode_local(g, l, lc);
#pragma unroll
  for (int d = 0; d < 4; ++d) n[d] = bc[d] * g.B[d] + lc[d];
  // upper triangles of the two 6x6 blocks: entry (r, c) with r = s*3 + a
  C acc[2][21];
#pragma unroll
  for (int chi = 0; chi < 2; ++chi)
#pragma unroll
    for (int q = 0; q < 21; ++q) acc[chi][q] = C{0.0, 0.0};
  int plane = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
      const M3 Q = leaves(g, U, mu, nu, n);
      // F = (Q - Q^+)/8, times i c_sw / 2
      M3 F;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const C a = Q.e[i * 3 + j], bt = conj(Q.e[j * 3 + i]);
          const C f = C{(a.re - bt.re) * 0.125, (a.im - bt.im) * 0.125};
          F.e[i * 3 + j] = C{-0.5 * csw * f.im, 0.5 * csw * f.re};  // (i csw/2) f
        }
#pragma unroll
      for (int chi = 0; chi < 2; ++chi) {
        int q = 0;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int c2 = r; c2 < 6; ++c2, ++q) {
            const int s1 = r / 3, a1 = r % 3, s2 = c2 / 3, a2 = c2 % 3;
            const C sg = C{sb.re[plane][chi][s1 * 2 + s2], sb.im[plane][chi][s1 * 2 + s2]};
            acc[chi][q] += sg * F.e[a1 * 3 + a2];
          }
      }
    }
  // pack: diagonals as three pairs, then the 15 off-diagonal entries
#pragma unroll
  for (int chi = 0; chi < 2; ++chi) {
    s64* o = out + ((long long)b * kCloverPairs + chi * 18) * g.bvol + l;
    double dg[6];
    int q = 0, k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c2 = r; c2 < 6; ++c2, ++q) {
        if (c2 == r) {
          dg[r] = acc[chi][q].re;
        } else {
          o[(long long)(k++) * g.bvol] = s64{acc[chi][q].re, acc[chi][q].im};
        }
      }
#pragma unroll
    for (int p = 0; p < 3; ++p) o[(long long)p * g.bvol] = s64{dg[2 * p], dg[2 * p + 1]};
  }
}

}  // namespace

SigmaBlocks sigma_blocks() {
  // gamma matrices of the chiral basis: g_k = [[0, -i s_k], [i s_k, 0]], g_t = [[0, 1], [1, 0]]
  typedef cplx<double> Cx;
  Cx s[3][4] = {{{0, 0}, {1, 0}, {1, 0}, {0, 0}},     // s_x
                {{0, 0}, {0, -1}, {0, 1}, {0, 0}},    // s_y
                {{1, 0}, {0, 0}, {0, 0}, {-1, 0}}};   // s_z
  Cx gam[4][16];
  for (int mu = 0; mu < 4; ++mu)
    for (int e = 0; e < 16; ++e) gam[mu][e] = Cx{0, 0};
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const Cx v = s[k][i * 2 + j];
        gam[k][i * 4 + (2 + j)] = Cx{v.im, -v.re};       // -i s_k (upper right)
        gam[k][(2 + i) * 4 + j] = Cx{-v.im, v.re};       // +i s_k (lower left)
      }
  for (int i = 0; i < 2; ++i) {
    gam[3][i * 4 + 2 + i] = Cx{1, 0};
    gam[3][(2 + i) * 4 + i] = Cx{1, 0};
  }
  auto mm = [&](const Cx* a, const Cx* b, Cx* r) {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        Cx t{0, 0};
        for (int k = 0; k < 4; ++k) t += a[i * 4 + k] * b[k * 4 + j];
        r[i * 4 + j] = t;
      }
  };
  SigmaBlocks sb;
  int plane = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
      Cx ab[16], ba[16];
      mm(gam[mu], gam[nu], ab);
      mm(gam[nu], gam[mu], ba);
      for (int chi = 0; chi < 2; ++chi)
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            const int e = (2 * chi + i) * 4 + 2 * chi + j;
            const Cx cm = ab[e] - ba[e];
            // sigma = (i/2) [g_mu, g_nu]
            sb.re[plane][chi][i * 2 + j] = -0.5 * cm.im;
            sb.im[plane][chi][i * 2 + j] = 0.5 * cm.re;
          }
    }
  return sb;
}

dw_status launch_clover_build(const Geom& g, const void* U64, double csw, double* out, hipStream_t s) {
  const unsigned grid = (unsigned)((g.V + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_clover_build, grid, kThreads, 0, s, g, (const s64*)U64, sigma_blocks(), csw, (s64*)out);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

}  // namespace dw
