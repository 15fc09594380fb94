// Lattice geometry and the internal block-tiled field layout.
//
// The lattice (extents L = Lx, Ly, Lz, Lt, periodic) is cut into
// hyper-rectangular domains of extents B (the SAP blocks, Section 2 of the
// paper). With an even number of blocks N_mu = L_mu / B_mu per direction,
// blocks are coloured by the parity of the sum of their block coordinates
// and blocks of one colour do not couple (Section 2, red/black colouring).
//
// Internal ordering (private to the library):
//   block index b in [0, nblk): lexicographic in the block coordinates,
//     b = bx + Nx*(by + Ny*(bz + Nz*bt)), so that neighbouring blocks are
//     close in memory and in launch order; the j-th block of a colour is
//     found by colour_block();
//   local site index l in [0, bvol): lx + Bx*(ly + By*(lz + Bz*lt));
//   spinor:  element (b, comp, l) at ((b*12 + comp)*bvol + l), comp = spin*3 + colour;
//   gauge:   element (b, mu, e, l) at (((b*4 + mu)*9 + e)*bvol + l), e = a*3 + b.
// Each block is one contiguous chunk; within it every component is a
// contiguous run over the block's sites (coalesced per wavefront).
// Canonical (boundary) ordering: site n = x + Lx*(y + Ly*(z + Lz*t)),
// spinor [n][spin][colour], gauge [mu][n][a][b], complex128 interleaved.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dw {

struct Geom {
  int L[4];        // lattice extents x, y, z, t
  int B[4];        // block extents
  int N[4];        // blocks per direction
  int bvol;        // sites per block
  int nblk;        // number of blocks
  int nbc;         // blocks per colour (nblk / 2)
  int lstride[4];  // local index stride per direction: 1, Bx, Bx*By, Bx*By*Bz
  long long V;     // sites
};

// Validates and fills a Geom. Returns 0 on success, else a static message.
inline const char* make_geom(const int L[4], const int B[4], Geom* g) {
  long long V = 1;
  int bvol = 1, nblk = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (L[mu] <= 0 || B[mu] <= 0) return "lattice and block extents must be positive";
    if (L[mu] % B[mu] != 0) return "block extent does not divide the lattice extent";
    int n = L[mu] / B[mu];
    if (n % 2 != 0) return "need an even number of blocks in every direction";
    g->L[mu] = L[mu];
    g->B[mu] = B[mu];
    g->N[mu] = n;
    V *= L[mu];
    bvol *= B[mu];
    nblk *= n;
  }
  if (bvol > 1024) return "block volume above 1024 sites is not supported";
  g->V = V;
  g->bvol = bvol;
  g->nblk = nblk;
  g->nbc = nblk / 2;
  g->lstride[0] = 1;
  g->lstride[1] = B[0];
  g->lstride[2] = B[0] * B[1];
  g->lstride[3] = B[0] * B[1] * B[2];
  return nullptr;
}

__host__ __device__ __forceinline__ void decode_block(const Geom& g, int b, int bc[4]) {
  bc[0] = b % g.N[0];
  int q = b / g.N[0];
  bc[1] = q % g.N[1];
  q /= g.N[1];
  bc[2] = q % g.N[2];
  bc[3] = q / g.N[2];
}

__host__ __device__ __forceinline__ int encode_block(const Geom& g, const int bc[4]) {
  return bc[0] + g.N[0] * (bc[1] + g.N[1] * (bc[2] + g.N[2] * bc[3]));
}

// j-th block (lexicographic order) among the blocks of `colour`, whose
// colour is the parity of the sum of the block coordinates; N_x is even,
// so every x-row of blocks holds N_x/2 blocks of each colour.
__host__ __device__ __forceinline__ int colour_block(const Geom& g, int colour, int j) {
  const int hx = g.N[0] >> 1;
  int q = j / hx;
  const int bx2 = j - q * hx;
  const int by = q % g.N[1];
  q /= g.N[1];
  const int bz = q % g.N[2];
  const int bt = q / g.N[2];
  const int bx = 2 * bx2 + ((colour + by + bz + bt) & 1);
  return bx + g.N[0] * (by + g.N[1] * (bz + g.N[2] * bt));
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2. Remapping launch index i so that XCD x receives the contiguous range
// [x*per, (x+1)*per) of work items keeps neighbouring blocks in one L2.
// Returns -1 for launch indices past the end (the grid is rounded up).
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ int xcd_remap(int i, int count) {
  const int per = (count + kXcds - 1) / kXcds;
  const int r = (i % kXcds) * per + i / kXcds;
  return r < count ? r : -1;
}
__host__ __device__ __forceinline__ int xcd_grid(int count) { return ((count + kXcds - 1) / kXcds) * kXcds; }

__host__ __device__ __forceinline__ void decode_local(const Geom& g, int l, int lc[4]) {
  lc[0] = l % g.B[0];
  int q = l / g.B[0];
  lc[1] = q % g.B[1];
  q /= g.B[1];
  lc[2] = q % g.B[2];
  lc[3] = q / g.B[2];
}

// canonical lexicographic site of internal (b, l)
__host__ __device__ __forceinline__ long long canonical_site(const Geom& g, int b, int l) {
  int bc[4], lc[4];
  decode_block(g, b, bc);
  decode_local(g, l, lc);
  long long x = bc[0] * g.B[0] + lc[0];
  long long y = bc[1] * g.B[1] + lc[1];
  long long z = bc[2] * g.B[2] + lc[2];
  long long t = bc[3] * g.B[3] + lc[3];
  return x + (long long)g.L[0] * (y + (long long)g.L[1] * (z + (long long)g.L[2] * t));
}

// Neighbour of site (b, l) with coordinates (bc, lc) in direction mu.
// Returns the neighbour's (block, local) pair and whether it stays in block b.
template <int DIR>
__device__ __forceinline__ bool neighbour(const Geom& g, int b, int l, const int bc[4], const int lc[4], int mu,
                                          int* nb, int* nl) {
  if (DIR > 0) {
    if (lc[mu] < g.B[mu] - 1) {
      *nb = b;
      *nl = l + g.lstride[mu];
      return true;
    }
    int c2[4] = {bc[0], bc[1], bc[2], bc[3]};
    c2[mu] = (bc[mu] + 1 == g.N[mu]) ? 0 : bc[mu] + 1;
    *nb = encode_block(g, c2);
    *nl = l - (g.B[mu] - 1) * g.lstride[mu];
    return false;
  } else {
    if (lc[mu] > 0) {
      *nb = b;
      *nl = l - g.lstride[mu];
      return true;
    }
    int c2[4] = {bc[0], bc[1], bc[2], bc[3]};
    c2[mu] = (bc[mu] == 0) ? g.N[mu] - 1 : bc[mu] - 1;
    *nb = encode_block(g, c2);
    *nl = l + (g.B[mu] - 1) * g.lstride[mu];
    return false;
  }
}

__host__ __device__ __forceinline__ long long spinor_index(const Geom& g, int b, int comp, int l) {
  return ((long long)b * 12 + comp) * g.bvol + l;
}
__host__ __device__ __forceinline__ long long gauge_index(const Geom& g, int b, int mu, int e, int l) {
  return (((long long)b * 4 + mu) * 9 + e) * g.bvol + l;
}

}  // namespace dw
