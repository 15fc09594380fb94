// Internal runtime structures and kernel launcher declarations.
#pragma once

#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dwsap.h"
#include "dw_geom.hpp"

namespace dw {
// Work tag of a launch inside a solver cycle: which right-hand sides it
// covers and which gate decides whether it does work for each of them
// (the kernels of a cycle are launched unconditionally and find their
// gates on the device). kind >= 0: an Arnoldi step of that column.
enum { kTagNone = -1, kTagFin = -2, kTagCycle = -3, kTagDefl = -4, kTagFresh = -5, kTagInject = -6 };
struct ProfTagV {
  int kind = kTagNone;
  unsigned long long mask = 0;  // right-hand sides 0..63 covered by the launch
};

struct Profiler {
  struct Rec {
    int kc;
    hipEvent_t a, b;
    double bytes, flops;
    ProfTagV tag;
  };
  std::mutex mu;
  bool on = false;
  std::vector<Rec> pending;
  std::vector<Rec> held;  // finished tagged launches, awaiting the outcome of their cycle
  std::vector<hipEvent_t> pool;
  dw_kernel_stats acc[DW_K_COUNT] = {};
};
}  // namespace dw

struct dw_ctx_s {
  int device;
  dw_allocator alloc;
  bool user_alloc;
  dw::Profiler prof;
  // the caller's handle plus one per live field: a destroyed context stays
  // until its last field is gone (the fields free through its allocator)
  std::atomic<int> refs{1};
};

struct dw_field_s {
  dw_ctx ctx;
  dw::Geom g;
  void* U[4];  // links per dw_prec, internal layout
  void* C[4];  // clover term per dw_prec (null without one)
  double csw;
  hipStream_t stream;  // stream the field was created on (its memory is freed there)
  // solver workspace and captured cycles kept for the next solve (DW_SOLVE_GRAPHS)
  void* solver_cache = nullptr;
  void (*solver_cache_free)(void*) = nullptr;
  // set by the server: the admission has reserved the memory of the whole
  // request, so a solve keeps all its right-hand sides in one batch
  bool memory_reserved = false;
};

namespace dw {

// drops one reference of a context, deleting it with the last one
void ctx_release(dw_ctx ctx);

// ---- errors -----------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define DW_CHECK_HIP(expr)                                                                    \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      ::dw::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return DW_EHIP;                                                                         \
    }                                                                                         \
  } while (0)

#define DW_CHECK_LAUNCH()                                                                     \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess) {                                                                   \
      ::dw::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
      return DW_EHIP;                                                                         \
    }                                                                                         \
  } while (0)

#define DW_TRY(expr)              \
  do {                            \
    dw_status s_ = (expr);        \
    if (s_ != DW_OK) return s_;   \
  } while (0)

// ---- kernel timing ----------------------------------------------------------------
// The entry points install their context's profiler for the calling thread;
// launchers bracket their kernels with KTimer.
struct ProfScope {
  Profiler* prev;
  explicit ProfScope(dw_ctx ctx);
  ~ProfScope();
};
struct KTimer {
  Profiler* p = nullptr;
  hipEvent_t a = nullptr;
  hipStream_t s = nullptr;
  int kc;
  KTimer(int kclass, hipStream_t stream);
  void done(double bytes, double flops);
};
// resolves finished timing records (of the calling thread's profiler if null);
// tagged records wait in `held` for prof_resolve
void prof_flush(Profiler* p = nullptr);
// sets the work tag of the calling thread's following launches
struct ProfTag {
  ProfTagV prev;
  ProfTag(int kind, unsigned long long mask);
  ~ProfTag();
};
// Accounts the held records of a finished cycle: active(kind, r) says
// whether right-hand side r did work under that tag; a launch counts with
// the fraction of its right-hand sides that did, and one that did none
// (every gate closed) is not counted at all.
Profiler* prof_current();
template <typename F>
void prof_resolve(F&& active) {
  Profiler* p = prof_current();
  if (!p) return;
  prof_flush(p);
  std::lock_guard<std::mutex> lk(p->mu);
  for (auto& r : p->held) {
    int n = 0, on = 0;
    for (int i = 0; i < 64; ++i)
      if ((r.tag.mask >> i) & 1ull) {
        ++n;
        if (active(r.tag.kind, i)) ++on;
      }
    float ms = 0.f;
    if (on > 0 && n > 0 && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      dw_kernel_stats& k = p->acc[r.kc];
      k.launches += 1;
      k.ms += ms;
      k.bytes += r.bytes * on / n;
      k.flops += r.flops * on / n;
    }
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->held.clear();
}

// ---- device memory ------------------------------------------------------------
void* dev_alloc(dw_ctx ctx, size_t bytes, hipStream_t stream);
void dev_free(dw_ctx ctx, void* p, hipStream_t stream);

// Scoped device buffer from the context allocator.
struct DevBuf {
  dw_ctx ctx = nullptr;
  hipStream_t stream = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  dw_status alloc(dw_ctx c, size_t n, hipStream_t s) {
    reset();
    ctx = c;
    stream = s;
    bytes = n;
    p = n ? dev_alloc(c, n, s) : nullptr;
    if (n && !p) {
      set_error("device allocation of %zu bytes failed", n);
      return DW_ENOMEM;
    }
    return DW_OK;
  }
  void reset() {
    if (p) dev_free(ctx, p, stream);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// bytes of one complex pair per precision
inline size_t pair_bytes(int prec) { return prec == DW_PREC_F64 ? 16 : prec == DW_PREC_F32 ? 8 : 4; }

// ---- launchers (kernels in the .hip files) --------------------------------------
// All counts in complex pairs; nrhs fields are stacked with stride V*12 pairs.
// dscale (may be null): a device factor per right-hand side r at dscale[r * dstride], multiplying scale
dw_status launch_pack_spinor(const Geom& g, int prec, const double* in, void* out, double scale, int nrhs,
                             hipStream_t s, const double* dscale = nullptr, int dstride = 0);
dw_status launch_unpack_spinor(const Geom& g, int prec, const void* in, double* out, double scale, int nrhs,
                               hipStream_t s, const double* dscale = nullptr, int dstride = 0);
dw_status launch_pack_gauge(const Geom& g, int prec, const double* in, void* out, hipStream_t s);
// sigma_{mu nu} chirality blocks (2x2) for the six planes mu < nu
struct SigmaBlocks {
  double re[6][2][4], im[6][2][4];
};
SigmaBlocks sigma_blocks();
// clover term (FP64, packed per dw_clover.hpp) from the FP64 internal links
dw_status launch_clover_build(const Geom& g, const void* U64, double csw, double* out, hipStream_t s);
// elementwise out = scale * (dscale ? dscale[0] : 1) * in over n pairs
// (precision conversion; dscale is a device scalar)
dw_status launch_convert(int pin, const void* in, int pout, void* out, double scale, long long n, hipStream_t s,
                         const double* dscale = nullptr, const int* gate = nullptr);

// y = scale * D x (mode 0) or y = b - scale * D x (mode 1), internal layout.
// prec_x: DW_PREC_F64 or DW_PREC_F32 input with FP64 links/output/arithmetic
// when outer = true; otherwise everything at precision prec_x (FP32 math).
// rlist (device, may be null): the nrhs right-hand-side indices to process.
// gate (device, may be null): right-hand side r is skipped when gate[r * gstride] == 0.
// dmass (device, may be null): the mass is read there instead of m0.
dw_status launch_dslash_outer(const Geom& g, double m0, int prec_x, const void* x, double scale, const void* U64,
                              double* y, const double* b, int mode, int nrhs, long long x_rhs_stride,
                              long long y_rhs_stride, hipStream_t s, const int* rlist = nullptr,
                              const void* C64 = nullptr, const int* gate = nullptr, int gstride = 0,
                              const double* dmass = nullptr);
dw_status launch_dslash_lowp(const Geom& g, double m0, int prec, const void* x, const void* U, void* y, int nrhs,
                             hipStream_t s, const void* C = nullptr);
// w = D z with FP32 vectors, FP32 links (and clover term) and FP32 arithmetic:
// the operator of the single-precision Arnoldi; mass from dmass (device)
dw_status launch_dslash_a32(const Geom& g, const void* x, const void* U32, void* y, int nrhs, long long xs,
                            long long ys, hipStream_t s, const int* rlist, const void* C32, const int* gate, int gstride,
                            const double* dmass);

// One SAP colour sweep: for every block of `colour`, r = v - D z on the
// block, nmr MR steps on D^l y = r, z += y. v at storage precision `prec`,
// z at FP64 (prec F64) or FP32 (otherwise). z_zero: z is zero on entry.
// gate, dmass as for launch_dslash_outer.
dw_status launch_sap_colour(const Geom& g, double m0, int prec, const void* v, void* z, const void* U, int colour,
                            int nmr, int z_zero, int nrhs, long long v_rhs_stride, long long z_rhs_stride,
                            hipStream_t s, const int* rlist = nullptr, const void* C = nullptr,
                            double mr_reduction = 0.0, const int* gate = nullptr, int gstride = 0,
                            const double* dmass = nullptr);

}  // namespace dw
