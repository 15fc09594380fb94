// Context, field and operator entry points of the C ABI.
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <new>
#include <string>

#include "dw_clover.hpp"
#include "dw_control.hpp"
#include "dw_internal.hpp"
#include "dw_kernels.hpp"
#include <math.h>

namespace dw {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

// Without a caller allocator, memory is stream-ordered (hipMallocAsync /
// hipFreeAsync on the call's stream), so that freeing a temporary at the end
// of an asynchronous call does not synchronise the device.
void ctx_release(dw_ctx ctx) {
  if (ctx->refs.fetch_sub(1) == 1) delete ctx;
}

void* dev_alloc(dw_ctx ctx, size_t bytes, hipStream_t stream) {
  if (ctx->user_alloc) return ctx->alloc.alloc(bytes, stream, ctx->alloc.user);
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, stream) != hipSuccess) return nullptr;
  return p;
}

void dev_free(dw_ctx ctx, void* p, hipStream_t stream) {
  if (!p) return;
  if (ctx->user_alloc) {
    ctx->alloc.release(p, stream, ctx->alloc.user);
    return;
  }
  (void)hipFreeAsync(p, stream);
}

}  // namespace dw

using namespace dw;

namespace {

// Device memory of dw_apply_noalloc: the internal-layout copies of x and y
// live in this file-scope array instead of allocated buffers. Each GPU the
// library runs on holds its own copy until the process ends. In host code
// the name stands for a host-side shadow, not a device address: host code
// uses only the address that hipGetSymbolAddress returned for the device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Looks up this device's copy of the scratch array once per device; the
// device must be current.
dw_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d beyond the %d devices the scratch table holds", device, kMaxDevices);
    return DW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return DW_OK;
  void* p = nullptr;
  DW_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) {
    set_error("hipGetSymbolAddress returned no address for the scratch array on device %d", device);
    return DW_EHIP;
  }
  g_scratch_ptr[device] = p;
  return DW_OK;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

dw_status check_device(dw_ctx ctx) {
  int cur = -1;
  DW_CHECK_HIP(hipGetDevice(&cur));
  if (cur != ctx->device) DW_CHECK_HIP(hipSetDevice(ctx->device));
  return DW_OK;
}

}  // namespace

extern "C" {

const char* dw_last_error(void) { return dw::g_last_error.c_str(); }

dw_status dw_ctx_create(int32_t device, const dw_allocator* alloc, dw_ctx* out) {
  clear_error();
  if (!out) {
    set_error("dw_ctx_create: null output pointer");
    return DW_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  DW_CHECK_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) {
    set_error("dw_ctx_create: device %d out of range (%d devices)", device, n);
    return DW_EINVAL;
  }
  if (alloc && (!alloc->alloc || !alloc->release)) {
    set_error("dw_ctx_create: allocator needs both alloc and release");
    return DW_EINVAL;
  }
  DW_CHECK_HIP(hipSetDevice(device));
  DW_TRY(scratch_setup(device));
  dw_ctx c = new (std::nothrow) dw_ctx_s;
  if (!c) {
    set_error("out of host memory");
    return DW_ENOMEM;
  }
  c->device = device;
  c->user_alloc = alloc != nullptr;
  if (alloc) c->alloc = *alloc;
  else memset(&c->alloc, 0, sizeof c->alloc);
  *out = c;
  return DW_OK;
}

dw_status dw_ctx_destroy(dw_ctx ctx) {
  clear_error();
  if (ctx) ctx_release(ctx);
  return DW_OK;
}

dw_status dw_field_create(dw_ctx ctx, const int32_t L[4], const int32_t block[4], const double* U_dev,
                          hipStream_t stream, dw_field* out) {
  clear_error();
  if (!ctx || !L || !block || !U_dev || !out) {
    set_error("dw_field_create: null argument");
    return DW_EINVAL;
  }
  *out = nullptr;
  Geom g;
  int Li[4] = {L[0], L[1], L[2], L[3]}, Bi[4] = {block[0], block[1], block[2], block[3]};
  if (const char* msg = make_geom(Li, Bi, &g)) {
    set_error("dw_field_create: %s (L = %d %d %d %d, block = %d %d %d %d)", msg, L[0], L[1], L[2], L[3], block[0],
              block[1], block[2], block[3]);
    return DW_EINVAL;
  }
  DW_TRY(check_device(ctx));
  ProfScope ps(ctx);
  dw_field f = new (std::nothrow) dw_field_s;
  if (!f) {
    set_error("out of host memory");
    return DW_ENOMEM;
  }
  f->ctx = ctx;
  f->g = g;
  f->stream = stream;
  f->csw = 0.0;
  for (int p = 0; p < 4; ++p) f->U[p] = f->C[p] = nullptr;
  for (int p = 0; p < 4; ++p) {
    size_t bytes = (size_t)g.V * 36 * pair_bytes(p);
    f->U[p] = dev_alloc(ctx, bytes, stream);
    if (!f->U[p]) {
      for (int q = 0; q < p; ++q) dev_free(ctx, f->U[q], stream);
      delete f;
      set_error("dw_field_create: allocation of %zu bytes failed", bytes);
      return DW_ENOMEM;
    }
    dw_status st = launch_pack_gauge(g, p, U_dev, f->U[p], stream);
    if (st != DW_OK) {
      for (int q = 0; q <= p; ++q) dev_free(ctx, f->U[q], stream);
      delete f;
      return st;
    }
  }
  ctx->refs.fetch_add(1);
  *out = f;
  return DW_OK;
}

dw_status dw_field_destroy(dw_field f) {
  clear_error();
  if (!f) return DW_OK;
  if (f->solver_cache) f->solver_cache_free(f->solver_cache);
  for (int p = 0; p < 4; ++p) {
    dev_free(f->ctx, f->U[p], f->stream);
    dev_free(f->ctx, f->C[p], f->stream);
  }
  dw_ctx ctx = f->ctx;
  delete f;
  ctx_release(ctx);
  return DW_OK;
}

dw_status dw_field_set_clover(dw_field f, double csw, hipStream_t stream) {
  clear_error();
  if (!f || !std::isfinite(csw)) {
    set_error("dw_field_set_clover: invalid argument");
    return DW_EINVAL;
  }
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  if (f->solver_cache) {
    // captured solver cycles read the old term
    DW_CHECK_HIP(hipStreamSynchronize(stream));
    f->solver_cache_free(f->solver_cache);
    f->solver_cache = nullptr;
    f->solver_cache_free = nullptr;
  }
  for (int p = 0; p < 4; ++p) {
    dev_free(f->ctx, f->C[p], stream);
    f->C[p] = nullptr;
  }
  f->csw = csw;
  if (csw == 0.0) return DW_OK;
  const long long n = f->g.V * kCloverPairs;
  for (int p = 0; p < 4; ++p) {
    const size_t bytes = (size_t)n * pair_bytes(p);
    f->C[p] = dev_alloc(f->ctx, bytes, stream);
    if (!f->C[p]) {
      for (int q = 0; q < p; ++q) {
        dev_free(f->ctx, f->C[q], stream);
        f->C[q] = nullptr;
      }
      f->csw = 0.0;
      set_error("dw_field_set_clover: allocation of %zu bytes failed", bytes);
      return DW_ENOMEM;
    }
  }
  DW_TRY(launch_clover_build(f->g, f->U[DW_PREC_F64], csw, (double*)f->C[DW_PREC_F64], stream));
  for (int p = 1; p < 4; ++p) DW_TRY(launch_convert(DW_PREC_F64, f->C[DW_PREC_F64], p, f->C[p], 1.0, n, stream));
  return DW_OK;
}

int64_t dw_field_volume(dw_field f) { return f ? (int64_t)f->g.V : 0; }

}  // extern "C"

namespace dw {

// Loads new links into an existing field in place (same lattice, block and
// presence of the clover term), keeping its buffers, so that captured solver
// cycles that read them stay valid. Asynchronous on `stream`.
dw_status field_reload(dw_field f, const double* U_dev, double csw, hipStream_t stream) {
  if (!f || !U_dev || (csw != 0.0) != (f->C[DW_PREC_F64] != nullptr) || !std::isfinite(csw)) {
    set_error("field_reload: invalid argument");
    return DW_EINVAL;
  }
  DW_TRY(check_device(f->ctx));
  for (int p = 0; p < 4; ++p) DW_TRY(launch_pack_gauge(f->g, p, U_dev, f->U[p], stream));
  f->csw = csw;
  if (csw != 0.0) {
    const long long n = f->g.V * kCloverPairs;
    DW_TRY(launch_clover_build(f->g, f->U[DW_PREC_F64], csw, (double*)f->C[DW_PREC_F64], stream));
    for (int p = 1; p < 4; ++p) DW_TRY(launch_convert(DW_PREC_F64, f->C[DW_PREC_F64], p, f->C[p], 1.0, n, stream));
  }
  return DW_OK;
}

}  // namespace dw

extern "C" {

size_t dw_internal_bytes(dw_field f, int32_t prec, int32_t nrhs) {
  if (!f || prec < 0 || prec > 3 || nrhs < 0) return 0;
  return (size_t)f->g.V * 12 * pair_bytes(prec) * (size_t)nrhs;
}

dw_status dw_apply(dw_field f, double m0, const double* x, double* y, int32_t nrhs, hipStream_t stream) {
  clear_error();
  if (!f || !x || !y || nrhs < 0) {
    set_error("dw_apply: invalid argument");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  if (x == y) {
    set_error("dw_apply: x and y must not overlap");
    return DW_EINVAL;
  }
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  const Geom& g = f->g;
  const size_t n = (size_t)g.V * 12;
  DevBuf xi, yi;
  DW_TRY(xi.alloc(f->ctx, n * 16 * nrhs, stream));
  DW_TRY(yi.alloc(f->ctx, n * 16 * nrhs, stream));
  DW_TRY(launch_pack_spinor(g, DW_PREC_F64, x, xi.p, 1.0, nrhs, stream));
  DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, xi.p, 1.0, f->U[DW_PREC_F64], yi.as<double>(), nullptr, 0, nrhs,
                             (long long)n, (long long)n, stream, nullptr, f->C[DW_PREC_F64]));
  return launch_unpack_spinor(g, DW_PREC_F64, yi.p, y, 1.0, nrhs, stream);
}

size_t dw_apply_noalloc_max_bytes(void) { return kScratchBytes; }

dw_status dw_apply_noalloc(dw_field f, double m0, const double* x, double* y, int32_t nrhs, hipStream_t stream) {
  clear_error();
  if (!f || !x || !y || nrhs < 0) {
    set_error("dw_apply_noalloc: invalid argument");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  if (x == y) {
    set_error("dw_apply_noalloc: x and y must not overlap");
    return DW_EINVAL;
  }
  const Geom& g = f->g;
  const size_t one = (size_t)g.V * 12 * 16 * (size_t)nrhs;  // one internal FP64 copy
  const size_t yofs = (one + 255) & ~(size_t)255;
  if (yofs + one > kScratchBytes) {
    set_error("dw_apply_noalloc: %d right-hand side(s) of %lld sites need %zu bytes of scratch, above its %zu bytes",
              (int)nrhs, (long long)g.V, yofs + one, kScratchBytes);
    return DW_EINVAL;
  }
  DW_TRY(check_device(f->ctx));
  unsigned char* base = (unsigned char*)scratch_ptr(f->ctx->device);
  if (!base) {
    set_error("dw_apply_noalloc: no scratch address for device %d", f->ctx->device);
    return DW_EHIP;
  }
  ProfScope ps(f->ctx);
  const long long n = g.V * 12;
  void* xi = base;
  double* yi = (double*)(base + yofs);
  DW_TRY(launch_pack_spinor(g, DW_PREC_F64, x, xi, 1.0, nrhs, stream));
  DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, xi, 1.0, f->U[DW_PREC_F64], yi, nullptr, 0, nrhs, n, n, stream,
                             nullptr, f->C[DW_PREC_F64]));
  return launch_unpack_spinor(g, DW_PREC_F64, yi, y, 1.0, nrhs, stream);
}

dw_status dw_apply_ex(dw_field f, double m0, int32_t prec, const void* x, void* y, int32_t nrhs, hipStream_t stream) {
  clear_error();
  if (!f || !x || !y || nrhs < 0 || prec < 0 || prec > 3 || x == y) {
    set_error("dw_apply_ex: invalid argument");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  return launch_dslash_lowp(f->g, m0, prec, x, f->U[prec], y, nrhs, stream, f->C[prec]);
}

dw_status dw_pack(dw_field f, int32_t prec, const double* x, void* xi, int32_t nrhs, hipStream_t stream) {
  clear_error();
  if (!f || !x || !xi || nrhs < 0 || prec < 0 || prec > 3) {
    set_error("dw_pack: invalid argument");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  return launch_pack_spinor(f->g, prec, x, xi, 1.0, nrhs, stream);
}

dw_status dw_unpack(dw_field f, int32_t prec, const void* xi, double* x, int32_t nrhs, hipStream_t stream) {
  clear_error();
  if (!f || !x || !xi || nrhs < 0 || prec < 0 || prec > 3) {
    set_error("dw_unpack: invalid argument");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  return launch_unpack_spinor(f->g, prec, xi, x, 1.0, nrhs, stream);
}

}  // extern "C"

namespace dw {

dw_status check_sap_params(const Geom& g, const sap_params* sp) {
  if (!sp) {
    set_error("null sap_params");
    return DW_EINVAL;
  }
  for (int mu = 0; mu < 4; ++mu)
    if (sp->block[mu] != g.B[mu]) {
      set_error("sap block %d %d %d %d differs from the field's block %d %d %d %d", sp->block[0], sp->block[1],
                sp->block[2], sp->block[3], g.B[0], g.B[1], g.B[2], g.B[3]);
      return DW_EINVAL;
    }
  if (sp->ncycles < 0 || sp->nmr < 0 || sp->storage < 0 || sp->storage > 3 || !(sp->mr_reduction >= 0.0) ||
      !(sp->mr_reduction < 1.0)) {
    set_error("invalid sap_params (ncycles %d, nmr %d, storage %d, mr_reduction %g)", sp->ncycles, sp->nmr,
              sp->storage, sp->mr_reduction);
    return DW_EINVAL;
  }
  return DW_OK;
}

// z (accumulator, FP64 for F64 storage else FP32) = M v, where v is already
// at storage precision in the internal layout. nrhs fields, stride V*12.
dw_status sap_apply_internal(dw_field f, double m0, const sap_params* sp, const void* v, void* z, int nrhs,
                             hipStream_t stream) {
  const Geom& g = f->g;
  const int prec = sp->storage;
  const long long n = g.V * 12;
  for (int cyc = 0; cyc < sp->ncycles; ++cyc)
    for (int colour = 0; colour < 2; ++colour)
      DW_TRY(launch_sap_colour(g, m0, prec, v, z, f->U[prec], colour, sp->nmr, cyc == 0 && colour == 0 ? 1 : 0, nrhs,
                               n, n, stream, nullptr, f->C[prec], sp->mr_reduction));
  return DW_OK;
}

}  // namespace dw

extern "C" dw_status sap_precondition(dw_field f, double m0, const sap_params* sp, const double* v, double* z,
                                      int32_t nrhs, hipStream_t stream) {
  clear_error();
  if (!f || !v || !z || nrhs < 0 || v == z) {
    set_error("sap_precondition: invalid argument");
    return DW_EINVAL;
  }
  DW_TRY(check_sap_params(f->g, sp));
  if (nrhs == 0) return DW_OK;
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  const Geom& g = f->g;
  const long long n = g.V * 12;
  const int prec = sp->storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  if (sp->ncycles == 0) {
    DW_CHECK_HIP(hipMemsetAsync(z, 0, (size_t)n * 16 * nrhs, stream));
    return DW_OK;
  }
  DevBuf vi, zi, part, nrm, sc;
  DW_TRY(vi.alloc(f->ctx, (size_t)n * pair_bytes(prec) * nrhs, stream));
  DW_TRY(zi.alloc(f->ctx, (size_t)n * pair_bytes(zprec) * nrhs, stream));
  if (prec != DW_PREC_F64) {
    // M is scale-equivariant (M(a v) = a M(v)); low-precision storage gets
    // each v scaled to unit RMS per entry so that FP16 keeps its range (the
    // factor is formed on the device, so the call does not synchronise)
    DW_TRY(part.alloc(f->ctx, (size_t)kBlasGrid * 16, stream));
    DW_TRY(nrm.alloc(f->ctx, (size_t)nrhs * 16, stream));
    DW_TRY(sc.alloc(f->ctx, (size_t)nrhs * 16, stream));
    for (int r = 0; r < nrhs; ++r) {
      const double* vr = v + 2 * (long long)r * n;
      DW_TRY(blas_dots(DW_PREC_F64, vr, n, 1, vr, n, part.as<double>(), nrm.as<double>() + 2 * r, 1, 0, stream));
    }
    DW_TRY(rms_scales(nrm.as<double>(), n, sc.as<double>(), nrhs, stream));
  }
  const double* sig = prec != DW_PREC_F64 ? sc.as<double>() : nullptr;
  const double* isig = prec != DW_PREC_F64 ? sc.as<double>() + 1 : nullptr;
  DW_TRY(launch_pack_spinor(g, prec, v, vi.p, 1.0, nrhs, stream, sig, 2));
  DW_TRY(sap_apply_internal(f, m0, sp, vi.p, zi.p, nrhs, stream));
  return launch_unpack_spinor(g, zprec, zi.p, z, 1.0, nrhs, stream, isig, 2);
}

extern "C" dw_status sap_solve(dw_field f, double m0, const sap_params* sp, const double* b, double* x, int32_t niter,
                               double* resid, hipStream_t stream) {
  clear_error();
  if (!f || !b || !x || !resid || niter < 0 || b == x) {
    set_error("sap_solve: invalid argument");
    return DW_EINVAL;
  }
  DW_TRY(check_sap_params(f->g, sp));
  DW_TRY(check_device(f->ctx));
  ProfScope ps(f->ctx);
  const Geom& g = f->g;
  const long long n = g.V * 12;
  const int prec = sp->storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  DevBuf bi, xi, ri, vi, zi, part, nrm, one;
  DW_TRY(bi.alloc(f->ctx, (size_t)n * 16, stream));
  DW_TRY(xi.alloc(f->ctx, (size_t)n * 16, stream));
  DW_TRY(ri.alloc(f->ctx, (size_t)n * 16, stream));
  DW_TRY(vi.alloc(f->ctx, (size_t)n * pair_bytes(prec), stream));
  DW_TRY(zi.alloc(f->ctx, (size_t)n * pair_bytes(zprec), stream));
  DW_TRY(part.alloc(f->ctx, (size_t)kBlasGrid * 16, stream));
  DW_TRY(nrm.alloc(f->ctx, 16, stream));
  DW_TRY(one.alloc(f->ctx, 16, stream));
  static const double kOne[2] = {1.0, 0.0};
  DW_CHECK_HIP(hipMemcpyAsync(one.p, kOne, sizeof kOne, hipMemcpyHostToDevice, stream));
  DW_TRY(launch_pack_spinor(g, DW_PREC_F64, b, bi.p, 1.0, 1, stream));
  DW_CHECK_HIP(hipMemsetAsync(xi.p, 0, (size_t)n * 16, stream));
  auto sqnorm = [&](const void* v, double& out) -> dw_status {
    DW_TRY(blas_dots(DW_PREC_F64, v, n, 1, (const double*)v, n, part.as<double>(), nrm.as<double>(), 1, 0, stream));
    double h[2];
    DW_CHECK_HIP(hipMemcpyAsync(h, nrm.p, sizeof h, hipMemcpyDeviceToHost, stream));
    DW_CHECK_HIP(hipStreamSynchronize(stream));
    out = h[0];
    return DW_OK;
  };
  double bb;
  DW_TRY(sqnorm(bi.p, bb));
  if (!(bb > 0)) {
    set_error("sap_solve: b = 0");
    return DW_EINVAL;
  }
  const double bnorm = sqrt(bb);
  for (int k = 0; k <= niter; ++k) {
    // r = b - D x_k (FP64 links, clover and arithmetic)
    DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, xi.p, 1.0, f->U[DW_PREC_F64], ri.as<double>(), bi.as<double>(), 1,
                               1, n, n, stream, nullptr, f->C[DW_PREC_F64]));
    double rr;
    DW_TRY(sqnorm(ri.p, rr));
    resid[k] = sqrt(rr) / bnorm;
    if (rr == 0) {
      for (int j = k + 1; j <= niter; ++j) resid[j] = 0;
      break;
    }
    if (k == niter || sp->ncycles == 0) continue;  // M = 0 without cycles
    // x_{k+1} = x_k + M r: the preconditioner input at storage precision,
    // scaled to unit RMS (M is scale-equivariant), the correction added in FP64
    const double sigma = prec == DW_PREC_F64 ? 1.0 : sqrt((double)n / rr);
    DW_TRY(launch_convert(DW_PREC_F64, ri.p, prec, vi.p, sigma, n, stream));
    DW_TRY(sap_apply_internal(f, m0, sp, vi.p, zi.p, 1, stream));
    DW_TRY(blas_combine(zprec, zi.p, n, 1, one.as<double>(), 1.0 / sigma, xi.as<double>(), n, stream));
  }
  DW_TRY(launch_unpack_spinor(g, DW_PREC_F64, xi.p, x, 1.0, 1, stream));
  DW_CHECK_HIP(hipStreamSynchronize(stream));
  return DW_OK;
}
