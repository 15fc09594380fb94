// Host-array entry points of the small dense steps of FGMRES-DR, so that
// they can be compared directly with a reference: the least-squares
// problem of Section 4.2 and the deflated restart of Section 4.4 (harmonic
// Ritz pairs of Lemma 1, G_{k+1}, its QR factorisation and H^_k). They run
// the same one-wavefront kernels the solver launches.
#include <string.h>

#include <hip/hip_runtime.h>

#include "dw_internal.hpp"
#include "dw_kernels.hpp"

using namespace dw;

namespace {

// copies a host column-major complex matrix (rows x cols, leading dim ld_in)
// into a kLd-leading device layout staged through host memory
dw_status upload_mat(const double* h, int rows, int cols, int ld_in, double* dev, hipStream_t s, double* stage) {
  memset(stage, 0, sizeof(double) * 2 * kLd * kMaxM);
  for (int q = 0; q < cols; ++q)
    for (int i = 0; i < rows; ++i) {
      stage[2 * (i + q * kLd)] = h[2 * (i + (long long)q * ld_in)];
      stage[2 * (i + q * kLd) + 1] = h[2 * (i + (long long)q * ld_in) + 1];
    }
  DW_CHECK_HIP(hipMemcpyAsync(dev, stage, sizeof(double) * 2 * kLd * kMaxM, hipMemcpyHostToDevice, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  return DW_OK;
}

struct DenseBufs {
  DevBuf H, c, eta, Q, ritz, scal;
  dw_status alloc(dw_ctx ctx, hipStream_t s) {
    DW_TRY(H.alloc(ctx, (size_t)kLd * kMaxM * 16, s));
    DW_TRY(c.alloc(ctx, (size_t)kLd * 16, s));
    DW_TRY(eta.alloc(ctx, (size_t)kMaxM * 16, s));
    DW_TRY(Q.alloc(ctx, (size_t)kLd * 25 * 16, s));
    DW_TRY(ritz.alloc(ctx, (size_t)kMaxM * 16, s));
    DW_TRY(scal.alloc(ctx, (size_t)kSclCount * 8, s));
    return DW_OK;
  }
};

dw_status set_device(dw_ctx ctx) {
  int cur = -1;
  DW_CHECK_HIP(hipGetDevice(&cur));
  if (cur != ctx->device) DW_CHECK_HIP(hipSetDevice(ctx->device));
  return DW_OK;
}

}  // namespace

extern "C" dw_status dw_dense_lsq(dw_ctx ctx, int32_t cols, const double* Hhat, const double* c, double* eta,
                                  double* resid) {
  clear_error();
  if (!ctx || !Hhat || !c || !eta || !resid || cols < 1 || cols > kMaxM) {
    set_error("dw_dense_lsq: invalid argument (cols %d, 1..%d)", (int)cols, kMaxM);
    return DW_EINVAL;
  }
  DW_TRY(set_device(ctx));
  ProfScope ps(ctx);
  hipStream_t s = nullptr;
  DenseBufs B;
  DW_TRY(B.alloc(ctx, s));
  static thread_local double stage[2 * kLd * kMaxM];
  DW_TRY(upload_mat(Hhat, cols + 1, cols, cols + 1, B.H.as<double>(), s, stage));
  DW_TRY(upload_mat(c, cols + 1, 1, cols + 1, B.c.as<double>(), s, stage));
  DW_TRY(dense_lsq(B.H.as<double>(), cols, B.c.as<double>(), B.eta.as<double>(), B.scal.as<double>(), s));
  double sc[kSclCount];
  DW_CHECK_HIP(hipMemcpyAsync(eta, B.eta.p, (size_t)cols * 16, hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipMemcpyAsync(sc, B.scal.p, sizeof sc, hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  *resid = sc[kSclResImp];
  return DW_OK;
}

extern "C" dw_status dw_dense_restart(dw_ctx ctx, int32_t mm, int32_t k, const double* Hhat, const double* c,
                                      const double* eta, double* ritz, double* Q, double* Hk, int32_t* status) {
  clear_error();
  if (!ctx || !Hhat || !c || !eta || !ritz || !Q || !Hk || !status || mm < 2 || mm > kMaxM || k < 1 || k >= mm ||
      k > 23) {
    set_error("dw_dense_restart: invalid argument (mm %d, k %d)", (int)mm, (int)k);
    return DW_EINVAL;
  }
  DW_TRY(set_device(ctx));
  ProfScope ps(ctx);
  hipStream_t s = nullptr;
  DenseBufs B;
  DW_TRY(B.alloc(ctx, s));
  static thread_local double stage[2 * kLd * kMaxM];
  DW_TRY(upload_mat(Hhat, mm + 1, mm, mm + 1, B.H.as<double>(), s, stage));
  DW_TRY(upload_mat(c, mm + 1, 1, mm + 1, B.c.as<double>(), s, stage));
  DW_TRY(upload_mat(eta, mm, 1, mm, B.eta.as<double>(), s, stage));
  DW_TRY(dense_deflate(B.H.as<double>(), mm, k, B.c.as<double>(), B.eta.as<double>(), B.Q.as<double>(),
                       B.ritz.as<double>(), B.scal.as<double>(), s));
  double sc[kSclCount];
  DW_CHECK_HIP(hipMemcpyAsync(sc, B.scal.p, sizeof sc, hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipMemcpyAsync(ritz, B.ritz.p, (size_t)mm * 16, hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipMemcpyAsync(stage, B.Q.p, (size_t)kLd * (k + 1) * 16, hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  for (int q = 0; q <= k; ++q)
    for (int i = 0; i <= mm; ++i) {
      Q[2 * (i + (long long)q * (mm + 1))] = stage[2 * (i + q * kLd)];
      Q[2 * (i + (long long)q * (mm + 1)) + 1] = stage[2 * (i + q * kLd) + 1];
    }
  DW_CHECK_HIP(hipMemcpyAsync(stage, B.H.p, (size_t)kLd * k * 16, hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < k; ++q)
    for (int i = 0; i <= k; ++i) {
      Hk[2 * (i + (long long)q * (k + 1))] = stage[2 * (i + q * kLd)];
      Hk[2 * (i + (long long)q * (k + 1)) + 1] = stage[2 * (i + q * kLd) + 1];
    }
  *status = (int32_t)sc[kSclStatus];
  return DW_OK;
}
