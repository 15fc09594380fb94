// FGMRES-DR driver (paper Section 4, Alg. 3 and Alg. 4, Section 4.7).
//
// The host sequences kernels on the caller's stream; all vector work and
// every small dense problem run on the GPU. The host reads back a handful
// of scalars per Arnoldi step (implicit residual, breakdown flag) and per
// cycle (explicit residual, deflation status) to steer the iteration.
//
// Per Arnoldi step j (flexible, Alg. 3):
//   z_j = M_j v_j   SAP at storage precision on sigma * v_j (sigma = sqrt(n)
//                   gives unit RMS entries; M is scale-equivariant) with an
//                   FP32 accumulator (FP64 for FP64 storage); the result is
//                   kept in Z at FP64, which holds it exactly, so that the
//                   rotated deflation basis Z_k = Z Q_k keeps A Z = V H^ to
//                   FP64 accuracy (an FP32 Z_k makes the implicit residual
//                   drift from the explicit one near convergence);
//   w = D z_j       FP64 operator on the stored z_j, so A Z = V H^ holds to
//                   FP64 accuracy whatever precision Z has;
//   classical Gram-Schmidt with one reorthogonalisation, delayed by one
//                   step: the sweep that projects w (first pass) also
//                   reorthogonalises the previous step's vector (second
//                   pass), so V is read twice per step instead of four
//                   times; the paper prints modified GS, all give the same
//                   H^ up to rounding;
//   h_{j+1,j} = ||w'||, implicit residual from the small least-squares
//                   problem (the last column is provisional until the next
//                   step's second pass, and is finalised at the cycle end).
// Per cycle: eta, x += Z eta, explicit FP64 residual r = b - D x; stop, or
// clean restart if ||r|| / ||r_implicit|| > t, or deflated restart:
// harmonic Ritz pairs, Q_{k+1}, V <- V Q_{k+1}, Z <- Z Q_k, H^_k, and
// c = [V_{k+1}^H r; 0] with the explicit residual r.
#include <math.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include <chrono>
#include <vector>

#include "dw_internal.hpp"
#include "dw_kernels.hpp"

namespace dw {
dw_status check_sap_params(const Geom& g, const sap_params* sp);
}

using namespace dw;

namespace {

struct Work {
  DevBuf V, Z, zs, w, r, x, b, vs, partials, H, c, eta, red, coef, nrm, Q, ritz, scal;
  double* scal_h = nullptr;
  ~Work() {
    if (scal_h) (void)hipHostFree(scal_h);
  }
};

dw_status alloc_work(dw_field f, const fgmresdr_params* P, Work& W, hipStream_t s) {
  const long long n = f->g.V * 12;
  const int prec = P->sap.storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  dw_ctx ctx = f->ctx;
  DW_TRY(W.V.alloc(ctx, (size_t)(P->m + 1) * n * 16, s));
  DW_TRY(W.Z.alloc(ctx, (size_t)P->m * n * 16, s));
  if (zprec != DW_PREC_F64) DW_TRY(W.zs.alloc(ctx, (size_t)n * pair_bytes(zprec), s));
  DW_TRY(W.w.alloc(ctx, (size_t)n * 16, s));
  DW_TRY(W.r.alloc(ctx, (size_t)n * 16, s));
  DW_TRY(W.x.alloc(ctx, (size_t)n * 16, s));
  DW_TRY(W.b.alloc(ctx, (size_t)n * 16, s));
  DW_TRY(W.vs.alloc(ctx, (size_t)n * pair_bytes(prec), s));
  DW_TRY(W.partials.alloc(ctx, (size_t)(2 * kLd + 6) * kBlasGrid * 16, s));
  DW_TRY(W.H.alloc(ctx, (size_t)kLd * kMaxM * 16, s));
  DW_TRY(W.c.alloc(ctx, (size_t)kLd * 16, s));
  DW_TRY(W.eta.alloc(ctx, (size_t)kMaxM * 16, s));
  DW_TRY(W.red.alloc(ctx, (size_t)(2 * kLd + 6) * 16, s));
  DW_TRY(W.coef.alloc(ctx, (size_t)(2 * kLd + 4) * 16, s));
  DW_TRY(W.nrm.alloc(ctx, 16, s));
  DW_TRY(W.Q.alloc(ctx, (size_t)kLd * 25 * 16, s));
  DW_TRY(W.ritz.alloc(ctx, (size_t)kMaxM * 16, s));
  DW_TRY(W.scal.alloc(ctx, (size_t)kSclCount * 8, s));
  DW_CHECK_HIP(hipHostMalloc((void**)&W.scal_h, 16 * sizeof(double), hipHostMallocDefault));
  return DW_OK;
}

// reads scal (kSclCount doubles) and nrm (one pair) to the host
dw_status readback(Work& W, hipStream_t s) {
  DW_CHECK_HIP(hipMemcpyAsync(W.scal_h, W.scal.p, kSclCount * sizeof(double), hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipMemcpyAsync(W.scal_h + kSclCount, W.nrm.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  prof_flush();
  return DW_OK;
}

dw_status solve_one(dw_field f, double m0, const fgmresdr_params* P, const double* b_can, double* x_can, Work& W,
                    dw_solve_stats* st, hipStream_t s) {
  const Geom& g = f->g;
  const long long n = g.V * 12;
  const int m = P->m, k = P->k;
  const int prec = P->sap.storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;  // SAP accumulator
  const size_t zb = 16;                                                  // Z is FP64
  const double sigma = prec == DW_PREC_F64 ? 1.0 : sqrt((double)n);
  const double bd_tol = 1e-14;
  double* V = W.V.as<double>();
  char* Z = W.Z.as<char>();
  double* partials = W.partials.as<double>();
  double* scal = W.scal.as<double>();
  auto t0 = std::chrono::steady_clock::now();

  DW_TRY(launch_pack_spinor(g, DW_PREC_F64, b_can, W.b.p, 1.0, 1, s));
  DW_CHECK_HIP(hipMemsetAsync(W.x.p, 0, (size_t)n * 16, s));
  DW_TRY(blas_dots(DW_PREC_F64, W.b.p, n, 1, W.b.as<double>(), n, partials, W.nrm.as<double>(), 1, 0, s));
  DW_TRY(readback(W, s));
  const double bnorm = sqrt(W.scal_h[kSclCount]);
  memset(st, 0, sizeof *st);
  if (bnorm == 0.0) {
    DW_CHECK_HIP(hipMemsetAsync(x_can, 0, (size_t)n * 16, s));
    DW_CHECK_HIP(hipStreamSynchronize(s));
    st->converged = 1;
    return DW_OK;
  }
  DW_CHECK_HIP(hipMemcpyAsync(W.r.p, W.b.p, (size_t)n * 16, hipMemcpyDeviceToDevice, s));

  int iters = 0, cycles = 0, clean = 0;
  double res_e = bnorm, res_i = bnorm;
  bool fresh = true, converged = false;
  while (true) {
    int j0;
    if (fresh) {
      // nrm holds ||r||^2 of the current explicit residual
      DW_TRY(dense_fresh(W.H.as<double>(), W.c.as<double>(), W.nrm.as<double>(), scal, s));
      DW_TRY(blas_scale(W.r.as<double>(), V, scal + kSclBetaInv, n, s));
      j0 = 0;
    } else {
      j0 = k;
    }
    int jend = j0;
    bool broke = false;
    bool lagged = false;  // V_j holds a once-orthogonalised, unnormalised vector
    double* red = W.red.as<double>();
    double* coef = W.coef.as<double>();
    for (int j = j0; j < m; ++j) {
      double* vj = V + 2 * (long long)j * n;
      double* vnext = V + 2 * (long long)(j + 1) * n;
      double* zj = (double*)(Z + (size_t)j * n * zb);
      void* zacc = zprec == DW_PREC_F64 ? (void*)zj : W.zs.p;
      // z_j = M_j applied to sigma * v_j (the lagged vector scaled by its
      // provisional norm; any z_j keeps A Z = V H^ exact in FGMRES)
      DW_TRY(launch_convert(DW_PREC_F64, vj, prec, W.vs.p, sigma, n, s, lagged ? scal + kSclHinv : nullptr));
      for (int cyc = 0; cyc < P->sap.ncycles; ++cyc)
        for (int colour = 0; colour < 2; ++colour)
          DW_TRY(launch_sap_colour(g, m0, prec, W.vs.p, zacc, f->U[prec], colour, P->sap.nmr,
                                   cyc == 0 && colour == 0 ? 1 : 0, 1, n, n, s));
      if (zprec != DW_PREC_F64) DW_TRY(launch_convert(zprec, zacc, DW_PREC_F64, zj, 1.0 / sigma, n, s));
      // w = D z_j in FP64 on the stored z_j
      DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, zj, 1.0, f->U[DW_PREC_F64], W.w.as<double>(), nullptr, 0, 1, n,
                                 n, s));
      // Gram-Schmidt with delayed reorthogonalisation: one sweep of dot
      // products finalises v_j (second pass) and projects w (first pass),
      // one update sweep writes v_j and the next lagged vector w'.
      const int nv = lagged ? j : j + 1;
      DW_TRY(gs_reduce(V, n, nv, lagged ? vj : nullptr, W.w.as<double>(), n, partials, red, s));
      DW_TRY(dense_gs_coef(W.H.as<double>(), nv, lagged ? j : -1, j, lagged ? 1 : 0, 1, red, coef, scal, bd_tol, s));
      DW_TRY(gs_update(V, n, nv, lagged ? j : -1, W.w.as<double>(), vnext, coef, n, partials, W.nrm.as<double>(), s));
      DW_TRY(dense_step2(W.H.as<double>(), j, W.nrm.as<double>(), W.c.as<double>(), scal, bd_tol, s));
      lagged = true;
      ++iters;
      jend = j + 1;
      DW_TRY(readback(W, s));
      res_i = W.scal_h[kSclResImp];
      broke = W.scal_h[kSclBreak] != 0.0;
      if (broke || res_i <= P->tol * bnorm || iters >= P->max_iter) break;
    }
    // finalise the last lagged vector (second Gram-Schmidt pass) so that
    // V_{jend+1} is orthonormal and H^ exact; after a breakdown it is unused
    if (lagged && !broke) {
      double* vl = V + 2 * (long long)jend * n;
      DW_TRY(gs_reduce(V, n, jend, vl, nullptr, n, partials, red, s));
      DW_TRY(dense_gs_coef(W.H.as<double>(), jend, jend, -1, 1, 0, red, coef, scal, bd_tol, s));
      DW_TRY(gs_update(V, n, jend, jend, nullptr, nullptr, coef, n, partials, nullptr, s));
    }
    // iterate and explicit FP64 residual
    DW_TRY(dense_lsq(W.H.as<double>(), jend, W.c.as<double>(), W.eta.as<double>(), scal, s));
    DW_TRY(blas_combine(DW_PREC_F64, Z, n, jend, W.eta.as<double>(), 1.0, W.x.as<double>(), n, s));
    DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, W.x.p, 1.0, f->U[DW_PREC_F64], W.r.as<double>(),
                               W.b.as<double>(), 1, 1, n, n, s));
    DW_TRY(blas_dots(DW_PREC_F64, W.r.p, n, 1, W.r.as<double>(), n, partials, W.nrm.as<double>(), 1, 0, s));
    DW_TRY(readback(W, s));
    res_i = W.scal_h[kSclResImp];
    res_e = sqrt(W.scal_h[kSclCount]);
    ++cycles;
    if (res_e <= P->tol * bnorm) {
      converged = true;
      break;
    }
    if (iters >= P->max_iter) break;
    if (k == 0) {
      fresh = true;
      continue;
    }
    if (broke || jend <= k || res_e > P->restart_t * fmax(res_i, 1e-300)) {
      ++clean;
      fresh = true;
      continue;
    }
    DW_TRY(dense_deflate(W.H.as<double>(), jend, k, W.c.as<double>(), W.eta.as<double>(), W.Q.as<double>(),
                         W.ritz.as<double>(), scal, s));
    DW_TRY(readback(W, s));
    if (W.scal_h[kSclStatus] != 0.0) {
      ++clean;
      fresh = true;
      continue;
    }
    DW_TRY(blas_rotate(DW_PREC_F64, V, n, jend + 1, W.Q.as<double>(), kLd, k + 1, n, s));
    DW_TRY(blas_rotate(DW_PREC_F64, Z, n, jend, W.Q.as<double>(), kLd, k, n, s));
    DW_CHECK_HIP(hipMemsetAsync(W.c.p, 0, (size_t)kLd * 16, s));
    DW_TRY(blas_dots(DW_PREC_F64, V, n, k + 1, W.r.as<double>(), n, partials, W.c.as<double>(), 1, 0, s));
    fresh = false;
  }
  DW_TRY(launch_unpack_spinor(g, DW_PREC_F64, W.x.p, x_can, 1.0, 1, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  st->converged = converged ? 1 : 0;
  st->iterations = iters;
  st->cycles = cycles;
  st->clean_restarts = clean;
  st->true_relres = res_e / bnorm;
  st->implicit_relres = res_i / bnorm;
  st->seconds = std::chrono::duration<double>(t1 - t0).count();
  return DW_OK;
}

}  // namespace

extern "C" dw_status fgmresdr_solve(dw_field f, double m0, const fgmresdr_params* P, const double* b, double* x,
                                    int32_t nrhs, dw_solve_stats* stats, hipStream_t stream) {
  clear_error();
  if (!f || !P || !b || !x || nrhs < 0 || b == x) {
    set_error("fgmresdr_solve: invalid argument");
    return DW_EINVAL;
  }
  if (P->m < 1 || P->m > kMaxM || P->k < 0 || P->k >= P->m || P->k > 23 || P->max_iter < 1 || !(P->tol > 0) ||
      !(P->restart_t > 0)) {
    set_error("fgmresdr_solve: invalid parameters (m %d, k %d, max_iter %d, tol %g, t %g); need 1 <= m <= %d, "
              "0 <= k < m, k <= 23",
              P->m, P->k, P->max_iter, P->tol, P->restart_t, kMaxM);
    return DW_EINVAL;
  }
  DW_TRY(check_sap_params(f->g, &P->sap));
  if (P->sap.ncycles < 1) {
    set_error("fgmresdr_solve: need at least one SAP cycle");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  int cur = -1;
  DW_CHECK_HIP(hipGetDevice(&cur));
  if (cur != f->ctx->device) DW_CHECK_HIP(hipSetDevice(f->ctx->device));
  ProfScope ps(f->ctx);
  Work W;
  DW_TRY(alloc_work(f, P, W, stream));
  const long long n = f->g.V * 12;
  bool all_conv = true;
  for (int r = 0; r < nrhs; ++r) {
    dw_solve_stats st;
    DW_TRY(solve_one(f, m0, P, b + 2 * (long long)r * n, x + 2 * (long long)r * n, W, &st, stream));
    if (stats) stats[r] = st;
    all_conv = all_conv && st.converged;
  }
  if (!all_conv) {
    set_error("fgmresdr_solve: max_iter reached before the tolerance");
    return DW_ENOTCONV;
  }
  return DW_OK;
}
