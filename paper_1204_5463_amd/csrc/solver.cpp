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
// c = [V_{k+1}^H r; 0] with the explicit residual r. With DW_SOLVE_INJECT the
// explicit residual also gives G_{k+1}'s last column (V^H r) and v_{k+1}
// (r orthonormalised against the rotated V_k, phase-matched to the rotated
// v_{k+1}), as Section 4.7 does for its low-precision Arnoldi.
#include <math.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "dw_internal.hpp"
#include "dw_kernels.hpp"

namespace dw {
dw_status check_sap_params(const Geom& g, const sap_params* sp);
}

using namespace dw;

namespace {

// Device and host state of a batch of right-hand sides solved in lock-step.
struct Work {
  int nr = 0, m = 0;
  long long n = 0;
  DevBuf V, Z, zs, w, r, x, b, vs, partials, H, c, eta, red, coef, nrm, Q, ritz, scal, rlist, proj, inj, zeta;
  double* scal_h = nullptr;  // nr x (kSclCount + 2): scalars and the pair nrm
  int* rlist_h = nullptr;
  double* inj_h = nullptr;  // nr x 4 doubles: v_{k+1}^H w and ||w||^2 of the injection, then its coefficient
  // captured Arnoldi steps, indexed by 2 j + lagged (single-RHS batches)
  std::vector<hipGraphExec_t> graphs;
  ~Work() {
    for (hipGraphExec_t g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    if (scal_h) (void)hipHostFree(scal_h);
    if (rlist_h) (void)hipHostFree(rlist_h);
    if (inj_h) (void)hipHostFree(inj_h);
  }
  int vprec = DW_PREC_F64;  // storage of the Krylov basis V
  // basis of RHS r, and its column j
  void* Vr(int r) const { return (char*)V.p + (size_t)r * (m + 1) * n * pair_bytes(vprec); }
  void* Vc(int r, int j) const { return (char*)Vr(r) + (size_t)j * n * pair_bytes(vprec); }
  double* Zr(int r) const { return Z.as<double>() + 2 * (long long)r * m * n; }
  double* vec(const DevBuf& d, int r) const { return d.as<double>() + 2 * (long long)r * n; }
  double* Hr(int r) const { return H.as<double>() + 2 * (long long)r * kLd * kMaxM; }
  double* cr(int r) const { return c.as<double>() + 2 * (long long)r * kLd; }
  double* etar(int r) const { return eta.as<double>() + 2 * (long long)r * kMaxM; }
  double* redr(int r) const { return red.as<double>() + 2 * (long long)r * (2 * kLd + 6); }
  double* coefr(int r) const { return coef.as<double>() + 2 * (long long)r * (2 * kLd + 4); }
  double* nrmr(int r) const { return nrm.as<double>() + 2 * (long long)r; }
  double* Qr(int r) const { return Q.as<double>() + 2 * (long long)r * kLd * 25; }
  double* ritzr(int r) const { return ritz.as<double>() + 2 * (long long)r * kMaxM; }
  double* scalr(int r) const { return scal.as<double>() + (long long)r * kSclCount; }
  double* partr(int r) const { return partials.as<double>() + 2 * (long long)r * (2 * kLd + 6) * kBlasGrid; }
  const double* sh(int r) const { return scal_h + (long long)r * (kSclCount + 2); }
  // shared-deflation projection: t = V_0^H r (kLd pairs), y (kMaxM), s = H_0 y (kLd)
  double* projr(int r) const { return proj.as<double>() + 2 * (long long)r * (2 * kLd + kMaxM); }
  // residual injection: G column V^H r (kLd pairs), t = V_k^H w (kLd), then
  // 4 pairs: v_{k+1}^H w, ||w||^2, coefficient
  double* injr(int r) const { return inj.as<double>() + 2 * (long long)r * (2 * kLd + 4); }
};

int basis_prec(const fgmresdr_params* P) { return (P->flags & DW_SOLVE_V32) ? DW_PREC_F32 : DW_PREC_F64; }

size_t bytes_per_rhs(long long n, int m, int prec, int vprec) {
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  return (size_t)n * pair_bytes(vprec) * (m + 1) + (size_t)n * 16 * (m + 4) + (size_t)n * pair_bytes(prec) +
         (zprec != DW_PREC_F64 ? (size_t)n * pair_bytes(zprec) : 0) + (size_t)(2 * kLd + 6) * kBlasGrid * 16;
}

dw_status alloc_work(dw_field f, const fgmresdr_params* P, int nr, Work& W, hipStream_t s) {
  const long long n = f->g.V * 12;
  const int prec = P->sap.storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  dw_ctx ctx = f->ctx;
  W.nr = nr;
  W.m = P->m;
  W.n = n;
  W.vprec = basis_prec(P);
  DW_TRY(W.V.alloc(ctx, (size_t)nr * (P->m + 1) * n * pair_bytes(W.vprec), s));
  DW_TRY(W.Z.alloc(ctx, (size_t)nr * P->m * n * 16, s));
  if (zprec != DW_PREC_F64) DW_TRY(W.zs.alloc(ctx, (size_t)nr * n * pair_bytes(zprec), s));
  DW_TRY(W.w.alloc(ctx, (size_t)nr * n * 16, s));
  DW_TRY(W.r.alloc(ctx, (size_t)nr * n * 16, s));
  DW_TRY(W.x.alloc(ctx, (size_t)nr * n * 16, s));
  DW_TRY(W.b.alloc(ctx, (size_t)nr * n * 16, s));
  DW_TRY(W.vs.alloc(ctx, (size_t)nr * n * pair_bytes(prec), s));
  DW_TRY(W.partials.alloc(ctx, (size_t)nr * (2 * kLd + 6) * kBlasGrid * 16, s));
  DW_TRY(W.H.alloc(ctx, (size_t)nr * kLd * kMaxM * 16, s));
  DW_TRY(W.c.alloc(ctx, (size_t)nr * kLd * 16, s));
  DW_TRY(W.eta.alloc(ctx, (size_t)nr * kMaxM * 16, s));
  DW_TRY(W.red.alloc(ctx, (size_t)nr * (2 * kLd + 6) * 16, s));
  DW_TRY(W.coef.alloc(ctx, (size_t)nr * (2 * kLd + 4) * 16, s));
  DW_TRY(W.nrm.alloc(ctx, (size_t)nr * 16, s));
  DW_TRY(W.Q.alloc(ctx, (size_t)nr * kLd * 25 * 16, s));
  DW_TRY(W.ritz.alloc(ctx, (size_t)nr * kMaxM * 16, s));
  DW_TRY(W.scal.alloc(ctx, (size_t)nr * kSclCount * 8, s));
  if (P->shared_defl && nr > 1) DW_TRY(W.proj.alloc(ctx, (size_t)nr * (2 * kLd + kMaxM) * 16, s));
  if (P->flags & DW_SOLVE_INJECT) {
    DW_TRY(W.inj.alloc(ctx, (size_t)nr * (2 * kLd + 4) * 16, s));
    DW_TRY(W.zeta.alloc(ctx, (size_t)kMaxM * 16, s));
    DW_CHECK_HIP(hipMemsetAsync(W.zeta.p, 0, (size_t)kMaxM * 16, s));
    DW_CHECK_HIP(hipHostMalloc((void**)&W.inj_h, (size_t)nr * 4 * sizeof(double), hipHostMallocDefault));
  }
  DW_TRY(W.rlist.alloc(ctx, (size_t)nr * sizeof(int), s));
  DW_CHECK_HIP(hipHostMalloc((void**)&W.scal_h, (size_t)nr * (kSclCount + 2) * sizeof(double), hipHostMallocDefault));
  DW_CHECK_HIP(hipHostMalloc((void**)&W.rlist_h, (size_t)nr * sizeof(int), hipHostMallocDefault));
  return DW_OK;
}

// reads every RHS's scalars and squared norm to the host (one sync)
dw_status readback(Work& W, hipStream_t s) {
  for (int r = 0; r < W.nr; ++r) {
    DW_CHECK_HIP(hipMemcpyAsync(W.scal_h + (long long)r * (kSclCount + 2), W.scalr(r), kSclCount * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    DW_CHECK_HIP(hipMemcpyAsync(W.scal_h + (long long)r * (kSclCount + 2) + kSclCount, W.nrmr(r), 2 * sizeof(double),
                                hipMemcpyDeviceToHost, s));
  }
  DW_CHECK_HIP(hipStreamSynchronize(s));
  prof_flush();
  return DW_OK;
}

// uploads the list of participating RHS; the pinned host copy is reused only
// after the next synchronisation, which every step performs
dw_status set_rlist(Work& W, const std::vector<int>& list, hipStream_t s) {
  for (size_t i = 0; i < list.size(); ++i) W.rlist_h[i] = list[i];
  DW_CHECK_HIP(hipMemcpyAsync(W.rlist.p, W.rlist_h, list.size() * sizeof(int), hipMemcpyHostToDevice, s));
  return DW_OK;
}

// v_{k+1} from the explicit residual r (Section 4.7): w = r orthogonalised
// against the rotated V_k (classical Gram-Schmidt, two passes), then
// v_{k+1} = e^{i theta} w / ||w|| with the phase of the rotated v_{k+1}
// (e^{i theta} = w^H v_{k+1} / |w^H v_{k+1}|), so that D Z_k = V_{k+1} H^_k
// keeps its coefficients. The rotated vector is kept when r lies in
// span(V_k) (||w|| <= 1e-12 ||r||), w is orthogonal to it, or a value is not
// finite. rnorm: ||r|| per entry of rot. Uses W.w as scratch; one
// synchronisation for the batch.
dw_status inject_residual(Work& W, const std::vector<int>& rot, const std::vector<double>& rnorm, int k,
                          hipStream_t s) {
  const long long n = W.n;
  for (size_t i = 0; i < rot.size(); ++i) {
    const int r = rot[i];
    double* w = W.vec(W.w, r);
    double* t = W.injr(r) + 2 * kLd;
    double* tail = W.injr(r) + 4 * kLd;
    DW_CHECK_HIP(hipMemcpyAsync(w, W.vec(W.r, r), (size_t)n * 16, hipMemcpyDeviceToDevice, s));
    for (int pass = 0; pass < 2; ++pass) {
      DW_TRY(blas_dots(W.vprec, W.Vr(r), n, k, w, n, W.partr(r), t, 1, 0, s));
      DW_TRY(blas_combine(W.vprec, W.Vr(r), n, k, t, -1.0, w, n, s));
    }
    DW_TRY(blas_dots(W.vprec, W.Vc(r, k), n, 1, w, n, W.partr(r), tail, 1, 0, s));
    DW_TRY(blas_dots(DW_PREC_F64, w, n, 1, w, n, W.partr(r), tail + 2, 1, 0, s));
    DW_CHECK_HIP(hipMemcpyAsync(W.inj_h + 4 * (long long)i, tail, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  DW_CHECK_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < rot.size(); ++i) {
    const int r = rot[i];
    double* h = W.inj_h + 4 * (long long)i;
    // h[0] + i h[1] = v_{k+1}^H w, h[2] = ||w||^2
    const double pm = hypot(h[0], h[1]), wn = sqrt(h[2]);
    if (!(pm > 0) || !(wn > 1e-12 * rnorm[i]) || !std::isfinite(pm) || !std::isfinite(wn)) continue;
    // coefficient e^{i theta} / ||w|| with e^{i theta} = conj(v^H w) / |v^H w|
    h[0] = h[0] / (pm * wn);
    h[1] = -h[1] / (pm * wn);
    double* coef = W.injr(r) + 4 * kLd + 4;
    DW_CHECK_HIP(hipMemcpyAsync(coef, h, 2 * sizeof(double), hipMemcpyHostToDevice, s));
    double* w = W.vec(W.w, r);
    if (W.vprec == DW_PREC_F64) {
      DW_CHECK_HIP(hipMemsetAsync(W.Vc(r, k), 0, (size_t)n * 16, s));
      DW_TRY(blas_combine(DW_PREC_F64, w, n, 1, coef, 1.0, (double*)W.Vc(r, k), n, s));
    } else {
      // w <- coefficient * w in place (FP64), then stored at the basis precision
      DW_TRY(blas_scale_c(w, coef, n, s));
      DW_TRY(launch_convert(DW_PREC_F64, w, W.vprec, W.Vc(r, k), 1.0, n, s));
    }
  }
  // the pinned coefficients stay in use until the copies above have run
  DW_CHECK_HIP(hipStreamSynchronize(s));
  return DW_OK;
}

struct Rhs {
  int j0 = 0, jend = 0, iters = 0, cycles = 0, clean = 0;
  bool lagged = false, broke = false, frozen = false, done = false, converged = false, fresh = true;
  double bnorm = 0, res_e = 0, res_i = 0;
};

// Solves nr right-hand sides in lock-step: at Arnoldi step j every RHS whose
// current cycle covers j takes part; the SAP sweeps and the FP64 operator
// cover all of them in one launch (each link read serves every RHS through
// L2), the Gram-Schmidt and small dense kernels run per RHS, and one host
// synchronisation per step serves the whole batch.
dw_status solve_batch(dw_field f, double m0, const fgmresdr_params* P, const double* b_can, double* x_can, int nr,
                      Work& W, dw_solve_stats* st, hipStream_t s) {
  const Geom& g = f->g;
  const long long n = g.V * 12;
  const int m = P->m, k = P->k;
  const int prec = P->sap.storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;  // SAP accumulator
  const double sigma = prec == DW_PREC_F64 ? 1.0 : sqrt((double)n);
  const double bd_tol = 1e-14;
  auto t0 = std::chrono::steady_clock::now();
  std::vector<Rhs> R(nr);
  bool donor_ok = false;
  // captured steps: single-RHS batches on a stream that can be captured,
  // without per-launch event timing
  const bool use_graphs = (P->flags & DW_SOLVE_GRAPHS) && nr == 1 && s != nullptr && !f->ctx->prof.on;  // RHS 0 holds a deflation space from a deflated restart

  DW_TRY(launch_pack_spinor(g, DW_PREC_F64, b_can, W.b.p, 1.0, nr, s));
  DW_CHECK_HIP(hipMemsetAsync(W.x.p, 0, (size_t)nr * n * 16, s));
  for (int r = 0; r < nr; ++r)
    DW_TRY(blas_dots(DW_PREC_F64, W.vec(W.b, r), n, 1, W.vec(W.b, r), n, W.partr(r), W.nrmr(r), 1, 0, s));
  DW_CHECK_HIP(hipMemcpyAsync(W.r.p, W.b.p, (size_t)nr * n * 16, hipMemcpyDeviceToDevice, s));
  DW_TRY(readback(W, s));
  for (int r = 0; r < nr; ++r) {
    R[r].bnorm = sqrt(W.sh(r)[kSclCount]);
    R[r].res_e = R[r].res_i = R[r].bnorm;
    if (R[r].bnorm == 0.0) {
      R[r].done = R[r].converged = true;
    }
  }

  std::vector<int> part;
  while (true) {
    // ---- cycle start
    std::vector<int> cyc;
    for (int r = 0; r < nr; ++r) {
      Rhs& q = R[r];
      if (q.done) continue;
      cyc.push_back(r);
      if (q.fresh) {
        // W.nrm(r) holds ||r||^2 of the current explicit residual
        DW_TRY(dense_fresh(W.Hr(r), W.cr(r), W.nrmr(r), W.scalr(r), s));
        if (W.vprec == DW_PREC_F64)
          DW_TRY(blas_scale(W.vec(W.r, r), (double*)W.Vr(r), W.scalr(r) + kSclBetaInv, n, s));
        else
          DW_TRY(launch_convert(DW_PREC_F64, W.vec(W.r, r), W.vprec, W.Vr(r), 1.0, n, s, W.scalr(r) + kSclBetaInv));
        q.j0 = 0;
      } else {
        q.j0 = k;
      }
      q.jend = q.j0;
      q.lagged = q.broke = q.frozen = false;
    }
    if (cyc.empty()) break;
    int jmin = m;
    for (int r : cyc) jmin = std::min(jmin, R[r].j0);

    // ---- lock-step Arnoldi steps
    for (int j = jmin; j < m; ++j) {
      part.clear();
      for (int r : cyc)
        if (!R[r].frozen && R[r].j0 <= j) part.push_back(r);
      if (part.empty()) break;
      DW_TRY(set_rlist(W, part, s));
      const int np = (int)part.size();
      auto enqueue_step = [&]() -> dw_status {
        // z_j = M_j applied to sigma * v_j (lagged vectors scaled by their
        // provisional norm; any z_j keeps A Z = V H^ exact in FGMRES)
        for (int r : part)
          DW_TRY(launch_convert(W.vprec, W.Vc(r, j), prec,
                                (char*)W.vs.p + (size_t)r * n * pair_bytes(prec), sigma, n, s,
                                R[r].lagged ? W.scalr(r) + kSclHinv : nullptr));
        void* zacc = zprec == DW_PREC_F64 ? (void*)(W.Z.as<double>() + 2 * (long long)j * n) : W.zs.p;
        const long long zstride = zprec == DW_PREC_F64 ? (long long)m * n : n;
        for (int cy = 0; cy < P->sap.ncycles; ++cy)
          for (int colour = 0; colour < 2; ++colour)
            DW_TRY(launch_sap_colour(g, m0, prec, W.vs.p, zacc, f->U[prec], colour, P->sap.nmr,
                                     cy == 0 && colour == 0 ? 1 : 0, np, n, zstride, s, W.rlist.as<int>(),
                                     f->C[prec], P->sap.mr_reduction));
        if (zprec != DW_PREC_F64)
          for (int r : part)
            DW_TRY(launch_convert(zprec, (char*)W.zs.p + (size_t)r * n * pair_bytes(zprec), DW_PREC_F64,
                                  W.Zr(r) + 2 * (long long)j * n, 1.0 / sigma, n, s));
        // w = D z_j in FP64 on the stored z_j, all participants in one launch
        DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, W.Z.as<double>() + 2 * (long long)j * n, 1.0,
                                   f->U[DW_PREC_F64], W.w.as<double>(), nullptr, 0, np, (long long)m * n, n, s,
                                   W.rlist.as<int>(), f->C[DW_PREC_F64]));
        // Gram-Schmidt with delayed reorthogonalisation, per RHS
        for (int r : part) {
          Rhs& q = R[r];
          void* V = W.Vr(r);
          const int nv = q.lagged ? j : j + 1;
          DW_TRY(gs_reduce(W.vprec, V, n, nv, q.lagged ? W.Vc(r, j) : nullptr, W.vec(W.w, r), n, W.partr(r),
                           W.redr(r), s));
          DW_TRY(dense_gs_coef(W.Hr(r), nv, q.lagged ? j : -1, j, q.lagged ? 1 : 0, 1, W.redr(r), W.coefr(r),
                               W.scalr(r), bd_tol, s));
          DW_TRY(gs_update(W.vprec, V, n, nv, q.lagged ? j : -1, W.vec(W.w, r), W.Vc(r, j + 1), W.coefr(r), n,
                           W.partr(r), W.nrmr(r), s));
          DW_TRY(dense_step2(W.Hr(r), j, W.nrmr(r), W.cr(r), W.scalr(r), bd_tol, s));
        }
        return DW_OK;
      };
      if (use_graphs) {
        // one HIP graph per (j, lagged): the step's launches are identical
        // in every cycle, so each is captured once and replayed
        const size_t key = 2 * (size_t)j + (R[part[0]].lagged ? 1 : 0);
        if (W.graphs.size() <= key) W.graphs.resize(key + 1, nullptr);
        if (!W.graphs[key]) {
          hipGraph_t gr = nullptr;
          DW_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          const dw_status es = enqueue_step();
          const hipError_t ce = hipStreamEndCapture(s, &gr);
          if (es != DW_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return es;
          }
          DW_CHECK_HIP(ce);
          const hipError_t ie = hipGraphInstantiate(&W.graphs[key], gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          DW_CHECK_HIP(ie);
        }
        DW_CHECK_HIP(hipGraphLaunch(W.graphs[key], s));
      } else {
        DW_TRY(enqueue_step());
      }
      DW_TRY(readback(W, s));
      for (int r : part) {
        Rhs& q = R[r];
        q.lagged = true;
        ++q.iters;
        q.jend = j + 1;
        q.res_i = W.sh(r)[kSclResImp];
        q.broke = W.sh(r)[kSclBreak] != 0.0;
        if (q.broke || q.res_i <= P->tol * q.bnorm || q.iters >= P->max_iter) q.frozen = true;
      }
    }

    // ---- cycle end: finalise the last lagged vector (second GS pass), then
    // iterate and explicit FP64 residual
    for (int r : cyc) {
      Rhs& q = R[r];
      void* V = W.Vr(r);
      if (q.lagged && !q.broke) {
        DW_TRY(gs_reduce(W.vprec, V, n, q.jend, W.Vc(r, q.jend), nullptr, n, W.partr(r), W.redr(r), s));
        DW_TRY(dense_gs_coef(W.Hr(r), q.jend, q.jend, -1, 1, 0, W.redr(r), W.coefr(r), W.scalr(r), bd_tol, s));
        DW_TRY(gs_update(W.vprec, V, n, q.jend, q.jend, nullptr, nullptr, W.coefr(r), n, W.partr(r), nullptr, s));
      }
      DW_TRY(dense_lsq(W.Hr(r), q.jend, W.cr(r), W.etar(r), W.scalr(r), s));
      DW_TRY(blas_combine(DW_PREC_F64, W.Zr(r), n, q.jend, W.etar(r), 1.0, W.vec(W.x, r), n, s));
    }
    DW_TRY(set_rlist(W, cyc, s));
    DW_TRY(launch_dslash_outer(g, m0, DW_PREC_F64, W.x.p, 1.0, f->U[DW_PREC_F64], W.r.as<double>(), W.b.as<double>(),
                               1, (int)cyc.size(), n, n, s, W.rlist.as<int>(), f->C[DW_PREC_F64]));
    // shared deflation space (multi-RHS): once RHS 0 has a deflation space,
    // every other RHS projects its restart residual onto it. The space
    // satisfies D Z_0 = V_0 H_0 (the k+1 leading columns of V_0, k of Z_0 and
    // the (k+1) x k block H_0 kept from RHS 0's last deflated restart), so
    // y = argmin ||V_0^H r - H_0 y|| minimises ||r - D Z_0 y||; then
    // x += Z_0 y, r -= V_0 H_0 y, and that RHS restarts from the projected
    // residual with a fresh Krylov space (the projected residual is no
    // longer in the span of its own deflation basis).
    std::vector<char> projected(nr, 0);
    if (P->shared_defl && nr > 1 && k > 0 && donor_ok) {
      for (int r : cyc) {
        if (r == 0) continue;
        projected[r] = 1;
        double* pr = W.projr(r);
        double* t = pr;
        double* y = pr + 2 * kLd;
        double* sv = y + 2 * kMaxM;
        DW_TRY(blas_dots(W.vprec, W.Vr(0), n, k + 1, W.vec(W.r, r), n, W.partr(r), t, 1, 0, s));
        DW_TRY(dense_project(W.Hr(0), k, t, y, sv, s));
        DW_TRY(blas_combine(DW_PREC_F64, W.Zr(0), n, k, y, 1.0, W.vec(W.x, r), n, s));
        DW_TRY(blas_combine(W.vprec, W.Vr(0), n, k + 1, sv, -1.0, W.vec(W.r, r), n, s));
      }
    }
    for (int r : cyc)
      DW_TRY(blas_dots(DW_PREC_F64, W.vec(W.r, r), n, 1, W.vec(W.r, r), n, W.partr(r), W.nrmr(r), 1, 0, s));
    DW_TRY(readback(W, s));
    std::vector<int> defl;
    for (int r : cyc) {
      Rhs& q = R[r];
      q.res_i = W.sh(r)[kSclResImp];
      q.res_e = sqrt(W.sh(r)[kSclCount]);
      ++q.cycles;
      q.fresh = true;
      if (q.res_e <= P->tol * q.bnorm) {
        q.done = q.converged = true;
      } else if (q.iters >= P->max_iter) {
        q.done = true;
      } else if (k == 0 || projected[r]) {
        // plain restarted FGMRES(m), or a restart from a projected residual
      } else if (q.broke || q.jend <= k || q.res_e > P->restart_t * fmax(q.res_i, 1e-300)) {
        ++q.clean;  // clean restart (Section 4.7)
        if (r == 0) donor_ok = false;
      } else {
        defl.push_back(r);
      }
    }
    const bool inject = (P->flags & DW_SOLVE_INJECT) != 0;
    if (!defl.empty()) {
      for (int r : defl) {
        if (inject) {
          // G_{k+1}'s last column from the explicit residual: V_{m+1}^H r with
          // eta = 0 (the kernel forms c - H^ eta)
          DW_TRY(blas_dots(W.vprec, W.Vr(r), n, R[r].jend + 1, W.vec(W.r, r), n, W.partr(r), W.injr(r), 1, 0, s));
          DW_TRY(dense_deflate(W.Hr(r), R[r].jend, k, W.injr(r), W.zeta.as<double>(), W.Qr(r), W.ritzr(r),
                               W.scalr(r), s));
        } else {
          DW_TRY(dense_deflate(W.Hr(r), R[r].jend, k, W.cr(r), W.etar(r), W.Qr(r), W.ritzr(r), W.scalr(r), s));
        }
      }
      DW_TRY(readback(W, s));
      std::vector<int> rot;
      for (int r : defl) {
        Rhs& q = R[r];
        if (W.sh(r)[kSclStatus] != 0.0) {
          ++q.clean;
          if (r == 0) donor_ok = false;
          continue;
        }
        if (r == 0) donor_ok = true;
        DW_TRY(blas_rotate(W.vprec, W.Vr(r), n, q.jend + 1, W.Qr(r), kLd, k + 1, n, s));
        DW_TRY(blas_rotate(DW_PREC_F64, W.Zr(r), n, q.jend, W.Qr(r), kLd, k, n, s));
        rot.push_back(r);
      }
      if (inject && !rot.empty()) {
        std::vector<double> rnorm;
        for (int r : rot) rnorm.push_back(R[r].res_e);
        DW_TRY(inject_residual(W, rot, rnorm, k, s));
      }
      for (int r : rot) {
        Rhs& q = R[r];
        DW_CHECK_HIP(hipMemsetAsync(W.cr(r), 0, (size_t)kLd * 16, s));
        DW_TRY(blas_dots(W.vprec, W.Vr(r), n, k + 1, W.vec(W.r, r), n, W.partr(r), W.cr(r), 1, 0, s));
        q.fresh = false;
      }
    }
  }
  DW_TRY(launch_unpack_spinor(g, DW_PREC_F64, W.x.p, x_can, 1.0, nr, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int r = 0; r < nr; ++r) {
    const Rhs& q = R[r];
    dw_solve_stats& o = st[r];
    memset(&o, 0, sizeof o);
    o.converged = q.converged ? 1 : 0;
    o.iterations = q.iters;
    o.cycles = q.cycles;
    o.clean_restarts = q.clean;
    o.true_relres = q.bnorm > 0 ? q.res_e / q.bnorm : 0.0;
    o.implicit_relres = q.bnorm > 0 ? q.res_i / q.bnorm : 0.0;
    o.seconds = secs;
  }
  return DW_OK;
}

}  // namespace

namespace dw {
size_t solver_bytes(long long sites, int m, int prec, int flags, int nrhs) {
  const int vprec = (flags & DW_SOLVE_V32) ? DW_PREC_F32 : DW_PREC_F64;
  return bytes_per_rhs(sites * 12, m, prec, vprec) * (size_t)nrhs + (size_t)nrhs * 64 * 1024;
}
}  // namespace dw

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
  if (P->flags & ~(DW_SOLVE_GRAPHS | DW_SOLVE_V32 | DW_SOLVE_INJECT)) {
    set_error("fgmresdr_solve: unknown flags 0x%x", (unsigned)P->flags);
    return DW_EINVAL;
  }
  if (P->shared_defl != 0 && P->shared_defl != 1) {
    set_error("fgmresdr_solve: shared_defl must be 0 or 1");
    return DW_EINVAL;
  }
  if (P->sap.ncycles < 1) {
    set_error("fgmresdr_solve: need at least one SAP cycle");
    return DW_EINVAL;
  }
  if (nrhs == 0) return DW_OK;
  int cur = -1;
  DW_CHECK_HIP(hipGetDevice(&cur));
  if (cur != f->ctx->device) DW_CHECK_HIP(hipSetDevice(f->ctx->device));
  ProfScope ps(f->ctx);
  const long long n = f->g.V * 12;
  // RHS per batch: as many as fit in free device memory (at least one)
  size_t free_b = 0, total_b = 0;
  DW_CHECK_HIP(hipMemGetInfo(&free_b, &total_b));
  const size_t per = bytes_per_rhs(n, P->m, P->sap.storage, basis_prec(P));
  int nb = (int)std::max<size_t>(1, (size_t)(0.9 * (double)free_b) / per);
  nb = std::min(nb, (int)nrhs);
  bool all_conv = true;
  std::vector<dw_solve_stats> st(nrhs);
  for (int r0 = 0; r0 < nrhs; r0 += nb) {
    const int nr = std::min(nb, nrhs - r0);
    Work W;
    DW_TRY(alloc_work(f, P, nr, W, stream));
    DW_TRY(solve_batch(f, m0, P, b + 2 * (long long)r0 * n, x + 2 * (long long)r0 * n, nr, W, st.data() + r0, stream));
  }
  for (int r = 0; r < nrhs; ++r) {
    if (stats) stats[r] = st[r];
    all_conv = all_conv && st[r].converged;
  }
  if (!all_conv) {
    set_error("fgmresdr_solve: max_iter reached before the tolerance");
    return DW_ENOTCONV;
  }
  return DW_OK;
}
