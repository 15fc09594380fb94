// FGMRES-DR driver (paper Section 4, Alg. 3 and Alg. 4, Section 4.7).
//
// The host enqueues kernels on the caller's stream; all vector work, every
// small dense problem and every decision of the cycle run on the GPU. Each
// right-hand side carries a control record on the device (dw_control.hpp):
// the step that reaches the tolerance (implicit residual), breaks down or
// exhausts the iteration budget stops the cycle for that right-hand side,
// and the remaining kernels of the cycle find their gate closed and return.
// At the cycle end the explicit FP64 residual decides on the device between
// stop, clean restart and deflated restart. The host reads the control
// records once per cycle, to learn which right-hand sides go on and how.
// A whole cycle (its Arnoldi steps, the cycle end and the restart) is
// therefore a fixed sequence of launches, which DW_SOLVE_GRAPHS captures as
// one HIP graph per cycle shape and replays.
//
// Per Arnoldi step j (flexible, Alg. 3):
//   z_j = M_j v_j   SAP at storage precision on sigma * v_j (sigma = sqrt(n)
//                   gives unit RMS entries; M is scale-equivariant) with an
//                   FP32 accumulator (FP64 for FP64 storage); the result is
//                   kept in Z at FP64, which holds it exactly, so that the
//                   rotated deflation basis Z_k = Z Q_k keeps A Z = V H^ to
//                   FP64 accuracy;
//   w = D z_j       FP64 operator on the stored z_j, so A Z = V H^ holds to
//                   FP64 accuracy whatever precision Z has;
//   classical Gram-Schmidt with one reorthogonalisation, delayed by one
//                   step: the sweep that projects w (first pass) also
//                   reorthogonalises the previous step's vector (second
//                   pass), so V is read twice per step instead of four
//                   times; all Gram-Schmidt variants give the same H^ up to
//                   rounding;
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
#include <memory>
#include <vector>

#include "dw_control.hpp"
#include "dw_internal.hpp"
#include "dw_kernels.hpp"

namespace dw {
dw_status check_sap_params(const Geom& g, const sap_params* sp);
}

using namespace dw;

namespace {

constexpr double kBdTol = 1e-14;  // breakdown: h_{j+1,j} <= kBdTol ||H^||
constexpr int kMaxBatch = 64;     // right-hand sides of one lock-step batch

unsigned long long rhs_mask(const std::vector<int>& rs) {
  unsigned long long m = 0;
  for (int r : rs) m |= 1ull << r;
  return m;
}

// One cycle shape: which right-hand sides take part and from which column
// (state 0: stopped, 1: fresh start at column 0, 2: deflated start at k),
// and whether the shared-deflation projection runs. Its launch lists live
// on the device for as long as its captured graph may be replayed.
struct Shape {
  std::vector<signed char> st;
  bool donor = false;
  DevBuf rl;  // (m + 1) x nr: row j lists the right-hand sides of step j, row m those of the cycle end
  hipGraphExec_t exec = nullptr;
  ~Shape() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// Device and host state of a batch of right-hand sides solved in lock-step.
struct Work {
  int nr = 0, m = 0, k = 0;
  long long n = 0;
  DevBuf V, Z, zs, w, r, x, b, vs, partials, H, c, eta, red, coef, nrm, Q, ritz, scal, proj, inj, zeta, ctl, ctld, mass;
  int* ctl_h = nullptr;
  double* ctld_h = nullptr;
  std::vector<std::unique_ptr<Shape>> shapes;
  // parameters the buffers and captured graphs were made for
  fgmresdr_params P{};
  const void* clover[2] = {};  // the field's clover terms the captured graphs read
  ~Work() {
    shapes.clear();
    if (ctl_h) (void)hipHostFree(ctl_h);
    if (ctld_h) (void)hipHostFree(ctld_h);
  }
  int vprec = DW_PREC_F64;  // storage of the Krylov basis V
  int zstore = DW_PREC_F64; // storage of the preconditioned basis Z
  bool a32 = false;         // single-precision Arnoldi (w = D z and Gram-Schmidt in FP32)
  // basis of RHS r, and its column j
  void* Vr(int r) const { return (char*)V.p + (size_t)r * (m + 1) * n * pair_bytes(vprec); }
  void* Vc(int r, int j) const { return (char*)Vr(r) + (size_t)j * n * pair_bytes(vprec); }
  void* Zr(int r) const { return (char*)Z.p + (size_t)r * m * n * pair_bytes(zstore); }
  void* Zc(int r, int j) const { return (char*)Zr(r) + (size_t)j * n * pair_bytes(zstore); }
  // w of RHS r at the Arnoldi's precision (the buffer holds FP64 pairs)
  void* wr(int r) const { return (char*)w.p + (size_t)r * n * (a32 ? 8 : 16); }
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
  int* ctlr(int r) const { return ctl.as<int>() + (long long)r * kCtl; }
  double* ctldr(int r) const { return ctld.as<double>() + (long long)r * kCtlD; }
  const int* gate(int r, int field) const { return ctlr(r) + field; }
  const int* hctl(int r) const { return ctl_h + (long long)r * kCtl; }
  const double* hctld(int r) const { return ctld_h + (long long)r * kCtlD; }
  // shared-deflation projection: t = V_0^H r (kLd pairs), y (kMaxM), s = H_0 y (kLd)
  double* projr(int r) const { return proj.as<double>() + 2 * (long long)r * (2 * kLd + kMaxM); }
  // residual injection: G column V^H r (kLd pairs), t = V_k^H w (kLd), then
  // 4 pairs: [v_{k+1}^H w, ||w||^2], coefficient
  double* injr(int r) const { return inj.as<double>() + 2 * (long long)r * (2 * kLd + 4); }
};

int basis_prec(const fgmresdr_params* P) {
  return (P->flags & (DW_SOLVE_V32 | DW_SOLVE_A32)) ? DW_PREC_F32 : DW_PREC_F64;
}
int zstore_prec(const fgmresdr_params* P) { return (P->flags & DW_SOLVE_A32) ? DW_PREC_F32 : DW_PREC_F64; }

// the SAP accumulator goes straight into Z when they share the precision
bool sap_into_z(int prec, int zstore) { return (prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32) == zstore; }

size_t bytes_per_rhs(long long n, int m, int prec, int vprec, int zstore) {
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  return (size_t)n * pair_bytes(vprec) * (m + 1) + (size_t)n * pair_bytes(zstore) * m + (size_t)n * 16 * 4 +
         (size_t)n * pair_bytes(prec) + (sap_into_z(prec, zstore) ? 0 : (size_t)n * pair_bytes(zprec)) +
         (size_t)(2 * kLd + 6) * kBlasGrid * 16;
}

dw_status alloc_work(dw_field f, const fgmresdr_params* P, int nr, Work& W, hipStream_t s) {
  const long long n = f->g.V * 12;
  const int prec = P->sap.storage;
  const int zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
  dw_ctx ctx = f->ctx;
  W.nr = nr;
  W.m = P->m;
  W.k = P->k;
  W.n = n;
  W.P = *P;
  W.clover[0] = f->C[prec];
  W.clover[1] = f->C[DW_PREC_F64];
  W.vprec = basis_prec(P);
  W.zstore = zstore_prec(P);
  W.a32 = (P->flags & DW_SOLVE_A32) != 0;
  DW_TRY(W.V.alloc(ctx, (size_t)nr * (P->m + 1) * n * pair_bytes(W.vprec), s));
  DW_TRY(W.Z.alloc(ctx, (size_t)nr * P->m * n * pair_bytes(W.zstore), s));
  if (!sap_into_z(prec, W.zstore)) DW_TRY(W.zs.alloc(ctx, (size_t)nr * n * pair_bytes(zprec), s));
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
  DW_TRY(W.ctl.alloc(ctx, (size_t)nr * kCtl * sizeof(int), s));
  DW_TRY(W.ctld.alloc(ctx, (size_t)nr * kCtlD * sizeof(double), s));
  DW_TRY(W.mass.alloc(ctx, 16, s));
  if (P->shared_defl && nr > 1) DW_TRY(W.proj.alloc(ctx, (size_t)nr * (2 * kLd + kMaxM) * 16, s));
  if (P->flags & DW_SOLVE_INJECT) {
    DW_TRY(W.inj.alloc(ctx, (size_t)nr * (2 * kLd + 4) * 16, s));
    DW_TRY(W.zeta.alloc(ctx, (size_t)kMaxM * 16, s));
  }
  DW_CHECK_HIP(hipHostMalloc((void**)&W.ctl_h, (size_t)nr * kCtl * sizeof(int), hipHostMallocDefault));
  DW_CHECK_HIP(hipHostMalloc((void**)&W.ctld_h, (size_t)nr * kCtlD * sizeof(double), hipHostMallocDefault));
  return DW_OK;
}

// reads every right-hand side's control record (the one synchronisation of a cycle)
dw_status readback(Work& W, hipStream_t s) {
  DW_CHECK_HIP(hipMemcpyAsync(W.ctl_h, W.ctl.p, (size_t)W.nr * kCtl * sizeof(int), hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipMemcpyAsync(W.ctld_h, W.ctld.p, (size_t)W.nr * kCtlD * sizeof(double), hipMemcpyDeviceToHost, s));
  DW_CHECK_HIP(hipStreamSynchronize(s));
  prof_flush();
  return DW_OK;
}

struct Solver {
  dw_field f;
  const fgmresdr_params* P;
  Work& W;
  hipStream_t s;
  int prec, zprec;
  double sigma;

  Solver(dw_field f_, const fgmresdr_params* P_, Work& W_, hipStream_t s_) : f(f_), P(P_), W(W_), s(s_) {
    prec = P->sap.storage;
    zprec = prec == DW_PREC_F64 ? DW_PREC_F64 : DW_PREC_F32;
    sigma = prec == DW_PREC_F64 ? 1.0 : sqrt((double)W.n);
  }

  // Restart preparation for every right-hand side in `rs` whose record asks
  // for a fresh start: H^ = 0, c = beta e_1, v_1 = r / beta. Then the
  // records open the next cycle.
  dw_status fresh_and_open(const std::vector<int>& rs, bool in_cycle = true) {
    const long long n = W.n;
    for (int r : rs) {
      const int* g = W.gate(r, kCFresh);
      ProfTag tag_f(in_cycle ? kTagFresh : kTagNone, 1ull << r);
      DW_TRY(dense_fresh(W.Hr(r), W.cr(r), W.nrmr(r), W.scalr(r), s, g));
      if (W.vprec == DW_PREC_F64)
        DW_TRY(blas_scale(W.vec(W.r, r), (double*)W.Vr(r), W.scalr(r) + kSclBetaInv, n, s, g));
      else
        DW_TRY(launch_convert(DW_PREC_F64, W.vec(W.r, r), W.vprec, W.Vr(r), 1.0, n, s, W.scalr(r) + kSclBetaInv, g));
    }
    return ctl_next(W.ctl.as<int>(), W.nr, W.m, W.k, s);
  }

  // b, x = 0, r = b, ||b||, the control records and the first cycle's start
  dw_status start(const double* b_can, double m0) {
    const Geom& g = f->g;
    const long long n = W.n;
    const int nr = W.nr;
    DW_TRY(set_double(W.mass.as<double>(), m0, s));
    DW_TRY(launch_pack_spinor(g, DW_PREC_F64, b_can, W.b.p, 1.0, nr, s));
    DW_TRY(fill_zero(W.x.as<double>(), 2 * (long long)nr * n, nullptr, s));
    std::vector<int> all(nr);
    for (int r = 0; r < nr; ++r) {
      all[r] = r;
      DW_TRY(blas_dots(DW_PREC_F64, W.vec(W.b, r), n, 1, W.vec(W.b, r), n, W.partr(r), W.nrmr(r), 1, 0, s));
    }
    DW_TRY(copy_doubles(W.b.as<double>(), W.r.as<double>(), 2 * (long long)nr * n, nullptr, s));
    DW_TRY(ctl_init(W.ctl.as<int>(), W.ctld.as<double>(), W.nrm.as<double>(), 2, nr, P->tol, P->restart_t,
                    P->max_iter, s));
    return fresh_and_open(all, false);
  }

  dw_status upload_lists(Shape& sh) {
    const int m = W.m, nr = W.nr;
    std::vector<int> tab((size_t)(m + 1) * nr, 0);
    for (int j = 0; j <= m; ++j) {
      int q = 0;
      for (int r = 0; r < nr; ++r) {
        const int st = sh.st[r];
        if (st == 0) continue;
        const int j0 = st == 2 ? W.k : 0;
        if (j == m || j0 <= j) tab[(size_t)j * nr + q++] = r;
      }
    }
    DW_TRY(sh.rl.alloc(f->ctx, tab.size() * sizeof(int), s));
    DW_CHECK_HIP(hipMemcpyAsync(sh.rl.p, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, s));
    DW_CHECK_HIP(hipStreamSynchronize(s));
    return DW_OK;
  }

  // One cycle of the given shape: Arnoldi steps, cycle end, restart.
  dw_status enqueue_cycle(const Shape& sh) {
    const Geom& g = f->g;
    const long long n = W.n;
    const int m = W.m, k = W.k, nr = W.nr;
    const bool inject = (P->flags & DW_SOLVE_INJECT) != 0;
    const int wprec = W.a32 ? DW_PREC_F32 : DW_PREC_F64;
    const double* mass = W.mass.as<double>();
    const int* gate_live = W.ctl.as<int>() + kCLive;
    const int* gate_cyc = W.ctl.as<int>() + kCInCycle;
    std::vector<int> present;
    int jstart = m;
    for (int r = 0; r < nr; ++r)
      if (sh.st[r]) {
        present.push_back(r);
        jstart = std::min(jstart, sh.st[r] == 2 ? k : 0);
      }
    auto j0_of = [&](int r) { return sh.st[r] == 2 ? k : 0; };

    // ---- Arnoldi steps
    for (int j = jstart; j < m; ++j) {
      std::vector<int> part;
      for (int r : present)
        if (j0_of(r) <= j) part.push_back(r);
      const int np = (int)part.size();
      const int* rl = sh.rl.as<int>() + (size_t)j * nr;
      ProfTag tag_step(j, rhs_mask(part));
      // z_j = M_j applied to sigma * v_j (lagged vectors scaled by their
      // provisional norm; any z_j keeps A Z = V H^ exact in FGMRES)
      for (int r : part) {
        ProfTag tag_rhs(j, 1ull << r);
        DW_TRY(launch_convert(W.vprec, W.Vc(r, j), prec, (char*)W.vs.p + (size_t)r * n * pair_bytes(prec), sigma, n,
                              s, j > j0_of(r) ? W.scalr(r) + kSclHinv : nullptr, W.gate(r, kCLive)));
      }
      // the accumulator is column j of Z itself when they share the
      // precision; with the low-precision SAP into an FP32 Z the column is
      // sigma M v_j, a scaled flexible preconditioner (A Z = V H^ holds for
      // the stored Z, and x = x0 + Z eta is unchanged)
      const bool direct = sap_into_z(prec, W.zstore);
      void* zacc = direct ? W.Zc(0, j) : W.zs.p;
      const long long zstride = direct ? (long long)m * n : n;
      for (int cy = 0; cy < P->sap.ncycles; ++cy)
        for (int colour = 0; colour < 2; ++colour)
          DW_TRY(launch_sap_colour(g, 0.0, prec, W.vs.p, zacc, f->U[prec], colour, P->sap.nmr,
                                   cy == 0 && colour == 0 ? 1 : 0, np, n, zstride, s, rl, f->C[prec],
                                   P->sap.mr_reduction, gate_live, kCtl, mass));
      if (!direct)
        for (int r : part) {
          ProfTag tag_rhs(j, 1ull << r);
          DW_TRY(launch_convert(zprec, (char*)W.zs.p + (size_t)r * n * pair_bytes(zprec), W.zstore, W.Zc(r, j),
                                1.0 / sigma, n, s, nullptr, W.gate(r, kCLive)));
        }
      // w = D z_j on the stored z_j, all participants in one launch: FP64,
      // so that A Z = V H^ holds to FP64 accuracy whatever precision Z has,
      // or FP32 (links, arithmetic and w) in the single-precision Arnoldi
      if (W.a32)
        DW_TRY(launch_dslash_a32(g, W.Zc(0, j), f->U[DW_PREC_F32], W.w.p, np, (long long)m * n, n, s, rl,
                                 f->C[DW_PREC_F32], gate_live, kCtl, mass));
      else
        DW_TRY(launch_dslash_outer(g, 0.0, DW_PREC_F64, W.Zc(0, j), 1.0, f->U[DW_PREC_F64], W.w.as<double>(),
                                   nullptr, 0, np, (long long)m * n, n, s, rl, f->C[DW_PREC_F64], gate_live, kCtl,
                                   mass));
      // Gram-Schmidt with delayed reorthogonalisation, per right-hand side
      for (int r : part) {
        ProfTag tag_rhs(j, 1ull << r);
        const bool lagged = j > j0_of(r);
        const int* gl = W.gate(r, kCLive);
        void* V = W.Vr(r);
        const int nv = lagged ? j : j + 1;
        DW_TRY(gs_reduce(W.vprec, V, n, nv, lagged ? W.Vc(r, j) : nullptr, W.wr(r), n, W.partr(r), W.redr(r), s,
                         gl, nullptr, wprec));
        DW_TRY(dense_gs_coef(W.Hr(r), nv, lagged ? j : -1, j, lagged ? 1 : 0, 1, W.redr(r), W.coefr(r), W.scalr(r),
                             kBdTol, s, gl));
        DW_TRY(gs_update(W.vprec, V, n, nv, lagged ? j : -1, W.wr(r), W.Vc(r, j + 1), W.coefr(r), n, W.partr(r),
                         W.nrmr(r), s, gl, nullptr, wprec));
        DW_TRY(dense_step2(W.Hr(r), j, W.nrmr(r), W.cr(r), W.scalr(r), kBdTol, s, W.ctlr(r), W.ctldr(r)));
      }
    }

    // ---- cycle end: finalise the last vector (second Gram-Schmidt pass),
    // then the iterate and the explicit FP64 residual
    DW_TRY(ctl_cycle_end(W.ctl.as<int>(), nr, s));
    for (int r : present) {
      const int* jend = W.gate(r, kCJend);
      const int* gfin = W.gate(r, kCFin);
      const int* gcyc = W.gate(r, kCInCycle);
      void* V = W.Vr(r);
      ProfTag tag_fin(kTagFin, 1ull << r);
      DW_TRY(gs_reduce(W.vprec, V, n, m, nullptr, nullptr, n, W.partr(r), W.redr(r), s, gfin, jend, wprec));
      DW_TRY(dense_gs_coef(W.Hr(r), m, m, -1, 1, 0, W.redr(r), W.coefr(r), W.scalr(r), kBdTol, s, gfin, jend));
      DW_TRY(gs_update(W.vprec, V, n, m, m, nullptr, nullptr, W.coefr(r), n, W.partr(r), nullptr, s, gfin, jend,
                       wprec));
      ProfTag tag_cyc(kTagCycle, 1ull << r);
      DW_TRY(dense_lsq(W.Hr(r), m, W.cr(r), W.etar(r), W.scalr(r), s, gcyc, jend));
      DW_TRY(blas_combine(W.zstore, W.Zr(r), n, m, W.etar(r), 1.0, W.vec(W.x, r), n, s, gcyc, jend));
    }
    const int* rl_end = sh.rl.as<int>() + (size_t)m * nr;
    ProfTag tag_end(kTagCycle, rhs_mask(present));
    DW_TRY(launch_dslash_outer(g, 0.0, DW_PREC_F64, W.x.p, 1.0, f->U[DW_PREC_F64], W.r.as<double>(),
                               W.b.as<double>(), 1, (int)present.size(), n, n, s, rl_end, f->C[DW_PREC_F64],
                               gate_cyc, kCtl, mass));
    // shared deflation space (multi-RHS): once RHS 0 has a deflation space,
    // every other RHS projects its restart residual onto it. The space
    // satisfies D Z_0 = V_0 H_0 (the k+1 leading columns of V_0, k of Z_0 and
    // the (k+1) x k block H_0 kept from RHS 0's last deflated restart), so
    // y = argmin ||V_0^H r - H_0 y|| minimises ||r - D Z_0 y||; then
    // x += Z_0 y, r -= V_0 H_0 y, and that RHS restarts from the projected
    // residual with a fresh Krylov space (the projected residual is no
    // longer in the span of its own deflation basis).
    unsigned long long projected = 0;
    if (sh.donor) {
      for (int r : present) {
        if (r == 0) continue;
        ProfTag tag_p(kTagCycle, 1ull << r);
        projected |= 1ull << r;
        const int* gcyc = W.gate(r, kCInCycle);
        double* pr = W.projr(r);
        double* t = pr;
        double* y = pr + 2 * kLd;
        double* sv = y + 2 * kMaxM;
        DW_TRY(blas_dots(W.vprec, W.Vr(0), n, k + 1, W.vec(W.r, r), n, W.partr(r), t, 1, 0, s, gcyc));
        DW_TRY(dense_project(W.Hr(0), k, t, y, sv, s, gcyc));
        DW_TRY(blas_combine(W.zstore, W.Zr(0), n, k, y, 1.0, W.vec(W.x, r), n, s, gcyc));
        DW_TRY(blas_combine(W.vprec, W.Vr(0), n, k + 1, sv, -1.0, W.vec(W.r, r), n, s, gcyc));
      }
    }
    for (int r : present) {
      ProfTag tag_n(kTagCycle, 1ull << r);
      DW_TRY(blas_dots(DW_PREC_F64, W.vec(W.r, r), n, 1, W.vec(W.r, r), n, W.partr(r), W.nrmr(r), 1, 0, s,
                       W.gate(r, kCInCycle)));
    }
    DW_TRY(ctl_decide(W.ctl.as<int>(), W.ctld.as<double>(), W.nrm.as<double>(), 2, W.scal.as<double>(), kSclCount,
                      nr, k, projected, s));

    // ---- deflated restart (Lemma 1, Section 4.4) where decided
    if (k > 0) {
      for (int r : present) {
        const int* gd = W.gate(r, kCDefl);
        const int* jend = W.gate(r, kCJend);
        ProfTag tag_d(kTagDefl, 1ull << r);
        if (inject) {
          // G_{k+1}'s last column from the explicit residual: V_{m+1}^H r with
          // eta = 0 (the kernel forms c - H^ eta)
          DW_TRY(fill_zero(W.injr(r), 2 * (long long)kLd, gd, s));
          DW_TRY(blas_dots(W.vprec, W.Vr(r), n, m + 1, W.vec(W.r, r), n, W.partr(r), W.injr(r), 1, 0, s, gd, jend,
                           1));
          DW_TRY(fill_zero(W.zeta.as<double>(), 2 * (long long)kMaxM, gd, s));
          DW_TRY(dense_deflate(W.Hr(r), m, k, W.injr(r), W.zeta.as<double>(), W.Qr(r), W.ritzr(r), W.scalr(r), s, gd,
                               jend));
        } else {
          DW_TRY(dense_deflate(W.Hr(r), m, k, W.cr(r), W.etar(r), W.Qr(r), W.ritzr(r), W.scalr(r), s, gd, jend));
        }
      }
      DW_TRY(ctl_after_deflate(W.ctl.as<int>(), W.scal.as<double>(), kSclCount, nr, s));
      for (int r : present) {
        const int* gd = W.gate(r, kCDefl);
        const int* jend = W.gate(r, kCJend);
        ProfTag tag_d(kTagDefl, 1ull << r);
        DW_TRY(blas_rotate(W.vprec, W.Vr(r), n, m + 1, W.Qr(r), kLd, k + 1, n, s, gd, jend, 1));
        DW_TRY(blas_rotate(W.zstore, W.Zr(r), n, m, W.Qr(r), kLd, k, n, s, gd, jend, 0));
      }
      if (inject)
        for (int r : present) DW_TRY(inject_vector(r));
      for (int r : present) {
        const int* gd = W.gate(r, kCDefl);
        ProfTag tag_d(kTagDefl, 1ull << r);
        DW_TRY(fill_zero(W.cr(r), 2 * (long long)kLd, gd, s));
        DW_TRY(blas_dots(W.vprec, W.Vr(r), n, k + 1, W.vec(W.r, r), n, W.partr(r), W.cr(r), 1, 0, s, gd));
      }
    }
    return fresh_and_open(present);
  }

  // v_{k+1} from the explicit residual r (Section 4.7): w = r orthogonalised
  // against the rotated V_k (classical Gram-Schmidt, two passes), then
  // v_{k+1} = e^{i theta} w / ||w|| with the phase of the rotated v_{k+1}
  // (e^{i theta} = w^H v_{k+1} / |w^H v_{k+1}|), so that D Z_k = V_{k+1} H^_k
  // keeps its coefficients. The rotated vector is kept when r lies in
  // span(V_k) (||w|| <= 1e-12 ||r||), w is orthogonal to it, or a value is not
  // finite. Uses W.w as scratch.
  dw_status inject_vector(int r) {
    const long long n = W.n;
    const int k = W.k;
    const int* gd = W.gate(r, kCDefl);
    ProfTag tag_d(kTagDefl, 1ull << r);
    double* w = W.vec(W.w, r);
    double* t = W.injr(r) + 2 * kLd;
    double* tail = W.injr(r) + 4 * kLd;
    double* coef = tail + 4;
    DW_TRY(copy_doubles(W.vec(W.r, r), w, 2 * n, gd, s));
    for (int pass = 0; pass < 2; ++pass) {
      DW_TRY(blas_dots(W.vprec, W.Vr(r), n, k, w, n, W.partr(r), t, 1, 0, s, gd));
      DW_TRY(blas_combine(W.vprec, W.Vr(r), n, k, t, -1.0, w, n, s, gd));
    }
    DW_TRY(blas_dots(W.vprec, W.Vc(r, k), n, 1, w, n, W.partr(r), tail, 1, 0, s, gd));
    DW_TRY(blas_dots(DW_PREC_F64, w, n, 1, w, n, W.partr(r), tail + 2, 1, 0, s, gd));
    DW_TRY(inject_coef(W.ctlr(r), W.ctldr(r), tail, coef, s));
    const int* gi = W.gate(r, kCInject);
    ProfTag tag_i(kTagInject, 1ull << r);
    if (W.vprec == DW_PREC_F64) {
      DW_TRY(fill_zero((double*)W.Vc(r, k), 2 * n, gi, s));
      DW_TRY(blas_combine(DW_PREC_F64, w, n, 1, coef, 1.0, (double*)W.Vc(r, k), n, s, gi));
    } else {
      // w <- coefficient * w in place (FP64), then stored at the basis precision
      DW_TRY(blas_scale_c(w, coef, n, s, gi));
      DW_TRY(launch_convert(DW_PREC_F64, w, W.vprec, W.Vc(r, k), 1.0, n, s, nullptr, gi));
    }
    return DW_OK;
  }

  dw_status run_cycle(Shape& sh, bool graphs) {
    if (!graphs) return enqueue_cycle(sh);
    if (!sh.exec) {
      hipGraph_t gr = nullptr;
      DW_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const dw_status es = enqueue_cycle(sh);
      const hipError_t ce = hipStreamEndCapture(s, &gr);
      if (es != DW_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return es;
      }
      DW_CHECK_HIP(ce);
      const hipError_t ie = hipGraphInstantiate(&sh.exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      DW_CHECK_HIP(ie);
    }
    DW_CHECK_HIP(hipGraphLaunch(sh.exec, s));
    return DW_OK;
  }

  Shape* shape_for(const std::vector<signed char>& st, bool donor) {
    for (auto& p : W.shapes)
      if (p->st == st && p->donor == donor) return p.get();
    return nullptr;
  }

  dw_status solve(double m0, const double* b_can, double* x_can, dw_solve_stats* stats, bool graphs) {
    const int nr = W.nr;
    auto t0 = std::chrono::steady_clock::now();
    DW_TRY(start(b_can, m0));
    std::vector<signed char> st(nr, 1);
    bool donor_ok = false;  // RHS 0 holds a deflation space from a deflated restart
    const bool shared = P->shared_defl && nr > 1 && W.k > 0;
    while (true) {
      const bool donor = shared && donor_ok;
      Shape* sh = shape_for(st, donor);
      if (!sh) {
        auto p = std::make_unique<Shape>();
        p->st = st;
        p->donor = donor;
        DW_TRY(upload_lists(*p));
        W.shapes.push_back(std::move(p));
        sh = W.shapes.back().get();
      }
      DW_TRY(run_cycle(*sh, graphs));
      DW_TRY(readback(W, s));
      // per-kernel timing: a launch counts for the right-hand sides whose gate was open
      prof_resolve([&](int kind, int r) {
        if (r >= nr) return false;
        const int* c = W.hctl(r);
        if (kind >= 0) return c[kCPrevInCycle] && kind >= c[kCPrevJ0] && kind < c[kCPrevJend];
        switch (kind) {
          case kTagFin: return c[kCPrevFin] != 0;
          case kTagCycle: return c[kCPrevInCycle] != 0;
          case kTagDefl: return c[kCPrevDefl] != 0;
          case kTagFresh: return c[kCPrevFresh] != 0;
          case kTagInject: return c[kCPrevInject] != 0;
          default: return true;
        }
      });
      bool any = false;
      for (int r = 0; r < nr; ++r) {
        const int* c = W.hctl(r);
        if (c[kCDone]) {
          st[r] = 0;
        } else {
          st[r] = c[kCDefl] ? 2 : 1;
          any = true;
        }
      }
      if (shared) {
        const int* c0 = W.hctl(0);
        if (c0[kCDefl]) donor_ok = true;
        else if (c0[kCFresh]) donor_ok = false;
      }
      if (!any) break;
    }
    DW_TRY(launch_unpack_spinor(f->g, DW_PREC_F64, W.x.p, x_can, 1.0, nr, s));
    DW_CHECK_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nr; ++r) {
      const int* c = W.hctl(r);
      const double* d = W.hctld(r);
      dw_solve_stats& o = stats[r];
      memset(&o, 0, sizeof o);
      o.converged = c[kCConv];
      o.iterations = c[kCIters];
      o.cycles = c[kCCycles];
      o.clean_restarts = c[kCClean];
      o.true_relres = d[kDBnorm] > 0 ? d[kDResE] / d[kDBnorm] : 0.0;
      o.implicit_relres = d[kDBnorm] > 0 ? d[kDResI] / d[kDBnorm] : 0.0;
      o.seconds = secs;
    }
    return DW_OK;
  }
};

bool same_params(const fgmresdr_params& a, const fgmresdr_params& b) {
  // the graphs flag only says whether cycles are captured; the workspace and
  // the captured cycles are the same either way
  const int32_t fa = a.flags & ~DW_SOLVE_GRAPHS, fb = b.flags & ~DW_SOLVE_GRAPHS;
  return a.m == b.m && a.k == b.k && a.shared_defl == b.shared_defl && fa == fb &&
         a.sap.ncycles == b.sap.ncycles && a.sap.nmr == b.sap.nmr && a.sap.storage == b.sap.storage &&
         a.sap.mr_reduction == b.sap.mr_reduction;
}

// workspace and captured cycles kept with a field between solves (DW_SOLVE_GRAPHS)
struct SolverCache {
  std::unique_ptr<Work> W;
};

void destroy_cache(void* p) { delete static_cast<SolverCache*>(p); }

}  // namespace

namespace dw {
size_t solver_bytes(long long sites, int m, int prec, int flags, int nrhs) {
  const int vprec = (flags & (DW_SOLVE_V32 | DW_SOLVE_A32)) ? DW_PREC_F32 : DW_PREC_F64;
  const int zstore = (flags & DW_SOLVE_A32) ? DW_PREC_F32 : DW_PREC_F64;
  return bytes_per_rhs(sites * 12, m, prec, vprec, zstore) * (size_t)nrhs + (size_t)nrhs * 64 * 1024;
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
  if (P->flags & ~(DW_SOLVE_GRAPHS | DW_SOLVE_V32 | DW_SOLVE_INJECT | DW_SOLVE_A32)) {
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
  // captured cycles need a stream that can be captured and no per-launch event timing
  const bool graphs = (P->flags & DW_SOLVE_GRAPHS) && stream != nullptr && !f->ctx->prof.on;
  SolverCache* cache = static_cast<SolverCache*>(f->solver_cache);
  // a workspace kept by an earlier solve with captured cycles serves this
  // solve too (captured or not) when it was made for the same shape; else it
  // goes before the free memory is counted
  const bool reuse = cache && cache->W && cache->W->nr == nrhs && same_params(cache->W->P, *P) &&
                     cache->W->clover[0] == f->C[P->sap.storage] && cache->W->clover[1] == f->C[DW_PREC_F64];
  if (cache && !reuse) {
    DW_CHECK_HIP(hipStreamSynchronize(stream));
    destroy_cache(cache);
    f->solver_cache = nullptr;
    f->solver_cache_free = nullptr;
    cache = nullptr;
  }
  // RHS per batch: as many as fit in free device memory (at least one), at
  // most kMaxBatch (the per-RHS masks of a batch are 64 bits wide)
  size_t free_b = 0, total_b = 0;
  DW_CHECK_HIP(hipMemGetInfo(&free_b, &total_b));
  {
    // memory that the stream-ordered allocator's pool holds unused is free too
    hipMemPool_t pool = nullptr;
    uint64_t res = 0, used = 0;
    if (hipDeviceGetDefaultMemPool(&pool, f->ctx->device) == hipSuccess && pool &&
        hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &res) == hipSuccess &&
        hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemCurrent, &used) == hipSuccess && res > used)
      free_b += (size_t)(res - used);
  }
  const size_t per = bytes_per_rhs(n, P->m, P->sap.storage, basis_prec(P), zstore_prec(P));
  int nb = (int)std::max<size_t>(1, (size_t)(0.9 * (double)free_b) / per);
  if (reuse || f->memory_reserved) nb = nrhs;
  nb = std::min(nb, (int)nrhs);
  nb = std::min(nb, kMaxBatch);
  // The count misses memory that the stream-ordered allocator keeps from
  // earlier solves (on this runtime its pool reports none reserved, yet the
  // device shows it as used), so a batch of all right-hand sides is tried
  // first; if it does not fit, the estimate stands.
  std::unique_ptr<Work> whole;
  if (nb < nrhs && nrhs <= kMaxBatch) {
    whole = std::make_unique<Work>();
    if (alloc_work(f, P, nrhs, *whole, stream) == DW_OK) {
      nb = nrhs;
    } else {
      whole.reset();
      (void)hipGetLastError();  // the failed allocation is not an error of this call
      clear_error();
    }
  }
  bool all_conv = true;
  std::vector<dw_solve_stats> st(nrhs);
  for (int r0 = 0; r0 < nrhs; r0 += nb) {
    const int nr = std::min(nb, nrhs - r0);
    const bool keep = graphs && nr == nrhs;  // a single batch keeps its workspace with the field
    std::unique_ptr<Work> own;
    Work* W = nullptr;
    if (reuse) {
      W = cache->W.get();
      W->P.max_iter = P->max_iter;
      W->P.tol = P->tol;
      W->P.restart_t = P->restart_t;
    } else if (whole) {
      own = std::move(whole);
      W = own.get();
    } else {
      own = std::make_unique<Work>();
      DW_TRY(alloc_work(f, P, nr, *own, stream));
      W = own.get();
    }
    Solver S(f, P, *W, stream);
    DW_TRY(S.solve(m0, b + 2 * (long long)r0 * n, x + 2 * (long long)r0 * n, st.data() + r0, graphs));
    if (keep && own) {
      SolverCache* c = new SolverCache;
      c->W = std::move(own);
      f->solver_cache = c;
      f->solver_cache_free = destroy_cache;
    }
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
