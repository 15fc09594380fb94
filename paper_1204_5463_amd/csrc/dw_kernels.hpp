// Launchers of the Krylov-space kernels (long vectors and small dense
// FP64 problems). All pointers are device pointers; complex numbers are
// (re, im) double pairs. Small matrices are column-major with leading
// dimension kLd (row i, column j at i + j*kLd).
#pragma once

#include "dw_internal.hpp"

namespace dw {

constexpr int kBlasGrid = 1024;  // workgroups of the multi-dot kernels (partials per column)
constexpr int kMaxM = 48;        // largest restart length m
constexpr int kLd = kMaxM + 1;   // leading dimension of small matrices

// out[c*ostride] (= or += per op) <- V_c^H w for c < ncols; partials holds
// ncols * kBlasGrid pairs of scratch
// gate (may be null): run only if *gate != 0; dn (may be null): the column
// count is *dn + dadd on the device (at most ncols)
dw_status blas_dots(int prec_v, const void* V, long long stride, int ncols, const double* w, long long n,
                    double* partials, double* out, int ostride, int op, hipStream_t s, const int* gate = nullptr,
                    const int* dn = nullptr, int dadd = 0);
// w -= sum_c h_c V_c
dw_status blas_sub_cols(const double* V, long long stride, int ncols, const double* h, double* w, long long n,
                        hipStream_t s);
// y = alpha[0] * x (alpha a device double)
dw_status blas_scale(const double* x, double* y, const double* alpha, long long n, hipStream_t s,
                     const int* gate = nullptr);
// x *= alpha[0] in place (alpha a device complex pair)
dw_status blas_scale_c(double* x, const double* alpha, long long n, hipStream_t s, const int* gate = nullptr);
// x += scale * sum_c coef_c Z_c
dw_status blas_combine(int prec_z, const void* Z, long long stride, int ncols, const double* coef, double scale,
                       double* x, long long n, hipStream_t s, const int* gate = nullptr, const int* dn = nullptr);
// in place V[:, 0:nout] = V[:, 0:nin] Q, Q column-major with leading dimension ldq
// with dn: nin = min(nin, *dn + dadd)
dw_status blas_rotate(int prec_v, void* V, long long stride, int nin, const double* Q, int ldq, int nout, long long n,
                      hipStream_t s, const int* gate = nullptr, const int* dn = nullptr, int dadd = 0);

// Gram-Schmidt with delayed reorthogonalisation (see k_blas.hip).
// gs_reduce: out[0..2nv+3) = [V^H u | V^H w | u^H u, u^H w, w^H w] over the
// nv final columns; u or w may be null. partials: (2 kMaxM + 5) * kBlasGrid pairs.
// V and u are stored at prec_v (FP64 or FP32), w is FP64.
// dcol (may be null): finalise column *dcol (u = V_{*dcol}, nv = *dcol <= nv)
// prec_w: storage of w, FP64, or FP32 with an FP32 basis: then the sweep's
// arithmetic is FP32 too (the single-precision Arnoldi), its per-workgroup
// sums combined in FP64
dw_status gs_reduce(int prec_v, const void* V, long long stride, int nv, const void* u, const void* w, long long n,
                    double* partials, double* out, hipStream_t s, const int* gate = nullptr,
                    const int* dcol = nullptr, int prec_w = DW_PREC_F64);
// gs_update: jcol >= 0: V_jcol <- (V_jcol - V a)/beta; w != null:
// wout <- w - V b - c V_jcol (c only if jcol >= 0), nrm2 <- ||wout||^2.
// coef as written by dense_gs_coef.
// V and wout are stored at prec_v (FP64 or FP32); with FP32 storage nrm2 is
// the squared norm of the stored (rounded) wout.
// dcol (may be null): nv = jcol = *dcol; prec_w as for gs_reduce
dw_status gs_update(int prec_v, void* V, long long stride, int nv, int jcol, const void* w, void* wout,
                    const double* coef, long long n, double* partials, double* nrm2, hipStream_t s,
                    const int* gate = nullptr, const int* dcol = nullptr, int prec_w = DW_PREC_F64);

// ---- small dense FP64 (one workgroup) ---------------------------------------------
// Scalars block written by dense_step / dense_cycle_end (doubles):
enum {
  kSclHnext = 0,      // h_{j+1,j}
  kSclHinv = 1,       // 1 / h_{j+1,j} (0 on breakdown)
  kSclResImp = 2,     // implicit residual norm ||c - H eta|| of the current step
  kSclBreak = 3,      // 1.0 if the step broke down
  kSclStatus = 4,     // deflation status (0 ok, 1 singular H_m, 2 eigen failure, 3 non-finite)
  kSclBeta = 5,       // norm used for a fresh start
  kSclBetaInv = 6,
  kSclCount = 8
};

// Completes Arnoldi step j: H(0:j, j) = h1 + h2, H(j+1, j) = sqrt(nrm2.re),
// breakdown test, implicit residual of the (j+2) x (j+1) least-squares
// problem with right-hand side c.
dw_status dense_step(double* H, int j, const double* h1, const double* h2, const double* nrm2, const double* c,
                     double* scal, double bd_tol, hipStream_t s);
// eta = argmin ||c(0:cols+1) - H(0:cols+1, 0:cols) eta||; scal[kSclResImp] = residual
dw_status dense_lsq(const double* H, int cols, const double* c, double* eta, double* scal, hipStream_t s,
                    const int* gate = nullptr, const int* dn = nullptr);
// Deflated restart of a cycle with mm columns (Lemma 1, Alg. 4):
// harmonic Ritz pairs, G_{k+1} = [[G_k; 0], c - H eta], QR -> Q ((mm+1) x (k+1), ld kLd),
// H <- [Q^H H Q_k in rows 0..k, cols 0..k-1; 0 elsewhere]; ritz <- all mm
// harmonic Ritz values sorted by modulus; scal[kSclStatus] = status.
// with dn: mm = *dn (at most the host mm)
dw_status dense_deflate(double* H, int mm, int k, const double* c, const double* eta, double* Q, double* ritz,
                        double* scal, hipStream_t s, const int* gate = nullptr, const int* dn = nullptr);
// Coefficients of one delayed-reorthogonalisation step from gs_reduce's
// output red. hu: the lagged vector u = V_jcol is finalised: a = V^H u,
// beta = sqrt(u^H u - |a|^2), H(0:jcol, jcol-1) += a, H(jcol, jcol-1) = beta.
// hw: column jw of H gets its first-pass entries b (rows 0..nv-1) and
// c = (u^H w - a^H b)/beta (row jcol) when hu. Writes coef for gs_update.
// with dcol: nv = jcol = *dcol (finalising the cycle's last vector; hu = 1, hw = 0)
dw_status dense_gs_coef(double* H, int nv, int jcol, int jw, int hu, int hw, const double* red, double* coef,
                        double* scal, double bd_tol, hipStream_t s, const int* gate = nullptr,
                        const int* dcol = nullptr);
// Completes step j after gs_update: H(j+1, j) = sqrt(nrm2), breakdown test,
// implicit residual of the (j+2) x (j+1) least-squares problem; also
// scal[kSclHinv] = 1/H(j+1, j) for scaling the next preconditioner input.
// ctl (may be null): the right-hand side's control record (dw_control.hpp);
// the step then runs only while it is live and records jend = j + 1 and the
// breakdown, and stops the cycle (live = 0) on breakdown, on an implicit
// residual <= ctld[kDTolAbs], or at the step limit.
dw_status dense_step2(double* H, int j, const double* nrm2, const double* c, double* scal, double bd_tol,
                      hipStream_t s, int* ctl = nullptr, const double* ctld = nullptr);
// projection onto a deflation space with D Z_k = V_{k+1} H_k (H_k the
// (k+1) x k leading block of H): y = argmin ||t - H_k y||, sv = H_k y
dw_status dense_project(const double* H, int k, const double* t, double* y, double* sv, hipStream_t s,
                        const int* gate = nullptr);
// fresh start: scal[kSclBeta] = sqrt(nrm2.re), scal[kSclBetaInv] = 1/beta, c = beta e_1, H = 0
dw_status dense_fresh(double* H, double* c, const double* nrm2, double* scal, hipStream_t s,
                      const int* gate = nullptr);

}  // namespace dw
