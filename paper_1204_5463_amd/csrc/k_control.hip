// Device-side control of the FGMRES-DR cycle (paper Alg. 4, Section 4.7).
//
// Every right-hand side of a lock-step batch has a small control record in
// device memory. The kernels of an Arnoldi step and of the cycle end read
// their gate from it, so a right-hand side that has stopped (converged
// implicit residual, breakdown, iteration limit) turns the rest of the
// cycle's kernels into no-ops without the host looking. The decisions at
// the cycle end (stop, clean restart, deflated restart) are taken here
// too, from the explicit FP64 residual; the host reads the records once per
// cycle. This is what lets a whole restart cycle be replayed as one HIP
// graph.
#include "dw_control.hpp"
#include "dw_internal.hpp"
#include "dw_kernels.hpp"

namespace dw {

namespace {

__global__ void k_ctl_init(int* __restrict__ ctl, double* __restrict__ ctld, const double* __restrict__ nrm,
                           int nrm_stride, int nr, double tol, double restart_t, int max_iter) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  int* c = ctl + r * kCtl;
  double* d = ctld + r * kCtlD;
  for (int i = 0; i < kCtl; ++i) c[i] = 0;
  for (int i = 0; i < kCtlD; ++i) d[i] = 0.0;
  const double bn = sqrt(fmax(nrm[(long long)r * nrm_stride], 0.0));
  d[kDBnorm] = bn;
  d[kDTolAbs] = tol * bn;
  d[kDResE] = bn;
  d[kDResI] = bn;
  d[kDRestartT] = restart_t;
  c[kCMaxIter] = max_iter;
  if (bn == 0.0) {
    c[kCDone] = 1;
    c[kCConv] = 1;
  } else {
    c[kCFresh] = 1;
  }
}

// after the explicit residual and its norm: stop, clean restart or
// deflated restart (same rules as the oracle's FGMRES-DR)
__global__ void k_ctl_decide(int* __restrict__ ctl, double* __restrict__ ctld, const double* __restrict__ nrm,
                             int nrm_stride, const double* __restrict__ scal, int scal_stride, int nr, int k,
                             unsigned long long projected) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  int* c = ctl + r * kCtl;
  double* d = ctld + r * kCtlD;
  c[kCDefl] = c[kCFresh] = 0;
  if (!c[kCInCycle]) return;
  c[kCIters] += c[kCJend] - c[kCJ0];
  c[kCCycles] += 1;
  const double res_e = sqrt(fmax(nrm[(long long)r * nrm_stride], 0.0));
  const double res_i = scal[(long long)r * scal_stride + kSclResImp];
  d[kDResE] = res_e;
  d[kDResI] = res_i;
  const bool proj = r < 64 && ((projected >> r) & 1ull);
  if (res_e <= d[kDTolAbs]) {
    c[kCDone] = 1;
    c[kCConv] = 1;
  } else if (c[kCIters] >= c[kCMaxIter]) {
    c[kCDone] = 1;
  } else if (k == 0 || proj) {
    c[kCFresh] = 1;  // restarted FGMRES(m), or a restart from a projected residual
  } else if (c[kCBroke] || c[kCJend] <= k || res_e > d[kDRestartT] * fmax(res_i, 1e-300)) {
    c[kCFresh] = 1;  // clean restart (Section 4.7)
    c[kCClean] += 1;
  } else {
    c[kCDefl] = 1;
  }
}

// a deflation whose small eigenproblem failed becomes a clean restart
__global__ void k_ctl_after_deflate(int* __restrict__ ctl, const double* __restrict__ scal, int scal_stride, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  int* c = ctl + r * kCtl;
  if (c[kCDefl] && scal[(long long)r * scal_stride + kSclStatus] != 0.0) {
    c[kCDefl] = 0;
    c[kCFresh] = 1;
    c[kCClean] += 1;
  }
}

// opens the next cycle: first column j0, step limit from the iteration budget
__global__ void k_ctl_next(int* __restrict__ ctl, int nr, int m, int k) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  int* c = ctl + r * kCtl;
  c[kCPrevInCycle] = c[kCInCycle];
  c[kCPrevJ0] = c[kCJ0];
  c[kCPrevJend] = c[kCJend];
  c[kCPrevFin] = c[kCFin];
  c[kCPrevDefl] = c[kCDefl];
  c[kCPrevFresh] = c[kCFresh];
  c[kCPrevInject] = c[kCInject];
  const int live = c[kCDone] ? 0 : 1;
  const int j0 = c[kCDefl] ? k : 0;
  c[kCJ0] = j0;
  c[kCJend] = j0;
  c[kCBroke] = 0;
  c[kCLive] = live;
  c[kCInCycle] = live;
  c[kCFin] = 0;
  c[kCInject] = 0;
  const int left = c[kCMaxIter] - c[kCIters];
  c[kCJlim] = j0 + left < m ? j0 + left : m;
}

// before the cycle end: the last vector needs its second Gram-Schmidt pass
// when the cycle took a step and did not break down
__global__ void k_ctl_cycle_end(int* __restrict__ ctl, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  int* c = ctl + r * kCtl;
  c[kCFin] = (c[kCInCycle] && c[kCJend] > c[kCJ0] && !c[kCBroke]) ? 1 : 0;
  c[kCLive] = 0;
}

__global__ void k_fill_zero(double* __restrict__ p, long long n, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, long long n,
                       const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// coefficient of the injected v_{k+1} (Section 4.7): from t = [v^H w, ||w||^2]
// (v the rotated v_{k+1}, w the explicit residual orthogonalised against
// V_k) the unit vector e^{i theta} w / ||w|| with the phase of v; kept only
// when w is not (numerically) in span(V_k) and everything is finite
__global__ void k_inject_coef(int* __restrict__ ctl, const double* __restrict__ ctld, const double* __restrict__ t,
                              double* __restrict__ coef) {
  if (threadIdx.x != 0 || !ctl[kCDefl]) return;
  const double pm = hypot(t[0], t[1]), wn = sqrt(fmax(t[2], 0.0));
  const double rnorm = ctld[kDResE];
  const bool use = pm > 0 && wn > 1e-12 * rnorm && isfinite(pm) && isfinite(wn);
  ctl[kCInject] = use ? 1 : 0;
  if (use) {
    coef[0] = t[0] / (pm * wn);
    coef[1] = -t[1] / (pm * wn);
  }
}

__global__ void k_set_double(double* p, double v) {
  if (threadIdx.x == 0) *p = v;
}

// per right-hand side r: sc[2r] = sqrt(n / ||v_r||^2) (1 for v_r = 0), sc[2r+1] = 1 / sc[2r]
__global__ void k_rms_scales(const double* __restrict__ nrm, long long n, double* __restrict__ sc, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  const double h = nrm[2 * (long long)r];
  const double sg = h > 0 ? sqrt((double)n / h) : 1.0;
  sc[2 * r] = sg;
  sc[2 * r + 1] = 1.0 / sg;
}

unsigned rhs_grid(int nr) { return (unsigned)((nr + 63) / 64); }

}  // namespace

dw_status ctl_init(int* ctl, double* ctld, const double* nrm, int nrm_stride, int nr, double tol, double restart_t,
                   int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, rhs_grid(nr), 64, 0, s, ctl, ctld, nrm, nrm_stride, nr, tol, restart_t, max_iter);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status ctl_decide(int* ctl, double* ctld, const double* nrm, int nrm_stride, const double* scal, int scal_stride,
                     int nr, int k, unsigned long long projected, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_decide, rhs_grid(nr), 64, 0, s, ctl, ctld, nrm, nrm_stride, scal, scal_stride, nr, k,
                     projected);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status ctl_after_deflate(int* ctl, const double* scal, int scal_stride, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_after_deflate, rhs_grid(nr), 64, 0, s, ctl, scal, scal_stride, nr);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status ctl_next(int* ctl, int nr, int m, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_next, rhs_grid(nr), 64, 0, s, ctl, nr, m, k);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status ctl_cycle_end(int* ctl, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_cycle_end, rhs_grid(nr), 64, 0, s, ctl, nr);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status fill_zero(double* p, long long ndoubles, const int* gate, hipStream_t s) {
  long long b = (ndoubles + 255) / 256;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_fill_zero, (unsigned)b, 256, 0, s, p, ndoubles, gate);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status copy_doubles(const double* a, double* b, long long ndoubles, const int* gate, hipStream_t s) {
  long long g = (ndoubles + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  KTimer kt(DW_K_SCALE, s);
  hipLaunchKernelGGL(k_copy, (unsigned)g, 256, 0, s, a, b, ndoubles, gate);
  DW_CHECK_LAUNCH();
  kt.done((double)ndoubles * 16, 0);
  return DW_OK;
}
dw_status rms_scales(const double* nrm, long long n, double* sc, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_rms_scales, rhs_grid(nr), 64, 0, s, nrm, n, sc, nr);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status set_double(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_double, 1, 64, 0, s, p, v);
  DW_CHECK_LAUNCH();
  return DW_OK;
}
dw_status inject_coef(int* ctl, const double* ctld, const double* t, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_inject_coef, 1, 64, 0, s, ctl, ctld, t, coef);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

}  // namespace dw
