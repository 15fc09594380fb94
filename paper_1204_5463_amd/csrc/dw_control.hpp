// Per right-hand-side control records of the FGMRES-DR cycle on the device
// (see k_control.hip), and gate conventions of the guarded kernels.
//
// A gated kernel takes `const int* gate` (null: always run) and returns at
// once when *gate == 0; batched kernels take a gate array indexed by the
// right-hand side with a stride. Counts that only the device knows (the
// columns of a cycle that ended early) are read through `const int* dn`.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/dwsap.h"

namespace dw {

// int fields (kCtl per right-hand side)
enum {
  kCLive = 0,     // takes part in the current cycle's Arnoldi steps
  kCJ0 = 1,       // first column of the cycle (0 fresh, k deflated)
  kCJend = 2,     // columns built in this cycle so far
  kCJlim = 3,     // the step building column j stops the cycle when j + 1 >= jlim
  kCBroke = 4,    // breakdown h_{j+1,j} ~ 0
  kCInCycle = 5,  // took part in the cycle (cycle end applies)
  kCFin = 6,      // the cycle's last vector needs its second Gram-Schmidt pass
  kCDone = 7,     // stopped (converged or iteration limit)
  kCConv = 8,     // converged
  kCFresh = 9,    // next cycle starts fresh (first cycle, k = 0, clean restart, projection)
  kCDefl = 10,    // next cycle starts from a deflated restart
  kCIters = 11,   // Arnoldi steps so far
  kCCycles = 12,  // cycles so far
  kCClean = 13,   // clean restarts so far
  kCInject = 14,  // the injected v_{k+1} is used (Section 4.7)
  kCMaxIter = 15, // iteration limit
  // the cycle just finished, kept when the next one opens (host accounting)
  kCPrevInCycle = 16,
  kCPrevJ0 = 17,
  kCPrevJend = 18,
  kCPrevFin = 19,
  kCPrevDefl = 20,
  kCPrevFresh = 21,
  kCPrevInject = 22,
  kCtl = 24
};
// double fields (kCtlD per right-hand side)
enum { kDBnorm = 0, kDTolAbs = 1, kDResE = 2, kDResI = 3, kDRestartT = 4, kCtlD = 8 };

dw_status ctl_init(int* ctl, double* ctld, const double* nrm, int nrm_stride, int nr, double tol, double restart_t,
                   int max_iter, hipStream_t s);
dw_status ctl_decide(int* ctl, double* ctld, const double* nrm, int nrm_stride, const double* scal, int scal_stride,
                     int nr, int k, unsigned long long projected, hipStream_t s);
dw_status ctl_after_deflate(int* ctl, const double* scal, int scal_stride, int nr, hipStream_t s);
dw_status ctl_next(int* ctl, int nr, int m, int k, hipStream_t s);
dw_status ctl_cycle_end(int* ctl, int nr, hipStream_t s);
// p[0..ndoubles) = 0 unless *gate == 0 (a kernel, so that it can be captured)
dw_status fill_zero(double* p, long long ndoubles, const int* gate, hipStream_t s);
dw_status copy_doubles(const double* a, double* b, long long ndoubles, const int* gate, hipStream_t s);
dw_status set_double(double* p, double v, hipStream_t s);
// sc[2r] = sqrt(n / nrm[2r]) (1 if nrm[2r] = 0), sc[2r+1] = 1 / sc[2r]: unit-RMS scaling per right-hand side
dw_status rms_scales(const double* nrm, long long n, double* sc, int nr, hipStream_t s);
dw_status inject_coef(int* ctl, const double* ctld, const double* t, double* coef, hipStream_t s);

}  // namespace dw
