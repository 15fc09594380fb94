// Small dense complex FP64 problems of FGMRES-DR, each solved by one
// workgroup of one wavefront (64 lanes) with its operands in LDS:
//
//   * per Arnoldi step: the new Hessenberg column and the implicit residual
//     norm of the small least-squares problem (Section 4.2 and Section 4.6;
//     the QR factorisation is recomputed by Householder reflections each
//     step, which also covers the dense leading block after a deflated
//     restart);
//   * per cycle: eta = argmin ||c - H^ eta||;
//   * per deflated restart (Lemma 1a, Alg. 4): f from H_m^H f = h_m (LU with
//     partial pivoting), the eigenpairs of H_m + f h_m^H (Householder
//     reduction to Hessenberg form, single-shift QR iteration with Wilkinson
//     shifts, eigenvectors by back substitution in the Schur form), the k
//     eigenvectors of smallest-modulus eigenvalues, G_{k+1}, its QR
//     factorisation and H^_k = Q_{k+1}^H H^ Q_k.
//
// Lanes work on rows or columns in parallel; serial steps (pivots, shifts,
// rotations) are computed redundantly by every lane from the same LDS data,
// so control flow is uniform across the wave.
#include "dw_control.hpp"
#include "dw_kernels.hpp"
#include "dw_types.hpp"

namespace dw {

namespace {

using C = cplx<double>;
constexpr int kL = 64;  // lanes

__device__ __forceinline__ double cabs(C a) { return sqrt(a.re * a.re + a.im * a.im); }
__device__ __forceinline__ C cdiv(C a, C b) {
  const double d = b.re * b.re + b.im * b.im;
  return C{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ C csqrt_(C z) {
  const double r = cabs(z);
  const double re = sqrt(0.5 * (r + z.re));
  double im = sqrt(0.5 * fmax(r - z.re, 0.0));
  if (z.im < 0) im = -im;
  return C{re, im};
}
__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
  for (int off = kL / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kL);
  return a;
}
__device__ __forceinline__ C ldc(const double* p, long long i) { return C{p[2 * i], p[2 * i + 1]}; }
__device__ __forceinline__ void stc(double* p, long long i, C v) {
  p[2 * i] = v.re;
  p[2 * i + 1] = v.im;
}

// Householder QR in place of A (rows x cols, column-major, leading dim lda)
// with optional right-hand side rhs. Reflector r is stored in column r of
// Uv (entries r..rows-1) with beta[r]; P_r = I - beta_r u_r u_r^H.
__device__ void hh_qr(C* A, int lda, int rows, int cols, C* rhs, C* Uv, int ldu, double* beta) {
  const int lane = threadIdx.x;
  for (int k = 0; k < cols && k < rows; ++k) {
    double part = 0;
    if (lane >= k && lane < rows) part = norm2(A[lane + k * lda]);
    const double nrm2 = wave_sum(part);
    const C x0 = A[k + k * lda];
    const double nrm = sqrt(nrm2);
    const double ax0 = cabs(x0);
    const C ph = ax0 > 0 ? C{x0.re / ax0, x0.im / ax0} : C{1.0, 0.0};
    const C alpha = C{-ph.re * nrm, -ph.im * nrm};
    const C u0 = x0 - alpha;
    const double un2 = nrm2 - ax0 * ax0 + norm2(u0);
    const double bk = (nrm > 0 && un2 > 0) ? 2.0 / un2 : 0.0;
    if (lane < rows) Uv[lane + k * ldu] = lane < k ? C{0, 0} : (lane == k ? u0 : A[lane + k * lda]);
    if (lane == 0) beta[k] = bk;
    __syncthreads();
    if (bk != 0.0) {
      // lane j updates column j (j >= k); lane kL-1 updates rhs
      C* col = nullptr;
      if (lane >= k && lane < cols) col = A + lane * lda;
      else if (lane == kL - 1 && rhs) col = rhs;
      if (col) {
        C s{0, 0};
        for (int i = k; i < rows; ++i) s += cdot(Uv[i + k * ldu], col[i]);
        s = bk * s;
        for (int i = k; i < rows; ++i) col[i] -= Uv[i + k * ldu] * s;
      }
    }
    __syncthreads();
    if (bk != 0.0 && lane < rows && lane >= k) A[lane + k * lda] = lane == k ? alpha : C{0, 0};
    __syncthreads();
  }
}

// solve R eta = rhs(0:cols) by back substitution (lane 0), R = upper part of A
__device__ void back_subst(const C* A, int lda, int cols, const C* rhs, C* eta) {
  if (threadIdx.x == 0) {
    for (int i = cols - 1; i >= 0; --i) {
      C s = rhs[i];
      for (int j = i + 1; j < cols; ++j) s -= A[i + j * lda] * eta[j];
      const C d = A[i + i * lda];
      eta[i] = (d.re == 0 && d.im == 0) ? C{0, 0} : cdiv(s, d);
    }
  }
  __syncthreads();
}

constexpr int kLdA = kMaxM;      // leading dimension of m x m work matrices
constexpr int kQCols = 25;       // at most k + 1 = 25 columns of Q

struct StepSmem {
  C A[kLd * kMaxM];
  C Uv[kLd * kMaxM];
  C rhs[kLd + 1];
  C eta[kMaxM];
  double beta[kMaxM];
};

__global__ void __launch_bounds__(kL) k_step(double* H, int j, const double* h1, const double* h2, const double* nrm2,
                                             const double* c, double* scal, double bd_tol) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  StepSmem& S = *reinterpret_cast<StepSmem*>(smem_raw);
  const int lane = threadIdx.x;
  const int rows = j + 2, cols = j + 1;
  if (lane <= j) stc(H, lane + (long long)j * kLd, ldc(h1, lane) + ldc(h2, lane));
  const double hn = sqrt(fmax(nrm2[0], 0.0));
  if (lane == 0) stc(H, j + 1 + (long long)j * kLd, C{hn, 0.0});
  __syncthreads();
  __threadfence_block();
  double part = 0;
  for (int t = lane; t < rows * cols; t += kL) {
    const int i = t % rows, q = t / rows;
    const C v = ldc(H, i + (long long)q * kLd);
    S.A[i + q * kLd] = v;
    part += norm2(v);
  }
  if (lane < rows) S.rhs[lane] = ldc(c, lane);
  const double hnorm = sqrt(wave_sum(part));
  __syncthreads();
  const bool broke = !(hn > bd_tol * hnorm);
  hh_qr(S.A, kLd, rows, cols, S.rhs, S.Uv, kLd, S.beta);
  if (lane == 0) {
    scal[kSclHnext] = hn;
    scal[kSclHinv] = broke ? 0.0 : 1.0 / hn;
    scal[kSclResImp] = cabs(S.rhs[rows - 1]);
    scal[kSclBreak] = broke ? 1.0 : 0.0;
  }
}


// Coefficients of a delayed-reorthogonalisation Gram-Schmidt step (see
// dense_gs_coef in dw_kernels.hpp). red: reduced slots of gs_reduce.
__global__ void __launch_bounds__(kL) k_gs_coef(double* H, int nv, int jcol, int jw, int hu, int hw,
                                                const double* red, double* coef, double* scal, const int* gate,
                                                const int* dcol) {
  if (gate && *gate == 0) return;
  if (dcol) nv = jcol = *dcol;
  const int lane = threadIdx.x;
  C a2sum{0, 0};
  double a2 = 0;
  C ab{0, 0};
  for (int i = lane; i < nv; i += kL) {
    const C ai = ldc(red, i), bi = ldc(red, nv + i);
    if (hu) a2 += norm2(ai);
    if (hu && hw) ab += cdot(ai, bi);
  }
  a2 = wave_sum(a2);
  ab.re = wave_sum(ab.re);
  ab.im = wave_sum(ab.im);
  (void)a2sum;
  double beta = 1.0, invbeta = 1.0;
  if (hu) {
    const double uu = red[2 * (2 * nv)];
    const double b2 = uu - a2;
    beta = b2 > 0 ? sqrt(b2) : 0.0;
    invbeta = beta > 0 ? 1.0 / beta : 0.0;
  }
  for (int i = lane; i < nv; i += kL) {
    const C ai = hu ? ldc(red, i) : C{0, 0};
    const C bi = hw ? ldc(red, nv + i) : C{0, 0};
    stc(coef, i, ai);
    stc(coef, nv + i, bi);
    if (hu && jcol >= 1) stc(H, i + (long long)(jcol - 1) * kLd, ldc(H, i + (long long)(jcol - 1) * kLd) + ai);
    if (hw) stc(H, i + (long long)jw * kLd, bi);
  }
  if (lane == 0) {
    C cj{0, 0};
    if (hu && hw && beta > 0) {
      const C uw = ldc(red, 2 * nv + 1);
      cj = invbeta * (uw - ab);
    }
    if (hu && jcol >= 1) stc(H, jcol + (long long)(jcol - 1) * kLd, C{beta, 0.0});
    if (hu && hw) stc(H, jcol + (long long)jw * kLd, cj);
    stc(coef, 2 * nv, cj);
    stc(coef, 2 * nv + 1, C{invbeta, 0.0});
    scal[kSclBeta] = beta;
  }
}

__global__ void __launch_bounds__(kL) k_step2(double* H, int j, const double* nrm2, const double* c, double* scal,
                                              double bd_tol, int* ctl, const double* ctld) {
  if (ctl && ctl[kCLive] == 0) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  StepSmem& S = *reinterpret_cast<StepSmem*>(smem_raw);
  const int lane = threadIdx.x;
  const int rows = j + 2, cols = j + 1;
  const double hn = sqrt(fmax(nrm2[0], 0.0));
  if (lane == 0) stc(H, j + 1 + (long long)j * kLd, C{hn, 0.0});
  __syncthreads();
  __threadfence_block();
  double part = 0;
  for (int t = lane; t < rows * cols; t += kL) {
    const int i = t % rows, q = t / rows;
    const C v = (i == j + 1 && q == j) ? C{hn, 0.0} : ldc(H, i + (long long)q * kLd);
    S.A[i + q * kLd] = v;
    part += norm2(v);
  }
  if (lane < rows) S.rhs[lane] = ldc(c, lane);
  const double hnorm = sqrt(wave_sum(part));
  __syncthreads();
  const bool broke = !(hn > bd_tol * hnorm);
  hh_qr(S.A, kLd, rows, cols, S.rhs, S.Uv, kLd, S.beta);
  if (lane == 0) {
    const double ri = cabs(S.rhs[rows - 1]);
    scal[kSclHnext] = hn;
    scal[kSclHinv] = broke ? 0.0 : 1.0 / hn;
    scal[kSclResImp] = ri;
    scal[kSclBreak] = broke ? 1.0 : 0.0;
    if (ctl) {
      ctl[kCJend] = j + 1;
      ctl[kCBroke] = broke ? 1 : 0;
      if (broke || ri <= ctld[kDTolAbs] || j + 1 >= ctl[kCJlim]) ctl[kCLive] = 0;
    }
  }
}

__global__ void __launch_bounds__(kL) k_lsq(const double* H, int cols, const double* c, double* eta, double* scal,
                                            const int* gate, const int* dn) {
  if (gate && *gate == 0) return;
  if (dn) cols = *dn;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  StepSmem& S = *reinterpret_cast<StepSmem*>(smem_raw);
  const int lane = threadIdx.x;
  const int rows = cols + 1;
  for (int t = lane; t < rows * cols; t += kL) {
    const int i = t % rows, q = t / rows;
    S.A[i + q * kLd] = ldc(H, i + (long long)q * kLd);
  }
  if (lane < rows) S.rhs[lane] = ldc(c, lane);
  __syncthreads();
  hh_qr(S.A, kLd, rows, cols, S.rhs, S.Uv, kLd, S.beta);
  back_subst(S.A, kLd, cols, S.rhs, S.eta);
  if (lane < cols) stc(eta, lane, S.eta[lane]);
  if (lane == 0) scal[kSclResImp] = cabs(S.rhs[rows - 1]);
}

// Projection onto a deflation space (D Z_k = V_{k+1} H_k): y = argmin ||t - H_k y||
// and s = H_k y, with H_k the (k+1) x k leading block of H.
__global__ void __launch_bounds__(kL) k_project(const double* H, int k, const double* t, double* y, double* sv,
                                                const int* gate) {
  if (gate && *gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  StepSmem& S = *reinterpret_cast<StepSmem*>(smem_raw);
  const int lane = threadIdx.x;
  const int rows = k + 1;
  for (int q = lane; q < rows * k; q += kL) {
    const int i = q % rows, c = q / rows;
    S.A[i + c * kLd] = ldc(H, i + (long long)c * kLd);
  }
  if (lane < rows) S.rhs[lane] = ldc(t, lane);
  __syncthreads();
  hh_qr(S.A, kLd, rows, k, S.rhs, S.Uv, kLd, S.beta);
  back_subst(S.A, kLd, k, S.rhs, S.eta);
  __syncthreads();
  if (lane < k) stc(y, lane, S.eta[lane]);
  if (lane < rows) {
    C acc{0, 0};
    for (int c = 0; c < k; ++c) {
      const C h = ldc(H, lane + (long long)c * kLd);
      const C e = S.eta[c];
      acc.re += h.re * e.re - h.im * e.im;
      acc.im += h.re * e.im + h.im * e.re;
    }
    stc(sv, lane, acc);
  }
}

__global__ void __launch_bounds__(kL) k_fresh(double* H, double* c, const double* nrm2, double* scal,
                                              const int* gate) {
  if (gate && *gate == 0) return;
  const int lane = threadIdx.x;
  const double beta = sqrt(fmax(nrm2[0], 0.0));
  for (int t = lane; t < kLd * kMaxM; t += kL) stc(H, t, C{0, 0});
  for (int t = lane; t < kLd; t += kL) stc(c, t, C{t == 0 ? beta : 0.0, 0.0});
  if (lane == 0) {
    scal[kSclBeta] = beta;
    scal[kSclBetaInv] = beta > 0 ? 1.0 / beta : 0.0;
  }
}

struct DeflSmem {
  C Hs[kLd * kMaxM];    // H^ (mm+1) x mm
  C A[kLdA * kMaxM];    // B = H_m^H, then H_m + f h^H, its Schur form T, then G_{k+1}, then H^ Q_k
  C Zm[kLdA * kMaxM];   // Schur vectors, then Householder vectors of G_{k+1}
  C Qs[kLd * kQCols];   // eigenvectors of T (k x mm), then Q_{k+1}
  C f[kMaxM];
  C u[kLd];
  C lam[kMaxM];
  C eta[kMaxM];
  double beta[kQCols];
  int order[kMaxM];
  C shift;
  int piv;
};

__global__ void __launch_bounds__(kL)
    k_deflate(double* H, int mm, int k, const double* c, const double* etag, double* Qg, double* ritz, double* scal,
              const int* gate, const int* dn) {
  if (gate && *gate == 0) return;
  if (dn) mm = *dn < mm ? *dn : mm;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  DeflSmem& S = *reinterpret_cast<DeflSmem*>(smem_raw);
  const int lane = threadIdx.x;
  const int n = mm;
  const double eps = 2.220446049250313e-16;

  // ---- 1. load H^ and eta
  for (int t = lane; t < (mm + 1) * mm; t += kL) {
    const int i = t % (mm + 1), q = t / (mm + 1);
    S.Hs[i + q * kLd] = ldc(H, i + (long long)q * kLd);
  }
  if (lane < mm) S.eta[lane] = ldc(etag, lane);
  __syncthreads();

  // ---- 2. f: H_m^H f = h_m with h_m = conj(last row of H^)
  for (int t = lane; t < n * n; t += kL) {
    const int i = t % n, q = t / n;
    S.A[i + q * kLdA] = conj(S.Hs[q + i * kLd]);
  }
  if (lane < n) S.f[lane] = conj(S.Hs[mm + lane * kLd]);
  __syncthreads();
  double bmax = 0;
  for (int t = lane; t < n * n; t += kL) bmax = fmax(bmax, cabs(S.A[(t % n) + (t / n) * kLdA]));
  for (int off = kL / 2; off > 0; off >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, off, kL));
  int status = 0;
  for (int q = 0; q < n; ++q) {
    if (lane == 0) {
      int p = q;
      double best = cabs(S.A[q + q * kLdA]);
      for (int i = q + 1; i < n; ++i) {
        const double a = cabs(S.A[i + q * kLdA]);
        if (a > best) {
          best = a;
          p = i;
        }
      }
      S.piv = p;
    }
    __syncthreads();
    const int p = S.piv;
    if (!(cabs(S.A[p + q * kLdA]) > 1e-14 * bmax)) {
      status = 1;
      break;
    }
    if (p != q) {
      for (int jj = lane; jj <= n; jj += kL) {
        if (jj < n) {
          C t0 = S.A[q + jj * kLdA];
          S.A[q + jj * kLdA] = S.A[p + jj * kLdA];
          S.A[p + jj * kLdA] = t0;
        } else {
          C t0 = S.f[q];
          S.f[q] = S.f[p];
          S.f[p] = t0;
        }
      }
    }
    __syncthreads();
    if (lane > q && lane < n) {
      const C lq = cdiv(S.A[lane + q * kLdA], S.A[q + q * kLdA]);
      for (int jj = q + 1; jj < n; ++jj) S.A[lane + jj * kLdA] -= lq * S.A[q + jj * kLdA];
      S.f[lane] -= lq * S.f[q];
      S.A[lane + q * kLdA] = C{0, 0};
    }
    __syncthreads();
  }
  if (status == 0) {
    back_subst(S.A, kLdA, n, S.f, S.u);  // f -> S.u
    if (lane < n) S.f[lane] = S.u[lane];
    __syncthreads();
  }

  // ---- 3. A = H_m + f h_m^H (h_m^H is the last row of H^), Zm = I
  if (status == 0) {
    for (int t = lane; t < n * n; t += kL) {
      const int i = t % n, q = t / n;
      S.A[i + q * kLdA] = S.Hs[i + q * kLd] + S.f[i] * S.Hs[mm + q * kLd];
      S.Zm[i + q * kLdA] = C{i == q ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    // ---- 4. Householder reduction to upper Hessenberg form, A <- P A P, Zm <- Zm P
    for (int q = 0; q + 2 < n; ++q) {
      double part = 0;
      if (lane > q && lane < n) part = norm2(S.A[lane + q * kLdA]);
      const double nrm2 = wave_sum(part);
      const C x0 = S.A[q + 1 + q * kLdA];
      const double nrm = sqrt(nrm2), ax0 = cabs(x0);
      const C ph = ax0 > 0 ? C{x0.re / ax0, x0.im / ax0} : C{1.0, 0.0};
      const C alpha = C{-ph.re * nrm, -ph.im * nrm};
      const C u0 = x0 - alpha;
      const double un2 = nrm2 - ax0 * ax0 + norm2(u0);
      if (!(nrm > 0 && un2 > 0)) {
        __syncthreads();
        continue;
      }
      const double bq = 2.0 / un2;
      if (lane < n) S.u[lane] = lane <= q ? C{0, 0} : (lane == q + 1 ? u0 : S.A[lane + q * kLdA]);
      __syncthreads();
      if (lane >= q && lane < n) {  // left: column `lane`
        C s{0, 0};
        for (int i = q + 1; i < n; ++i) s += cdot(S.u[i], S.A[i + lane * kLdA]);
        s = bq * s;
        for (int i = q + 1; i < n; ++i) S.A[i + lane * kLdA] -= S.u[i] * s;
      }
      __syncthreads();
      if (lane < n) {  // right: row `lane` of A and of Zm
        C s{0, 0}, sz{0, 0};
        for (int jj = q + 1; jj < n; ++jj) {
          s += S.A[lane + jj * kLdA] * S.u[jj];
          sz += S.Zm[lane + jj * kLdA] * S.u[jj];
        }
        s = bq * s;
        sz = bq * sz;
        for (int jj = q + 1; jj < n; ++jj) {
          S.A[lane + jj * kLdA] -= s * conj(S.u[jj]);
          S.Zm[lane + jj * kLdA] -= sz * conj(S.u[jj]);
        }
      }
      __syncthreads();
      if (lane > q + 1 && lane < n) S.A[lane + q * kLdA] = C{0, 0};
      __syncthreads();
    }

    // ---- 5. shifted QR iteration (complex, single shift) to upper triangular T
    double anorm = 0;
    for (int t = lane; t < n * n; t += kL) anorm = fmax(anorm, cabs(S.A[(t % n) + (t / n) * kLdA]));
    for (int off = kL / 2; off > 0; off >>= 1) anorm = fmax(anorm, __shfl_xor(anorm, off, kL));
    int hi = n - 1, its = 0, total = 0;
    while (hi > 0) {
      int l = hi;
      while (l > 0) {
        double sc = cabs(S.A[l - 1 + (l - 1) * kLdA]) + cabs(S.A[l + l * kLdA]);
        if (sc == 0) sc = anorm;
        if (cabs(S.A[l + (l - 1) * kLdA]) <= eps * sc) break;
        --l;
      }
      if (l > 0) {
        __syncthreads();
        if (lane == 0) S.A[l + (l - 1) * kLdA] = C{0, 0};
        __syncthreads();
      }
      if (l == hi) {
        --hi;
        its = 0;
        continue;
      }
      if (++total > 60 * n) {
        status = 2;
        break;
      }
      ++its;
      C mu;
      const C a = S.A[hi - 1 + (hi - 1) * kLdA], b = S.A[hi - 1 + hi * kLdA];
      const C cc = S.A[hi + (hi - 1) * kLdA], d = S.A[hi + hi * kLdA];
      if (its % 11 == 10) {
        // exceptional shift to break cycles
        mu = d + C{0.75 * cabs(cc), 0.0};
      } else {
        const C t = 0.5 * (a - d);
        const C disc = csqrt_(t * t + b * cc);
        const C m1 = d + t + disc, m2 = d + t - disc;
        mu = cabs(m1 - d) < cabs(m2 - d) ? m1 : m2;
      }
      for (int q = l; q < hi; ++q) {
        C x, y;
        if (q == l) {
          x = S.A[l + l * kLdA] - mu;
          y = S.A[l + 1 + l * kLdA];
        } else {
          x = S.A[q + (q - 1) * kLdA];
          y = S.A[q + 1 + (q - 1) * kLdA];
        }
        // rotation G = [[cs, sn], [-conj(sn), cs]] with G [x; y] = [r; 0]
        const double ax = cabs(x), ay = cabs(y);
        double cs;
        C sn;
        if (ay == 0) {
          cs = 1;
          sn = C{0, 0};
        } else if (ax == 0) {
          cs = 0;
          sn = C{y.re / ay, -y.im / ay};
        } else {
          const double r = sqrt(ax * ax + ay * ay);
          cs = ax / r;
          const C ph = C{x.re / ax, x.im / ax};
          sn = (1.0 / r) * (ph * conj(y));
        }
        __syncthreads();
        const int j0 = q == l ? l : q - 1;
        if (lane >= j0 && lane < n) {  // rows q, q+1
          const C r0 = S.A[q + lane * kLdA], r1 = S.A[q + 1 + lane * kLdA];
          S.A[q + lane * kLdA] = cs * r0 + sn * r1;
          S.A[q + 1 + lane * kLdA] = cs * r1 - conj(sn) * r0;
        }
        __syncthreads();
        const int imax = q + 2 < hi ? q + 2 : hi;
        if (lane <= imax) {  // columns q, q+1 (times G^H)
          const C c0 = S.A[lane + q * kLdA], c1 = S.A[lane + (q + 1) * kLdA];
          S.A[lane + q * kLdA] = cs * c0 + conj(sn) * c1;
          S.A[lane + (q + 1) * kLdA] = cs * c1 - sn * c0;
        }
        if (lane < n) {
          const C z0 = S.Zm[lane + q * kLdA], z1 = S.Zm[lane + (q + 1) * kLdA];
          S.Zm[lane + q * kLdA] = cs * z0 + conj(sn) * z1;
          S.Zm[lane + (q + 1) * kLdA] = cs * z1 - sn * z0;
        }
        __syncthreads();
        if (q > l && lane == 0) S.A[q + 1 + (q - 1) * kLdA] = C{0, 0};
        __syncthreads();
      }
    }
  }

  // ---- 6. eigenvalues, stable sort by modulus
  if (status == 0) {
    if (lane < n) S.lam[lane] = S.A[lane + lane * kLdA];
    __syncthreads();
    if (lane < n) {
      const double me = cabs(S.lam[lane]);
      if (!(me == me)) status = 3;
      int rank = 0;
      for (int i = 0; i < n; ++i) {
        const double o = cabs(S.lam[i]);
        if (o < me || (o == me && i < lane)) ++rank;
      }
      S.order[rank] = lane;
    }
    int bad = status;
    for (int off = kL / 2; off > 0; off >>= 1) bad = max(bad, __shfl_xor(bad, off, kL));
    status = bad;
    __syncthreads();
  }

  if (status == 0) {
    // ---- 7. eigenvectors of T for the k smallest: lane qv back-substitutes
    double tnorm = 0;
    for (int t = lane; t < n * n; t += kL) tnorm = fmax(tnorm, cabs(S.A[(t % n) + (t / n) * kLdA]));
    for (int off = kL / 2; off > 0; off >>= 1) tnorm = fmax(tnorm, __shfl_xor(tnorm, off, kL));
    const double smin = fmax(eps * tnorm, 1e-300);
    if (lane < k) {
      const int p = S.order[lane];
      const C lp = S.lam[p];
      C* y = S.Qs + lane * kMaxM;
      for (int i = 0; i < n; ++i) y[i] = C{i == p ? 1.0 : 0.0, 0.0};
      for (int i = p - 1; i >= 0; --i) {
        C s{0, 0};
        for (int jj = i + 1; jj <= p; ++jj) s += S.A[i + jj * kLdA] * y[jj];
        C den = S.A[i + i * kLdA] - lp;
        if (cabs(den) < smin) den = C{smin, 0.0};
        y[i] = -cdiv(s, den);
      }
    }
    __syncthreads();
    // G_k = Zm Y into A as the first k columns of G_{k+1} ((mm+1) x (k+1), leading dim kLd)
    if (lane <= n) {
      for (int qv = 0; qv < k; ++qv) {
        const int p = S.order[qv];
        const C* y = S.Qs + qv * kMaxM;
        C s{0, 0};
        if (lane < n)
          for (int jj = 0; jj <= p; ++jj) s += S.Zm[lane + jj * kLdA] * y[jj];
        S.A[lane + qv * kLd] = s;
      }
    }
    __syncthreads();
    if (lane < k) {
      double nn = 0;
      for (int i = 0; i < n; ++i) nn += norm2(S.A[i + lane * kLd]);
      const double inv = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
      for (int i = 0; i < n; ++i) S.A[i + lane * kLd] = inv * S.A[i + lane * kLd];
    }
    // ---- 8. last column: the small residual c - H^ eta
    if (lane <= mm) {
      C s = ldc(c, lane);
      for (int jj = 0; jj < mm; ++jj) s -= S.Hs[lane + jj * kLd] * S.eta[jj];
      S.A[lane + k * kLd] = s;
    }
    __syncthreads();
    // ---- 9. QR of G_{k+1}; reflectors into Zm, explicit Q_{k+1} into Qs
    hh_qr(S.A, kLd, mm + 1, k + 1, nullptr, S.Zm, kLd, S.beta);
    if (lane <= k) {
      C* col = S.Qs + lane * kLd;
      for (int i = 0; i <= mm; ++i) col[i] = C{i == lane ? 1.0 : 0.0, 0.0};
      for (int r = k; r >= 0; --r) {
        const double br = S.beta[r];
        if (br == 0.0) continue;
        C sacc{0, 0};
        for (int i = r; i <= mm; ++i) sacc += cdot(S.Zm[i + r * kLd], col[i]);
        sacc = br * sacc;
        for (int i = r; i <= mm; ++i) col[i] -= S.Zm[i + r * kLd] * sacc;
      }
    }
    __syncthreads();
    // ---- 10. H^_k = Q^H H^ Q_k (Q_k = Q(0:mm-1, 0:k-1)); T1 = H^ Q_k into A
    if (lane <= mm) {
      for (int cq = 0; cq < k; ++cq) {
        C s{0, 0};
        for (int jj = 0; jj < mm; ++jj) s += S.Hs[lane + jj * kLd] * S.Qs[jj + cq * kLd];
        S.A[lane + cq * kLd] = s;
      }
    }
    for (int t = lane; t < kLd * kMaxM; t += kL) stc(H, t, C{0, 0});
    __syncthreads();
    __threadfence_block();
    if (lane <= k) {
      for (int cq = 0; cq < k; ++cq) {
        C s{0, 0};
        for (int i = 0; i <= mm; ++i) s += cdot(S.Qs[i + lane * kLd], S.A[i + cq * kLd]);
        stc(H, lane + (long long)cq * kLd, s);
      }
    }
    for (int t = lane; t < (mm + 1) * (k + 1); t += kL) {
      const int i = t % (mm + 1), q = t / (mm + 1);
      stc(Qg, i + (long long)q * kLd, S.Qs[i + q * kLd]);
    }
    if (lane < n) stc(ritz, lane, S.lam[S.order[lane]]);
  }
  if (lane == 0) scal[kSclStatus] = (double)status;
}

template <typename K>
dw_status set_lds(K kernel, size_t bytes) {
  if (bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
      set_error("hipFuncSetAttribute(LDS %zu) failed: %s", bytes, hipGetErrorString(e));
      return DW_EHIP;
    }
  }
  return DW_OK;
}

}  // namespace

dw_status dense_step(double* H, int j, const double* h1, const double* h2, const double* nrm2, const double* c,
                     double* scal, double bd_tol, hipStream_t s) {
  if (j < 0 || j >= kMaxM) {
    set_error("dense_step: column %d out of range", j);
    return DW_EINVAL;
  }
  DW_TRY(set_lds(k_step, sizeof(StepSmem)));
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_step, 1, kL, sizeof(StepSmem), s, H, j, h1, h2, nrm2, c, scal, bd_tol);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

dw_status dense_lsq(const double* H, int cols, const double* c, double* eta, double* scal, hipStream_t s,
                    const int* gate, const int* dn) {
  if (cols < 1 || cols > kMaxM) {
    set_error("dense_lsq: %d columns out of range", cols);
    return DW_EINVAL;
  }
  DW_TRY(set_lds(k_lsq, sizeof(StepSmem)));
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_lsq, 1, kL, sizeof(StepSmem), s, H, cols, c, eta, scal, gate, dn);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

dw_status dense_project(const double* H, int k, const double* t, double* y, double* sv, hipStream_t s,
                        const int* gate) {
  if (k < 1 || k >= kMaxM) {
    set_error("dense_project: k = %d out of range", k);
    return DW_EINVAL;
  }
  DW_TRY(set_lds(k_project, sizeof(StepSmem)));
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_project, 1, kL, sizeof(StepSmem), s, H, k, t, y, sv, gate);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

dw_status dense_deflate(double* H, int mm, int k, const double* c, const double* eta, double* Q, double* ritz,
                        double* scal, hipStream_t s, const int* gate, const int* dn) {
  if (mm < 1 || mm > kMaxM || k < 1 || k >= mm || k + 1 > kQCols) {
    set_error("dense_deflate: unsupported sizes mm %d, k %d", mm, k);
    return DW_EINVAL;
  }
  DW_TRY(set_lds(k_deflate, sizeof(DeflSmem)));
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_deflate, 1, kL, sizeof(DeflSmem), s, H, mm, k, c, eta, Q, ritz, scal, gate, dn);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

dw_status dense_gs_coef(double* H, int nv, int jcol, int jw, int hu, int hw, const double* red, double* coef,
                        double* scal, double bd_tol, hipStream_t s, const int* gate, const int* dcol) {
  (void)bd_tol;
  if (nv < 0 || nv > kLd || jcol > kMaxM || jw >= kMaxM || (hw && jw < 0) || (hu && jcol < 0)) {
    set_error("dense_gs_coef: bad sizes (nv %d, jcol %d, jw %d)", nv, jcol, jw);
    return DW_EINVAL;
  }
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_gs_coef, 1, kL, 0, s, H, nv, jcol, jw, hu, hw, red, coef, scal, gate, dcol);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

dw_status dense_step2(double* H, int j, const double* nrm2, const double* c, double* scal, double bd_tol,
                      hipStream_t s, int* ctl, const double* ctld) {
  if (j < 0 || j >= kMaxM) {
    set_error("dense_step2: column %d out of range", j);
    return DW_EINVAL;
  }
  DW_TRY(set_lds(k_step2, sizeof(StepSmem)));
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_step2, 1, kL, sizeof(StepSmem), s, H, j, nrm2, c, scal, bd_tol, ctl, ctld);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

dw_status dense_fresh(double* H, double* c, const double* nrm2, double* scal, hipStream_t s, const int* gate) {
  KTimer kt(DW_K_DENSE, s);
  hipLaunchKernelGGL(k_fresh, 1, kL, 0, s, H, c, nrm2, scal, gate);
  DW_CHECK_LAUNCH();
  kt.done(0, 0);
  return DW_OK;
}

}  // namespace dw
