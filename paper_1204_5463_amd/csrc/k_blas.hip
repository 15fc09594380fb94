// Long-vector kernels of the flexible Arnoldi process and the deflated
// restart (paper Section 4): block inner products V^H w, column updates
// w -= V h, combinations x += Z eta and in-place basis rotations V <- V Q.
//
// Vectors are complex FP64 (the Krylov basis V, residuals, iterate) or FP32
// (the preconditioned basis Z at low SAP precision), stored as flat arrays
// of complex pairs; columns of a basis are `stride` pairs apart.
// All reductions are two-stage with a fixed grid and a fixed summation
// order, so results are bitwise reproducible run to run.
// Every kernel streams each column once: they are HBM-bandwidth bound.
#include "dw_internal.hpp"
#include "dw_kernels.hpp"
#include "dw_types.hpp"

namespace dw {

namespace {

constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr int kDotCols = 8;   // columns per multi-dot pass
constexpr int kRotMax = 24;   // output columns of one rotation pass

__device__ __forceinline__ double wsum(double a) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
  return a;
}

// partials[c * gridDim.x + block] = sum over this block's elements of conj(V_c) w
template <typename SV>
__global__ void __launch_bounds__(kThreads)
    k_dots(const SV* __restrict__ V, long long stride, int ncols, const s64* __restrict__ w, long long n,
           s64* __restrict__ partials) {
  __shared__ double red[kThreads / kWave][kDotCols][2];
  cplx<double> acc[kDotCols];
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) acc[c] = mk(0.0, 0.0);
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) {
    cplx<double> wv = ld<double>(w + i);
#pragma unroll
    for (int c = 0; c < kDotCols; ++c)
      if (c < ncols) acc[c] += cdot(ld<double>(V + c * stride + i), wv);
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) {
    double re = wsum(acc[c].re), im = wsum(acc[c].im);
    if (lane == 0) {
      red[wave][c][0] = re;
      red[wave][c][1] = im;
    }
  }
  __syncthreads();
  if (threadIdx.x < ncols) {
    const int c = threadIdx.x;
    double re = 0, im = 0;
    for (int q = 0; q < kThreads / kWave; ++q) {
      re += red[q][c][0];
      im += red[q][c][1];
    }
    partials[(long long)c * gridDim.x + blockIdx.x] = s64{re, im};
  }
}

// out[c*ostride] (op 0: =, op 1: +=) sum_g partials[c*G + g]; one wave per column
__global__ void __launch_bounds__(kThreads)
    k_reduce(const s64* __restrict__ partials, int G, int ncols, s64* __restrict__ out, int ostride, int op) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (int c = wave; c < ncols; c += kThreads / kWave) {
    double re = 0, im = 0;
    for (int g = lane; g < G; g += kWave) {
      re += partials[(long long)c * G + g].x;
      im += partials[(long long)c * G + g].y;
    }
    re = wsum(re);
    im = wsum(im);
    if (lane == 0) {
      s64* o = out + (long long)c * ostride;
      if (op == 1) {
        re += o->x;
        im += o->y;
      }
      *o = s64{re, im};
    }
  }
}

// w -= sum_c h[c] V_c   (h on the device)
template <typename SV>
__global__ void __launch_bounds__(kThreads)
    k_sub_cols(const SV* __restrict__ V, long long stride, int ncols, const s64* __restrict__ h, s64* __restrict__ w,
               long long n) {
  __shared__ cplx<double> hs[64];
  for (int c = threadIdx.x; c < ncols; c += kThreads) hs[c] = ld<double>(h + c);
  __syncthreads();
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) {
    cplx<double> a = ld<double>(w + i);
    for (int c = 0; c < ncols; ++c) a -= hs[c] * ld<double>(V + c * stride + i);
    st(w + i, a);
  }
}

// y = x * (alpha[0] if alpha_is_inv == 0 else 1/alpha[0]) with alpha a device
// scalar stored as the real part of a complex pair
__global__ void __launch_bounds__(kThreads)
    k_scale(const s64* __restrict__ x, s64* __restrict__ y, const double* __restrict__ alpha, long long n) {
  const double a = alpha[0];
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) st(y + i, a * ld<double>(x + i));
}

// x += scale * sum_c coef[c] Z_c
template <typename SZ>
__global__ void __launch_bounds__(kThreads)
    k_combine(const SZ* __restrict__ Z, long long stride, int ncols, const s64* __restrict__ coef, double scale,
              s64* __restrict__ x, long long n) {
  __shared__ cplx<double> cs[64];
  for (int c = threadIdx.x; c < ncols; c += kThreads) cs[c] = scale * ld<double>(coef + c);
  __syncthreads();
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) {
    cplx<double> a = ld<double>(x + i);
    for (int c = 0; c < ncols; ++c) a += cs[c] * ld<double>(Z + c * stride + i);
    st(x + i, a);
  }
}

// in place: V_c <- sum_{i<nin} V_i Q[i + c*ldq] for c < nout (nout <= kRotMax).
// Each thread reads all nin inputs of its element before writing any output.
template <typename SV>
__global__ void __launch_bounds__(kThreads)
    k_rotate(SV* __restrict__ V, long long stride, int nin, const s64* __restrict__ Q, int ldq, int nout, long long n) {
  __shared__ cplx<double> qs[49 * kRotMax];
  for (int t = threadIdx.x; t < nin * nout; t += kThreads) {
    const int i = t % nin, c = t / nin;
    qs[c * 49 + i] = ld<double>(Q + i + (long long)c * ldq);
  }
  __syncthreads();
  const long long step = (long long)gridDim.x * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n; e += step) {
    cplx<double> acc[kRotMax];
#pragma unroll
    for (int c = 0; c < kRotMax; ++c) acc[c] = mk(0.0, 0.0);
    for (int i = 0; i < nin; ++i) {
      const cplx<double> v = ld<double>(V + i * stride + e);
#pragma unroll
      for (int c = 0; c < kRotMax; ++c)
        if (c < nout) acc[c] += v * qs[c * 49 + i];
    }
#pragma unroll
    for (int c = 0; c < kRotMax; ++c)
      if (c < nout) st(V + c * stride + e, acc[c]);
  }
}

unsigned grid_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b > kBlasGrid) b = kBlasGrid;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

dw_status blas_dots(int prec_v, const void* V, long long stride, int ncols, const double* w, long long n,
                    double* partials, double* out, int ostride, int op, hipStream_t s) {
  const unsigned G = grid_for(n);
  for (int c0 = 0; c0 < ncols; c0 += kDotCols) {
    const int nc = ncols - c0 < kDotCols ? ncols - c0 : kDotCols;
    s64* part = (s64*)partials + (long long)c0 * G;
    if (prec_v == DW_PREC_F64)
      hipLaunchKernelGGL(k_dots<s64>, G, kThreads, 0, s, (const s64*)V + c0 * stride, stride, nc, (const s64*)w, n, part);
    else
      hipLaunchKernelGGL(k_dots<s32>, G, kThreads, 0, s, (const s32*)V + c0 * stride, stride, nc, (const s64*)w, n, part);
    DW_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_reduce, 1, kThreads, 0, s, (const s64*)partials, (int)G, ncols, (s64*)out, ostride, op);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

dw_status blas_sub_cols(const double* V, long long stride, int ncols, const double* h, double* w, long long n,
                        hipStream_t s) {
  if (ncols > 64) {
    set_error("blas_sub_cols: too many columns");
    return DW_EINVAL;
  }
  hipLaunchKernelGGL(k_sub_cols<s64>, grid_for(n), kThreads, 0, s, (const s64*)V, stride, ncols, (const s64*)h, (s64*)w, n);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

dw_status blas_scale(const double* x, double* y, const double* alpha, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, grid_for(n), kThreads, 0, s, (const s64*)x, (s64*)y, alpha, n);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

dw_status blas_combine(int prec_z, const void* Z, long long stride, int ncols, const double* coef, double scale,
                       double* x, long long n, hipStream_t s) {
  if (ncols > 64) {
    set_error("blas_combine: too many columns");
    return DW_EINVAL;
  }
  if (prec_z == DW_PREC_F64)
    hipLaunchKernelGGL(k_combine<s64>, grid_for(n), kThreads, 0, s, (const s64*)Z, stride, ncols, (const s64*)coef, scale, (s64*)x, n);
  else
    hipLaunchKernelGGL(k_combine<s32>, grid_for(n), kThreads, 0, s, (const s32*)Z, stride, ncols, (const s64*)coef, scale, (s64*)x, n);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

dw_status blas_rotate(int prec_v, void* V, long long stride, int nin, const double* Q, int ldq, int nout, long long n,
                      hipStream_t s) {
  if (nin > 49 || nout > kRotMax || nout > nin) {
    set_error("blas_rotate: unsupported shape %d -> %d", nin, nout);
    return DW_EINVAL;
  }
  if (prec_v == DW_PREC_F64)
    hipLaunchKernelGGL(k_rotate<s64>, grid_for(n), kThreads, 0, s, (s64*)V, stride, nin, (const s64*)Q, ldq, nout, n);
  else
    hipLaunchKernelGGL(k_rotate<s32>, grid_for(n), kThreads, 0, s, (s32*)V, stride, nin, (const s64*)Q, ldq, nout, n);
  DW_CHECK_LAUNCH();
  return DW_OK;
}

}  // namespace dw
