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
#include <type_traits>

#include "dw_internal.hpp"
#include "dw_kernels.hpp"
#include "dw_types.hpp"

namespace dw {

namespace {

constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr int kDotCols = 8;   // columns per multi-dot pass
constexpr int kRotMax = 24;   // output columns of one rotation pass
constexpr int kGsCols = 8;    // columns per pass of the Gram-Schmidt reduction
constexpr int kUpd = 8;       // columns loaded together by the Gram-Schmidt update

__device__ __forceinline__ double wsum(double a) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
  return a;
}

// partials[c * gridDim.x + block] = sum over this block's elements of conj(V_c) w
template <typename SV>
__global__ void __launch_bounds__(kThreads)
    k_dots(const SV* __restrict__ V, long long stride, int ncols, const s64* __restrict__ w, long long n,
           s64* __restrict__ partials, const int* __restrict__ gate, const int* __restrict__ dn, int dadd, int c0) {
  if (gate && *gate == 0) return;
  if (dn) {
    // columns c0.. of a device-side count
    const int left = *dn + dadd - c0;
    if (left <= 0) return;
    ncols = left < kDotCols ? left : kDotCols;
  }
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
    k_reduce(const s64* __restrict__ partials, int G, int ncols, s64* __restrict__ out, int ostride, int op,
             const int* __restrict__ gate, const int* __restrict__ dn, int dmul, int dadd) {
  if (gate && *gate == 0) return;
  if (dn) ncols = dmul * *dn + dadd;
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
    k_scale(const s64* __restrict__ x, s64* __restrict__ y, const double* __restrict__ alpha, long long n,
            const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const double a = alpha[0];
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) st(y + i, a * ld<double>(x + i));
}

// x *= alpha (complex, device)
__global__ void __launch_bounds__(kThreads)
    k_scale_c(s64* __restrict__ x, const s64* __restrict__ alpha, long long n, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const cplx<double> a = ld<double>(alpha);
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) st(x + i, a * ld<double>(x + i));
}

// x += scale * sum_c coef[c] Z_c
template <typename SZ>
__global__ void __launch_bounds__(kThreads)
    k_combine(const SZ* __restrict__ Z, long long stride, int ncols, const s64* __restrict__ coef, double scale,
              s64* __restrict__ x, long long n, const int* __restrict__ gate, const int* __restrict__ dn) {
  if (gate && *gate == 0) return;
  if (dn) ncols = *dn < ncols ? *dn : ncols;
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
    k_rotate(SV* __restrict__ V, long long stride, int nin, const s64* __restrict__ Q, int ldq, int nout, long long n,
             const int* __restrict__ gate, const int* __restrict__ dn, int dadd) {
  if (gate && *gate == 0) return;
  if (dn) nin = *dn + dadd < nin ? *dn + dadd : nin;
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


// ---- Gram-Schmidt with delayed reorthogonalisation ---------------------------
// One reduction sweep computes, over the final basis columns V_0..V_{nv-1},
//   a = V^H u (u: the previous step's once-orthogonalised vector),
//   b = V^H w (w: the new vector A z_j), and u^H u, u^H w, w^H w;
// one update sweep forms v = (u - V a) / beta and w' = w - V b - c v.
// Partial-sum slots: [0, nv) a, [nv, 2 nv) b, 2 nv: u^H u, 2 nv + 1: u^H w,
// 2 nv + 2: w^H w.
// SW: storage of w; T: arithmetic (double, or float for the single-precision
// Arnoldi); the per-workgroup sums are combined in double.
template <bool HU, bool HW, typename SV, typename SW, typename T>
__global__ void __launch_bounds__(kThreads)
    k_gs_reduce(const SV* __restrict__ V, long long stride, int c0, int nc, int nv, const SV* __restrict__ u,
                const SW* __restrict__ w, long long n, int first, s64* __restrict__ partials,
                const int* __restrict__ gate, const int* __restrict__ dcol, int chunk) {
  constexpr int NA = kGsCols;
  if (gate && *gate == 0) return;
  if (dcol) {
    // finalising column nv = *dcol against the nv columns before it: the
    // chunk split of the host-side form, on the device-side count
    nv = *dcol;
    u = V + (long long)nv * stride;
    const int nchunks = nv > 0 ? (nv + NA - 1) / NA : 1;
    if (chunk >= nchunks) return;
    const int per = nv > 0 ? (nv + nchunks - 1) / nchunks : 0;
    c0 = chunk * per;
    nc = nv - c0 < per ? nv - c0 : per;
    first = chunk == 0;
  }
  __shared__ double red[kThreads / kWave][2 * NA + 3][2];
  cplx<T> au[NA], aw[NA], uu = mk<T>(0, 0), uw = mk<T>(0, 0), ww = mk<T>(0, 0);
#pragma unroll
  for (int c = 0; c < NA; ++c) {
    au[c] = mk<T>(0, 0);
    aw[c] = mk<T>(0, 0);
  }
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) {
    cplx<T> uv = mk<T>(0, 0), wv = mk<T>(0, 0);
    if constexpr (HU) uv = ld<T>(u + i);
    if constexpr (HW) wv = ld<T>(w + i);
#pragma unroll
    for (int c = 0; c < NA; ++c)
      if (c < nc) {
        const cplx<T> vc = ld<T>(V + (long long)(c0 + c) * stride + i);
        if constexpr (HU) au[c] += cdot(vc, uv);
        if constexpr (HW) aw[c] += cdot(vc, wv);
      }
    if (first) {
      if constexpr (HU) uu.re += norm2(uv);
      if constexpr (HU && HW) uw += cdot(uv, wv);
      if constexpr (HW) ww.re += norm2(wv);
    }
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  auto put = [&](int slot, cplx<T> v) {
    const double re = wsum((double)v.re), im = wsum((double)v.im);
    if (lane == 0) {
      red[wave][slot][0] = re;
      red[wave][slot][1] = im;
    }
  };
#pragma unroll
  for (int c = 0; c < NA; ++c) {
    if (HU) put(c, au[c]);
    if (HW) put(NA + c, aw[c]);
  }
  put(2 * NA, uu);
  put(2 * NA + 1, uw);
  put(2 * NA + 2, ww);
  __syncthreads();
  const int G = gridDim.x;
  for (int t = threadIdx.x; t < 2 * NA + 3; t += kThreads) {
    int slot;
    if (t < NA) {
      if (!HU || t >= nc) continue;
      slot = c0 + t;
    } else if (t < 2 * NA) {
      if (!HW || t - NA >= nc) continue;
      slot = nv + c0 + (t - NA);
    } else {
      if (!first) continue;
      slot = 2 * nv + (t - 2 * NA);
    }
    double re = 0, im = 0;
    for (int q = 0; q < kThreads / kWave; ++q) {
      re += red[q][t][0];
      im += red[q][t][1];
    }
    partials[(long long)slot * G + blockIdx.x] = s64{re, im};
  }
}

// coef: a[0..nv), b[0..nv), c (slot 2 nv), 1/beta (slot 2 nv + 1, real part).
// HU: V_jcol <- (V_jcol - V a) / beta (in place); HW: wout <- w - V b - c V_jcol,
// partials[block] = sum |wout|^2 over the block's elements.
template <bool HU, bool HW, typename SV, typename SW, typename T>
__global__ void __launch_bounds__(kThreads)
    k_gs_update(SV* __restrict__ V, long long stride, int nv, int jcol, const SW* __restrict__ w,
                SV* __restrict__ wout, const s64* __restrict__ coef, long long n, s64* __restrict__ partials,
                const int* __restrict__ gate, const int* __restrict__ dcol) {
  if (gate && *gate == 0) return;
  if (dcol) nv = jcol = *dcol;
  __shared__ cplx<T> ca[kMaxM + 1], cb[kMaxM + 1];
  __shared__ double red[kThreads / kWave];
  for (int c = threadIdx.x; c < nv; c += kThreads) {
    ca[c] = ld<T>(coef + c);
    cb[c] = ld<T>(coef + nv + c);
  }
  __syncthreads();
  const cplx<T> cj = ld<T>(coef + 2 * nv);
  const T invbeta = (T)coef[2 * nv + 1].x;
  double nrm = 0;
  const long long step = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) {
    cplx<T> uu = mk<T>(0, 0), wa = mk<T>(0, 0);
    if constexpr (HU) uu = ld<T>(V + (long long)jcol * stride + i);
    if constexpr (HW) wa = ld<T>(w + i);
    // columns in groups of kUpd with all loads of a group issued together,
    // so that each thread keeps several HBM reads in flight
    int c = 0;
    for (; c + kUpd <= nv; c += kUpd) {
      cplx<T> vc[kUpd];
#pragma unroll
      for (int q = 0; q < kUpd; ++q) vc[q] = ld<T>(V + (long long)(c + q) * stride + i);
#pragma unroll
      for (int q = 0; q < kUpd; ++q) {
        if constexpr (HU) uu -= ca[c + q] * vc[q];
        if constexpr (HW) wa -= cb[c + q] * vc[q];
      }
    }
    for (; c < nv; ++c) {
      const cplx<T> vc = ld<T>(V + (long long)c * stride + i);
      if constexpr (HU) uu -= ca[c] * vc;
      if constexpr (HW) wa -= cb[c] * vc;
    }
    if constexpr (HU) {
      uu = invbeta * uu;
      st(V + (long long)jcol * stride + i, uu);
      if constexpr (HW) wa -= cj * uu;
    }
    if constexpr (HW) {
      st(wout + i, wa);
      if constexpr (sizeof(SV) == 2 * sizeof(T)) nrm += (double)norm2(wa);  // stored without rounding
      else nrm += norm2(ld<double>(wout + i));                               // the stored, rounded vector
    }
  }
  if constexpr (HW) {
    nrm = wsum(nrm);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) red[wave] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int q = 0; q < kThreads / kWave; ++q) t += red[q];
      partials[blockIdx.x] = s64{t, 0.0};
    }
  }
}

unsigned grid_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b > kBlasGrid) b = kBlasGrid;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

dw_status blas_dots(int prec_v, const void* V, long long stride, int ncols, const double* w, long long n,
                    double* partials, double* out, int ostride, int op, hipStream_t s, const int* gate, const int* dn,
                    int dadd) {
  const unsigned G = grid_for(n);
  for (int c0 = 0; c0 < ncols; c0 += kDotCols) {
    const int nc = ncols - c0 < kDotCols ? ncols - c0 : kDotCols;
    s64* part = (s64*)partials + (long long)c0 * G;
    KTimer kt(DW_K_DOTS, s);
    if (prec_v == DW_PREC_F64)
      hipLaunchKernelGGL(k_dots<s64>, G, kThreads, 0, s, (const s64*)V + c0 * stride, stride, nc, (const s64*)w, n,
                         part, gate, dn, dadd, c0);
    else
      hipLaunchKernelGGL(k_dots<s32>, G, kThreads, 0, s, (const s32*)V + c0 * stride, stride, nc, (const s64*)w, n,
                         part, gate, dn, dadd, c0);
    DW_CHECK_LAUNCH();
    kt.done((double)n * (nc * (double)pair_bytes(prec_v) + 16), (double)n * nc * 8);
  }
  KTimer kr(DW_K_REDUCE, s);
  hipLaunchKernelGGL(k_reduce, 1, kThreads, 0, s, (const s64*)partials, (int)G, ncols, (s64*)out, ostride, op, gate,
                     dn, 1, dadd);
  DW_CHECK_LAUNCH();
  kr.done((double)G * ncols * 16, (double)G * ncols * 2);
  return DW_OK;
}

dw_status blas_sub_cols(const double* V, long long stride, int ncols, const double* h, double* w, long long n,
                        hipStream_t s) {
  if (ncols > 64) {
    set_error("blas_sub_cols: too many columns");
    return DW_EINVAL;
  }
  KTimer kt(DW_K_SUBCOLS, s);
  hipLaunchKernelGGL(k_sub_cols<s64>, grid_for(n), kThreads, 0, s, (const s64*)V, stride, ncols, (const s64*)h, (s64*)w, n);
  DW_CHECK_LAUNCH();
  kt.done((double)n * (ncols + 2) * 16, (double)n * ncols * 8);
  return DW_OK;
}

dw_status blas_scale(const double* x, double* y, const double* alpha, long long n, hipStream_t s, const int* gate) {
  KTimer kt(DW_K_SCALE, s);
  hipLaunchKernelGGL(k_scale, grid_for(n), kThreads, 0, s, (const s64*)x, (s64*)y, alpha, n, gate);
  DW_CHECK_LAUNCH();
  kt.done((double)n * 32, (double)n * 2);
  return DW_OK;
}

dw_status blas_scale_c(double* x, const double* alpha, long long n, hipStream_t s, const int* gate) {
  KTimer kt(DW_K_SCALE, s);
  hipLaunchKernelGGL(k_scale_c, grid_for(n), kThreads, 0, s, (s64*)x, (const s64*)alpha, n, gate);
  DW_CHECK_LAUNCH();
  kt.done((double)n * 32, (double)n * 6);
  return DW_OK;
}

dw_status blas_combine(int prec_z, const void* Z, long long stride, int ncols, const double* coef, double scale,
                       double* x, long long n, hipStream_t s, const int* gate, const int* dn) {
  if (ncols > 64) {
    set_error("blas_combine: too many columns");
    return DW_EINVAL;
  }
  KTimer kt(DW_K_COMBINE, s);
  if (prec_z == DW_PREC_F64)
    hipLaunchKernelGGL(k_combine<s64>, grid_for(n), kThreads, 0, s, (const s64*)Z, stride, ncols, (const s64*)coef, scale, (s64*)x, n, gate, dn);
  else
    hipLaunchKernelGGL(k_combine<s32>, grid_for(n), kThreads, 0, s, (const s32*)Z, stride, ncols, (const s64*)coef, scale, (s64*)x, n, gate, dn);
  DW_CHECK_LAUNCH();
  kt.done((double)n * (ncols * (double)pair_bytes(prec_z) + 32), (double)n * ncols * 8);
  return DW_OK;
}

dw_status blas_rotate(int prec_v, void* V, long long stride, int nin, const double* Q, int ldq, int nout, long long n,
                      hipStream_t s, const int* gate, const int* dn, int dadd) {
  if (nin > 49 || nout > kRotMax || nout > nin) {
    set_error("blas_rotate: unsupported shape %d -> %d", nin, nout);
    return DW_EINVAL;
  }
  KTimer kt(DW_K_ROTATE, s);
  if (prec_v == DW_PREC_F64)
    hipLaunchKernelGGL(k_rotate<s64>, grid_for(n), kThreads, 0, s, (s64*)V, stride, nin, (const s64*)Q, ldq, nout, n, gate, dn, dadd);
  else
    hipLaunchKernelGGL(k_rotate<s32>, grid_for(n), kThreads, 0, s, (s32*)V, stride, nin, (const s64*)Q, ldq, nout, n, gate, dn, dadd);
  DW_CHECK_LAUNCH();
  kt.done((double)n * (nin + nout) * pair_bytes(prec_v), (double)n * nin * nout * 8);
  return DW_OK;
}

}  // namespace dw

namespace dw {

template <typename SV, typename SW, typename T>
dw_status gs_reduce_t(const SV* Vp, long long stride, int nv, const SV* up, const SW* wp, long long n,
                      double* partials, double* out, hipStream_t s, const int* gate, const int* dcol) {
  const bool hu = up != nullptr || dcol != nullptr, hw = wp != nullptr;
  const unsigned G = grid_for(n);
  // the columns in as few passes as possible, split evenly (u and w are
  // re-read by every pass); with dcol the device picks the split of its
  // count and nv bounds it
  const int nchunks = nv > 0 ? (nv + kGsCols - 1) / kGsCols : 1;
  const int per = nv > 0 ? (nv + nchunks - 1) / nchunks : 0;
  for (int q = 0; q < nchunks; ++q) {
    const int c0 = q * per;
    const int nc = nv - c0 < per ? nv - c0 : per;
    KTimer kt(DW_K_DOTS, s);
    s64* part = (s64*)partials;
    if (hu && hw)
      hipLaunchKernelGGL((k_gs_reduce<true, true, SV, SW, T>), G, kThreads, 0, s, Vp, stride, c0, nc, nv, up, wp, n, q == 0,
                         part, gate, dcol, q);
    else if (hu)
      hipLaunchKernelGGL((k_gs_reduce<true, false, SV, SW, T>), G, kThreads, 0, s, Vp, stride, c0, nc, nv, up, wp, n,
                         q == 0, part, gate, dcol, q);
    else
      hipLaunchKernelGGL((k_gs_reduce<false, true, SV, SW, T>), G, kThreads, 0, s, Vp, stride, c0, nc, nv, up, wp, n,
                         q == 0, part, gate, dcol, q);
    DW_CHECK_LAUNCH();
    kt.done((double)n * (sizeof(SV) * (nc + (hu ? 1 : 0)) + (hw ? sizeof(SW) : 0)),
            (double)n * 8 * nc * ((hu ? 1 : 0) + (hw ? 1 : 0)));
  }
  KTimer kr(DW_K_REDUCE, s);
  hipLaunchKernelGGL(k_reduce, 1, kThreads, 0, s, (const s64*)partials, (int)G, 2 * nv + 3, (s64*)out, 1, 0, gate,
                     dcol, 2, 3);
  DW_CHECK_LAUNCH();
  kr.done((double)G * (2 * nv + 3) * 16, 0);
  return DW_OK;
}

dw_status gs_reduce(int prec_v, const void* V, long long stride, int nv, const void* u, const void* w, long long n,
                    double* partials, double* out, hipStream_t s, const int* gate, const int* dcol, int prec_w) {
  if (nv < 0 || nv > kMaxM + 1 || (!u && !w && !dcol) || (prec_v != DW_PREC_F64 && prec_v != DW_PREC_F32) ||
      (prec_w == DW_PREC_F32 && prec_v != DW_PREC_F32) || (prec_w != DW_PREC_F64 && prec_w != DW_PREC_F32)) {
    set_error("gs_reduce: bad arguments");
    return DW_EINVAL;
  }
  if (prec_w == DW_PREC_F32)
    return gs_reduce_t<s32, s32, float>((const s32*)V, stride, nv, (const s32*)u, (const s32*)w, n, partials, out, s,
                                        gate, dcol);
  if (prec_v == DW_PREC_F64)
    return gs_reduce_t<s64, s64, double>((const s64*)V, stride, nv, (const s64*)u, (const s64*)w, n, partials, out,
                                         s, gate, dcol);
  return gs_reduce_t<s32, s64, double>((const s32*)V, stride, nv, (const s32*)u, (const s64*)w, n, partials, out, s,
                                       gate, dcol);
}

template <typename SV, typename SW, typename T>
dw_status gs_update_t(SV* Vp, long long stride, int nv, int jcol, const SW* w, SV* wout, const double* coef,
                      long long n, double* partials, double* nrm2, hipStream_t s, const int* gate, const int* dcol) {
  const bool hu = jcol >= 0 || dcol != nullptr, hw = w != nullptr;
  const unsigned G = grid_for(n);
  KTimer kt(DW_K_SUBCOLS, s);
  if (hu && hw)
    hipLaunchKernelGGL((k_gs_update<true, true, SV, SW, T>), G, kThreads, 0, s, Vp, stride, nv, jcol, w, wout,
                       (const s64*)coef, n, (s64*)partials, gate, dcol);
  else if (hu)
    hipLaunchKernelGGL((k_gs_update<true, false, SV, SW, T>), G, kThreads, 0, s, Vp, stride, nv, jcol, w, wout,
                       (const s64*)coef, n, (s64*)partials, gate, dcol);
  else
    hipLaunchKernelGGL((k_gs_update<false, true, SV, SW, T>), G, kThreads, 0, s, Vp, stride, nv, jcol, w, wout,
                       (const s64*)coef, n, (s64*)partials, gate, dcol);
  DW_CHECK_LAUNCH();
  kt.done((double)n * (sizeof(SV) * (nv + (hu ? 2 : 0) + (hw ? 1 : 0)) + (hw ? sizeof(SW) : 0)),
          (double)n * 8 * nv * ((hu ? 1 : 0) + (hw ? 1 : 0)));
  if (hw) {
    KTimer kr(DW_K_REDUCE, s);
    hipLaunchKernelGGL(k_reduce, 1, kThreads, 0, s, (const s64*)partials, (int)G, 1, (s64*)nrm2, 1, 0, gate,
                       (const int*)nullptr, 0, 0);
    DW_CHECK_LAUNCH();
    kr.done((double)G * 16, 0);
  }
  return DW_OK;
}

dw_status gs_update(int prec_v, void* V, long long stride, int nv, int jcol, const void* w, void* wout,
                    const double* coef, long long n, double* partials, double* nrm2, hipStream_t s, const int* gate,
                    const int* dcol, int prec_w) {
  if (nv < 0 || nv > kMaxM + 1 || (jcol < 0 && !w && !dcol) || (prec_v != DW_PREC_F64 && prec_v != DW_PREC_F32) ||
      (prec_w == DW_PREC_F32 && prec_v != DW_PREC_F32) || (prec_w != DW_PREC_F64 && prec_w != DW_PREC_F32)) {
    set_error("gs_update: bad arguments");
    return DW_EINVAL;
  }
  if (prec_w == DW_PREC_F32)
    return gs_update_t<s32, s32, float>((s32*)V, stride, nv, jcol, (const s32*)w, (s32*)wout, coef, n, partials,
                                        nrm2, s, gate, dcol);
  if (prec_v == DW_PREC_F64)
    return gs_update_t<s64, s64, double>((s64*)V, stride, nv, jcol, (const s64*)w, (s64*)wout, coef, n, partials,
                                         nrm2, s, gate, dcol);
  return gs_update_t<s32, s64, double>((s32*)V, stride, nv, jcol, (const s64*)w, (s32*)wout, coef, n, partials,
                                       nrm2, s, gate, dcol);
}

}  // namespace dw
