// Layout and precision conversion kernels: canonical complex128 fields to
// and from the internal block-tiled layout, and elementwise conversions.
#include "dw_internal.hpp"
#include "dw_types.hpp"

namespace dw {

namespace {

constexpr int kThreads = 256;

// one thread per (internal site, rhs): reads the site's 12 canonical
// complex numbers, writes 12 coalesced internal entries
template <typename S>
__global__ void __launch_bounds__(kThreads) k_pack_spinor(Geom g, const s64* __restrict__ in, S* __restrict__ out,
                                                          double scale, const double* __restrict__ dscale,
                                                          int dstride) {
  long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= g.V) return;
  if (dscale) scale *= dscale[(long long)blockIdx.y * dstride];
  const long long rhs_off = (long long)blockIdx.y * g.V * 12;
  const int b = (int)(s / g.bvol);
  const int l = (int)(s - (long long)b * g.bvol);
  const long long n = canonical_site(g, b, l);
  const s64* src = in + rhs_off + n * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cplx<double> v = ld<double>(src + c);
    st(out + rhs_off + spinor_index(g, b, c, l), scale * v);
  }
}

template <typename S>
__global__ void __launch_bounds__(kThreads) k_unpack_spinor(Geom g, const S* __restrict__ in, s64* __restrict__ out,
                                                            double scale, const double* __restrict__ dscale,
                                                            int dstride) {
  long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= g.V) return;
  if (dscale) scale *= dscale[(long long)blockIdx.y * dstride];
  const long long rhs_off = (long long)blockIdx.y * g.V * 12;
  const int b = (int)(s / g.bvol);
  const int l = (int)(s - (long long)b * g.bvol);
  const long long n = canonical_site(g, b, l);
  s64* dst = out + rhs_off + n * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cplx<double> v = ld<double>(in + rhs_off + spinor_index(g, b, c, l));
    st(dst + c, scale * v);
  }
}

template <typename S>
__global__ void __launch_bounds__(kThreads) k_pack_gauge(Geom g, const s64* __restrict__ in, S* __restrict__ out) {
  long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= g.V) return;
  const int b = (int)(s / g.bvol);
  const int l = (int)(s - (long long)b * g.bvol);
  const long long n = canonical_site(g, b, l);
  for (int mu = 0; mu < 4; ++mu) {
    const s64* src = in + ((long long)mu * g.V + n) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) st(out + gauge_index(g, b, mu, e, l), ld<double>(src + e));
  }
}

template <typename SI, typename SO>
__global__ void __launch_bounds__(kThreads) k_convert(const SI* __restrict__ in, SO* __restrict__ out, double scale,
                                                      const double* __restrict__ dscale, long long n,
                                                      const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  if (dscale) scale *= dscale[0];
  long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long stride = (long long)gridDim.x * kThreads;
  for (; i < n; i += stride) st(out + i, scale * ld<double>(in + i));
}

dim3 site_grid(const Geom& g, int nrhs) { return dim3((unsigned)((g.V + kThreads - 1) / kThreads), (unsigned)nrhs); }

}  // namespace

dw_status launch_pack_spinor(const Geom& g, int prec, const double* in, void* out, double scale, int nrhs,
                             hipStream_t s, const double* dscale, int dstride) {
  const s64* src = reinterpret_cast<const s64*>(in);
  dim3 grid = site_grid(g, nrhs);
  KTimer kt(DW_K_CONVERT, s);
  switch (prec) {
    case DW_PREC_F64: hipLaunchKernelGGL(k_pack_spinor<s64>, grid, kThreads, 0, s, g, src, (s64*)out, scale, dscale, dstride); break;
    case DW_PREC_F32: hipLaunchKernelGGL(k_pack_spinor<s32>, grid, kThreads, 0, s, g, src, (s32*)out, scale, dscale, dstride); break;
    case DW_PREC_F16: hipLaunchKernelGGL(k_pack_spinor<s16>, grid, kThreads, 0, s, g, src, (s16*)out, scale, dscale, dstride); break;
    case DW_PREC_BF16: hipLaunchKernelGGL(k_pack_spinor<sbf>, grid, kThreads, 0, s, g, src, (sbf*)out, scale, dscale, dstride); break;
    default: set_error("unknown precision %d", prec); return DW_EINVAL;
  }
  DW_CHECK_LAUNCH();
  kt.done((double)g.V * 12 * nrhs * (16 + pair_bytes(prec)), 0);
  return DW_OK;
}

dw_status launch_unpack_spinor(const Geom& g, int prec, const void* in, double* out, double scale, int nrhs,
                               hipStream_t s, const double* dscale, int dstride) {
  s64* dst = reinterpret_cast<s64*>(out);
  dim3 grid = site_grid(g, nrhs);
  KTimer kt(DW_K_CONVERT, s);
  switch (prec) {
    case DW_PREC_F64: hipLaunchKernelGGL(k_unpack_spinor<s64>, grid, kThreads, 0, s, g, (const s64*)in, dst, scale, dscale, dstride); break;
    case DW_PREC_F32: hipLaunchKernelGGL(k_unpack_spinor<s32>, grid, kThreads, 0, s, g, (const s32*)in, dst, scale, dscale, dstride); break;
    case DW_PREC_F16: hipLaunchKernelGGL(k_unpack_spinor<s16>, grid, kThreads, 0, s, g, (const s16*)in, dst, scale, dscale, dstride); break;
    case DW_PREC_BF16: hipLaunchKernelGGL(k_unpack_spinor<sbf>, grid, kThreads, 0, s, g, (const sbf*)in, dst, scale, dscale, dstride); break;
    default: set_error("unknown precision %d", prec); return DW_EINVAL;
  }
  DW_CHECK_LAUNCH();
  kt.done((double)g.V * 12 * nrhs * (16 + pair_bytes(prec)), 0);
  return DW_OK;
}

dw_status launch_pack_gauge(const Geom& g, int prec, const double* in, void* out, hipStream_t s) {
  const s64* src = reinterpret_cast<const s64*>(in);
  dim3 grid = site_grid(g, 1);
  KTimer kt(DW_K_CONVERT, s);
  switch (prec) {
    case DW_PREC_F64: hipLaunchKernelGGL(k_pack_gauge<s64>, grid, kThreads, 0, s, g, src, (s64*)out); break;
    case DW_PREC_F32: hipLaunchKernelGGL(k_pack_gauge<s32>, grid, kThreads, 0, s, g, src, (s32*)out); break;
    case DW_PREC_F16: hipLaunchKernelGGL(k_pack_gauge<s16>, grid, kThreads, 0, s, g, src, (s16*)out); break;
    case DW_PREC_BF16: hipLaunchKernelGGL(k_pack_gauge<sbf>, grid, kThreads, 0, s, g, src, (sbf*)out); break;
    default: set_error("unknown precision %d", prec); return DW_EINVAL;
  }
  DW_CHECK_LAUNCH();
  kt.done((double)g.V * 36 * (16 + pair_bytes(prec)), 0);
  return DW_OK;
}

namespace {
template <typename SI>
dw_status convert_from(const SI* in, int pout, void* out, double scale, const double* ds, long long n,
                       hipStream_t s, const int* gate) {
  long long nb = (n + kThreads - 1) / kThreads;
  unsigned grid = (unsigned)(nb < 8192 ? (nb > 0 ? nb : 1) : 8192);
  KTimer kt(DW_K_CONVERT, s);
  switch (pout) {
    case DW_PREC_F64: hipLaunchKernelGGL((k_convert<SI, s64>), grid, kThreads, 0, s, in, (s64*)out, scale, ds, n, gate); break;
    case DW_PREC_F32: hipLaunchKernelGGL((k_convert<SI, s32>), grid, kThreads, 0, s, in, (s32*)out, scale, ds, n, gate); break;
    case DW_PREC_F16: hipLaunchKernelGGL((k_convert<SI, s16>), grid, kThreads, 0, s, in, (s16*)out, scale, ds, n, gate); break;
    case DW_PREC_BF16: hipLaunchKernelGGL((k_convert<SI, sbf>), grid, kThreads, 0, s, in, (sbf*)out, scale, ds, n, gate); break;
    default: set_error("unknown precision %d", pout); return DW_EINVAL;
  }
  DW_CHECK_LAUNCH();
  kt.done((double)n * (sizeof(SI) + pair_bytes(pout)), 0);
  return DW_OK;
}
}  // namespace

dw_status launch_convert(int pin, const void* in, int pout, void* out, double scale, long long n, hipStream_t s,
                         const double* dscale, const int* gate) {
  switch (pin) {
    case DW_PREC_F64: return convert_from((const s64*)in, pout, out, scale, dscale, n, s, gate);
    case DW_PREC_F32: return convert_from((const s32*)in, pout, out, scale, dscale, n, s, gate);
    case DW_PREC_F16: return convert_from((const s16*)in, pout, out, scale, dscale, n, s, gate);
    case DW_PREC_BF16: return convert_from((const sbf*)in, pout, out, scale, dscale, n, s, gate);
    default: set_error("unknown precision %d", pin); return DW_EINVAL;
  }
}

}  // namespace dw
