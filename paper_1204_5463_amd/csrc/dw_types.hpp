// Complex arithmetic and storage formats for the Wilson-Dirac kernels.
//
// Fields are stored as arrays of complex pairs in one of four storage
// formats (FP64, FP32, FP16, BF16). Kernels load a pair, convert it to the
// compute type (double or float) and convert back when storing.
// Conversions from a wider to a narrower format round to nearest even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dw {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T>& operator+=(cplx<T>& a, cplx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T>& operator-=(cplx<T>& a, cplx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cdot(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// acc += a b and acc -= a b as four fused multiply-adds (one rounding per term)
template <typename T>
__host__ __device__ __forceinline__ void cmac(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
template <typename T>
__host__ __device__ __forceinline__ void cmsub(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(-a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(-a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// multiply by +i and -i
template <typename T>
__host__ __device__ __forceinline__ cplx<T> mul_i(cplx<T> a) { return {-a.im, a.re}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) { return {a.im, -a.re}; }

// ---- storage formats -------------------------------------------------------

struct __attribute__((aligned(16))) s64 { double x, y; };
struct __attribute__((aligned(8))) s32 { float x, y; };
struct __attribute__((aligned(4))) s16 { _Float16 x, y; };
struct __attribute__((aligned(4))) sbf { uint16_t x, y; };

__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// round to nearest even; NaN stays NaN
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename S>
struct storage_traits;

template <>
struct storage_traits<s64> {
  template <typename T>
  __device__ static __forceinline__ cplx<T> load(const s64& s) { return {(T)s.x, (T)s.y}; }
  template <typename T>
  __device__ static __forceinline__ s64 store(cplx<T> c) { return s64{(double)c.re, (double)c.im}; }
};
template <>
struct storage_traits<s32> {
  template <typename T>
  __device__ static __forceinline__ cplx<T> load(const s32& s) { return {(T)s.x, (T)s.y}; }
  template <typename T>
  __device__ static __forceinline__ s32 store(cplx<T> c) { return s32{(float)c.re, (float)c.im}; }
};
template <>
struct storage_traits<s16> {
  template <typename T>
  __device__ static __forceinline__ cplx<T> load(const s16& s) { return {(T)(float)s.x, (T)(float)s.y}; }
  template <typename T>
  __device__ static __forceinline__ s16 store(cplx<T> c) { return s16{(_Float16)(float)c.re, (_Float16)(float)c.im}; }
};
template <>
struct storage_traits<sbf> {
  template <typename T>
  __device__ static __forceinline__ cplx<T> load(const sbf& s) { return {(T)bf16_to_f32(s.x), (T)bf16_to_f32(s.y)}; }
  template <typename T>
  __device__ static __forceinline__ sbf store(cplx<T> c) { return sbf{f32_to_bf16((float)c.re), f32_to_bf16((float)c.im)}; }
};

template <typename T, typename S>
__device__ __forceinline__ cplx<T> ld(const S* p) { return storage_traits<S>::template load<T>(*p); }

// Streaming (non-temporal) load and store of one complex pair: for data read
// or written once per kernel, so that it does not evict reused data from
// the caches. The pair moves as one vector of its own size.
template <int BYTES> struct nt_vec;
template <> struct nt_vec<16> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct nt_vec<8> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct nt_vec<4> { typedef uint32_t type; };

template <typename S>
__device__ __forceinline__ S ld_nt_raw(const S* p) {
  using V = typename nt_vec<sizeof(S)>::type;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  S s;
  __builtin_memcpy(&s, &v, sizeof(S));
  return s;
}
template <typename T, typename S>
__device__ __forceinline__ cplx<T> ld_nt(const S* p) { return storage_traits<S>::template load<T>(ld_nt_raw(p)); }
template <typename T, typename S>
__device__ __forceinline__ void st_nt(S* p, cplx<T> c) {
  using V = typename nt_vec<sizeof(S)>::type;
  const S s = storage_traits<S>::template store<T>(c);
  V v;
  __builtin_memcpy(&v, &s, sizeof(S));
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}
template <typename T, typename S>
__device__ __forceinline__ void st(S* p, cplx<T> c) { *p = storage_traits<S>::template store<T>(c); }

}  // namespace dw
