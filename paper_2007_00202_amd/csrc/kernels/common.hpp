// Device-side helpers shared by the HIP kernels: interleaved complex values
// and the MFMA fragment layouts of gfx950.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfmf {

template <class T>
struct cplx {
  T re, im;
};

template <class T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <class T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
// a / b by scaling with the larger component of b (Smith's algorithm)
template <class T>
__device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  T ar = fabs(b.re), ai = fabs(b.im);
  if (ar >= ai) {
    T r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  T r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
template <class T>
__device__ __forceinline__ T cabs1(cplx<T> a) {
  return fabs(a.re) + fabs(a.im);
}

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// One 16x16x4 real MFMA step.  Operand layout (both precisions): lane l holds
// A(row l%16, k l/16) and B(k l/16, col l%16).  Result layout (measured on
// gfx950): f32 lane l item r holds D(4*(l/16)+r, l%16); f64 lane l item r
// holds D(l/16 + 4*r, l%16).
template <class T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4_t acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return lane / 16 + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef f4_t acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

}  // namespace bfmf
