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

// Device-memory access through the global address space.  A generic (flat)
// access also counts against the LDS wait counter, so in a kernel that mixes
// memory and LDS traffic every wait for an LDS result would wait for the
// memory accesses in flight as well.  The pointer is made from the address's
// integer value (a cast between pointer types can be dropped again by the
// optimizer); complex values move component by component.
template <class T>
using gmem_t = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const gmem_t<T>*)(uintptr_t)p;
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(gmem_t<T>*)(uintptr_t)p = v;
}
template <class T>
__device__ __forceinline__ cplx<T> gld(const cplx<T>* p) {
  const gmem_t<T>* q = (const gmem_t<T>*)(uintptr_t)p;
  return cplx<T>{q[0], q[1]};
}
template <class T>
__device__ __forceinline__ void gst(cplx<T>* p, cplx<T> v) {
  gmem_t<T>* q = (gmem_t<T>*)(uintptr_t)p;
  q[0] = v.re;
  q[1] = v.im;
}

// Workgroups are handed to the chip's 8 XCDs in turn (block b to XCD b mod 8), each with its own L2. Runs of
// XCD_RUN consecutive tiles, which mostly belong to one task and share its operand panels, are given to
// one XCD; the runs still alternate between XCDs, so the load stays balanced. A bijection of
// [0, nb): blocks past the last whole group of 8 runs keep their own tile.
constexpr int64_t XCDS = 8, XCD_RUN = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t full = nb / (XCDS * XCD_RUN) * (XCDS * XCD_RUN);
  if (b >= full) return b;
  const int64_t x = b % XCDS, j = b / XCDS;
  return (x + XCDS * (j / XCD_RUN)) * XCD_RUN + j % XCD_RUN;
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
