// Complex GEMM tile on MFMA: C = beta*C + alpha * op(A) * B, column-major.
//
// One 256-thread workgroup computes a 64x64 tile of C; each of the four
// 64-wide waves owns a 32x32 quarter made of 2x2 MFMA 16x16 blocks, with the
// real and imaginary parts in separate accumulators (4 real MFMAs per
// complex multiply-add).  A and B tiles of depth 16 are staged through LDS.
#pragma once
#include "common.hpp"

namespace bfmf {

constexpr int GEMM_TM = 64, GEMM_TN = 64, GEMM_TK = 16;

template <class T>
struct GemmSmem {
  cplx<T> a[GEMM_TK][GEMM_TM];
  cplx<T> b[GEMM_TK][GEMM_TN];
};

// Computes tile (tm, tn).  opA: OP_N -> A is M x K (lda); OP_T / OP_C -> A is
// stored K x M (lda) and used transposed / conjugate-transposed.  opB: OP_N ->
// B is K x N (ldb); OP_T / OP_C -> B is stored N x K.
template <class T>
__device__ __forceinline__ void gemm_tile(const cplx<T>* __restrict__ A, int64_t lda, int opA,
                                          const cplx<T>* __restrict__ B, int64_t ldb, cplx<T>* __restrict__ C,
                                          int64_t ldc, int M, int N, int K, cplx<T> alpha, int beta, int tm, int tn,
                                          GemmSmem<T>& sm, int opB = OP_N) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int row0 = tm * GEMM_TM, col0 = tn * GEMM_TN;
  acc_t accr[2][2], acci[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        accr[i][j][r] = 0;
        acci[i][j][r] = 0;
      }
  const cplx<T> zero = {0, 0};
  for (int k0 = 0; k0 < K; k0 += GEMM_TK) {
    // stage A: 64 rows x 16 k
    if (opA == OP_N) {
      const int k = tid >> 4, rb = (tid & 15) * 4;
      const int gk = k0 + k;
      for (int q = 0; q < 4; ++q) {
        const int gr = row0 + rb + q;
        sm.a[k][rb + q] = (gk < K && gr < M) ? A[(int64_t)gr + (int64_t)gk * lda] : zero;
      }
    } else {
      const int r = tid >> 2, kb = (tid & 3) * 4;
      const int gr = row0 + r;
      for (int q = 0; q < 4; ++q) {
        const int gk = k0 + kb + q;
        cplx<T> v = (gk < K && gr < M) ? A[(int64_t)gk + (int64_t)gr * lda] : zero;
        if (opA == OP_C) v.im = -v.im;
        sm.a[kb + q][r] = v;
      }
    }
    // stage B: 16 k x 64 cols
    if (opB == OP_N) {
      const int c = tid >> 2, kb = (tid & 3) * 4;
      const int gc = col0 + c;
      for (int q = 0; q < 4; ++q) {
        const int gk = k0 + kb + q;
        sm.b[kb + q][c] = (gk < K && gc < N) ? B[(int64_t)gk + (int64_t)gc * ldb] : zero;
      }
    } else {
      const int k = tid >> 4, cb = (tid & 15) * 4;
      const int gk = k0 + k;
      for (int q = 0; q < 4; ++q) {
        const int gc = col0 + cb + q;
        cplx<T> v = (gk < K && gc < N) ? B[(int64_t)gc + (int64_t)gk * ldb] : zero;
        if (opB == OP_C) v.im = -v.im;
        sm.b[k][cb + q] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GEMM_TK; kk += 4) {
      const int k = kk + (lane >> 4);
      cplx<T> a[2], b[2];
      for (int i = 0; i < 2; ++i) a[i] = sm.a[k][wr + i * 16 + (lane & 15)];
      for (int j = 0; j < 2; ++j) b[j] = sm.b[k][wc + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accr[i][j] = Mfma<T>::step(a[i].re, b[j].re, accr[i][j]);
          accr[i][j] = Mfma<T>::step(-a[i].im, b[j].im, accr[i][j]);
          acci[i][j] = Mfma<T>::step(a[i].re, b[j].im, acci[i][j]);
          acci[i][j] = Mfma<T>::step(a[i].im, b[j].re, acci[i][j]);
        }
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + i * 16 + Mfma<T>::row(lane, r);
        const int gc = col0 + wc + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          const T pr = accr[i][j][r], pi = acci[i][j][r];
          cplx<T> v = {alpha.re * pr - alpha.im * pi, alpha.re * pi + alpha.im * pr};
          cplx<T>* dst = C + (int64_t)gr + (int64_t)gc * ldc;
          if (beta) v = cadd(*dst, v);
          *dst = v;
        }
      }
}

}  // namespace bfmf
