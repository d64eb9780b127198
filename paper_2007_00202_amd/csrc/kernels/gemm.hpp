// Complex GEMM tile on MFMA: C = beta*C + alpha * op(A) * B, column-major.
//
// One 256-thread workgroup computes a 64x64 tile of C; each of the four
// 64-wide waves owns a 32x32 quarter made of 2x2 MFMA 16x16 blocks, with the
// real and imaginary parts in separate accumulators (4 real MFMAs per
// complex multiply-add).  A and B tiles of depth 16 are staged through LDS,
// the next one prefetched into registers while the current one is used.
#pragma once
#include "common.hpp"

namespace bfmf {

constexpr int GEMM_TM = 64, GEMM_TN = 64, GEMM_TK = 16;

// *p when ok, else 0 (a guarded load: a select between the global address and
// a local zero would put the zero in scratch memory)
template <class T>
__device__ __forceinline__ cplx<T> load_or_zero(const cplx<T>* p, bool ok) {
  cplx<T> v = {0, 0};
  if (ok) v = *p;
  return v;
}

template <class TO, class TI>
__device__ __forceinline__ cplx<TO> to_cplx(cplx<TI> v) {
  return cplx<TO>{(TO)v.re, (TO)v.im};
}

template <class T>
struct GemmSmem {
  cplx<T> a[GEMM_TK][GEMM_TM];
  cplx<T> b[GEMM_TK][GEMM_TN];
};

// Computes tile (tm, tn).  opA: OP_N -> A is M x K (lda); OP_T / OP_C -> A is
// stored K x M (lda) and used transposed / conjugate-transposed.  opB: OP_N ->
// B is K x N (ldb); OP_T / OP_C -> B is stored N x K.
// TL is the storage type of A, B and C; T that of the arithmetic (MFMA and
// accumulation): with TL = double and T = float the operands are rounded to
// complex64 as they are staged and the tile is added to C in double.
template <class T, class TL = T>
__device__ __forceinline__ void gemm_tile(const cplx<TL>* __restrict__ A, int64_t lda, int opA,
                                          const cplx<TL>* __restrict__ B, int64_t ldb, cplx<TL>* __restrict__ C,
                                          int64_t ldc, int M, int N, int K, cplx<T> alpha, int beta, int tm, int tn,
                                          GemmSmem<T>& sm, int opB = OP_N) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int row0 = tm * GEMM_TM, col0 = tn * GEMM_TN;
  acc_t accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accr[i][j][r] = 0;
        acci[i][j][r] = 0;
      }
  // Each thread stages 4 A and 4 B entries per k-block of depth 16.  The
  // next block is fetched into registers before the MFMAs of the current
  // block run, so its global-memory latency overlaps the arithmetic.
  cplx<T> ra[4], rb[4];
  auto fetch = [&](int k0) {
    if (opA == OP_N) {
      const int k = tid >> 4, rb0 = (tid & 15) * 4;
      const int gk = k0 + k;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = row0 + rb0 + q;
        ra[q] = to_cplx<T>(load_or_zero(A + (int64_t)gr + (int64_t)gk * lda, gk < K && gr < M));
      }
    } else {
      const int r = tid >> 2, kb = (tid & 3) * 4;
      const int gr = row0 + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gk = k0 + kb + q;
        cplx<T> v = to_cplx<T>(load_or_zero(A + (int64_t)gk + (int64_t)gr * lda, gk < K && gr < M));
        if (opA == OP_C) v.im = -v.im;
        ra[q] = v;
      }
    }
    if (opB == OP_N) {
      const int c = tid >> 2, kb = (tid & 3) * 4;
      const int gc = col0 + c;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gk = k0 + kb + q;
        rb[q] = to_cplx<T>(load_or_zero(B + (int64_t)gk + (int64_t)gc * ldb, gk < K && gc < N));
      }
    } else {
      const int k = tid >> 4, cb = (tid & 15) * 4;
      const int gk = k0 + k;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gc = col0 + cb + q;
        cplx<T> v = to_cplx<T>(load_or_zero(B + (int64_t)gc + (int64_t)gk * ldb, gk < K && gc < N));
        if (opB == OP_C) v.im = -v.im;
        rb[q] = v;
      }
    }
  };
  auto stage = [&]() {
    if (opA == OP_N) {
      const int k = tid >> 4, rb0 = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.a[k][rb0 + q] = ra[q];
    } else {
      const int r = tid >> 2, kb = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.a[kb + q][r] = ra[q];
    }
    if (opB == OP_N) {
      const int c = tid >> 2, kb = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.b[kb + q][c] = rb[q];
    } else {
      const int k = tid >> 4, cb = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.b[k][cb + q] = rb[q];
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += GEMM_TK) {
    stage();
    __syncthreads();
    if (k0 + GEMM_TK < K) fetch(k0 + GEMM_TK);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < GEMM_TK; kk += 4) {
      const int k = kk + (lane >> 4);
      cplx<T> a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sm.a[k][wr + i * 16 + (lane & 15)];
#pragma unroll
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
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + i * 16 + Mfma<T>::row(lane, r);
        const int gc = col0 + wc + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          const T pr = accr[i][j][r], pi = acci[i][j][r];
          const cplx<T> v = {alpha.re * pr - alpha.im * pi, alpha.re * pi + alpha.im * pr};
          cplx<TL>* dst = C + (int64_t)gr + (int64_t)gc * ldc;
          cplx<TL> w = to_cplx<TL>(v);
          if (beta) w = cadd(*dst, w);
          *dst = w;
        }
      }
}

// ------------------------------------------------------------ tile shapes
// The grouped GEMM of butterfly products runs one of several tile shapes
// per launch.  A 256-thread workgroup (four waves) computes a TM x TN tile of
// C; the waves form a WI x WJ grid and each wave computes BI x BJ blocks of
// 16 x 16 (MFMA 16x16x4, four real MFMAs per complex multiply-add).  Every
// shape adds the products of an output entry in the same order (k in steps of
// 16 through LDS, 4 per MFMA), so all shapes give the same result bit for bit.
template <int BI_, int BJ_, int WI_, int WJ_>
struct TileCfg {
  static constexpr int BI = BI_, BJ = BJ_, WI = WI_, WJ = WJ_;
  static constexpr int TM = 16 * BI * WI, TN = 16 * BJ * WJ, TK = 16;
  static_assert(WI * WJ == 4, "four waves per workgroup");
  static_assert(TM * TK % 256 == 0 && TN * TK % 256 == 0, "whole staging loads per thread");
};

// One padding entry per row: operands stored with k contiguous (B untransposed,
// A transposed) are written down a column, 16 lanes at a row stride that
// would otherwise map them all to the same LDS banks.
template <class T, class C>
struct TileSmem {
  cplx<T> a[C::TK][C::TM + 1];
  cplx<T> b[C::TK][C::TN + 1];
};

// Tile (tm, tn) of C = beta C + alpha op(A) op(B); operand conventions as in gemm_tile.
template <class T, class C>
__device__ __forceinline__ void gemm_tile_cfg(const cplx<T>* __restrict__ A, int64_t lda, int opA,
                                              const cplx<T>* __restrict__ B, int64_t ldb, int opB,
                                              cplx<T>* __restrict__ Cm, int64_t ldc, int M, int N, int K,
                                              cplx<T> alpha, int beta, int tm, int tn, TileSmem<T, C>& sm) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int TM = C::TM, TN = C::TN, TK = C::TK, BI = C::BI, BJ = C::BJ;
  constexpr int NA = TM * TK / 256, NB = TN * TK / 256;  // staged entries per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave % C::WI) * 16 * BI, wc = (wave / C::WI) * 16 * BJ;
  const int row0 = tm * TM, col0 = tn * TN;
  acc_t accr[BI][BJ], acci[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accr[i][j][r] = 0;
        acci[i][j][r] = 0;
      }
  // staged entry e = tid + 256 q: consecutive threads take consecutive
  // addresses of the operand's contiguous dimension
  cplx<T> ra[NA], rb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      if (opA == OP_N) {
        const int gr = row0 + e % TM, gk = k0 + e / TM;
        ra[q] = load_or_zero(A + (int64_t)gr + (int64_t)gk * lda, gk < K && gr < M);
      } else {
        const int gk = k0 + e % TK, gr = row0 + e / TK;
        cplx<T> v = load_or_zero(A + (int64_t)gk + (int64_t)gr * lda, gk < K && gr < M);
        if (opA == OP_C) v.im = -v.im;
        ra[q] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      if (opB == OP_N) {
        const int gk = k0 + e % TK, gc = col0 + e / TK;
        rb[q] = load_or_zero(B + (int64_t)gk + (int64_t)gc * ldb, gk < K && gc < N);
      } else {
        const int gc = col0 + e % TN, gk = k0 + e / TN;
        cplx<T> v = load_or_zero(B + (int64_t)gc + (int64_t)gk * ldb, gk < K && gc < N);
        if (opB == OP_C) v.im = -v.im;
        rb[q] = v;
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      if (opA == OP_N)
        sm.a[e / TM][e % TM] = ra[q];
      else
        sm.a[e % TK][e / TK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      if (opB == OP_N)
        sm.b[e % TK][e / TK] = rb[q];
      else
        sm.b[e / TN][e % TN] = rb[q];
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += TK) {
    stage();
    __syncthreads();
    if (k0 + TK < K) fetch(k0 + TK);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int k = kk + (lane >> 4);
      cplx<T> a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = sm.a[k][wr + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = sm.b[k][wc + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
          accr[i][j] = Mfma<T>::step(a[i].re, b[j].re, accr[i][j]);
          accr[i][j] = Mfma<T>::step(-a[i].im, b[j].im, accr[i][j]);
          acci[i][j] = Mfma<T>::step(a[i].re, b[j].im, acci[i][j]);
          acci[i][j] = Mfma<T>::step(a[i].im, b[j].re, acci[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + i * 16 + Mfma<T>::row(lane, r);
        const int gc = col0 + wc + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          const T pr = accr[i][j][r], pi = acci[i][j][r];
          cplx<T> v = {alpha.re * pr - alpha.im * pi, alpha.re * pi + alpha.im * pr};
          cplx<T>* dst = Cm + (int64_t)gr + (int64_t)gc * ldc;
          if (beta) v = cadd(*dst, v);
          *dst = v;
        }
      }
}

// Skinny product for at most 16 right-hand sides: C = beta C + alpha A B with
// A (M x K, column-major, not transposed) streamed from memory once.  A
// workgroup computes rows [256 tm, 256 tm + 256) and all N <= 16 columns; wave
// w owns 64 rows as four 16x16 MFMA blocks and loads its A operands straight
// into registers in the MFMA layout (lane l: row l%16, k l/16: 16 consecutive
// rows per k, coalesced), four k-steps ahead of their use.  No LDS.
constexpr int SKINNY_TM = 256, SKINNY_TN = 16;

// RB row blocks of 16 per wave (the workgroup covers 64 RB rows); fewer blocks
// hold fewer registers, so more waves share a SIMD.
template <class T, int RB = 4>
__device__ __forceinline__ void gemm_tile_skinny(const cplx<T>* __restrict__ A, int64_t lda,
                                                 const cplx<T>* __restrict__ B, int64_t ldb, cplx<T>* __restrict__ C,
                                                 int64_t ldc, int M, int N, int K, cplx<T> alpha, int beta, int tm) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rbase = tm * 64 * RB + wave * 16 * RB;
  if (rbase >= M) return;  // no barrier below: idle waves may leave
  const int lr = lane & 15, lk = lane >> 4;
  acc_t accr[RB], acci[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      accr[i][r] = 0;
      acci[i][r] = 0;
    }
  constexpr int U = 4;  // k-steps of 4 per batch of loads
  cplx<T> a0[U][RB], b0[U], a1[U][RB], b1[U];  // two named batches: no dynamically indexed registers
  auto load = [&](cplx<T>(&aa)[U][RB], cplx<T>(&bb)[U], int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 4 * u + lk;
      const bool kin = k < K;
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int row = rbase + 16 * i + lr;
        aa[u][i] = load_or_zero(A + (int64_t)row + (int64_t)k * lda, kin && row < M);
      }
      bb[u] = load_or_zero(B + (int64_t)k + (int64_t)lr * ldb, kin && lr < N);
    }
  };
  auto mma = [&](cplx<T>(&aa)[U][RB], cplx<T>(&bb)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const cplx<T> bv = bb[u];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const cplx<T> av = aa[u][i];
        accr[i] = Mfma<T>::step(av.re, bv.re, accr[i]);
        accr[i] = Mfma<T>::step(-av.im, bv.im, accr[i]);
        acci[i] = Mfma<T>::step(av.re, bv.im, acci[i]);
        acci[i] = Mfma<T>::step(av.im, bv.re, acci[i]);
      }
    }
  };
  if (K > 0) load(a0, b0, 0);
  for (int k0 = 0; k0 < K; k0 += 8 * U) {
    if (k0 + 4 * U < K) load(a1, b1, k0 + 4 * U);  // in flight during the MFMAs of a0
    mma(a0, b0);
    if (k0 + 4 * U >= K) break;
    if (k0 + 8 * U < K) load(a0, b0, k0 + 8 * U);  // in flight during the MFMAs of a1
    mma(a1, b1);
  }
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = rbase + 16 * i + Mfma<T>::row(lane, r);
      const int gc = lr;
      if (gr < M && gc < N) {
        const T pr = accr[i][r], pi = acci[i][r];
        cplx<T> v = {alpha.re * pr - alpha.im * pi, alpha.re * pi + alpha.im * pr};
        cplx<T>* dst = C + (int64_t)gr + (int64_t)gc * ldc;
        if (beta) v = cadd(*dst, v);
        *dst = v;
      }
    }
}

}  // namespace bfmf
