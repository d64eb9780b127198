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

// Operands in device memory are read through the global address space: a
// generic (flat) load also counts against the LDS wait counter, so every wait
// for a staged LDS operand would wait for the next block's prefetch as well.
// The global pointer is made from the address's integer value (a cast between
// pointer types can be dropped again by the optimizer).
template <class T>
using gcptr = const __attribute__((address_space(1))) cplx<T>*;
template <class T>
__device__ __forceinline__ gcptr<T> as_global(const cplx<T>* p) {
  return (gcptr<T>)(uintptr_t)p;
}

// *p when ok, else 0 (a guarded load: a select between the global address and
// a local zero would put the zero in scratch memory)
template <class T>
__device__ __forceinline__ cplx<T> load_or_zero(gcptr<T> p, bool ok) {
  cplx<T> v = {0, 0};
  if (ok) {
    v.re = p->re;
    v.im = p->im;
  }
  return v;
}
template <class T>
__device__ __forceinline__ cplx<T> load_or_zero(const cplx<T>* p, bool ok) {
  return load_or_zero(as_global(p), ok);
}

template <class TO, class TI>
__device__ __forceinline__ cplx<TO> to_cplx(cplx<TI> v) {
  return cplx<TO>{(TO)v.re, (TO)v.im};
}

// LDS layout of a staged operand block (TK = 16 rows k, a row of t entries m):
// row stride lds_ld(t), congruent to 16 modulo 32 entries, and entry (k, m)
// stored at column m ^ k, which permutes each aligned run of 16 entries.  A
// wave's MFMA operand read (rows k..k+3, 16 consecutive m each) and both
// staging patterns (consecutive m in a row, or consecutive k down a column)
// then fall on distinct banks in every group of lanes the LDS serves at once.
__host__ __device__ constexpr int lds_ld(int t) { return t % 32 == 0 ? t + 16 : t; }
__device__ __forceinline__ int lds_swz(int k, int m) { return m ^ (k & 15); }

// Real and imaginary parts in separate planes: every LDS access moves 8
// (or 4) contiguous bytes per lane, so a wave's access covers distinct banks.
template <class T, int TK, int TM, int TN>
struct SplitSmem {
  T are[TK][lds_ld(TM)], aim[TK][lds_ld(TM)];
  T bre[TK][lds_ld(TN)], bim[TK][lds_ld(TN)];
  __device__ __forceinline__ void put_a(int k, int m, cplx<T> v) {
    const int c = lds_swz(k, m);
    are[k][c] = v.re;
    aim[k][c] = v.im;
  }
  __device__ __forceinline__ void put_b(int k, int n, cplx<T> v) {
    const int c = lds_swz(k, n);
    bre[k][c] = v.re;
    bim[k][c] = v.im;
  }
  __device__ __forceinline__ cplx<T> get_a(int k, int m) const {
    const int c = lds_swz(k, m);
    return cplx<T>{are[k][c], aim[k][c]};
  }
  __device__ __forceinline__ cplx<T> get_b(int k, int n) const {
    const int c = lds_swz(k, n);
    return cplx<T>{bre[k][c], bim[k][c]};
  }
};

template <class T>
struct GemmSmem : SplitSmem<T, GEMM_TK, GEMM_TM, GEMM_TN> {};

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
  // Each thread stages 4 A and 4 B entries per k-block of depth 16, entry
  // e = tid + 256 q: consecutive threads take consecutive addresses of the
  // operand's contiguous dimension.  The next block is fetched into registers
  // as stored before the MFMAs of the current block run, so its global-memory
  // latency overlaps the arithmetic; conversion and conjugation wait for the
  // staging.
  cplx<TL> ra[4], rb[4];
  const gcptr<TL> Ag = as_global(A), Bg = as_global(B);
  // one guarded load per entry, its address chosen without branches: loads in
  // alternative branches would share destination registers, and the compiler
  // then waits for each load before issuing the next
  const bool an = opA == OP_N, bn = opB == OP_N;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ar = row0 + (an ? e % GEMM_TM : e / GEMM_TK), ak = k0 + (an ? e / GEMM_TM : e % GEMM_TK);
      ra[q] = load_or_zero(Ag + (an ? (int64_t)ar + (int64_t)ak * lda : (int64_t)ak + (int64_t)ar * lda),
                           ak < K && ar < M);
      const int bc = col0 + (bn ? e / GEMM_TK : e % GEMM_TN), bk = k0 + (bn ? e % GEMM_TK : e / GEMM_TN);
      rb[q] = load_or_zero(Bg + (bn ? (int64_t)bk + (int64_t)bc * ldb : (int64_t)bc + (int64_t)bk * ldb),
                           bk < K && bc < N);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      cplx<T> va = to_cplx<T>(ra[q]), vb = to_cplx<T>(rb[q]);
      if (opA == OP_C) va.im = -va.im;
      if (opB == OP_C) vb.im = -vb.im;
      if (opA == OP_N)
        sm.put_a(e / GEMM_TM, e % GEMM_TM, va);
      else
        sm.put_a(e % GEMM_TK, e / GEMM_TK, va);
      if (opB == OP_N)
        sm.put_b(e % GEMM_TK, e / GEMM_TK, vb);
      else
        sm.put_b(e / GEMM_TN, e % GEMM_TN, vb);
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
      for (int i = 0; i < 2; ++i) a[i] = sm.get_a(k, wr + i * 16 + (lane & 15));
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sm.get_b(k, wc + j * 16 + (lane & 15));
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
  // workgroups per CU the registers must allow: two for shapes of four 16x16 blocks per wave and
  // sides of at most 128 (two waves per SIMD hide each other's barriers and staging), one for the
  // others (which would spill)
  static constexpr int MINB = BI * BJ <= 4 && TM <= 128 && TN <= 128 ? 2 : 1;
  static_assert(WI * WJ == 4, "four waves per workgroup");
  static_assert(TM * TK % 256 == 0 && TN * TK % 256 == 0, "whole staging loads per thread");
};

// The layout of lds_ld / lds_swz: operands stored with k contiguous (B
// untransposed, A transposed) are written down a column, the others along a
// row, and both are read four rows at a time by the MFMA operand loads.
template <class T, class C>
struct TileSmem : SplitSmem<T, C::TK, C::TM, C::TN> {};

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
  const gcptr<T> Ag = as_global(A), Bg = as_global(B);
  // one guarded load per entry, its address chosen without branches: loads in
  // alternative branches would share destination registers, and the compiler
  // then waits for each load before issuing the next
  const bool an = opA == OP_N, bn = opB == OP_N;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      const int ar = row0 + (an ? e % TM : e / TK), ak = k0 + (an ? e / TM : e % TK);
      ra[q] = load_or_zero(Ag + (an ? (int64_t)ar + (int64_t)ak * lda : (int64_t)ak + (int64_t)ar * lda),
                           ak < K && ar < M);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      const int bc = col0 + (bn ? e / TK : e % TN), bk = k0 + (bn ? e % TK : e / TN);
      rb[q] = load_or_zero(Bg + (bn ? (int64_t)bk + (int64_t)bc * ldb : (int64_t)bc + (int64_t)bk * ldb),
                           bk < K && bc < N);
    }
  };
  // conjugation at staging, so that nothing waits for a prefetched value before its staging
  auto stage = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      cplx<T> v = ra[q];
      if (opA == OP_C) v.im = -v.im;
      if (opA == OP_N)
        sm.put_a(e / TM, e % TM, v);
      else
        sm.put_a(e % TK, e / TK, v);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      cplx<T> v = rb[q];
      if (opB == OP_C) v.im = -v.im;
      if (opB == OP_N)
        sm.put_b(e % TK, e / TK, v);
      else
        sm.put_b(e / TN, e % TN, v);
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
      for (int i = 0; i < BI; ++i) a[i] = sm.get_a(k, wr + i * 16 + (lane & 15));
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = sm.get_b(k, wc + j * 16 + (lane & 15));
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

// Skinny product for at most 16 (or 32) right-hand sides: C = beta C + alpha A B
// with A (M x K, column-major, not transposed) streamed from memory once.  A
// workgroup computes rows [256 tm, 256 tm + 256) and all N <= 16 columns; wave
// w owns 64 rows as four 16x16 MFMA blocks and loads its A operands straight
// into registers in the MFMA layout (lane l: row l%16, k l/16: 16 consecutive
// rows per k, coalesced), four k-steps ahead of their use.  No LDS.  The
// products of an entry are added in the order of the LDS tiles (k in steps of
// 4, increasing), so the results are those of the other tile shapes.
constexpr int SKINNY_TM = 256, SKINNY_TN = 16;

// RB row blocks of 16 per wave (the workgroup covers 64 RB rows); fewer blocks
// hold fewer registers, so more waves share a SIMD.  NB column blocks of 16
// (N <= 16 NB): each A operand serves NB blocks of MFMAs.
template <class T, int RB = 4, int NB = 1>
__device__ __forceinline__ void gemm_tile_skinny(const cplx<T>* __restrict__ A, int64_t lda,
                                                 const cplx<T>* __restrict__ B, int64_t ldb, cplx<T>* __restrict__ C,
                                                 int64_t ldc, int M, int N, int K, cplx<T> alpha, int beta, int tm) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rbase = tm * 64 * RB + wave * 16 * RB;
  if (rbase >= M) return;  // no barrier below: idle waves may leave
  const int lr = lane & 15, lk = lane >> 4;
  const gcptr<T> Ag = as_global(A), Bg = as_global(B);
  acc_t accr[RB][NB], acci[RB][NB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accr[i][j][r] = 0;
        acci[i][j][r] = 0;
      }
  constexpr int U = NB == 1 ? 4 : 2;  // k-steps of 4 per batch of loads
  cplx<T> a0[U][RB], b0[U][NB], a1[U][RB], b1[U][NB];  // two named batches: no dynamically indexed registers
  auto load = [&](cplx<T>(&aa)[U][RB], cplx<T>(&bb)[U][NB], int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 4 * u + lk;
      const bool kin = k < K;
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int row = rbase + 16 * i + lr;
        aa[u][i] = load_or_zero(Ag + (int64_t)row + (int64_t)k * lda, kin && row < M);
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int col = 16 * j + lr;
        bb[u][j] = load_or_zero(Bg + (int64_t)k + (int64_t)col * ldb, kin && col < N);
      }
    }
  };
  auto mma = [&](cplx<T>(&aa)[U][RB], cplx<T>(&bb)[U][NB]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const cplx<T> av = aa[u][i];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const cplx<T> bv = bb[u][j];
          accr[i][j] = Mfma<T>::step(av.re, bv.re, accr[i][j]);
          accr[i][j] = Mfma<T>::step(-av.im, bv.im, accr[i][j]);
          acci[i][j] = Mfma<T>::step(av.re, bv.im, acci[i][j]);
          acci[i][j] = Mfma<T>::step(av.im, bv.re, acci[i][j]);
        }
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
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = rbase + 16 * i + Mfma<T>::row(lane, r);
        const int gc = 16 * j + lr;
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
