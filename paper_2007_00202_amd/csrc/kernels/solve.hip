// Forward / backward sweeps through the dense fronts (paper Sec. 2, Alg. 1
// last step; Sec. 5: forward applies F11^-1 then F21 from the leaves to the
// root, backward applies F12 then F11^-1 from the root to the leaves), and the
// FP64 vector kernels of GMRES (Sec. 6).
//
// Sweeps are written in gather form: front f owns a workspace W_f (n x nrhs);
// in the forward sweep rows ns..n-1 of W_f end up holding the update vector
// that the parent extend-adds (through the same inverse maps as the
// factorization), so no two fronts ever write the same memory.
#include "../devtypes.hpp"
#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace bfmf {

template <class T>
__global__ void permute_in_kernel(const cplx<double>* __restrict__ B, int64_t ldb, cplx<T>* __restrict__ y,
                                  const int64_t* __restrict__ perm, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const cplx<double> v = B[perm[i] + c * ldb];
  y[i + c * N] = cplx<T>{(T)v.re, (T)v.im};
}

template <class T>
__global__ void permute_out_kernel(const cplx<T>* __restrict__ x, cplx<double>* __restrict__ X, int64_t ldx,
                                   const int64_t* __restrict__ perm, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const cplx<T> v = x[i + c * N];
  X[perm[i] + c * ldx] = cplx<double>{(double)v.re, (double)v.im};
}

// W_f(i, c) = [y(sbeg + r, c) if r < ns] (+) child updates at r, in child order, with r = i except
// for the rows of a dense front's F11, where r = pperm[i]: the gather applies the row interchanges
// of the partial pivoting (P^T) on the way in.
template <class T>
__global__ __launch_bounds__(256) void fwd_gather_kernel(const FrontDesc* __restrict__ fds,
                                                         const cplx<T>* __restrict__ y, int64_t N, int nrhs) {
  const FrontDesc& fd = fds[blockIdx.y];
  const int n = fd.n, ns = fd.ns;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int r = (fd.P && i < ns) ? fd.pperm[i] : i;
  const int k1 = fd.nchild > 0 ? fd.inv[0][r] : -1;
  const int k2 = fd.nchild > 1 ? fd.inv[1][r] : -1;
  cplx<T>* W = (cplx<T>*)fd.W;
  for (int c = 0; c < nrhs; ++c) {
    cplx<T> v = {0, 0};
    if (r < ns) v = y[fd.sbeg + r + c * N];
    if (k1 >= 0) v = cadd(v, ((const cplx<T>*)fd.cw[0])[k1 + c * fd.cw_ld[0]]);
    if (k2 >= 0) v = cadd(v, ((const cplx<T>*)fd.cw[1])[k2 + c * fd.cw_ld[1]]);
    W[i + (int64_t)c * n] = v;
  }
}

// Unit-lower substitution on W_f(0:ns, :) (already interchanged by the
// gather), one workgroup per front; threads own rows, one synchronisation
// per column.  Complex64 fronts only (the double-precision ones take the
// blocked sweeps).
template <class T>
__global__ __launch_bounds__(256) void fwd_trsv_kernel(const FrontDesc* __restrict__ fds, int nrhs) {
  const FrontDesc& fd = fds[blockIdx.x];
  const int n = fd.n, ns = fd.ns;
  if (ns == 0) return;
  const cplx<T>* F = (const cplx<T>*)fd.P;  // [L U; F21'], ld n
  cplx<T>* W = (cplx<T>*)fd.W;
  for (int j = 0; j < ns - 1; ++j) {
    const cplx<T>* Lj = F + (int64_t)j * n;
    for (int r = j + 1 + threadIdx.x; r < ns; r += 256) {
      const cplx<T> l = Lj[r];
      for (int c = 0; c < nrhs; ++c) {
        cplx<T>* w = W + (int64_t)c * n;
        w[r] = csub(w[r], cmul(l, w[j]));
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ blocked sweeps
// The dense fronts' substitutions on the matrix cores.  A workgroup takes
// BLK_RC right-hand sides of one front and keeps W_f(0:ns, those columns) in
// the accumulators of its four waves: row block b (16 rows) in wave b % 4,
// slot b / 4, in the f64 16x16x4 result layout (lane l, item r: row
// l/16 + 4r, column l%16).  Diagonal block by diagonal block of F11, the
// owner wave solves its 16 x 16 triangle in registers (the triangle staged
// in LDS, each solved row broadcast to the lanes of its columns by
// shuffles) and publishes the 16 solved rows through LDS; then every wave
// subtracts the product of the panel of L below (U above) the block with
// them from its own row blocks (f64 MFMA, the panel read once per
// workgroup).  Two barriers per 16 columns.  Workgroups of one front are
// adjacent in the XCD order, so the other column groups find the panels in
// the same L2.
constexpr int BLK_RC = 16;
constexpr int BLK_MAXNS = 1024;   // up to 16 row blocks per wave
constexpr int PERM_MAXNS = 16384;  // pivot permutations built in LDS (64 KiB)

// LDS entries that other lanes of the same wave read without a barrier in
// between (the triangle solves): volatile, so that every store is performed
// in program order and no value is forwarded in registers (one wave's LDS
// operations complete in order)
__device__ __forceinline__ cplx<double> vld(const volatile cplx<double>* p) { return cplx<double>{p->re, p->im}; }
__device__ __forceinline__ void vst(volatile cplx<double>* p, cplx<double> v) {
  p->re = v.re;
  p->im = v.im;
}

// one product step Y_b -= A Y_jb on 16 x 16 blocks: A from F (rows gi, columns
// 16 jb + 4q + lr), Y_jb from LDS
__device__ __forceinline__ void blk_update(d4_t& yr, d4_t& yi, const cplx<double>* __restrict__ F, int64_t n,
                                           int gi, int jb, int ns, int lr, int col,
                                           const cplx<double> (*Ys)[17]) {
  cplx<double> a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gk = 16 * jb + 4 * q + lr;
    const bool ok = gi < ns && gk < ns;
    a[q] = load_or_zero(F + (ok ? gi : 0) + (int64_t)(ok ? gk : 0) * n, ok);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const cplx<double> bv = Ys[4 * q + lr][col];
    // the real and imaginary chains alternate, so consecutive MFMAs are independent
    yr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[q].re, bv.re, yr, 0, 0, 0);
    yi = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[q].re, bv.im, yi, 0, 0, 0);
    yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].im, bv.im, yr, 0, 0, 0);
    yi = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[q].im, bv.re, yi, 0, 0, 0);
  }
}

// The rows a blocked sweep takes in one launch: the whole F11 (seg < 0) of a
// front with ns <= BLK_MAXNS, or rows [r0, r1) = segment seg of 1024 rows of a
// larger front (the others' segments come with their own launches, and the
// panels between segments with sweep_seg_gemm_kernel).  False: not this launch's.
__device__ __forceinline__ bool blk_range(const FrontDesc& fd, int seg, int& r0, int& r1) {
  if (seg < 0) {
    r0 = 0;
    r1 = fd.ns;
    return fd.ns > 0 && fd.ns <= BLK_MAXNS;
  }
  r0 = seg * BLK_MAXNS;
  r1 = min(fd.ns, r0 + BLK_MAXNS);
  return fd.ns > BLK_MAXNS && r0 < fd.ns;
}

// W_f(r0:r1) <- L(r0:r1, r0:r1)^-1 W_f(r0:r1) (the interchanges were applied by the gather) for
// the rows blk_range gives, at most 64 MB of them
template <int MB>
__global__ __launch_bounds__(256) void fwd_trsv_blk_kernel(const FrontDesc* __restrict__ fds, int nfront, int nrhs,
                                                           int seg) {
  __shared__ cplx<double> Ls[2][16][17];  // Ls[buf][k][i] = L(16 jb + i, 16 jb + k), strictly lower
  __shared__ cplx<double> Ys[2][16][17];  // Ys[buf][k][c] = Y(16 jb + k, c)
  const int ngrp = (nrhs + BLK_RC - 1) / BLK_RC;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int fi = (int)(tile / ngrp), grp = (int)(tile % ngrp);
  if (fi >= nfront) return;
  const FrontDesc& fd = fds[fi];
  int r0, r1;
  if (!blk_range(fd, seg, r0, r1) || r1 - r0 > 64 * MB) return;  // uniform; the host never sends the latter
  const int n = fd.n, ns = r1 - r0;  // from here on rows are relative to r0
  const int c0 = grp * BLK_RC, ncl = min(BLK_RC, nrhs - c0);
  const cplx<double>* F = (const cplx<double>*)fd.P + r0 + (int64_t)r0 * n;  // L(r0:, r0:), ld n
  cplx<double>* W = (cplx<double>*)fd.W + r0 + (int64_t)c0 * n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, lr = lane >> 4;
  const int nb = (ns + 15) / 16;
  d4_t yr[MB], yi[MB];
#pragma unroll
  for (int s = 0; s < MB; ++s)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * (4 * s + wave) + lr + 4 * r;
      const bool ok = row < ns && col < ncl;
      const cplx<double> v = load_or_zero(W + (ok ? row + (int64_t)col * n : 0), ok);
      yr[s][r] = v.re;
      yi[s][r] = v.im;
    }
  for (int jb = 0; jb < nb; ++jb) {
    const int buf = jb & 1, sj = jb >> 2;
    {
      const int i = tid & 15, k = tid >> 4, gi = 16 * jb + i, gk = 16 * jb + k;
      const bool ok = i > k && gi < ns;
      Ls[buf][k][i] = load_or_zero(F + (ok ? gi + (int64_t)gk * n : 0), ok);
    }
    __syncthreads();
    if (wave == (jb & 3)) {  // the owner: block jb to LDS, its triangle there, then out to W
      volatile cplx<double>(*V)[17] = Ys[buf];
#pragma unroll
      for (int s = 0; s < MB; ++s)
        if (s == sj)
#pragma unroll
          for (int r = 0; r < 4; ++r) vst(&V[lr + 4 * r][col], cplx<double>{yr[s][r], yi[s][r]});
#pragma unroll
      for (int k = 0; k < 15; ++k) {
        const cplx<double> yk = vld(&V[k][col]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = lr + 4 * r;
          if (i > k) vst(&V[i][col], csub(vld(&V[i][col]), cmul(Ls[buf][k][i], yk)));
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * jb + lr + 4 * r;
        if (row < ns && col < ncl) W[row + (int64_t)col * n] = vld(&V[lr + 4 * r][col]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < MB; ++s2) {
      const int b2 = 4 * s2 + wave;
      if (b2 > jb && b2 < nb) blk_update(yr[s2], yi[s2], F, n, 16 * b2 + col, jb, ns, lr, col, Ys[buf]);
    }
  }
}

// x(r0:r1) <- U(r0:r1, r0:r1)^-1 W_f(r0:r1) for the rows blk_range gives (W_f(r0:r1) already
// holds W - F12 x(I^u) minus the segments below); a segment's solution also goes back to W_f
// for the panel product above it
template <int MB>
__global__ __launch_bounds__(256) void bwd_trsv_blk_kernel(const FrontDesc* __restrict__ fds, int nfront,
                                                           cplx<double>* __restrict__ x, int64_t N, int nrhs,
                                                           int seg) {
  __shared__ cplx<double> Us[2][16][17];  // Us[buf][k][i] = U(16 jb + i, 16 jb + k), upper with the diagonal
  __shared__ cplx<double> Ys[2][16][17];
  const int ngrp = (nrhs + BLK_RC - 1) / BLK_RC;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int fi = (int)(tile / ngrp), grp = (int)(tile % ngrp);
  if (fi >= nfront) return;
  const FrontDesc& fd = fds[fi];
  int r0, r1;
  if (!blk_range(fd, seg, r0, r1) || r1 - r0 > 64 * MB) return;  // uniform
  const int n = fd.n, ns = r1 - r0;
  const int c0 = grp * BLK_RC, ncl = min(BLK_RC, nrhs - c0);
  const cplx<double>* F = (const cplx<double>*)fd.P + r0 + (int64_t)r0 * n;
  cplx<double>* W = (cplx<double>*)fd.W + r0 + (int64_t)c0 * n;
  cplx<double>* xs = x + fd.sbeg + r0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, lr = lane >> 4;
  const int nb = (ns + 15) / 16;
  d4_t yr[MB], yi[MB];
#pragma unroll
  for (int s = 0; s < MB; ++s)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * (4 * s + wave) + lr + 4 * r;
      const bool ok = row < ns && col < ncl;
      const cplx<double> v = load_or_zero(W + (ok ? row + (int64_t)col * n : 0), ok);
      yr[s][r] = v.re;
      yi[s][r] = v.im;
    }
  for (int jb = nb - 1; jb >= 0; --jb) {
    const int buf = jb & 1, sj = jb >> 2;
    {
      const int i = tid & 15, k = tid >> 4, gi = 16 * jb + i, gk = 16 * jb + k;
      const bool ok = i <= k && gk < ns;
      Us[buf][k][i] = load_or_zero(F + (ok ? gi + (int64_t)gk * n : 0), ok);
    }
    __syncthreads();
    if (wave == (jb & 3)) {
      volatile cplx<double>(*V)[17] = Ys[buf];
#pragma unroll
      for (int s = 0; s < MB; ++s)
        if (s == sj)
#pragma unroll
          for (int r = 0; r < 4; ++r) vst(&V[lr + 4 * r][col], cplx<double>{yr[s][r], yi[s][r]});
      const int kmax = min(16, ns - 16 * jb);  // rows of the block inside the front
#pragma unroll
      for (int k = 15; k >= 0; --k) {
        if (k < kmax) {  // uniform
          if (lr == (k & 3)) vst(&V[k][col], cdiv(vld(&V[k][col]), Us[buf][k][k]));
          const cplx<double> yk = vld(&V[k][col]);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = lr + 4 * r;
            if (i < k) vst(&V[i][col], csub(vld(&V[i][col]), cmul(Us[buf][k][i], yk)));
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * jb + lr + 4 * r;
        if (row < ns && col < ncl) {
          const cplx<double> v = vld(&V[lr + 4 * r][col]);
          xs[row + (int64_t)(c0 + col) * N] = v;
          if (seg >= 0) W[row + (int64_t)col * n] = v;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < MB; ++s2) {
      const int b2 = 4 * s2 + wave;
      if (b2 < jb) blk_update(yr[s2], yi[s2], F, n, 16 * b2 + col, jb, ns, lr, col, Ys[buf]);
    }
  }
}

// The interchanges of F11's partial pivoting (row k swapped with piv[k], k
// ascending) as one permutation, applied to an index vector: pperm[i] is the
// row of F11 that ends up at position i.  One workgroup per dense front.
__global__ __launch_bounds__(256) void pivot_perm_kernel(const FrontDesc* __restrict__ fds, int nfront) {
  extern __shared__ int32_t perm_smem[];
  const FrontDesc& fd = fds[blockIdx.x];
  const int ns = fd.ns;
  if (!fd.P || ns == 0) return;  // compressed fronts
  int32_t* idx = ns <= PERM_MAXNS ? perm_smem : fd.pperm;  // the largest fronts in place in memory
  for (int i = threadIdx.x; i < ns; i += 256) idx[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < ns; ++k) {
      const int p = fd.piv[k];
      if (p != k && p >= 0 && p < ns) {
        const int t = idx[k];
        idx[k] = idx[p];
        idx[p] = t;
      }
    }
  __syncthreads();
  if (ns <= PERM_MAXNS)
    for (int i = threadIdx.x; i < ns; i += 256) fd.pperm[i] = idx[i];
}

// Panel products between the segments of a front with ns > BLK_MAXNS, after segment seg =
// rows [r0, r1) is solved: forward (mode 0) W(r1:n) -= P(r1:n, r0:r1) W(r0:r1), which for the
// last segment includes F21 (rows ns..n of P); backward (mode 1) W(0:r0) -= U(0:r0, r0:r1) x(r0:r1).
template <class C>
__global__ __launch_bounds__(256) void sweep_seg_gemm_kernel(const FrontDesc* __restrict__ fds, int nrhs, int seg,
                                                             int mode) {
  __shared__ TileSmem<double, C> sm;
  const FrontDesc& fd = fds[blockIdx.y];
  int r0, r1;
  if (!blk_range(fd, seg, r0, r1)) return;
  const int n = fd.n;
  const cplx<double>* F = (const cplx<double>*)fd.P;
  cplx<double>* W = (cplx<double>*)fd.W;
  const int M = mode == 0 ? n - r1 : r0, K = r1 - r0;
  if (M <= 0) return;
  const int tm = (M + C::TM - 1) / C::TM, tn = (nrhs + C::TN - 1) / C::TN;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  if (mode == 0)
    gemm_tile_cfg<double, C>(F + r1 + (int64_t)r0 * n, n, OP_N, W + r0, n, OP_N, W + r1, n, M, nrhs, K,
                             cplx<double>{-1, 0}, 1, t % tm, t / tm, sm);
  else
    gemm_tile_cfg<double, C>(F + (int64_t)r0 * n, n, OP_N, W + r0, n, OP_N, W, n, M, nrhs, K, cplx<double>{-1, 0}, 1,
                             t % tm, t / tm, sm);
}

typedef TileCfg<2, 2, 4, 1> SweepTile128x32;

// Upper substitution on W_f(0:ns, :) and scatter of the result into x.
template <class T>
__global__ __launch_bounds__(256) void bwd_trsv_kernel(const FrontDesc* __restrict__ fds, cplx<T>* __restrict__ x,
                                                       int64_t N, int nrhs) {
  const FrontDesc& fd = fds[blockIdx.x];
  const int n = fd.n, ns = fd.ns;
  if (ns == 0) return;
  const cplx<T>* F = (const cplx<T>*)fd.P;  // [L U; F21'], ld n
  cplx<T>* W = (cplx<T>*)fd.W;
  for (int j = ns - 1; j >= 0; --j) {
    const cplx<T>* Uj = F + (int64_t)j * n;
    const cplx<T> d = Uj[j];
    for (int c = threadIdx.x; c < nrhs; c += 256) {
      cplx<T>* w = W + (int64_t)c * n;
      w[j] = cdiv(w[j], d);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < j; r += 256) {
      const cplx<T> u = Uj[r];
      for (int c = 0; c < nrhs; ++c) {
        cplx<T>* w = W + (int64_t)c * n;
        w[r] = csub(w[r], cmul(u, w[j]));
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < ns * nrhs; e += 256) {
    const int r = e % ns, c = e / ns;
    x[fd.sbeg + r + (int64_t)c * N] = W[r + (int64_t)c * n];
  }
}

// W_f(ns + k, c) = x(I^u[k], c)
template <class T>
__global__ __launch_bounds__(256) void bwd_gather_kernel(const FrontDesc* __restrict__ fds,
                                                         const cplx<T>* __restrict__ x, int64_t N, int nrhs) {
  const FrontDesc& fd = fds[blockIdx.y];
  const int n = fd.n, ns = fd.ns;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n - ns) return;
  const int64_t g = fd.iu[k];
  cplx<T>* W = (cplx<T>*)fd.W;
  for (int c = 0; c < nrhs; ++c) W[ns + k + (int64_t)c * n] = x[g + c * N];
}

// mode 0: W(ns:n) -= F21 W(0:ns)   (forward update)
// mode 1: W(0:ns) -= F12 W(ns:n)   (backward update)
template <class T>
__global__ __launch_bounds__(256) void sweep_gemm_kernel(const FrontDesc* __restrict__ fds, int nrhs, int mode) {
  __shared__ GemmSmem<T> sm;
  const FrontDesc& fd = fds[blockIdx.y];
  const int n = fd.n, ns = fd.ns, nu = n - ns;
  if (ns == 0 || nu == 0) return;
  if (sizeof(T) == 8 && mode == 0 && ns > BLK_MAXNS) return;  // the segment panels carry F21
  const cplx<T>* F = (const cplx<T>*)fd.P;  // [L U; F21'], ld n
  cplx<T>* W = (cplx<T>*)fd.W;
  const int M = mode == 0 ? nu : ns;
  const int tm = (M + GEMM_TM - 1) / GEMM_TM, tn = (nrhs + GEMM_TN - 1) / GEMM_TN;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  if (mode == 0)
    gemm_tile<T>(F + ns, n, OP_N, W, n, W + ns, n, nu, nrhs, ns, cplx<T>{-1, 0}, 1, t % tm, t / tm, sm);
  else
    gemm_tile<T>((const cplx<T>*)fd.F12, fd.ld12, OP_N, W + ns, n, W, n, ns, nrhs, nu, cplx<T>{-1, 0}, 1, t % tm,
                 t / tm, sm);
}

// the same products for at most 16 right-hand sides: 256-row streaming tiles (F21 / F12 read once)
// rows of a sweep product per workgroup: two 16-row blocks per wave in double precision (fewer
// registers, more waves per SIMD for this bandwidth-bound stream), four in single
template <class T>
constexpr int sweep_skinny_tm() {
  return sizeof(T) == 8 ? 128 : 256;
}

// NB column blocks of 16: at most 16 NB right-hand sides (two workgroups per CU: the stream's latency is
// hidden by the other workgroup's MFMAs)
template <class T, int NB = 1>
__global__ __launch_bounds__(256, 2) void sweep_gemm_skinny_kernel(const FrontDesc* __restrict__ fds, int nrhs, int mode) {
  constexpr int RB = sweep_skinny_tm<T>() / 64;
  const FrontDesc& fd = fds[blockIdx.y];
  const int n = fd.n, ns = fd.ns, nu = n - ns;
  if (ns == 0 || nu == 0 || nrhs > SKINNY_TN * NB) return;
  if (sizeof(T) == 8 && mode == 0 && ns > BLK_MAXNS) return;  // the segment panels carry F21
  const cplx<T>* F = (const cplx<T>*)fd.P;  // [L U; F21'], ld n
  cplx<T>* W = (cplx<T>*)fd.W;
  const int M = mode == 0 ? nu : ns;
  const int t = blockIdx.x;
  if (t * sweep_skinny_tm<T>() >= M) return;
  if (mode == 0)
    gemm_tile_skinny<T, RB, NB>(F + ns, n, W, n, W + ns, n, nu, nrhs, ns, cplx<T>{-1, 0}, 1, t);
  else
    gemm_tile_skinny<T, RB, NB>((const cplx<T>*)fd.F12, fd.ld12, W + ns, n, W, n, ns, nrhs, nu, cplx<T>{-1, 0}, 1,
                                t);
}

// ------------------------------------------------------------ GMRES vectors
// Y = A X (alpha = 0) or Y = B - A X (residual), CSR complex128, nrhs columns
__global__ void spmv_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                            const cplx<double>* __restrict__ val, const cplx<double>* __restrict__ X, int64_t ldx,
                            cplx<double>* __restrict__ Y, int64_t ldy, const cplx<double>* __restrict__ B, int64_t ldb,
                            int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const cplx<double>* x = X + c * ldx;
  cplx<double> s = {0, 0};
  for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) s = cadd(s, cmul(val[t], x[colind[t]]));
  if (B) s = csub(B[i + c * ldb], s);
  Y[i + c * ldy] = s;
}

// partial[b, c] = sum over the block's rows of conj(V) W (or |W|^2 if V null)
__global__ __launch_bounds__(256) void dot_partial_kernel(const cplx<double>* __restrict__ V, int64_t ldv,
                                                          const cplx<double>* __restrict__ Wv, int64_t ldw, int64_t N,
                                                          cplx<double>* __restrict__ partial) {
  const int c = blockIdx.y;
  __shared__ double sr[256], si[256];
  double ar = 0, ai = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const cplx<double> w = Wv[i + c * ldw];
    if (V) {
      const cplx<double> v = V[i + c * ldv];
      ar += v.re * w.re + v.im * w.im;
      ai += v.re * w.im - v.im * w.re;
    } else {
      ar += w.re * w.re + w.im * w.im;
    }
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x + (int64_t)c * gridDim.x] = cplx<double>{sr[0], si[0]};
}

// out[c] = sum_b partial[b, c] in a fixed order (deterministic)
__global__ void dot_final_kernel(const cplx<double>* __restrict__ partial, int nblk, int nrhs,
                                 cplx<double>* __restrict__ out, int sqrt_mode) {
  for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
    cplx<double> s = {0, 0};
    for (int b = 0; b < nblk; ++b) s = cadd(s, partial[b + (int64_t)c * nblk]);
    if (sqrt_mode) s = cplx<double>{sqrt(s.re), 0};
    out[c] = s;
  }
}

// W(:, c) += sign * a[c] * V(:, c)
__global__ void axpy_cols_kernel(const cplx<double>* __restrict__ a, double sign, const cplx<double>* __restrict__ V,
                                 int64_t ldv, cplx<double>* __restrict__ Wv, int64_t ldw, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const cplx<double> s = {sign * a[c].re, sign * a[c].im};
  Wv[i + c * ldw] = cadd(Wv[i + c * ldw], cmul(s, V[i + c * ldv]));
}

// V(:, c) = W(:, c) / nrm[c].re (0 if nrm is 0)
__global__ void scale_cols_kernel(const cplx<double>* __restrict__ nrm, const cplx<double>* __restrict__ Wv,
                                  int64_t ldw, cplx<double>* __restrict__ V, int64_t ldv, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const double d = nrm[c].re;
  const double s = d > 0 ? 1.0 / d : 0.0;
  const cplx<double> w = Wv[i + c * ldw];
  V[i + c * ldv] = cplx<double>{w.re * s, w.im * s};
}

// X(:, c) += sum_{i < m} y[i, c] * Vbasis_i(:, c); basis i at V + i * vstride
__global__ void basis_update_kernel(const cplx<double>* __restrict__ y, int ldy, int m,
                                    const cplx<double>* __restrict__ V, int64_t vstride, int64_t ldv,
                                    cplx<double>* __restrict__ X, int64_t ldx, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  cplx<double> s = X[i + c * ldx];
  for (int k = 0; k < m; ++k) s = cadd(s, cmul(y[k + c * ldy], V[k * vstride + i + c * ldv]));
  X[i + c * ldx] = s;
}

// ------------------------------------------------ slot GMRES (serving)
// Columns ("slots") of a serving batch each run their own GMRES cycle and may
// be at different steps; these kernels take per-column arguments.

// Vcur(:, c) = *src[c] (null: zero)
__global__ void slot_gather_kernel(const cplx<double>* const* __restrict__ src, cplx<double>* __restrict__ Vcur,
                                   int64_t ld, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const cplx<double>* p = src[c];
  Vcur[i + c * ld] = p ? p[i] : cplx<double>{0, 0};
}

// mode[c] = 1 (restart): T(:, c) = B(:, c) - T(:, c); mode 0 (idle): T(:, c) = 0; mode 2: unchanged
__global__ void slot_fix_kernel(const int32_t* __restrict__ mode, const cplx<double>* __restrict__ B, int64_t ldb,
                                cplx<double>* __restrict__ T, int64_t ldt, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N) return;
  const int md = mode[c];
  if (md == 2) return;
  cplx<double> v = {0, 0};
  if (md == 1) v = csub(B[i + c * ldb], T[i + c * ldt]);
  T[i + c * ldt] = v;
}

// W(:, c) += sign a[c] V(:, c) for the columns with step >= i (lim[c] >= i)
__global__ void axpy_cols_masked_kernel(const cplx<double>* __restrict__ a, double sign,
                                        const cplx<double>* __restrict__ V, int64_t ldv, cplx<double>* __restrict__ Wv,
                                        int64_t ldw, int64_t N, const int32_t* __restrict__ lim, int i0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N || lim[c] < i0) return;
  const cplx<double> s = {sign * a[c].re, sign * a[c].im};
  Wv[i + c * ldw] = cadd(Wv[i + c * ldw], cmul(s, V[i + c * ldv]));
}

// *dst[c] = W(:, c) / nrm[c].re (0 if nrm is 0) for the columns with a destination
__global__ void scale_cols_to_kernel(const cplx<double>* __restrict__ nrm, const cplx<double>* __restrict__ Wv,
                                     int64_t ldw, cplx<double>* const* __restrict__ dst, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  cplx<double>* d = dst[c];
  if (i >= N || !d) return;
  const double r = nrm[c].re;
  const double sc = r > 0 ? 1.0 / r : 0.0;
  const cplx<double> w = Wv[i + c * ldw];
  d[i] = cplx<double>{w.re * sc, w.im * sc};
}

// X(:, c) += sum_{k < mc[c]} y[k, c] Vbasis_k(:, c) for the columns with mc[c] > 0
__global__ void basis_update_masked_kernel(const cplx<double>* __restrict__ y, int ldy, const int32_t* __restrict__ mc,
                                           const cplx<double>* __restrict__ V, int64_t vstride, int64_t ldv,
                                           cplx<double>* __restrict__ X, int64_t ldx, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const int m = mc[c];
  if (i >= N || m <= 0) return;
  cplx<double> s = X[i + c * ldx];
  for (int k = 0; k < m; ++k) s = cadd(s, cmul(y[k + c * ldy], V[k * vstride + i + c * ldv]));
  X[i + c * ldx] = s;
}

// ------------------------------------------------------------------ launchers
#define KCHECK(expr)                   \
  do {                                 \
    hipError_t e__ = (expr);           \
    if (e__ != hipSuccess) return e__; \
  } while (0)

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <class T>
hipError_t launch_permute_in(const void* B, int64_t ldb, void* y, const int64_t* perm, int64_t N, int nrhs,
                             hipStream_t s) {
  hipLaunchKernelGGL((permute_in_kernel<T>), dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s,
                     (const cplx<double>*)B, ldb, (cplx<T>*)y, perm, N);
  return hipGetLastError();
}
template <class T>
hipError_t launch_permute_out(const void* x, void* X, int64_t ldx, const int64_t* perm, int64_t N, int nrhs,
                              hipStream_t s) {
  hipLaunchKernelGGL((permute_out_kernel<T>), dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s,
                     (const cplx<T>*)x, (cplx<double>*)X, ldx, perm, N);
  return hipGetLastError();
}

// the sweep products of a level (mode 0: W(ns:n) -= F21 W(0:ns); mode 1: W(0:ns) -= F12 W(ns:n)): F21 or
// F12 streamed once by the register-operand kernel for up to 32 right-hand sides, tiles through LDS beyond
template <class T>
hipError_t launch_sweep_product(const FrontDesc* d_fds, int nbatch, int maxn, int nrhs, int mode, hipStream_t s) {
  const dim3 sgrid((unsigned)blocks_for(maxn, sweep_skinny_tm<T>()), nbatch);
  if (nrhs <= SKINNY_TN) {
    hipLaunchKernelGGL((sweep_gemm_skinny_kernel<T, 1>), sgrid, dim3(256), 0, s, d_fds, nrhs, mode);
  } else if (nrhs <= 2 * SKINNY_TN) {
    hipLaunchKernelGGL((sweep_gemm_skinny_kernel<T, 2>), sgrid, dim3(256), 0, s, d_fds, nrhs, mode);
  } else {
    const int tiles = (int)(blocks_for(maxn, GEMM_TM) * blocks_for(nrhs, GEMM_TN));
    hipLaunchKernelGGL((sweep_gemm_kernel<T>), dim3(tiles, nbatch), dim3(256), 0, s, d_fds, nrhs, mode);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_forward_level(const FrontDesc* d_fds, int nbatch, int maxn, int maxnu, int maxns, const void* y,
                                int64_t N, int nrhs, hipStream_t s) {
  if (nbatch == 0) return hipSuccess;
  (void)maxnu;
  hipLaunchKernelGGL((fwd_gather_kernel<T>), dim3(blocks_for(maxn, 256), nbatch), dim3(256), 0, s, d_fds,
                     (const cplx<T>*)y, N, nrhs);
  KCHECK(hipGetLastError());
  if (sizeof(T) == 8 && maxns > 0) {
    // fronts with ns <= BLK_MAXNS whole (the kernel for the level's largest of them), then the
    // larger ones segment by segment with the panel products in between
    const dim3 grid((unsigned)((int64_t)nbatch * ((nrhs + BLK_RC - 1) / BLK_RC)));
    const int small = maxns <= BLK_MAXNS ? maxns : BLK_MAXNS;
    if (small <= 64)
      hipLaunchKernelGGL((fwd_trsv_blk_kernel<1>), grid, dim3(256), 0, s, d_fds, nbatch, nrhs, -1);
    else if (small <= 128)
      hipLaunchKernelGGL((fwd_trsv_blk_kernel<2>), grid, dim3(256), 0, s, d_fds, nbatch, nrhs, -1);
    else if (small <= 256)
      hipLaunchKernelGGL((fwd_trsv_blk_kernel<4>), grid, dim3(256), 0, s, d_fds, nbatch, nrhs, -1);
    else if (small <= 512)
      hipLaunchKernelGGL((fwd_trsv_blk_kernel<8>), grid, dim3(256), 0, s, d_fds, nbatch, nrhs, -1);
    else
      hipLaunchKernelGGL((fwd_trsv_blk_kernel<16>), grid, dim3(256), 0, s, d_fds, nbatch, nrhs, -1);
    KCHECK(hipGetLastError());
    const int tiles = (int)(blocks_for(maxn, SweepTile128x32::TM) * blocks_for(nrhs, SweepTile128x32::TN));
    for (int seg = 0; seg * BLK_MAXNS < maxns && maxns > BLK_MAXNS; ++seg) {
      hipLaunchKernelGGL((fwd_trsv_blk_kernel<16>), grid, dim3(256), 0, s, d_fds, nbatch, nrhs, seg);
      KCHECK(hipGetLastError());
      hipLaunchKernelGGL((sweep_seg_gemm_kernel<SweepTile128x32>), dim3(tiles, nbatch), dim3(256), 0, s, d_fds, nrhs,
                         seg, 0);
      KCHECK(hipGetLastError());
    }
  } else {  // complex64: one workgroup per front, one barrier per column
    hipLaunchKernelGGL((fwd_trsv_kernel<T>), dim3(nbatch), dim3(256), 0, s, d_fds, nrhs);
  }
  KCHECK(hipGetLastError());
  return launch_sweep_product<T>(d_fds, nbatch, maxn, nrhs, 0, s);
}

template <class T>
hipError_t launch_backward_level(const FrontDesc* d_fds, int nbatch, int maxn, int maxnu, int maxns, void* x,
                                 int64_t N, int nrhs, hipStream_t s) {
  if (nbatch == 0) return hipSuccess;
  if (maxnu > 0) {
    hipLaunchKernelGGL((bwd_gather_kernel<T>), dim3(blocks_for(maxnu, 256), nbatch), dim3(256), 0, s, d_fds,
                       (const cplx<T>*)x, N, nrhs);
    KCHECK(hipGetLastError());
    KCHECK(launch_sweep_product<T>(d_fds, nbatch, maxn, nrhs, 1, s));
  }
  if (sizeof(T) == 8 && maxns > 0) {
    const dim3 grid((unsigned)((int64_t)nbatch * ((nrhs + BLK_RC - 1) / BLK_RC)));
    cplx<double>* xd = (cplx<double>*)x;
    const int tiles = (int)(blocks_for(maxn, SweepTile128x32::TM) * blocks_for(nrhs, SweepTile128x32::TN));
    // the larger fronts segment by segment from the bottom, then the others whole
    for (int seg = (maxns - 1) / BLK_MAXNS; seg >= 0 && maxns > BLK_MAXNS; --seg) {
      hipLaunchKernelGGL((bwd_trsv_blk_kernel<16>), grid, dim3(256), 0, s, d_fds, nbatch, xd, N, nrhs, seg);
      KCHECK(hipGetLastError());
      hipLaunchKernelGGL((sweep_seg_gemm_kernel<SweepTile128x32>), dim3(tiles, nbatch), dim3(256), 0, s, d_fds, nrhs,
                         seg, 1);
      KCHECK(hipGetLastError());
    }
    const int small = maxns <= BLK_MAXNS ? maxns : BLK_MAXNS;
    if (small <= 64)
      hipLaunchKernelGGL((bwd_trsv_blk_kernel<1>), grid, dim3(256), 0, s, d_fds, nbatch, xd, N, nrhs, -1);
    else if (small <= 128)
      hipLaunchKernelGGL((bwd_trsv_blk_kernel<2>), grid, dim3(256), 0, s, d_fds, nbatch, xd, N, nrhs, -1);
    else if (small <= 256)
      hipLaunchKernelGGL((bwd_trsv_blk_kernel<4>), grid, dim3(256), 0, s, d_fds, nbatch, xd, N, nrhs, -1);
    else if (small <= 512)
      hipLaunchKernelGGL((bwd_trsv_blk_kernel<8>), grid, dim3(256), 0, s, d_fds, nbatch, xd, N, nrhs, -1);
    else
      hipLaunchKernelGGL((bwd_trsv_blk_kernel<16>), grid, dim3(256), 0, s, d_fds, nbatch, xd, N, nrhs, -1);
  } else {
    hipLaunchKernelGGL((bwd_trsv_kernel<T>), dim3(nbatch), dim3(256), 0, s, d_fds, (cplx<T>*)x, N, nrhs);
  }
  return hipGetLastError();
}

hipError_t launch_pivot_perm(const FrontDesc* d_fds, int nfront, hipStream_t s) {
  if (nfront == 0) return hipSuccess;
  hipLaunchKernelGGL(pivot_perm_kernel, dim3(nfront), dim3(256), PERM_MAXNS * sizeof(int32_t), s, d_fds, nfront);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fwd_gather(const FrontDesc* d_fds, int nbatch, int maxn, const void* y, int64_t N, int nrhs,
                             hipStream_t s) {
  if (nbatch == 0 || maxn == 0) return hipSuccess;
  hipLaunchKernelGGL((fwd_gather_kernel<T>), dim3(blocks_for(maxn, 256), nbatch), dim3(256), 0, s, d_fds,
                     (const cplx<T>*)y, N, nrhs);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bwd_gather(const FrontDesc* d_fds, int nbatch, int maxnu, const void* x, int64_t N, int nrhs,
                             hipStream_t s) {
  if (nbatch == 0 || maxnu == 0) return hipSuccess;
  hipLaunchKernelGGL((bwd_gather_kernel<T>), dim3(blocks_for(maxnu, 256), nbatch), dim3(256), 0, s, d_fds,
                     (const cplx<T>*)x, N, nrhs);
  return hipGetLastError();
}

hipError_t launch_spmv(const int64_t* rowptr, const int32_t* colind, const void* val, const void* X, int64_t ldx,
                       void* Y, int64_t ldy, const void* B, int64_t ldb, int64_t N, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(spmv_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s, rowptr, colind,
                     (const cplx<double>*)val, (const cplx<double>*)X, ldx, (cplx<double>*)Y, ldy,
                     (const cplx<double>*)B, ldb, N);
  return hipGetLastError();
}

hipError_t launch_dots(const void* V, int64_t ldv, const void* Wv, int64_t ldw, int64_t N, int nrhs, void* partial,
                       int nblk, void* out, bool norm, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nblk, nrhs), dim3(256), 0, s, (const cplx<double>*)V, ldv,
                     (const cplx<double>*)Wv, ldw, N, (cplx<double>*)partial);
  KCHECK(hipGetLastError());
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, (const cplx<double>*)partial, nblk, nrhs,
                     (cplx<double>*)out, norm ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(const void* a, double sign, const void* V, int64_t ldv, void* Wv, int64_t ldw, int64_t N,
                            int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(axpy_cols_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s, (const cplx<double>*)a,
                     sign, (const cplx<double>*)V, ldv, (cplx<double>*)Wv, ldw, N);
  return hipGetLastError();
}

hipError_t launch_scale_cols(const void* nrm, const void* Wv, int64_t ldw, void* V, int64_t ldv, int64_t N, int nrhs,
                             hipStream_t s) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s, (const cplx<double>*)nrm,
                     (const cplx<double>*)Wv, ldw, (cplx<double>*)V, ldv, N);
  return hipGetLastError();
}

hipError_t launch_basis_update(const void* y, int ldy, int m, const void* V, int64_t vstride, int64_t ldv, void* X,
                               int64_t ldx, int64_t N, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(basis_update_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s, (const cplx<double>*)y,
                     ldy, m, (const cplx<double>*)V, vstride, ldv, (cplx<double>*)X, ldx, N);
  return hipGetLastError();
}

hipError_t launch_slot_gather(const void* const* d_src, void* Vcur, int64_t ld, int64_t N, int ncol, hipStream_t s) {
  if (ncol == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(slot_gather_kernel, dim3(blocks_for(N, 256), ncol), dim3(256), 0, s,
                     (const cplx<double>* const*)d_src, (cplx<double>*)Vcur, ld, N);
  return hipGetLastError();
}

hipError_t launch_slot_fix(const int32_t* d_mode, const void* B, int64_t ldb, void* T, int64_t ldt, int64_t N, int ncol,
                           hipStream_t s) {
  if (ncol == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(slot_fix_kernel, dim3(blocks_for(N, 256), ncol), dim3(256), 0, s, d_mode,
                     (const cplx<double>*)B, ldb, (cplx<double>*)T, ldt, N);
  return hipGetLastError();
}

hipError_t launch_axpy_cols_masked(const void* a, double sign, const void* V, int64_t ldv, void* Wv, int64_t ldw,
                                   int64_t N, int nrhs, const int32_t* d_lim, int i0, hipStream_t s) {
  if (nrhs == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_cols_masked_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s,
                     (const cplx<double>*)a, sign, (const cplx<double>*)V, ldv, (cplx<double>*)Wv, ldw, N, d_lim, i0);
  return hipGetLastError();
}

hipError_t launch_scale_cols_to(const void* nrm, const void* Wv, int64_t ldw, void* const* d_dst, int64_t N, int nrhs,
                                hipStream_t s) {
  if (nrhs == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_to_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s,
                     (const cplx<double>*)nrm, (const cplx<double>*)Wv, ldw, (cplx<double>* const*)d_dst, N);
  return hipGetLastError();
}

hipError_t launch_basis_update_masked(const void* y, int ldy, const int32_t* d_mc, const void* V, int64_t vstride,
                                      int64_t ldv, void* X, int64_t ldx, int64_t N, int nrhs, hipStream_t s) {
  if (nrhs == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(basis_update_masked_kernel, dim3(blocks_for(N, 256), nrhs), dim3(256), 0, s,
                     (const cplx<double>*)y, ldy, d_mc, (const cplx<double>*)V, vstride, ldv, (cplx<double>*)X, ldx,
                     N);
  return hipGetLastError();
}

template hipError_t launch_permute_in<double>(const void*, int64_t, void*, const int64_t*, int64_t, int, hipStream_t);
template hipError_t launch_permute_in<float>(const void*, int64_t, void*, const int64_t*, int64_t, int, hipStream_t);
template hipError_t launch_permute_out<double>(const void*, void*, int64_t, const int64_t*, int64_t, int, hipStream_t);
template hipError_t launch_permute_out<float>(const void*, void*, int64_t, const int64_t*, int64_t, int, hipStream_t);
template hipError_t launch_forward_level<double>(const FrontDesc*, int, int, int, int, const void*, int64_t, int, hipStream_t);
template hipError_t launch_forward_level<float>(const FrontDesc*, int, int, int, int, const void*, int64_t, int, hipStream_t);
template hipError_t launch_fwd_gather<double>(const FrontDesc*, int, int, const void*, int64_t, int, hipStream_t);
template hipError_t launch_bwd_gather<double>(const FrontDesc*, int, int, const void*, int64_t, int, hipStream_t);
template hipError_t launch_backward_level<double>(const FrontDesc*, int, int, int, int, void*, int64_t, int, hipStream_t);
template hipError_t launch_backward_level<float>(const FrontDesc*, int, int, int, int, void*, int64_t, int, hipStream_t);

// B(rows[e], cols[e]) = vals[e] for the nonzeros of a block of right-hand
// sides (each (row, column) once)
__global__ void scatter_nz_kernel(cplx<double>* __restrict__ B, int64_t ldb, const int32_t* __restrict__ rows,
                                  const int32_t* __restrict__ cols, const double* __restrict__ vals, int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  B[rows[e] + (int64_t)cols[e] * ldb] = cplx<double>{vals[2 * e], vals[2 * e + 1]};
}

hipError_t launch_scatter_nz(void* B, int64_t ldb, const int32_t* rows, const int32_t* cols, const double* vals,
                             int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_nz_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, (cplx<double>*)B, ldb,
                     rows, cols, vals, nnz);
  return hipGetLastError();
}

}  // namespace bfmf
