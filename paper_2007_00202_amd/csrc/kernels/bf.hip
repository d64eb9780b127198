// Kernels of the butterfly algorithms (paper Sec. 3 and 4):
//   grouped GEMM      every block-diagonal butterfly factor level is one
//                     launch of independent ragged products (Sec. 3.1: a
//                     butterfly matvec is a chain of block-diagonal factors)
//   cpqr_id           interpolative decomposition of many small blocks by
//                     truncated column-pivoted Householder QR (Sec. 3)
//   id_expand         interpolation matrix U = P [I; (R11^-1 R12)^T]
//   front_extract     entries of a compressed front from the sparse matrix and
//                     the children's contribution blocks (Sec. 5, list routing)
//   philox_gauss      complex Gaussian probe vectors supported on one tree node
//   small_solve       X A = B for many small systems (least-squares centre)
//   leaf_inverse      explicit inverses of the dense HOD-BF leaves (Alg. 4)
#include <hip/hip_ext.h>

#include "../devtypes.hpp"
#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace bfmf {

// ------------------------------------------------------------ grouped GEMM
// the task owning grid tile `tile` (tile_start: first tile of each task) and the tile's index in it
__device__ __forceinline__ int find_task(const int64_t* __restrict__ tile_start, int ntasks, int64_t tile) {
  int lo = 0, hi = ntasks - 1;  // last task with tile_start <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// operand address = base + offset, in integer arithmetic; base 4 is zero (the offset is the
// operand's address in elements, for operands scattered over several allocations)
template <class T>
__device__ __forceinline__ uintptr_t task_addr(int i, int64_t off, void* b0, void* b1, void* b2, void* b3) {
  const uintptr_t b = i == 0 ? (uintptr_t)b0 : i == 1 ? (uintptr_t)b1 : i == 2 ? (uintptr_t)b2 : i == 3 ? (uintptr_t)b3 : 0;
  return b + (uintptr_t)off * sizeof(cplx<T>);
}

template <class T, class C>
__device__ __forceinline__ void grouped_gemm_run(const GTask* __restrict__ tasks,
                                                 const int64_t* __restrict__ tile_start, int ntasks, void* b0,
                                                 void* b1, void* b2, void* b3, TileSmem<T, C>& sm) {
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int lo = find_task(tile_start, ntasks, tile);
  const GTask& t = tasks[lo];
  const int64_t local = tile - tile_start[lo];
  const int tm = (t.M + C::TM - 1) / C::TM;
  const int tn = (t.N + C::TN - 1) / C::TN;
  if (local >= (int64_t)tm * tn || t.M <= 0 || t.N <= 0) return;
  const cplx<T>* A = (const cplx<T>*)task_addr<T>(t.abase, t.a_off, b0, b1, b2, b3);
  const cplx<T>* B = (const cplx<T>*)task_addr<T>(t.bbase, t.b_off, b0, b1, b2, b3);
  cplx<T>* Cm = (cplx<T>*)task_addr<T>(t.cbase, t.c_off, b0, b1, b2, b3);
  const cplx<T> alpha = {(T)t.alpha_re, (T)t.alpha_im};
  gemm_tile_cfg<T, C>(A, t.lda, t.opA, B, t.ldb, t.opB, Cm, t.ldc, t.M, t.N, t.K, alpha, t.beta, (int)(local % tm),
                      (int)(local / tm), sm);
}

// butterfly products (and every other grouped product but the Gram matrices of the IDs)
template <class T, class C>
__global__ __launch_bounds__(256, C::MINB) void grouped_gemm_kernel(const GTask* __restrict__ tasks,
                                                           const int64_t* __restrict__ tile_start, int ntasks,
                                                           void* b0, void* b1, void* b2, void* b3) {
  __shared__ TileSmem<T, C> sm;
  grouped_gemm_run<T, C>(tasks, tile_start, ntasks, b0, b1, b2, b3, sm);
}

// the same product for the Gram matrices G = A^H A of the interpolative decompositions (a kernel of
// its own name, so that profiles tell the two classes apart)
template <class T, class C>
__global__ __launch_bounds__(256, C::MINB) void gram_gemm_kernel(const GTask* __restrict__ tasks,
                                                        const int64_t* __restrict__ tile_start, int ntasks,
                                                        void* b0, void* b1, void* b2, void* b3) {
  __shared__ TileSmem<T, C> sm;
  grouped_gemm_run<T, C>(tasks, tile_start, ntasks, b0, b1, b2, b3, sm);
}

// the LDS tile shapes of the launcher's cfg index (GEMM_CFG_TM / GEMM_CFG_TN)
typedef TileCfg<2, 2, 2, 2> Tile64x64;
typedef TileCfg<2, 2, 1, 4> Tile32x128;
typedef TileCfg<2, 2, 4, 1> Tile128x32;
typedef TileCfg<1, 4, 1, 4> Tile16x256;
typedef TileCfg<4, 1, 4, 1> Tile256x16;
typedef TileCfg<3, 2, 1, 4> Tile48x128;
typedef TileCfg<3, 2, 2, 2> Tile96x64;
static_assert(Tile64x64::TM == GEMM_CFG_TM[0] && Tile64x64::TN == GEMM_CFG_TN[0], "tile table");
static_assert(Tile32x128::TM == GEMM_CFG_TM[1] && Tile32x128::TN == GEMM_CFG_TN[1], "tile table");
static_assert(Tile128x32::TM == GEMM_CFG_TM[2] && Tile128x32::TN == GEMM_CFG_TN[2], "tile table");
static_assert(Tile16x256::TM == GEMM_CFG_TM[3] && Tile16x256::TN == GEMM_CFG_TN[3], "tile table");
static_assert(Tile256x16::TM == GEMM_CFG_TM[4] && Tile256x16::TN == GEMM_CFG_TN[4], "tile table");
static_assert(SKINNY_TM == GEMM_CFG_TM[GEMM_CFG_SKINNY] && SKINNY_TN == GEMM_CFG_TN[GEMM_CFG_SKINNY], "tile table");
static_assert(Tile48x128::TM == GEMM_CFG_TM[6] && Tile48x128::TN == GEMM_CFG_TN[6], "tile table");
static_assert(Tile96x64::TM == GEMM_CFG_TM[7] && Tile96x64::TN == GEMM_CFG_TN[7], "tile table");

// phases whose tasks are all C = beta C + alpha A B (no transposes) with N <= 16: 256-row tiles
template <class T>
__global__ __launch_bounds__(256) void grouped_gemm_skinny_kernel(const GTask* __restrict__ tasks,
                                                                  const int64_t* __restrict__ tile_start, int ntasks,
                                                                  void* b0, void* b1, void* b2, void* b3) {
  const int64_t tile = blockIdx.x;
  const int lo = find_task(tile_start, ntasks, tile);
  const GTask& t = tasks[lo];
  const int64_t local = tile - tile_start[lo];
  const int tm = (t.M + SKINNY_TM - 1) / SKINNY_TM;
  if (local >= tm || t.M <= 0 || t.N <= 0 || t.N > SKINNY_TN) return;
  const cplx<T>* A = (const cplx<T>*)task_addr<T>(t.abase, t.a_off, b0, b1, b2, b3);
  const cplx<T>* B = (const cplx<T>*)task_addr<T>(t.bbase, t.b_off, b0, b1, b2, b3);
  cplx<T>* C = (cplx<T>*)task_addr<T>(t.cbase, t.c_off, b0, b1, b2, b3);
  const cplx<T> alpha = {(T)t.alpha_re, (T)t.alpha_im};
  gemm_tile_skinny<T>(A, t.lda, B, t.ldb, C, t.ldc, t.M, t.N, t.K, alpha, t.beta, (int)local);
}

// ---------------------------------------------------------------- CPQR ID
// One workgroup of CPQR_THREADS threads per block.  Columns of A (q x p) are
// pivoted by largest remaining norm (first maximum); the factorization stops
// at the first |R_kk| <= tol |R_00| (rank k) or at maxrank.  Householder
// vectors live in LDS; one wave applies a reflector to one column at a time,
// so the trailing columns of a step stream through the CU with 16 waves in
// flight.  The column norms and the permutation live in dynamic LDS: maxp
// doubles, then maxp ints.
constexpr int ID_MAXQ = CPQR_MAXQ;
constexpr int CPQR_THREADS = 1024;
constexpr int CPQR_WAVES = CPQR_THREADS / 64;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// the workgroup's largest v (first index i on ties) into bv, bi for every thread; red_v and
// red_i hold one entry per wave and are not read again before the caller's next barrier
__device__ __forceinline__ void cpqr_argmax(double v, int i, double* red_v, int* red_i, double& bv, int& bi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(i, o);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red_v[wave] = v;
    red_i[wave] = i;
  }
  __syncthreads();
  bv = red_v[0];
  bi = red_i[0];
  for (int w = 1; w < CPQR_WAVES; ++w)
    if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bi)) {
      bv = red_v[w];
      bi = red_i[w];
    }
}

// the workgroup's sum of v for every thread, added in wave order (the same value in every thread)
__device__ __forceinline__ double cpqr_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < CPQR_WAVES; ++w) t += red[w];
  return t;
}

template <class T>
__global__ __launch_bounds__(CPQR_THREADS) void cpqr_id_kernel(const IdTask* __restrict__ tasks, double tol, int maxp) {
  const IdTask& tk = tasks[blockIdx.x];
  const int q = tk.q, p = tk.p;
  const int64_t lda = tk.lda;
  cplx<T>* A = (cplx<T>*)tk.A;
  if (q > ID_MAXQ || p > maxp || q < 0 || p < 0) {  // the host never sends these; refuse, never overflow LDS
    if (threadIdx.x == 0) *tk.rank = -1;
    return;
  }
  extern __shared__ __align__(16) unsigned char cpqr_smem[];
  double* nrm = (double*)cpqr_smem;
  int* perm = (int*)(cpqr_smem + (size_t)maxp * sizeof(double));
  __shared__ cplx<T> v[ID_MAXQ];
  // per-wave partials, two sets each used on alternate steps: a set is written again only two
  // steps later, after several barriers, so no barrier is needed behind its readers
  __shared__ double red_v[2][CPQR_WAVES];
  __shared__ int red_i[2][CPQR_WAVES];
  __shared__ double red_s[2][CPQR_WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = wave; j < p; j += CPQR_WAVES) {  // squared column norms, one column per wave
    const cplx<T>* a = A + (int64_t)j * lda;
    double s = 0;
    for (int i = lane; i < q; i += 64) s += (double)a[i].re * a[i].re + (double)a[i].im * a[i].im;
    s = wave_sum(s);
    if (lane == 0) {
      nrm[j] = s;
      perm[j] = j;
    }
  }
  __syncthreads();
  const int kmax = min(min(p, q), tk.maxrank);
  double ref = 0;  // |R_00|
  int k = 0;
  for (; k < kmax; ++k) {
    // pivot: largest remaining norm, first index on ties
    double best = -1;
    int bi = p;
    for (int j = k + tid; j < p; j += CPQR_THREADS)
      if (nrm[j] > best) {
        best = nrm[j];
        bi = j;
      }
    double bv;
    int jp;
    cpqr_argmax(best, bi, red_v[k & 1], red_i[k & 1], bv, jp);
    if (jp != k && jp < p) {
      cplx<T>* a = A + (int64_t)k * lda;
      cplx<T>* b = A + (int64_t)jp * lda;
      for (int i = tid; i < q; i += CPQR_THREADS) {
        const cplx<T> t = a[i];
        a[i] = b[i];
        b[i] = t;
      }
      if (tid == 0) {
        const double tn = nrm[k];
        nrm[k] = nrm[jp];
        nrm[jp] = tn;
        const int tp = perm[k];
        perm[k] = perm[jp];
        perm[jp] = tp;
      }
    }
    __syncthreads();
    // exact norm of the trailing part of column k
    cplx<T>* ak = A + (int64_t)k * lda;
    double s = 0;
    for (int i = k + tid; i < q; i += CPQR_THREADS) s += (double)ak[i].re * ak[i].re + (double)ak[i].im * ak[i].im;
    const double alpha = sqrt(cpqr_sum(s, red_s[k & 1]));
    if (k == 0) ref = alpha;
    if (!(alpha > tol * ref) || alpha == 0) break;
    // Householder vector v = x + s alpha e1, tau = 1 / (alpha (alpha + |x0|))
    const cplx<T> x0 = ak[k];
    const double ax0 = sqrt((double)x0.re * x0.re + (double)x0.im * x0.im);
    const double sr = ax0 > 0 ? x0.re / ax0 : 1.0, si = ax0 > 0 ? x0.im / ax0 : 0.0;
    const double tau = 1.0 / (alpha * (alpha + ax0));
    for (int i = k + tid; i < q; i += CPQR_THREADS) {
      cplx<T> x = ak[i];
      if (i == k) {
        x.re = (T)(x.re + sr * alpha);
        x.im = (T)(x.im + si * alpha);
      }
      v[i] = x;
    }
    __syncthreads();
    if (tid == 0) {
      ak[k] = cplx<T>{(T)(-sr * alpha), (T)(-si * alpha)};  // R_kk
    }
    // apply H to columns k+1..p-1: a -= tau v (v^H a), two columns per wave at a time (j and
    // j + CPQR_WAVES) for twice the independent loads in flight; each column's sums run in the
    // same order as with one column at a time
    for (int j = k + 1 + wave; j < p; j += 2 * CPQR_WAVES) {
      const bool two = j + CPQR_WAVES < p;
      cplx<T>* a = A + (int64_t)j * lda;
      cplx<T>* b = A + (int64_t)(two ? j + CPQR_WAVES : j) * lda;  // read only, as a, when !two
      double wr = 0, wi = 0, xr = 0, xi = 0;
      for (int i = k + lane; i < q; i += 64) {
        const cplx<T> vi = v[i], ai = a[i], bi = b[i];
        wr += (double)vi.re * ai.re + (double)vi.im * ai.im;
        wi += (double)vi.re * ai.im - (double)vi.im * ai.re;
        xr += (double)vi.re * bi.re + (double)vi.im * bi.im;
        xi += (double)vi.re * bi.im - (double)vi.im * bi.re;
      }
      wr = wave_sum(wr);
      wi = wave_sum(wi);
      xr = wave_sum(xr);
      xi = wave_sum(xi);
      const double cr = tau * wr, ci = tau * wi, dr = tau * xr, di = tau * xi;
      for (int i = k + lane; i < q; i += 64) {
        const cplx<T> vi = v[i];
        a[i].re -= (T)(vi.re * cr - vi.im * ci);
        a[i].im -= (T)(vi.re * ci + vi.im * cr);
        if (two) {
          b[i].re -= (T)(vi.re * dr - vi.im * di);
          b[i].im -= (T)(vi.re * di + vi.im * dr);
        }
      }
    }
    __syncthreads();
    // downdate the remaining column norms with the new row k of R
    for (int j = k + 1 + tid; j < p; j += CPQR_THREADS) {
      const cplx<T> r = A[k + (int64_t)j * lda];
      const double d = nrm[j] - ((double)r.re * r.re + (double)r.im * r.im);
      nrm[j] = d > 0 ? d : 0;
    }
    __syncthreads();
  }
  const int rank = k;
  if (tid == 0) *tk.rank = rank;
  for (int j = tid; j < p; j += CPQR_THREADS) tk.perm[j] = perm[j];
  // T = R11^-1 R12: back substitution, one thread per column of R12
  cplx<T>* Tout = (cplx<T>*)tk.T;
  const int ldt = tk.maxrank;
  for (int j = rank + tid; j < p; j += CPQR_THREADS) {
    cplx<T>* tcol = Tout + (int64_t)(j - rank) * ldt;
    for (int i = rank - 1; i >= 0; --i) {
      cplx<T> s = A[i + (int64_t)j * lda];
      for (int l = i + 1; l < rank; ++l) s = csub(s, cmul(A[i + (int64_t)l * lda], tcol[l]));
      tcol[i] = cdiv(s, A[i + (int64_t)i * lda]);
    }
  }
}

// ------------------------------------------------------------ Gram ID
// The same decomposition from the Gram matrix G = A^H A = R^H R: pivoted
// Cholesky, left-looking (row k of R from G's pivot column and the k rows
// before it), chooses at each step the largest remaining squared column norm
// d_j (first index on ties) and stops at the first d <= tol^2 d_0, which in
// exact arithmetic are the pivots and the rank of the column-pivoted QR.
// T = R11^-1 R12 by back substitution over the whole workgroup.
// Rounding in G limits the accuracy of T to about eps p / tol^2 (relative),
// so the host uses this variant only for tolerances where that is small.

// R (rows 0 .. kmax-1 of the factor, row i at R + i p) lives in LDS when it fits
// the launch's dynamic LDS, else in the task's workspace; the body is the same.
// One workgroup of GRAM_THREADS threads per block: the steps are latency-bound
// (each needs the previous step's pivot), so more lanes per block shorten the
// dot products of a step.
constexpr int GRAM_THREADS = 1024;
// RG: R in device memory (else in LDS)
template <class T, bool RG>
__device__ __forceinline__ void gram_id_body(const IdTask& tk, double tol, cplx<T>* __restrict__ R,
                                             unsigned char* __restrict__ aux, int maxp) {
  const int p = tk.p;
  const cplx<T>* G = (const cplx<T>*)tk.G;
  auto rget = [&](int64_t i) -> cplx<T> {
    if constexpr (RG)
      return gld(R + i);
    else
      return R[i];
  };
  auto rput = [&](int64_t i, cplx<T> v) {
    if constexpr (RG)
      gst(R + i, v);
    else
      R[i] = v;
  };
  // per-column state in the launch's dynamic LDS (maxp entries each; maxp is a multiple of 16)
  cplx<T>* rc = (cplx<T>*)aux;  // R(0:k, pivot) of the step
  cplx<T>* tl = rc + maxp;      // row i of T in the back substitution
  double* d = (double*)(tl + maxp);
  int* sel = (int*)(d + maxp);  // step at which a column was chosen, or -1
  int* piv = sel + maxp;
  int* pl = piv + maxp;         // the permutation
  __shared__ double red_v[2][GRAM_THREADS / 64];
  __shared__ int red_i[2][GRAM_THREADS / 64];
  const int tid = threadIdx.x;
  for (int j = tid; j < p; j += GRAM_THREADS) {
    d[j] = (double)gld(G + j + (int64_t)j * p).re;
    sel[j] = -1;
  }
  __syncthreads();
  const int kmax = min(tk.maxrank, p);
  // lanes per column in the row update: GRAM_THREADS / p rounded down to a power of two, at most 16
  int tpc = 1;
  while (tpc < 16 && 2 * tpc * p <= GRAM_THREADS) tpc *= 2;
  const int pcols = (p + GRAM_THREADS / tpc - 1) / (GRAM_THREADS / tpc) * (GRAM_THREADS / tpc);  // columns padded to whole passes
  const int part = tid & (tpc - 1);
  const int wave = tid >> 6, lane = tid & 63;
  // the pivot search of a step: each thread's candidate (largest d, first index on ties), the wave's
  // by shuffles, the four waves' through a double-buffered exchange behind the step's one barrier
  auto publish = [&](double v, int vi, int buf) {
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(v, o);
      const int oi = __shfl_xor(vi, o);
      if (ov > v || (ov == v && oi < vi)) {
        v = ov;
        vi = oi;
      }
    }
    if (lane == 0) {
      red_v[buf][wave] = v;
      red_i[buf][wave] = vi;
    }
  };
  {
    double v = -1;
    int vi = p;
    for (int j = tid; j < p; j += GRAM_THREADS)
      if (d[j] > v) {
        v = d[j];
        vi = j;
      }
    publish(v, vi, 0);
  }
  __syncthreads();
  double d0 = 0;
  int k = 0;
  for (; k < kmax; ++k) {
    double dmax = red_v[k & 1][0];
    int pi = red_i[k & 1][0];
    for (int w = 1; w < GRAM_THREADS / 64; ++w)
      if (red_v[k & 1][w] > dmax || (red_v[k & 1][w] == dmax && red_i[k & 1][w] < pi)) {
        dmax = red_v[k & 1][w];
        pi = red_i[k & 1][w];
      }
    if (k == 0) d0 = dmax;
    if (!(dmax > tol * tol * d0) || !(dmax > 0) || pi >= p) break;  // the same decision in every thread
    const double rkk = sqrt(dmax);
    // row k: R(k, j) = (G(pi, j) - sum_i conj(R(i, pi)) R(i, j)) / rkk, G(pi, j) = conj(G(j, pi));
    // tpc adjacent lanes share a column's sum (lane part takes i = part, part + tpc, ...)
    double v = -1;  // this thread's candidate for the next pivot
    int vi = p;
    for (int j = tid / tpc; j < pcols; j += GRAM_THREADS / tpc) {
      const bool live = j < p && j != pi && sel[j] < 0;
      // G(j, pi) requested before the sum so that its latency overlaps the sum
      cplx<T> g = {0, 0};
      if (live && part == 0) g = gld(G + j + (int64_t)pi * p);
      double sr = 0, si = 0;
      if (live)
        for (int i = part; i < k; i += tpc) {
          const cplx<T> a = rget((int64_t)i * p + pi), b = rget((int64_t)i * p + j);
          sr += (double)a.re * b.re + (double)a.im * b.im;  // conj(a) b
          si += (double)a.re * b.im - (double)a.im * b.re;
        }
      for (int o = 1; o < tpc; o <<= 1) {  // lanes of one column are adjacent within a wave
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
      }
      if (part == 0 && j < p) {
        cplx<T> out = {0, 0};
        if (j == pi) {
          out.re = (T)rkk;
        } else if (live) {
          const double gr = (double)g.re - sr, gi = -(double)g.im - si;
          out.re = (T)(gr / rkk);
          out.im = (T)(gi / rkk);
          double nd = d[j] - (gr * gr + gi * gi) / dmax;
          nd = nd > 0 ? nd : 0;
          d[j] = nd;
          if (nd > v) {  // columns are visited in ascending order: the first on ties is kept
            v = nd;
            vi = j;
          }
        }
        rput((int64_t)k * p + j, out);
      }
    }
    if (tid == 0) {
      sel[pi] = k;
      piv[k] = pi;
    }
    publish(v, vi, (k + 1) & 1);
    __syncthreads();  // row k, d, sel and the next pivot are visible
  }
  const int rank = k;
  // perm: the pivots, then the other columns in ascending order
  if (tid == 0) {
    gst(tk.rank, (int32_t)rank);
    int c = rank;
    for (int j = 0; j < p; ++j) {
      if (sel[j] >= 0)
        pl[sel[j]] = j;
      else
        pl[c++] = j;
    }
  }
  __syncthreads();
  for (int j = tid; j < p; j += GRAM_THREADS) gst(tk.perm + j, (int32_t)pl[j]);
  // T = R11^-1 R12 with R11(i, m) = R(i, piv[m]) (upper triangular) and R12(:, c) = R(:, pl[rank + c]):
  // back substitution by columns of R11, every (row, column) update of a step in parallel
  cplx<T>* Tout = (cplx<T>*)tk.T;
  const int ldt = tk.maxrank;
  const int nc = p - rank;
  for (int e = tid; e < rank * nc; e += GRAM_THREADS) {
    const int i = e % rank, c = e / rank;
    gst(Tout + i + (int64_t)c * ldt, rget((int64_t)i * p + pl[rank + c]));
  }
  __syncthreads();
  for (int i = rank - 1; i >= 0; --i) {
    const cplx<T> rii = rget((int64_t)i * p + piv[i]);
    for (int c = tid; c < nc; c += GRAM_THREADS) {
      cplx<T>* tp = Tout + i + (int64_t)c * ldt;
      const cplx<T> t = cdiv(gld(tp), rii);
      gst(tp, t);
      tl[c] = t;
    }
    for (int m = tid; m < i; m += GRAM_THREADS) rc[m] = rget((int64_t)m * p + piv[i]);
    __syncthreads();
    for (int e = tid; e < i * nc; e += GRAM_THREADS) {
      const int m = e % i, c = e / i;
      cplx<T>* tp = Tout + m + (int64_t)c * ldt;
      gst(tp, csub(gld(tp), cmul(rc[m], tl[c])));
    }
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(GRAM_THREADS) void gram_id_kernel(const IdTask* __restrict__ tasks, double tol, int lds_entries,
                                                      int maxp) {
  extern __shared__ __align__(16) unsigned char gram_smem[];
  const IdTask& tk = tasks[blockIdx.x];
  const int p = tk.p;
  if (p > maxp || p > GRAM_MAXP || p < 0 || tk.q < 0) {  // the host never sends these; refuse, never overflow LDS
    if (threadIdx.x == 0) *tk.rank = -1;
    return;
  }
  unsigned char* aux = gram_smem;
  cplx<T>* Rl = (cplx<T>*)(gram_smem + gram_aux_bytes(maxp));
  if ((int64_t)min(tk.maxrank, p) * p <= lds_entries)
    gram_id_body<T, false>(tk, tol, Rl, aux, maxp);
  else
    gram_id_body<T, true>(tk, tol, (cplx<T>*)tk.R, aux, maxp);
}

// U (p x rank, ld p): U[perm[i], i] = 1 (i < rank), U[perm[rank + j], :] = T[:, j]^T,
// or its conjugate transpose layout Ut (rank x p) when transpose_out (column ID).
template <class T>
__global__ void id_expand_kernel(const IdTask* __restrict__ tasks, void* const* __restrict__ outs,
                                 const int64_t* __restrict__ ldo, int transpose_out, int conj_out) {
  const IdTask& tk = tasks[blockIdx.x];
  const int p = tk.p, rank = *tk.rank;
  cplx<T>* U = (cplx<T>*)outs[blockIdx.x];
  const int64_t ld = ldo[blockIdx.x];
  const cplx<double>* Tm = (const cplx<double>*)tk.T;  // decompositions are computed in FP64
  const int ldt = tk.maxrank;
  for (int e = threadIdx.x; e < p * rank; e += blockDim.x) {
    const int row = e % p, col = e / p;  // position in the pivoted order, basis column
    cplx<T> val;
    if (row < rank) {
      val = cplx<T>{(T)(row == col ? 1 : 0), 0};
    } else {
      const cplx<double> t = Tm[col + (int64_t)(row - rank) * ldt];
      val = cplx<T>{(T)t.re, (T)t.im};
    }
    if (conj_out) val.im = -val.im;
    const int r = tk.perm[row];
    if (transpose_out)
      U[col + (int64_t)r * ld] = val;
    else
      U[r + (int64_t)col * ld] = val;
  }
}

// ------------------------------------------------------------ extraction
// node k of a sorted boundary list b[0..n] with b[k] <= x < b[k + 1] (empty nodes skipped)
__device__ __forceinline__ int node_of(const int32_t* __restrict__ b, int n, int x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (b[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// K(x, y) of a butterfly in centre form: one dot product of the centre block's rank (FP64 sums)
template <class TE>
__device__ double2 centre_dot(const BfCentreDev& B, int x, int y) {
  const int t = node_of(B.tb, B.nt, x), v = node_of(B.vb, B.nv, y);
  const int blk = t * B.nv + v;
  const int r = B.rk[blk];
  const int64_t lde = B.tb[t + 1] - B.tb[t];
  const cplx<TE>* E = (const cplx<TE>*)B.E[blk] + (x - B.tb[t]);
  const cplx<TE>* G = (const cplx<TE>*)B.G[blk] + (int64_t)(y - B.vb[v]) * r;
  double re = 0, im = 0;
  for (int k = 0; k < r; ++k) {
    const cplx<TE> e = E[k * lde], g = G[k];
    re += (double)e.re * (double)g.re - (double)e.im * (double)g.im;
    im += (double)e.re * (double)g.im + (double)e.im * (double)g.re;
  }
  return make_double2(re, im);
}

__device__ __forceinline__ double2 bf_entry(const BfCentreDev& B, int x, int y) {
  return B.single ? centre_dot<float>(B, x, y) : centre_dot<double>(B, x, y);
}

// C(i, j) of a contribution block in HOD-BF form (Sec. 4): descend while i and j fall on the
// same side of a node; a leaf gives a dense entry, a split the entry of that node's
// off-diagonal butterfly (extract_HODBF through extract_BF)
__device__ double2 hodbf_entry(const HodbfDev& H, int i, int j) {
  int node = 0;
  for (int d = 0; d <= H.depth; ++d) {
    const HodbfNodeDev& nd = H.nodes[node];
    if (nd.left < 0) {
      const int64_t k = (int64_t)(i - nd.beg) + (int64_t)(j - nd.beg) * (nd.end - nd.beg);
      if (H.single) {
        const cplx<float> v = ((const cplx<float>*)nd.leaf)[k];
        return make_double2(v.re, v.im);
      }
      const cplx<double> v = ((const cplx<double>*)nd.leaf)[k];
      return make_double2(v.re, v.im);
    }
    const bool si = i >= nd.mid, sj = j >= nd.mid;
    if (si == sj) {
      node = si ? nd.right : nd.left;
      continue;
    }
    const int b = si ? nd.b21 : nd.b12;
    if (b < 0) return make_double2(0.0, 0.0);
    return si ? bf_entry(H.bfs[b], i - nd.mid, j - nd.beg) : bf_entry(H.bfs[b], i - nd.beg, j - nd.mid);
  }
  return make_double2(0.0, 0.0);  // not reached for a well-formed tree
}

// out(i, j) = alpha K(rows[i], cols[j]) (+ out when accumulate) for butterflies in centre form
template <class TO>
__global__ __launch_bounds__(256) void bf_extract_kernel(const BfExtractTask* __restrict__ tasks) {
  const BfExtractTask& tk = tasks[blockIdx.x];
  cplx<TO>* out = (cplx<TO>*)tk.out;
  const int nr = tk.nr, nc = tk.nc;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < (int64_t)nr * nc; e += (int64_t)gridDim.y * 256) {
    const int ii = (int)(e % nr), jj = (int)(e / nr);
    const double2 v = bf_entry(*tk.bf, tk.rows[ii], tk.cols[jj]);
    cplx<TO>* dst = tk.trans ? out + jj + (int64_t)ii * tk.ldo : out + ii + (int64_t)jj * tk.ldo;
    double re = tk.alpha * v.x, im = tk.alpha * v.y;
    if (tk.accumulate) {
      re += (double)dst->re;
      im += (double)dst->im;
    }
    *dst = cplx<TO>{(TO)re, (TO)im};
  }
}

// out(i, j) = F(rows[i], cols[j]) with F = [A(Is,Is) A(Is,Iu); A(Iu,Is) 0]
// (+) C_nu1 (+) C_nu2 (list routing: the sparse matrix, then each child's
// contribution block, dense or in HOD-BF form); one workgroup per task,
// threads over entries.
template <class T, class TC>
__global__ __launch_bounds__(256) void front_extract_kernel(const ExtractTask* __restrict__ tasks,
                                                            const cplx<double>* __restrict__ values) {
  const ExtractTask& tk = tasks[blockIdx.x];
  const FrontDesc* fd = tk.fd;
  cplx<T>* out = (cplx<T>*)tk.out;
  const int nr = tk.nr, nc = tk.nc;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < (int64_t)nr * nc; e += (int64_t)gridDim.y * 256) {
    const int ii = (int)(e % nr), jj = (int)(e / nr);
    const int i = tk.rows[ii], j = tk.cols[jj];
    cplx<T>* dst = tk.trans ? out + jj + (int64_t)ii * tk.ldo : out + ii + (int64_t)jj * tk.ldo;
    if (tk.dense) {  // dense source of the launch's source type
      const TC v = ((const TC*)tk.dense)[i + (int64_t)j * tk.ldd];
      *dst = cplx<T>{(T)v.re, (T)v.im};
      continue;
    }
    double vr = 0, vi = 0;
    for (int64_t t = fd->a_ptr[j]; t < fd->a_ptr[j + 1]; ++t)
      if (fd->a_row[t] == i) {
        const cplx<double> a = values[fd->a_vidx[t]];
        vr += a.re;
        vi += a.im;
      }
    for (int c = 0; c < fd->nchild; ++c) {
      const int ki = fd->inv[c][i], kj = fd->inv[c][j];
      if (ki >= 0 && kj >= 0) {
        if (fd->chb[c]) {
          const double2 v = hodbf_entry(*fd->chb[c], ki, kj);
          vr += v.x;
          vi += v.y;
        } else {
          const TC v = ((const TC*)fd->cb[c])[ki + (int64_t)kj * fd->cb_ld[c]];
          vr += v.re;
          vi += v.im;
        }
      }
    }
    *dst = cplx<T>{(T)vr, (T)vi};
  }
}

// ------------------------------------------------------------ Philox probes
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// multiply-xor round function with the published multipliers and Weyl key
// increments; a 4x32 counter gives 4 uniforms, Box-Muller turns 2 uniforms
// into one complex Gaussian of unit variance (E|z|^2 = 1).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k0 += W0;
    k1 += W1;
  }
}

// Omega (n x ncol, ld n): column c belongs to group g = c / width; group g is
// supported on rows [gbeg[g], gend[g]) and zero elsewhere.
template <class T>
__device__ __forceinline__ cplx<T> probe_entry(int64_t i, int c, uint64_t seed, uint64_t stream_id) {
  uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)c, (uint32_t)stream_id};
  philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)(stream_id >> 32));
  const double u1 = ((double)ctr[0] + 1.0) * (1.0 / 4294967296.0);  // (0, 1]
  const double u2 = (double)ctr[1] * (1.0 / 4294967296.0);
  const double rad = sqrt(-log(u1));  // |z|^2 ~ Exp(1): unit variance complex
  return cplx<T>{(T)(rad * cos(6.283185307179586 * u2)), (T)(rad * sin(6.283185307179586 * u2))};
}

template <class T>
__global__ void philox_gauss_kernel(cplx<T>* __restrict__ Om, int64_t ld, int64_t n, int ncol, int width,
                                    const int32_t* __restrict__ gbeg, const int32_t* __restrict__ gend,
                                    uint64_t seed, uint64_t stream_id) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= ncol) return;
  const int g = c / width;
  cplx<T> z = {0, 0};
  if (i >= gbeg[g] && i < gend[g]) z = probe_entry<T>(i, c, seed, stream_id);
  Om[i + (int64_t)c * ld] = z;
}

// the same probe blocks for many tasks in one launch (grid row = task)
template <class T>
__global__ __launch_bounds__(256) void philox_gauss_batch_kernel(const ProbeTask* __restrict__ tasks,
                                                                 const int32_t* __restrict__ gbeg,
                                                                 const int32_t* __restrict__ gend, uint64_t seed) {
  const ProbeTask& t = tasks[blockIdx.x];
  const int64_t tot = t.n * t.ncol;
  cplx<T>* Om = (cplx<T>*)t.Om;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.y * 256) {
    const int64_t i = e % t.n;
    const int c = (int)(e / t.n);
    const int g = t.g0 + c / t.width;
    cplx<T> z = {0, 0};
    if (i >= gbeg[g] && i < gend[g]) z = probe_entry<T>(i, c, seed, t.stream_id);
    Om[i + (int64_t)c * t.ld] = z;
  }
}

// ------------------------------------------------------------ small solves
// X A = B for each task: A k x k (lda), B r x k (ldb, overwritten by X).
// Gaussian elimination with partial pivoting on A^T, one workgroup per task,
// A is destroyed.  Per column: the pivot (first row maximising |Re| + |Im|)
// by wave shuffles and one exchange between the waves, the interchange, the
// multipliers, then the trailing update of A^T and the same row operations
// on B^T with every entry in parallel.  Back substitution by columns of the
// triangle (x_c for all rows of B, then its contribution to the columns
// before it), again every entry in parallel.  SOLVE_THREADS lanes per task:
// the steps are sequential, so more lanes shorten each step.
constexpr int SOLVE_THREADS = 1024;

template <class T>
__global__ __launch_bounds__(SOLVE_THREADS) void small_solve_right_kernel(const SolveTask* __restrict__ tasks) {
  const SolveTask& tk = tasks[blockIdx.x];
  const int k = tk.k, r = tk.r;
  cplx<T>* A = (cplx<T>*)tk.A;
  cplx<T>* B = (cplx<T>*)tk.B;
  const int64_t lda = tk.lda, ldb = tk.ldb;
  // X A = B  <=>  A^T X^T = B^T.  Work on At(i, j) = A(j, i): rows of A^T are
  // columns of A.  Eliminate with row pivoting on A^T == column pivoting of A.
  __shared__ double red_v[2][SOLVE_THREADS / 64];
  __shared__ int red_i[2][SOLVE_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = 0; c < k; ++c) {
    const int buf = c & 1;
    // pivot among At rows c..k-1 of column c: At(i, c) = A(c, i)
    double best = -1;
    int bi = c;
    for (int i = c + tid; i < k; i += SOLVE_THREADS) {
      const double a = cabs1(A[c + (int64_t)i * lda]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[buf][wave] = best;
      red_i[buf][wave] = bi;
    }
    __syncthreads();
    double pv = red_v[buf][0];
    int pr = red_i[buf][0];
    for (int w = 1; w < SOLVE_THREADS / 64; ++w)
      if (red_v[buf][w] > pv || (red_v[buf][w] == pv && red_i[buf][w] < pr)) {
        pv = red_v[buf][w];
        pr = red_i[buf][w];
      }
    if (pr != c) {  // swap At rows c and pr: columns c, pr of A; columns c, pr of B
      for (int j = tid; j < k; j += SOLVE_THREADS) {
        const cplx<T> t = A[j + (int64_t)c * lda];
        A[j + (int64_t)c * lda] = A[j + (int64_t)pr * lda];
        A[j + (int64_t)pr * lda] = t;
      }
      for (int j = tid; j < r; j += SOLVE_THREADS) {
        const cplx<T> t = B[j + (int64_t)c * ldb];
        B[j + (int64_t)c * ldb] = B[j + (int64_t)pr * ldb];
        B[j + (int64_t)pr * ldb] = t;
      }
    }
    __syncthreads();
    const cplx<T> d = A[c + (int64_t)c * lda];
    const bool ok = cabs1(d) > 0;
    // multipliers l_i = At(i, c) / At(c, c), kept in At(i, c)
    for (int i = c + 1 + tid; i < k; i += SOLVE_THREADS)
      A[c + (int64_t)i * lda] = ok ? cdiv(A[c + (int64_t)i * lda], d) : cplx<T>{0, 0};
    __syncthreads();
    // At(i, j) -= l_i At(c, j) for i, j > c, and B(:, i) -= l_i B(:, c)
    const int kr = k - c - 1;
    for (int e = tid; e < kr * kr; e += SOLVE_THREADS) {
      const int i = c + 1 + e / kr, j = c + 1 + e % kr;
      A[j + (int64_t)i * lda] = csub(A[j + (int64_t)i * lda], cmul(A[c + (int64_t)i * lda], A[j + (int64_t)c * lda]));
    }
    for (int e = tid; e < r * kr; e += SOLVE_THREADS) {
      const int row = e % r, i = c + 1 + e / r;
      B[row + (int64_t)i * ldb] = csub(B[row + (int64_t)i * ldb], cmul(A[c + (int64_t)i * lda], B[row + (int64_t)c * ldb]));
    }
    __syncthreads();
  }
  // back substitution on the upper triangle of At: x_c, then B(:, j) -= At(j, c) x_c for j < c
  for (int c = k - 1; c >= 0; --c) {
    const cplx<T> d = A[c + (int64_t)c * lda];
    const bool ok = cabs1(d) > 0;
    for (int row = tid; row < r; row += SOLVE_THREADS) {
      const cplx<T> s = B[row + (int64_t)c * ldb];
      B[row + (int64_t)c * ldb] = ok ? cdiv(s, d) : cplx<T>{0, 0};
    }
    __syncthreads();
    for (int e = tid; e < r * c; e += SOLVE_THREADS) {
      const int row = e % r, j = e / r;
      B[row + (int64_t)j * ldb] = csub(B[row + (int64_t)j * ldb], cmul(A[c + (int64_t)j * lda], B[row + (int64_t)c * ldb]));
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ leaf inverses
// In-place inverse of many small dense blocks (Gauss-Jordan with partial
// pivoting), n <= 128, one workgroup per block; records singular blocks.
template <class T>
__global__ __launch_bounds__(256) void leaf_inverse_kernel(const InvTask* __restrict__ tasks, int* status) {
  const InvTask& tk = tasks[blockIdx.x];
  const int n = tk.n;
  cplx<T>* A = (cplx<T>*)tk.A;
  const int64_t lda = tk.lda;
  __shared__ int piv[128];
  __shared__ double rv[256];
  __shared__ int ri[256];
  const int tid = threadIdx.x;
  for (int c = 0; c < n; ++c) {
    double best = -1;
    int bi = c;
    for (int i = c + tid; i < n; i += 256) {
      const double a = cabs1(A[i + (int64_t)c * lda]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    rv[tid] = best;
    ri[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s && (rv[tid + s] > rv[tid] || (rv[tid + s] == rv[tid] && ri[tid + s] < ri[tid]))) {
        rv[tid] = rv[tid + s];
        ri[tid] = ri[tid + s];
      }
      __syncthreads();
    }
    const int pr = ri[0];
    const bool sing = !(rv[0] > 0);
    __syncthreads();
    if (tid == 0) {
      piv[c] = pr;
      if (sing && status) atomicExch(status, 1);
    }
    if (pr != c)
      for (int j = tid; j < n; j += 256) {
        const cplx<T> t = A[c + (int64_t)j * lda];
        A[c + (int64_t)j * lda] = A[pr + (int64_t)j * lda];
        A[pr + (int64_t)j * lda] = t;
      }
    __syncthreads();
    const cplx<T> d = A[c + (int64_t)c * lda];
    const cplx<T> dinv = sing ? cplx<T>{0, 0} : cdiv(cplx<T>{1, 0}, d);
    __syncthreads();
    // scale row c, then eliminate column c from every other row
    for (int j = tid; j < n; j += 256) {
      if (j == c)
        A[c + (int64_t)j * lda] = dinv;
      else
        A[c + (int64_t)j * lda] = cmul(A[c + (int64_t)j * lda], dinv);
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int i = e % n, j = e / n;
      if (i == c) continue;
      const cplx<T> f = A[i + (int64_t)c * lda];
      if (j == c) continue;
      A[i + (int64_t)j * lda] = csub(A[i + (int64_t)j * lda], cmul(f, A[c + (int64_t)j * lda]));
    }
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
      if (i == c) continue;
      A[i + (int64_t)c * lda] = cmul(cplx<T>{-A[i + (int64_t)c * lda].re, -A[i + (int64_t)c * lda].im}, dinv);
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int c = n - 1; c >= 0; --c) {
    const int pr = piv[c];
    if (pr != c)
      for (int i = tid; i < n; i += 256) {
        const cplx<T> t = A[i + (int64_t)c * lda];
        A[i + (int64_t)c * lda] = A[i + (int64_t)pr * lda];
        A[i + (int64_t)pr * lda] = t;
      }
    __syncthreads();
  }
}

// ------------------------------------------------------------ misc
// Y(i, c) = X(rows[i], c) (gather rows) or Y(rows[i], c) = X(i, c) (scatter)
template <class T>
__global__ void gather_rows_kernel(const cplx<T>* __restrict__ X, int64_t ldx, cplx<T>* __restrict__ Y, int64_t ldy,
                                   const int32_t* __restrict__ rows, int nr, int ncol, int scatter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= nr || c >= ncol) return;
  if (scatter)
    Y[rows[i] + (int64_t)c * ldy] = X[i + (int64_t)c * ldx];
  else
    Y[i + (int64_t)c * ldy] = X[rows[i] + (int64_t)c * ldx];
}

// Y = a X + b Y (elementwise, m x n blocks with lds)
template <class T>
__global__ void axpby_kernel(cplx<T>* __restrict__ Y, int64_t ldy, const cplx<T>* __restrict__ X, int64_t ldx,
                             int64_t m, double a, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= m) return;
  const cplx<T> x = X ? X[i + (int64_t)c * ldx] : cplx<T>{0, 0};
  cplx<T> y = {0, 0};
  if (b != 0) y = Y[i + (int64_t)c * ldy];  // b = 0 overwrites (old contents may be garbage)
  y.re = (T)(a * x.re + b * y.re);
  y.im = (T)(a * x.im + b * y.im);
  Y[i + (int64_t)c * ldy] = y;
}

// y_t = a x_t + b y_t for every task t of a batch (b = 0 overwrites); blockIdx.x
// is the task, the threads of blockIdx.y stride over its entries
template <class T>
__global__ __launch_bounds__(256) void axpby_batch_kernel(const AxpbyTask* __restrict__ tasks, double a, double b) {
  const AxpbyTask& t = tasks[blockIdx.x];
  const int64_t tot = t.m * t.ncol;
  cplx<T>* Y = (cplx<T>*)t.Y;
  const cplx<T>* X = (const cplx<T>*)t.X;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.y * 256) {
    const int64_t i = e % t.m, c = e / t.m;
    const cplx<T> x = X ? X[i + c * t.ldx] : cplx<T>{0, 0};
    cplx<T> y = {0, 0};
    if (b != 0) y = Y[i + c * t.ldy];
    y.re = (T)(a * x.re + b * y.re);
    y.im = (T)(a * x.im + b * y.im);
    Y[i + c * t.ldy] = y;
  }
}

// Y (T1) = a X (T2) + b Y + diag E on each task's m x ncol block, in double,
// with E(i, c) = 1 where i == c + task.pad (X null: zero; b = 0 overwrites Y);
// grid row = task
template <class T1, class T2>
__global__ __launch_bounds__(256) void mix_batch_kernel(const AxpbyTask* __restrict__ tasks, double a, double b,
                                                        double diag) {
  const AxpbyTask& t = tasks[blockIdx.x];
  const int64_t tot = t.m * t.ncol;
  cplx<T1>* Y = (cplx<T1>*)t.Y;
  const cplx<T2>* X = (const cplx<T2>*)t.X;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.y * 256) {
    const int64_t i = e % t.m, c = e / t.m;
    double xr = 0, xi = 0, yr = 0, yi = 0;
    if (X) {
      const cplx<T2> x = X[i + c * t.ldx];
      xr = x.re;
      xi = x.im;
    }
    if (b != 0) {
      const cplx<T1> y = Y[i + c * t.ldy];
      yr = y.re;
      yi = y.im;
    }
    Y[i + c * t.ldy] = cplx<T1>{(T1)(a * xr + b * yr + (i == c + t.pad ? diag : 0.0)), (T1)(a * xi + b * yi)};
  }
}

// Bordered fronts of the SMW dense base, one per task (Y: 2n x 2n, ld 2n; X:
// n x n, ld n, written too; n = m): F = [I I; -I 0] and E = I.  The caller
// then adds K to the leading block (F11 = I + K).
template <class T>
__global__ __launch_bounds__(256) void smw_border_kernel(const AxpbyTask* __restrict__ tasks) {
  const AxpbyTask& t = tasks[blockIdx.x];
  const int64_t n = t.m, n2 = 2 * t.m, tot = n2 * n2;
  cplx<T>* F = (cplx<T>*)t.Y;
  cplx<T>* E = (cplx<T>*)const_cast<void*>(t.X);
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.y * 256) {
    const int64_t i = e % n2, c = e / n2;
    T v = 0;
    if (i < n && c < n)
      v = i == c ? (T)1 : (T)0;
    else if (i < n)
      v = c - n == i ? (T)1 : (T)0;
    else if (c < n)
      v = i - n == c ? (T)-1 : (T)0;
    F[i + c * n2] = cplx<T>{v, (T)0};
    if (i < n && c < n) E[i + c * n] = cplx<T>{i == c ? (T)1 : (T)0, (T)0};
  }
}

// Y(i, j) = v if i == j + off, else 0, on an m x ncol block
template <class T>
__global__ void set_eye_kernel(cplx<T>* __restrict__ Y, int64_t ldy, int64_t m, int ncol, int64_t off, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int c = blockIdx.y; c < ncol; c += gridDim.y)
    Y[i + (int64_t)c * ldy] = cplx<T>{(T)(i == (int64_t)c + off ? v : 0.0), (T)0};
}

// Y (T1) = a X (T2) + b Y on an m x ncol block (b = 0 overwrites)
template <class T1, class T2>
__global__ void axpby_mixed_kernel(cplx<T1>* __restrict__ Y, int64_t ldy, const cplx<T2>* __restrict__ X, int64_t ldx,
                                   int64_t m, double a, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= m) return;
  const cplx<T2> x = X[i + (int64_t)c * ldx];
  double yr = 0, yi = 0;
  if (b != 0) {
    const cplx<T1> y = Y[i + (int64_t)c * ldy];
    yr = b * (double)y.re;
    yi = b * (double)y.im;
  }
  Y[i + (int64_t)c * ldy] = cplx<T1>{(T1)(a * (double)x.re + yr), (T1)(a * (double)x.im + yi)};
}

// Y (T1) = X (T2), elementwise conversion of an m x n block
template <class T1, class T2>
__global__ void convert_kernel(cplx<T1>* __restrict__ Y, int64_t ldy, const cplx<T2>* __restrict__ X, int64_t ldx,
                               int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= m) return;
  const cplx<T2> x = X[i + (int64_t)c * ldx];
  Y[i + (int64_t)c * ldy] = cplx<T1>{(T1)x.re, (T1)x.im};
}

// ------------------------------------------------------------ launchers
#define KCHECK(expr)                   \
  do {                                 \
    hipError_t e__ = (expr);           \
    if (e__ != hipSuccess) return e__; \
  } while (0)

template <class T>
hipError_t launch_grouped_gemm(const GTask* d_tasks, const int64_t* d_tile_start, int ntasks, int64_t ntiles,
                               void* const bases[4], int cfg, hipStream_t s, hipEvent_t ev_start,
                               hipEvent_t ev_stop, bool gram) {
  if (ntasks == 0 || ntiles == 0) return hipSuccess;
  if (cfg < 0 || cfg >= GEMM_CFGS) return hipErrorInvalidValue;
  // grids are limited to 2^31 - 1 blocks in x (the host checks ntiles)
  const dim3 grid((unsigned)ntiles), block(256);
  auto go = [&](auto kernel) {
    if (ev_start)
      hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev_start, ev_stop, 0, d_tasks, d_tile_start, ntasks, bases[0],
                            bases[1], bases[2], bases[3]);
    else
      hipLaunchKernelGGL(kernel, grid, block, 0, s, d_tasks, d_tile_start, ntasks, bases[0], bases[1], bases[2],
                         bases[3]);
  };
  if (gram && cfg != GEMM_CFG_SKINNY) {
    switch (cfg) {
      case 0: go(gram_gemm_kernel<T, Tile64x64>); break;
      case 1: go(gram_gemm_kernel<T, Tile32x128>); break;
      case 2: go(gram_gemm_kernel<T, Tile128x32>); break;
      case 3: go(gram_gemm_kernel<T, Tile16x256>); break;
      case 6: go(gram_gemm_kernel<T, Tile48x128>); break;
      case 7: go(gram_gemm_kernel<T, Tile96x64>); break;
      default: go(gram_gemm_kernel<T, Tile256x16>); break;
    }
    return hipGetLastError();
  }
  switch (cfg) {
    case 0: go(grouped_gemm_kernel<T, Tile64x64>); break;
    case 1: go(grouped_gemm_kernel<T, Tile32x128>); break;
    case 2: go(grouped_gemm_kernel<T, Tile128x32>); break;
    case 3: go(grouped_gemm_kernel<T, Tile16x256>); break;
    case 4: go(grouped_gemm_kernel<T, Tile256x16>); break;
    case 6: go(grouped_gemm_kernel<T, Tile48x128>); break;
    case 7: go(grouped_gemm_kernel<T, Tile96x64>); break;
    default: go(grouped_gemm_skinny_kernel<T>); break;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cpqr_id(const IdTask* d_tasks, int ntasks, double tol, int maxp, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  if (maxp <= 0 || maxp > CPQR_WIDE_MAXP) return hipErrorInvalidValue;
  const size_t bytes = (size_t)maxp * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL((cpqr_id_kernel<T>), dim3(ntasks), dim3(CPQR_THREADS), bytes, s, d_tasks, tol, maxp);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gram_id(const IdTask* d_tasks, int ntasks, double tol, int lds_entries, int maxp, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  if (lds_entries < 0 || lds_entries > GRAM_LDS_MAX || maxp <= 0 || maxp > GRAM_MAXP || maxp % 16 != 0 ||
      sizeof(cplx<T>) != 16)
    return hipErrorInvalidValue;
  const size_t bytes = gram_aux_bytes(maxp) + (size_t)lds_entries * sizeof(cplx<T>);
  if (bytes > GRAM_LDS_BYTES) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gram_id_kernel<T>), dim3(ntasks), dim3(GRAM_THREADS), bytes, s, d_tasks, tol, lds_entries, maxp);
  return hipGetLastError();
}

template <class T>
hipError_t launch_id_expand(const IdTask* d_tasks, int ntasks, void* const* d_outs, const int64_t* d_ldo,
                            bool transpose_out, bool conj_out, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL((id_expand_kernel<T>), dim3(ntasks), dim3(256), 0, s, d_tasks, d_outs, d_ldo,
                     transpose_out ? 1 : 0, conj_out ? 1 : 0);
  return hipGetLastError();
}

template <class T>
hipError_t launch_front_extract(const ExtractTask* d_tasks, int ntasks, int yblocks, const void* values, bool src_single,
                                hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  dim3 grid(ntasks, yblocks > 0 ? yblocks : 1);
  if (src_single)
    hipLaunchKernelGGL((front_extract_kernel<T, cplx<float>>), grid, dim3(256), 0, s, d_tasks,
                       (const cplx<double>*)values);
  else
    hipLaunchKernelGGL((front_extract_kernel<T, cplx<double>>), grid, dim3(256), 0, s, d_tasks,
                       (const cplx<double>*)values);
  return hipGetLastError();
}

template <class TO>
hipError_t launch_bf_extract(const void* d_tasks, int ntasks, int yblocks, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL((bf_extract_kernel<TO>), dim3(ntasks, yblocks > 0 ? yblocks : 1), dim3(256), 0, s,
                     (const BfExtractTask*)d_tasks);
  return hipGetLastError();
}

template <class T>
hipError_t launch_philox_gauss(void* Om, int64_t ld, int64_t n, int ncol, int width, const int32_t* d_gbeg,
                               const int32_t* d_gend, uint64_t seed, uint64_t stream_id, hipStream_t s) {
  if (ncol == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL((philox_gauss_kernel<T>), dim3((unsigned)((n + 255) / 256), ncol), dim3(256), 0, s,
                     (cplx<T>*)Om, ld, n, ncol, width, d_gbeg, d_gend, seed, stream_id);
  return hipGetLastError();
}

template <class T>
hipError_t launch_small_solve_right(const void* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL((small_solve_right_kernel<T>), dim3(ntasks), dim3(SOLVE_THREADS), 0, s, (const SolveTask*)d_tasks);
  return hipGetLastError();
}

template <class T>
hipError_t launch_leaf_inverse(const void* d_tasks, int ntasks, int* d_status, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL((leaf_inverse_kernel<T>), dim3(ntasks), dim3(256), 0, s, (const InvTask*)d_tasks, d_status);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gather_rows(const void* X, int64_t ldx, void* Y, int64_t ldy, const int32_t* rows, int nr, int ncol,
                              bool scatter, hipStream_t s) {
  if (nr == 0 || ncol == 0) return hipSuccess;
  hipLaunchKernelGGL((gather_rows_kernel<T>), dim3((nr + 255) / 256, ncol), dim3(256), 0, s, (const cplx<T>*)X, ldx,
                     (cplx<T>*)Y, ldy, rows, nr, ncol, scatter ? 1 : 0);
  return hipGetLastError();
}

template <class T>
hipError_t launch_axpby(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol, double a, double b,
                        hipStream_t s) {
  if (m == 0 || ncol == 0) return hipSuccess;
  hipLaunchKernelGGL((axpby_kernel<T>), dim3((unsigned)((m + 255) / 256), ncol), dim3(256), 0, s, (cplx<T>*)Y, ldy,
                     (const cplx<T>*)X, ldx, m, a, b);
  return hipGetLastError();
}

template <class T>
hipError_t launch_axpby_batch(const AxpbyTask* d_tasks, int ntasks, int64_t max_entries, double a, double b,
                              hipStream_t s) {
  if (ntasks == 0 || max_entries == 0) return hipSuccess;
  const unsigned yb = (unsigned)std::min<int64_t>(64, std::max<int64_t>(1, (max_entries + 4095) / 4096));
  hipLaunchKernelGGL((axpby_batch_kernel<T>), dim3(ntasks, yb), dim3(256), 0, s, d_tasks, a, b);
  return hipGetLastError();
}

static unsigned batch_rows(int64_t max_entries) {
  return (unsigned)std::min<int64_t>(64, std::max<int64_t>(1, (max_entries + 4095) / 4096));
}

template <class T1, class T2>
hipError_t launch_mix_batch(const AxpbyTask* d_tasks, int ntasks, int64_t max_entries, double a, double b,
                            double diag, hipStream_t s) {
  if (ntasks == 0 || max_entries == 0) return hipSuccess;
  hipLaunchKernelGGL((mix_batch_kernel<T1, T2>), dim3(ntasks, batch_rows(max_entries)), dim3(256), 0, s, d_tasks, a,
                     b, diag);
  return hipGetLastError();
}

template <class T>
hipError_t launch_smw_border(const AxpbyTask* d_tasks, int ntasks, int64_t max_n, hipStream_t s) {
  if (ntasks == 0 || max_n == 0) return hipSuccess;
  hipLaunchKernelGGL((smw_border_kernel<T>), dim3(ntasks, batch_rows(4 * max_n * max_n)), dim3(256), 0, s, d_tasks);
  return hipGetLastError();
}

template <class T>
hipError_t launch_philox_gauss_batch(const ProbeTask* d_tasks, int ntasks, int64_t max_entries,
                                     const int32_t* d_gbeg, const int32_t* d_gend, uint64_t seed, hipStream_t s) {
  if (ntasks == 0 || max_entries == 0) return hipSuccess;
  hipLaunchKernelGGL((philox_gauss_batch_kernel<T>), dim3(ntasks, batch_rows(max_entries)), dim3(256), 0, s, d_tasks,
                     d_gbeg, d_gend, seed);
  return hipGetLastError();
}

template <class T>
hipError_t launch_set_eye(void* Y, int64_t ldy, int64_t m, int ncol, int64_t off, double v, hipStream_t s) {
  if (m == 0 || ncol == 0) return hipSuccess;
  hipLaunchKernelGGL((set_eye_kernel<T>), dim3((unsigned)((m + 255) / 256), (unsigned)std::min(ncol, 65535)), dim3(256),
                     0, s, (cplx<T>*)Y, ldy, m, ncol, off, v);
  return hipGetLastError();
}

template <class T1, class T2>
hipError_t launch_axpby_mixed(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol, double a,
                              double b, hipStream_t s) {
  if (m == 0 || ncol == 0) return hipSuccess;
  hipLaunchKernelGGL((axpby_mixed_kernel<T1, T2>), dim3((unsigned)((m + 255) / 256), ncol), dim3(256), 0, s,
                     (cplx<T1>*)Y, ldy, (const cplx<T2>*)X, ldx, m, a, b);
  return hipGetLastError();
}

template <class T1, class T2>
hipError_t launch_convert(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol, hipStream_t s) {
  if (m == 0 || ncol == 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<T1, T2>), dim3((unsigned)((m + 255) / 256), ncol), dim3(256), 0, s,
                     (cplx<T1>*)Y, ldy, (const cplx<T2>*)X, ldx, m);
  return hipGetLastError();
}

#define INST(T)                                                                                                       \
  template hipError_t launch_grouped_gemm<T>(const GTask*, const int64_t*, int, int64_t, void* const[4], int,         \
                                             hipStream_t, hipEvent_t, hipEvent_t, bool);                              \
  template hipError_t launch_cpqr_id<T>(const IdTask*, int, double, int, hipStream_t);                                \
  template hipError_t launch_gram_id<T>(const IdTask*, int, double, int, int, hipStream_t);                           \
  template hipError_t launch_id_expand<T>(const IdTask*, int, void* const*, const int64_t*, bool, bool, hipStream_t);  \
  template hipError_t launch_front_extract<T>(const ExtractTask*, int, int, const void*, bool, hipStream_t);          \
  template hipError_t launch_bf_extract<T>(const void*, int, int, hipStream_t);                                       \
  template hipError_t launch_philox_gauss<T>(void*, int64_t, int64_t, int, int, const int32_t*, const int32_t*,       \
                                             uint64_t, uint64_t, hipStream_t);                                        \
  template hipError_t launch_small_solve_right<T>(const void*, int, hipStream_t);                                     \
  template hipError_t launch_leaf_inverse<T>(const void*, int, int*, hipStream_t);                                    \
  template hipError_t launch_gather_rows<T>(const void*, int64_t, void*, int64_t, const int32_t*, int, int, bool,     \
                                            hipStream_t);                                                             \
  template hipError_t launch_axpby<T>(void*, int64_t, const void*, int64_t, int64_t, int, double, double, hipStream_t); \
  template hipError_t launch_set_eye<T>(void*, int64_t, int64_t, int, int64_t, double, hipStream_t);               \
  template hipError_t launch_axpby_batch<T>(const AxpbyTask*, int, int64_t, double, double, hipStream_t);           \
  template hipError_t launch_smw_border<T>(const AxpbyTask*, int, int64_t, hipStream_t);                             \
  template hipError_t launch_philox_gauss_batch<T>(const ProbeTask*, int, int64_t, const int32_t*, const int32_t*,    \
                                                   uint64_t, hipStream_t);
INST(double)
INST(float)
template hipError_t launch_mix_batch<double, double>(const AxpbyTask*, int, int64_t, double, double, double,
                                                     hipStream_t);
template hipError_t launch_mix_batch<double, float>(const AxpbyTask*, int, int64_t, double, double, double,
                                                    hipStream_t);
template hipError_t launch_mix_batch<float, double>(const AxpbyTask*, int, int64_t, double, double, double,
                                                    hipStream_t);
template hipError_t launch_mix_batch<float, float>(const AxpbyTask*, int, int64_t, double, double, double,
                                                   hipStream_t);
template hipError_t launch_axpby_mixed<double, float>(void*, int64_t, const void*, int64_t, int64_t, int, double,
                                                      double, hipStream_t);
template hipError_t launch_axpby_mixed<float, double>(void*, int64_t, const void*, int64_t, int64_t, int, double,
                                                      double, hipStream_t);
template hipError_t launch_axpby_mixed<double, double>(void*, int64_t, const void*, int64_t, int64_t, int, double,
                                                       double, hipStream_t);
template hipError_t launch_convert<double, float>(void*, int64_t, const void*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_convert<float, double>(void*, int64_t, const void*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_convert<double, double>(void*, int64_t, const void*, int64_t, int64_t, int, hipStream_t);

}  // namespace bfmf
