// Dense front kernels: extend-add assembly and partial LU with pivoting
// restricted to F11 (paper Sec. 2, Alg. 1).
//
// The partial factorization of F = [F11 F12; F21 F22] (ns fully-summed
// variables) is right-looking over the block row [F11 F12] in panels of
// KB columns:
//   panel   : LU with partial pivoting of F11(k0:ns, k0:k0+jb); the pivot is
//             the first row maximising |Re| + |Im| (LAPACK getrf convention)
//   laswp   : the panel's row interchanges applied to the other columns of
//             rows 0..ns-1 (so F12 becomes P^T F12)
//   trsm_ll : F(k0:k0+jb, k0+jb:n) <- L_kk^-1 F(k0:k0+jb, k0+jb:n)
//   trsm_ru : F21(:, k0:k0+jb) <- F21(:, k0:k0+jb) U_kk^-1
//   trailing: F11/F12 rows below the panel and F21 columns right of it get
//             the rank-jb update (MFMA GEMM)
// and finally the Schur complement C = F22 - F21 F12 is one GEMM of depth ns.
// Pivot search never looks at F21 (Sec. 2: the pivoting in F11 does not use
// the values of F21 and F12).
#include "../devtypes.hpp"
#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace bfmf {

// ---------------------------------------------------------------- assembly
// F_tau = [A(Is,Is) A(Is,Iu); A(Iu,Is) 0] (+) C_nu1 (+) C_nu2, computed in
// gather form: every entry is ((0 + a) + c1) + c2 in that order.  One wave
// per front column; the column's few A entries are held in registers.
template <class T, class TC>
__global__ __launch_bounds__(256) void assemble_kernel(const FrontDesc* __restrict__ fds,
                                                       const cplx<double>* __restrict__ values) {
  const FrontDesc& fd = fds[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n = fd.n;
  if (j >= n) return;
  cplx<T>* F = (cplx<T>*)fd.F + (int64_t)j * n;
  const int64_t a0 = fd.a_ptr[j], a1 = fd.a_ptr[j + 1];
  const int inv1j = fd.nchild > 0 ? fd.inv[0][j] : -1;
  const int inv2j = fd.nchild > 1 ? fd.inv[1][j] : -1;
  const TC* cb1 = inv1j >= 0 ? (const TC*)fd.cb[0] + (int64_t)inv1j * fd.cb_ld[0] : nullptr;
  const TC* cb2 = inv2j >= 0 ? (const TC*)fd.cb[1] + (int64_t)inv2j * fd.cb_ld[1] : nullptr;
  const int na = (int)(a1 - a0);
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    cplx<T> v = {0, 0};
    // entries t0..t0+63 of this column, one per lane, broadcast by shuffles;
    // every lane of the wave runs the same trip counts
    for (int t0 = 0; t0 < na; t0 += 64) {
      int myrow = -1;
      double mr = 0, mi = 0;
      if (t0 + lane < na) {
        myrow = fd.a_row[a0 + t0 + lane];
        const cplx<double> a = values[fd.a_vidx[a0 + t0 + lane]];
        mr = a.re;
        mi = a.im;
      }
      const int cnt = min(64, na - t0);
      for (int t = 0; t < cnt; ++t) {
        const int r = __shfl(myrow, t);
        const double vr = __shfl(mr, t), vi = __shfl(mi, t);
        if (r == i) {
          v.re += (T)vr;
          v.im += (T)vi;
        }
      }
    }
    if (i < n) {
      if (cb1) {
        const int k = fd.inv[0][i];
        if (k >= 0) {
          const TC c = cb1[k];
          v.re += (T)c.re;
          v.im += (T)c.im;
        }
      }
      if (cb2) {
        const int k = fd.inv[1][i];
        if (k >= 0) {
          const TC c = cb2[k];
          v.re += (T)c.re;
          v.im += (T)c.im;
        }
      }
      F[i] = v;
    }
  }
}

// ------------------------------------------------------------------ panel
// One workgroup per front: unblocked LU with partial pivoting of the
// (ns-k0) x jb panel F11(k0:ns, k0:k0+jb).  Per column: the pivot (largest
// |Re| + |Im|, first row on ties) by wave shuffles and one exchange between
// the four waves; the row interchange inside the panel; then every thread
// scales its rows of the column and updates the same rows of the panel's
// remaining columns.  Three barriers per column.
template <class T>
__global__ __launch_bounds__(256) void panel_kernel(const FrontDesc* __restrict__ fds, int k0, int kb,
                                                    int* __restrict__ status) {
  const FrontDesc& fd = fds[blockIdx.x];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(kb, ns - k0);
  cplx<T>* F = (cplx<T>*)fd.F;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ T red_v[2][4];
  __shared__ int red_i[2][4];
  for (int jj = 0; jj < jb; ++jj) {
    const int col = k0 + jj;
    cplx<T>* Fc = F + (int64_t)col * n;
    T best = -1;
    int bi = ns;
    for (int r = col + tid; r < ns; r += 256) {
      const T a = cabs1(Fc[r]);
      if (a > best) {
        best = a;
        bi = r;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {  // wave maximum, first index on ties
      const T ov = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[jj & 1][wave] = best;
      red_i[jj & 1][wave] = bi;
    }
    __syncthreads();
    T pv = red_v[jj & 1][0];
    int p = red_i[jj & 1][0];
    for (int w = 1; w < 4; ++w) {
      const T ov = red_v[jj & 1][w];
      const int oi = red_i[jj & 1][w];
      if (ov > pv || (ov == pv && oi < p)) {
        pv = ov;
        p = oi;
      }
    }
    const bool singular = !(pv > 0) || p >= ns;
    if (singular) p = col;
    if (tid == 0) {
      fd.piv[col] = p;
      if (singular && atomicCAS(&status[0], 0, 1) == 0) {
        status[1] = fd.front;
        status[2] = col;
      }
    }
    if (p != col) {
      for (int c = k0 + tid; c < k0 + jb; c += 256) {
        cplx<T>* Fcc = F + (int64_t)c * n;
        const cplx<T> t = Fcc[col];
        Fcc[col] = Fcc[p];
        Fcc[p] = t;
      }
    }
    __syncthreads();  // the interchanged rows are visible
    const cplx<T> d = Fc[col];
    for (int r = col + 1 + tid; r < ns; r += 256) {
      cplx<T> l = Fc[r];
      if (!singular) {
        l = cdiv(l, d);
        Fc[r] = l;
      }
      for (int c = col + 1; c < k0 + jb; ++c) {
        cplx<T>* Fcc = F + (int64_t)c * n;
        Fcc[r] = csub(Fcc[r], cmul(l, Fcc[col]));
      }
    }
    __syncthreads();  // the updated panel is visible to the next pivot search
  }
}

// The same factorization of a panel of at most PR_ROWS rows, held in registers.
// 512 threads; thread t owns panel rows t and t + 512 (relative to k0) of a
// half-panel of up to 16 columns at a time, rotated so that the current column
// is always register slot 0 (no register index depends on the column).  A
// finished column goes to memory at once; later row interchanges are applied
// to the finished columns in memory (thread c swaps column c).
//   left half : columns k0 .. k0+15 factored column by column as above;
//   right half: loaded with all of the left half's row interchanges applied
//               (each row read from its source position), then the left
//               half's rank-1 updates in column order (the interchanges of a
//               later column only exchange rows below the current one, so
//               every entry receives the same operations in the same order as
//               in panel_kernel), then factored like the left half.
// Every arithmetic operation is panel_kernel's in the same order, so the two
// kernels give identical factors and pivots.  A column costs two barriers: the
// pivot exchange, then the pivot-row broadcast (double-buffered LDS slots).
constexpr int PR_THREADS = 512, PR_ROWS = 2 * PR_THREADS, PR_HALF = 16;

template <class T>
__global__ __launch_bounds__(PR_THREADS) void panel_reg_kernel(const FrontDesc* __restrict__ fds, int k0, int kb,
                                                               int* __restrict__ status) {
  const FrontDesc& fd = fds[blockIdx.x];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(kb, ns - k0);
  const int m = ns - k0;  // panel rows; the launcher guarantees m <= PR_ROWS
  cplx<T>* F = (cplx<T>*)fd.F;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ T red_v[2][PR_THREADS / 64];
  __shared__ int red_i[2][PR_THREADS / 64];
  __shared__ cplx<T> urow[2][PR_HALF];  // the step's pivot row (slots of the current half)
  __shared__ cplx<T> jrow[2][PR_HALF];  // the row it replaces
  __shared__ int pl[PR_HALF];           // the left half's pivots (relative rows)
  const int rowq[2] = {tid, tid + PR_THREADS};
  cplx<T> a[2][PR_HALF];
  int st = 0;  // LDS slot parity, advanced after every step that uses a slot

  auto at = [&](int r, int c) __attribute__((always_inline)) -> cplx<T>* {
    return F + (int64_t)(k0 + r) + (int64_t)(k0 + c) * n;
  };
  // column by column LU of the half-panel in registers (panel columns c0 .. c0+w-1)
  auto factor_half = [&](int c0, int w) __attribute__((always_inline)) {
    for (int jj = 0; jj < w; ++jj) {
      const int cr = c0 + jj;  // relative pivot row / column
      const int buf = st & 1;
      T best = -1;
      int bi = m;
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (rowq[q] >= cr && rowq[q] < m) {
          const T v = cabs1(a[q][0]);
          if (v > best) {  // rows in ascending order: the first on ties is kept
            best = v;
            bi = rowq[q];
          }
        }
      for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(best, o);
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
      T pv = red_v[buf][0];
      int p = red_i[buf][0];
      for (int w2 = 1; w2 < PR_THREADS / 64; ++w2) {
        const T ov = red_v[buf][w2];
        const int oi = red_i[buf][w2];
        if (ov > pv || (ov == pv && oi < p)) {
          pv = ov;
          p = oi;
        }
      }
      const bool singular = !(pv > 0) || p >= m;
      if (singular) p = cr;
      if (tid == 0) {
        gst(fd.piv + k0 + cr, (int32_t)(k0 + p));
        if (c0 == 0) pl[jj] = p;
        if (singular && atomicCAS(&status[0], 0, 1) == 0) {
          status[1] = fd.front;
          status[2] = k0 + cr;
        }
      }
      // the pivot row (row p) and, on an interchange, row cr through LDS
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (rowq[q] == p)
#pragma unroll
          for (int c = 0; c < PR_HALF; ++c) urow[buf][c] = a[q][c];
        if (p != cr && rowq[q] == cr)
#pragma unroll
          for (int c = 0; c < PR_HALF; ++c) jrow[buf][c] = a[q][c];
      }
      if (p != cr && tid < cr) {  // the interchange in the finished columns (in memory)
        cplx<T>* x = at(cr, tid);
        cplx<T>* y = at(p, tid);
        const cplx<T> t = gld(x);
        gst(x, gld(y));
        gst(y, t);
      }
      __syncthreads();
      const cplx<T> d = urow[buf][0];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (p != cr) {
          if (rowq[q] == cr) {
#pragma unroll
            for (int c = 0; c < PR_HALF; ++c) a[q][c] = urow[buf][c];
          } else if (rowq[q] == p) {
#pragma unroll
            for (int c = 0; c < PR_HALF; ++c) a[q][c] = jrow[buf][c];
          }
        }
        if (rowq[q] > cr && rowq[q] < m) {
          cplx<T> l = a[q][0];
          if (!singular) {
            l = cdiv(l, d);
            a[q][0] = l;
          }
#pragma unroll
          for (int c = 1; c < PR_HALF; ++c)
            if (c < w - jj) a[q][c] = csub(a[q][c], cmul(l, urow[buf][c]));
        }
        if (rowq[q] < m) gst(at(rowq[q], cr), a[q][0]);  // column cr is final (interchanges aside)
#pragma unroll
        for (int c = 0; c + 1 < PR_HALF; ++c) a[q][c] = a[q][c + 1];
      }
      ++st;
    }
  };

  const int w1 = min(jb, PR_HALF);
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int c = 0; c < PR_HALF; ++c) a[q][c] = (rowq[q] < m && c < w1) ? gld(at(rowq[q], c)) : cplx<T>{0, 0};
  factor_half(0, w1);
  if (jb <= PR_HALF) return;
  const int w2 = jb - PR_HALF;
  __syncthreads();  // the left half is in memory and its pivots in LDS
  // right half with the left half's interchanges applied: position r holds the row at position
  // s_0(s_1(...s_15(r))), s_j the interchange of rows j and pl[j]
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int src = rowq[q];
    for (int j = PR_HALF - 1; j >= 0; --j) {
      const int pj = pl[j];
      if (src == j)
        src = pj;
      else if (src == pj)
        src = j;
    }
#pragma unroll
    for (int c = 0; c < PR_HALF; ++c)
      a[q][c] = (rowq[q] < m && c < w2) ? gld(at(src, PR_HALF + c)) : cplx<T>{0, 0};
  }
  __syncthreads();  // every thread has read the right half before any of it is written again
  // the left half's rank-1 updates, in column order
  for (int jj = 0; jj < PR_HALF; ++jj) {
    const int buf = st & 1;
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (rowq[q] == jj)
#pragma unroll
        for (int c = 0; c < PR_HALF; ++c) urow[buf][c] = a[q][c];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (rowq[q] > jj && rowq[q] < m) {
        const cplx<T> l = gld(at(rowq[q], jj));
#pragma unroll
        for (int c = 0; c < PR_HALF; ++c)
          if (c < w2) a[q][c] = csub(a[q][c], cmul(l, urow[buf][c]));
      }
    ++st;
  }
  factor_half(PR_HALF, w2);
}

// Row interchanges of the pivot rows [k0, k0+jb) applied to columns outside
// the panel, rows 0..ns-1 only (F21 rows are never swapped): columns
// [cbeg, k0) and then [max(k0+jb, cfrom), min(cend, n)).
template <class T>
__global__ __launch_bounds__(256) void laswp_kernel(const FrontDesc* __restrict__ fds, int k0, int kb, int cbeg,
                                                    int cfrom, int cend) {
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(kb, ns - k0);
  const int idx = blockIdx.x * 256 + threadIdx.x, nleft = max(k0 - cbeg, 0);
  const int c = idx < nleft ? cbeg + idx : max(k0 + jb, cfrom) + (idx - nleft);
  if (c >= min(cend, n)) return;
  cplx<T>* Fc = (cplx<T>*)fd.F + (int64_t)c * n;
  for (int k = k0; k < k0 + jb; ++k) {
    const int p = fd.piv[k];
    if (p != k) {
      const cplx<T> t = Fc[k];
      Fc[k] = Fc[p];
      Fc[p] = t;
    }
  }
}

// The value v of lane j (j uniform over the wave), through the scalar unit.
__device__ __forceinline__ double lane_value(double v, int j) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, j), hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ float lane_value(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// F(k0:k0+jb, c) <- L_kk^-1 F(k0:k0+jb, c) for c in [max(k0+jb, cfrom),
// min(cend, n)), forward substitution with lane i holding row k0+i.  A wave
// solves TRSM_CW consecutive columns together (one read of L per step for all
// of them, the step's pivot values read from lane j), and a workgroup takes
// TRSM_COLS columns so that its copy of L_kk in LDS serves all of them.
constexpr int TRSM_CW = 4, TRSM_GR = 2, TRSM_COLS = 4 * TRSM_CW * TRSM_GR;
template <class T, int KB>
__global__ __launch_bounds__(256) void trsm_ll_kernel(const FrontDesc* __restrict__ fds, int k0, int cfrom,
                                                      int cend) {
  static_assert(KB <= 64, "one lane per row of the block");
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(KB, ns - k0);
  const int c0 = max(k0 + jb, cfrom) + blockIdx.x * TRSM_COLS, c1 = min(cend, n);
  if (c0 >= c1) return;  // the same for the whole workgroup
  // strictly lower part of L_kk, zero elsewhere (rows past jb included)
  __shared__ cplx<T> L[KB][KB + 1];
  cplx<T>* F = (cplx<T>*)fd.F;
  for (int e = threadIdx.x; e < KB * KB; e += 256) {
    const int i = e % KB, j = e / KB;
    L[i][j] = (i > j && i < jb) ? gld(F + (int64_t)(k0 + i) + (int64_t)(k0 + j) * n) : cplx<T>{0, 0};
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane < KB ? lane : 0;  // row 0 of the strictly lower part is zero
  for (int g = 0; g < TRSM_GR; ++g) {
    const int cb = c0 + (g * 4 + w) * TRSM_CW;
    if (cb >= c1) break;  // the same for the whole wave
    cplx<T> x[TRSM_CW];
#pragma unroll
    for (int q = 0; q < TRSM_CW; ++q)
      x[q] = (lane < jb && cb + q < c1) ? gld(F + (int64_t)(cb + q) * n + k0 + lane) : cplx<T>{0, 0};
    for (int j = 0; j < jb - 1; ++j) {
      const cplx<T> l = L[li][j];
#pragma unroll
      for (int q = 0; q < TRSM_CW; ++q) {
        const cplx<T> xj = {lane_value(x[q].re, j), lane_value(x[q].im, j)};
        x[q] = csub(x[q], cmul(l, xj));
      }
    }
#pragma unroll
    for (int q = 0; q < TRSM_CW; ++q)
      if (lane < jb && cb + q < c1) gst(F + (int64_t)(cb + q) * n + k0 + lane, x[q]);
  }
}

// F21(r, k0:k0+jb) <- F21(r, k0:k0+jb) U_kk^-1 for rows r in [ns, n): one
// thread per row, the row vector kept in registers.
template <class T, int KB>
__global__ __launch_bounds__(256) void trsm_ru_kernel(const FrontDesc* __restrict__ fds, int k0) {
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(KB, ns - k0);
  __shared__ cplx<T> U[KB][KB + 1];
  cplx<T>* F = (cplx<T>*)fd.F;
  for (int e = threadIdx.x; e < KB * KB; e += 256) {
    const int i = e % KB, j = e / KB;
    U[i][j] = (i < jb && j < jb) ? gld(F + (int64_t)(k0 + i) + (int64_t)(k0 + j) * n) : cplx<T>{1, 0};
  }
  __syncthreads();
  const int r = ns + blockIdx.x * 256 + threadIdx.x;
  // with F21 = -I at the start, rows ns + i with i >= k0 + jb are still zero in these columns
  const int rend = fd.f21_unit ? min(n, ns + k0 + jb) : n;
  if (r >= rend) return;
  cplx<T> x[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) x[c] = c < jb ? gld(F + (int64_t)r + (int64_t)(k0 + c) * n) : cplx<T>{0, 0};
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    cplx<T> s = x[c];
#pragma unroll
    for (int d = 0; d < c; ++d) s = csub(s, cmul(x[d], U[d][c]));
    x[c] = c < jb ? cdiv(s, U[c][c]) : s;
  }
#pragma unroll
  for (int c = 0; c < KB; ++c)
    if (c < jb) gst(F + (int64_t)r + (int64_t)(k0 + c) * n, x[c]);
}

// Rank-jb update after the panel of columns [k0, k0+jb): rows [k0+jb, ns) x
// cols [k0+jb, ce) and rows [ns, n) x cols [k0+jb, min(ce, ns)), ce = min(cend, n).
template <class T>
__global__ __launch_bounds__(256, 2) void trailing_kernel(const FrontDesc* __restrict__ fds, int k0, int kb, int cend) {
  __shared__ GemmSmem<T> sm;
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(kb, ns - k0);
  const int r0 = k0 + jb;
  const int ce = min(cend, n);
  cplx<T>* F = (cplx<T>*)fd.F;
  const int M1 = ns - r0, N1 = ce - r0;
  // with F21 = -I at the start, F21(:, k0:r0) is zero below row ns + r0
  const int M2 = fd.f21_unit ? min(n - ns, r0) : n - ns, N2 = min(ce, ns) - r0;
  const int tm1 = (M1 + GEMM_TM - 1) / GEMM_TM, tn1 = (N1 + GEMM_TN - 1) / GEMM_TN;
  const int tm2 = (M2 + GEMM_TM - 1) / GEMM_TM, tn2 = (N2 + GEMM_TN - 1) / GEMM_TN;
  const int t1 = (M1 > 0 && N1 > 0) ? tm1 * tn1 : 0;
  const int t2 = (M2 > 0 && N2 > 0) ? tm2 * tn2 : 0;
  int t = blockIdx.x;
  const cplx<T> m1 = {-1, 0};
  if (t < t1) {
    gemm_tile<T>(F + r0 + (int64_t)k0 * n, n, OP_N, F + k0 + (int64_t)r0 * n, n, F + r0 + (int64_t)r0 * n, n, M1,
                 N1, jb, m1, 1, t % tm1, t / tm1, sm);
    return;
  }
  t -= t1;
  if (t < t2) {
    gemm_tile<T>(F + ns + (int64_t)k0 * n, n, OP_N, F + k0 + (int64_t)r0 * n, n, F + ns + (int64_t)r0 * n, n,
                 M2, N2, jb, m1, 1, t % tm2, t / tm2, sm);
  }
}

// Rows [k0+jb, min(rend, ns)) x cols [max(k0+jb, cfrom), min(cend, n)) -= F(rows, k0:k0+jb) F(k0:k0+jb, cols):
// the product between the two halves of a row-block solve taller than one wave's 64 lanes.
template <class T>
__global__ __launch_bounds__(256, 2) void rowblock_update_kernel(const FrontDesc* __restrict__ fds, int k0, int kb,
                                                              int rend, int cfrom, int cend) {
  __shared__ GemmSmem<T> sm;
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n;
  if (k0 >= ns) return;
  const int jb = min(kb, ns - k0);
  const int r0 = k0 + jb, c0 = max(r0, cfrom);
  const int M = min(rend, ns) - r0, N = min(cend, n) - c0;
  if (M <= 0 || N <= 0) return;
  const int tm = (M + GEMM_TM - 1) / GEMM_TM, tn = (N + GEMM_TN - 1) / GEMM_TN;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  cplx<T>* F = (cplx<T>*)fd.F;
  gemm_tile<T>(F + r0 + (int64_t)k0 * n, n, OP_N, F + k0 + (int64_t)c0 * n, n, F + r0 + (int64_t)c0 * n, n, M, N, jb,
               cplx<T>{-1, 0}, 1, t % tm, t / tm, sm);
}

// Schur complement C = F22 - F21 F12 (depth ns).
template <class T>
__global__ __launch_bounds__(256, 2) void schur_kernel(const FrontDesc* __restrict__ fds) {
  __shared__ GemmSmem<T> sm;
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n, nu = n - ns;
  if (nu <= 0 || ns <= 0) return;
  const int tm = (nu + GEMM_TM - 1) / GEMM_TM, tn = tm;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  cplx<T>* F = (cplx<T>*)fd.F;
  gemm_tile<T>(F + ns, n, OP_N, F + (int64_t)ns * n, n, F + ns + (int64_t)ns * n, n, nu, nu, ns, cplx<T>{-1, 0},
               1, t % tm, t / tm, sm);
}

// The same Schur complement with the product on FP32 MFMA: F21 and F12 rounded
// to complex64 as they are staged, the product accumulated in FP32 and
// subtracted from F22 in double (the complex64 form of the dense fronts).
__global__ __launch_bounds__(256, 2) void schur_mixed_kernel(const FrontDesc* __restrict__ fds) {
  __shared__ GemmSmem<float> sm;
  const FrontDesc& fd = fds[blockIdx.y];
  const int ns = fd.ns, n = fd.n, nu = n - ns;
  if (nu <= 0 || ns <= 0) return;
  const int tm = (nu + GEMM_TM - 1) / GEMM_TM, tn = tm;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  cplx<double>* F = (cplx<double>*)fd.F;
  gemm_tile<float, double>(F + ns, n, OP_N, F + (int64_t)ns * n, n, F + ns + (int64_t)ns * n, n, nu, nu, ns,
                           cplx<float>{-1, 0}, 1, t % tm, t / tm, sm);
}

// ------------------------------------------------------------------ launchers
#define KCHECK(expr)                       \
  do {                                     \
    hipError_t e__ = (expr);               \
    if (e__ != hipSuccess) return e__;     \
  } while (0)

template <class T>
hipError_t launch_assemble(const FrontDesc* d_fds, int nbatch, int maxn, const void* values, bool cb_single,
                           hipStream_t s) {
  if (nbatch == 0 || maxn == 0) return hipSuccess;
  dim3 grid((maxn + 3) / 4, nbatch);
  if (cb_single)
    hipLaunchKernelGGL((assemble_kernel<T, cplx<float>>), grid, dim3(256), 0, s, d_fds,
                       (const cplx<double>*)values);
  else
    hipLaunchKernelGGL((assemble_kernel<T, cplx<double>>), grid, dim3(256), 0, s, d_fds,
                       (const cplx<double>*)values);
  return hipGetLastError();
}

template <class T>
hipError_t launch_partial_lu(const FrontDesc* d_fds, int nbatch, const int* h_n, const int* h_ns, int* d_status,
                             hipStream_t s) {
  if (nbatch == 0) return hipSuccess;
  constexpr int KB = 32;
  int maxns = 0, maxn = 0;
  for (int b = 0; b < nbatch; ++b) {
    maxns = h_ns[b] > maxns ? h_ns[b] : maxns;
    maxn = h_n[b] > maxn ? h_n[b] : maxn;
  }
  static_assert(KB <= 2 * PR_HALF, "the register panel holds two half-panels");
  // Columns in blocks of 4 KB, each made of two blocks of 2 KB, each made of two panels of KB (the
  // register panel). A block's interchanges, row-block solve and right-looking update reach only the
  // columns of the enclosing block until the block is complete; then one solve and one rank-w update
  // (w = 2 KB, 4 KB) cover the enclosing block's columns (or everything to the right, for the outermost
  // blocks). The panels see exactly the values of a KB-column right-looking sweep, so the pivots are the
  // same; the trailing matrix is rewritten once per 4 KB columns.
  auto tiles_for = [&](int k0, int kb, int cend) {
    int mt = 0;
    for (int b = 0; b < nbatch; ++b) {
      if (k0 >= h_ns[b]) continue;
      const int jb = (h_ns[b] - k0) < kb ? (h_ns[b] - k0) : kb;
      const int r0 = k0 + jb, ce = cend < h_n[b] ? cend : h_n[b];
      const int M1 = h_ns[b] - r0, N1 = ce - r0, M2 = h_n[b] - h_ns[b], N2 = (ce < h_ns[b] ? ce : h_ns[b]) - r0;
      int t = 0;
      if (M1 > 0 && N1 > 0) t += ((M1 + 63) / 64) * ((N1 + 63) / 64);
      if (M2 > 0 && N2 > 0) t += ((M2 + 63) / 64) * ((N2 + 63) / 64);
      mt = t > mt ? t : mt;
    }
    return mt;
  };
  int maxnu = 0;
  for (int b = 0; b < nbatch; ++b) maxnu = (h_n[b] - h_ns[b]) > maxnu ? (h_n[b] - h_ns[b]) : maxnu;
  // does any front have columns in [k0+jb, min(cend, n)) for the pivot rows [k0, k0+jb)?
  auto right_cols = [&](int k0, int kb, int cend) {
    for (int b = 0; b < nbatch; ++b) {
      if (k0 >= h_ns[b]) continue;
      const int jb = (h_ns[b] - k0) < kb ? (h_ns[b] - k0) : kb;
      if (k0 + jb < (cend < h_n[b] ? cend : h_n[b])) return true;
    }
    return false;
  };
  auto half = [&](int k0, int cend) -> hipError_t {  // factor columns [k0, k0+KB); update columns up to cend
    if (maxns - k0 <= PR_ROWS)  // every front's panel fits the register kernel
      hipLaunchKernelGGL((panel_reg_kernel<T>), dim3(nbatch), dim3(PR_THREADS), 0, s, d_fds, k0, KB, d_status);
    else
      hipLaunchKernelGGL((panel_kernel<T>), dim3(nbatch), dim3(256), 0, s, d_fds, k0, KB, d_status);
    KCHECK(hipGetLastError());
    hipLaunchKernelGGL((laswp_kernel<T>), dim3((cend + 255) / 256, nbatch), dim3(256), 0, s, d_fds, k0, KB, 0, 0,
                       cend);
    KCHECK(hipGetLastError());
    if (right_cols(k0, KB, cend)) {
      hipLaunchKernelGGL((trsm_ll_kernel<T, KB>), dim3((cend - k0 + TRSM_COLS - 1) / TRSM_COLS, nbatch), dim3(256), 0,
                         s, d_fds, k0, 0, cend);
      KCHECK(hipGetLastError());
    }
    if (maxnu > 0) {
      hipLaunchKernelGGL((trsm_ru_kernel<T, KB>), dim3((maxnu + 255) / 256, nbatch), dim3(256), 0, s, d_fds, k0);
      KCHECK(hipGetLastError());
    }
    const int mt = tiles_for(k0, KB, cend);
    if (mt > 0) {
      hipLaunchKernelGGL((trailing_kernel<T>), dim3(mt, nbatch), dim3(256), 0, s, d_fds, k0, KB, cend);
      KCHECK(hipGetLastError());
    }
    return hipSuccess;
  };
  // pivot rows [k0, k0+w) applied to columns [cfrom, cend): interchanges, row-block solve (rows of a 64-row
  // half one lane each; for w = 4 KB two halves with the product between them), rank-w update
  auto block_update = [&](int k0, int w, int cfrom, int cend) -> hipError_t {
    const int ncol = cend - cfrom;
    hipLaunchKernelGGL((laswp_kernel<T>), dim3((ncol + 255) / 256, nbatch), dim3(256), 0, s, d_fds, k0, w, k0, cfrom,
                       cend);
    KCHECK(hipGetLastError());
    const dim3 sgrid((ncol + TRSM_COLS - 1) / TRSM_COLS, nbatch);
    hipLaunchKernelGGL((trsm_ll_kernel<T, 2 * KB>), sgrid, dim3(256), 0, s, d_fds, k0, cfrom, cend);
    KCHECK(hipGetLastError());
    if (w > 2 * KB) {
      hipLaunchKernelGGL((rowblock_update_kernel<T>), dim3((ncol + GEMM_TN - 1) / GEMM_TN, nbatch), dim3(256), 0, s,
                         d_fds, k0, 2 * KB, k0 + w, cfrom, cend);
      KCHECK(hipGetLastError());
      hipLaunchKernelGGL((trsm_ll_kernel<T, 2 * KB>), sgrid, dim3(256), 0, s, d_fds, k0 + 2 * KB, cfrom, cend);
      KCHECK(hipGetLastError());
    }
    const int mt = tiles_for(k0, w, cend);
    if (mt > 0) {
      hipLaunchKernelGGL((trailing_kernel<T>), dim3(mt, nbatch), dim3(256), 0, s, d_fds, k0, w, cend);
      KCHECK(hipGetLastError());
    }
    return hipSuccess;
  };
  // columns [k0, k0 + 2 KB), right updates up to cend
  auto block2 = [&](int k0, int cend) -> hipError_t {
    const int kend = k0 + 2 * KB;
    KCHECK(half(k0, kend));
    if (k0 + KB < maxns) KCHECK(half(k0 + KB, kend));
    if (maxn > kend && cend > kend) KCHECK(block_update(k0, 2 * KB, kend, cend));
    return hipSuccess;
  };
  for (int k0 = 0; k0 < maxns; k0 += 4 * KB) {
    const int kend = k0 + 4 * KB;
    KCHECK(block2(k0, kend));
    if (k0 + 2 * KB < maxns) KCHECK(block2(k0 + 2 * KB, kend));
    if (maxn > kend) KCHECK(block_update(k0, 4 * KB, kend, maxn));
  }
  return hipSuccess;
}

template <class T>
hipError_t launch_schur(const FrontDesc* d_fds, int nbatch, const int* h_n, const int* h_ns, hipStream_t s) {
  int maxtiles = 0;
  for (int b = 0; b < nbatch; ++b) {
    const int nu = h_n[b] - h_ns[b];
    if (nu <= 0 || h_ns[b] <= 0) continue;
    const int t = ((nu + 63) / 64) * ((nu + 63) / 64);
    maxtiles = t > maxtiles ? t : maxtiles;
  }
  if (maxtiles > 0) {
    hipLaunchKernelGGL((schur_kernel<T>), dim3(maxtiles, nbatch), dim3(256), 0, s, d_fds);
    KCHECK(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t launch_schur_mixed(const FrontDesc* d_fds, int nbatch, const int* h_n, const int* h_ns, hipStream_t s) {
  int maxtiles = 0;
  for (int b = 0; b < nbatch; ++b) {
    const int nu = h_n[b] - h_ns[b];
    if (nu <= 0 || h_ns[b] <= 0) continue;
    const int t = ((nu + 63) / 64) * ((nu + 63) / 64);
    maxtiles = t > maxtiles ? t : maxtiles;
  }
  if (maxtiles > 0) {
    hipLaunchKernelGGL(schur_mixed_kernel, dim3(maxtiles, nbatch), dim3(256), 0, s, d_fds);
    KCHECK(hipGetLastError());
  }
  return hipSuccess;
}

// Kept factor of one front from its working storage: the first ns columns
// ([L U; F21'], contiguous since ld = n) and F12' (rows 0..ns of the last nu
// columns) repacked with ld = ns.  One grid row per front; the element index
// runs over both parts, so consecutive threads touch consecutive addresses of
// both source and destination except at column ends of F12'.
template <class T>
__global__ __launch_bounds__(256) void store_factor_kernel(const FrontDesc* __restrict__ fds) {
  const FrontDesc& fd = fds[blockIdx.y];
  const int64_t n = fd.n, ns = fd.ns, nu = n - ns;
  const int64_t panel = n * ns, total = panel + ns * nu;
  const cplx<T>* F = (const cplx<T>*)fd.F;
  cplx<T>* P = (cplx<T>*)fd.P;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    if (e < panel) {
      P[e] = F[e];
    } else {
      const int64_t q = e - panel, r = q % ns, c = q / ns;
      P[e] = F[r + (ns + c) * n];
    }
  }
}

template <class T>
hipError_t launch_store_factor(const FrontDesc* d_fds, int nbatch, int64_t max_elems, hipStream_t s) {
  if (nbatch == 0 || max_elems == 0) return hipSuccess;
  // about 8 elements per thread for the largest front, at most 1024 workgroups per front
  const int64_t gx = std::min<int64_t>(1024, std::max<int64_t>(1, (max_elems + 2047) / 2048));
  hipLaunchKernelGGL((store_factor_kernel<T>), dim3((unsigned)gx, nbatch), dim3(256), 0, s, d_fds);
  return hipGetLastError();
}

template hipError_t launch_store_factor<double>(const FrontDesc*, int, int64_t, hipStream_t);
template hipError_t launch_assemble<double>(const FrontDesc*, int, int, const void*, bool, hipStream_t);
template hipError_t launch_assemble<float>(const FrontDesc*, int, int, const void*, bool, hipStream_t);
template hipError_t launch_partial_lu<double>(const FrontDesc*, int, const int*, const int*, int*, hipStream_t);
template hipError_t launch_partial_lu<float>(const FrontDesc*, int, const int*, const int*, int*, hipStream_t);
template hipError_t launch_schur<double>(const FrontDesc*, int, const int*, const int*, hipStream_t);
template hipError_t launch_schur<float>(const FrontDesc*, int, const int*, const int*, hipStream_t);

}  // namespace bfmf
