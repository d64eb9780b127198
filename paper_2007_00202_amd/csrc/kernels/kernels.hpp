// Host-callable launchers of the HIP kernels.  All pointers are device
// pointers; every launcher queues work on stream `s` and returns the launch
// status.  T is the real type of the complex arithmetic (double: complex128,
// float: complex64).  Complex vectors and matrices are interleaved and
// column-major.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../devtypes.hpp"

namespace bfmf {

// ---- dense fronts (front.hip)
// Extend-add assembly of nbatch fronts (maxn = largest front).  Child
// contribution blocks are complex64 when cb_single, else complex128.
// values: the CSR values of A (complex128).
template <class T>
hipError_t launch_assemble(const FrontDesc* d_fds, int nbatch, int maxn, const void* values, bool cb_single,
                           hipStream_t s);
// Partial LU of nbatch fronts with restricted pivoting: F11 = P L U,
// F12 <- L^-1 P^T F12, F21 <- F21 U^-1 (right-looking, panels of 32).
// h_n / h_ns: host copies of the front sizes.  d_status[0..2]: singular flag,
// front, local index (first zero pivot).
template <class T>
hipError_t launch_partial_lu(const FrontDesc* d_fds, int nbatch, const int* h_n, const int* h_ns, int* d_status,
                             hipStream_t s);
// Schur complement C = F22 - F21 F12 of nbatch fronts (after the LU loop).
template <class T>
hipError_t launch_schur(const FrontDesc* d_fds, int nbatch, const int* h_n, const int* h_ns, hipStream_t s);
// the same on FP32 MFMA: complex128 fronts, operands rounded to complex64, product subtracted in double
hipError_t launch_schur_mixed(const FrontDesc* d_fds, int nbatch, const int* h_n, const int* h_ns, hipStream_t s);
// copy of the factor panels of dense fronts from F to P / F12 (null P: the host never sends these)
template <class T>
hipError_t launch_store_factor(const FrontDesc* d_fds, int nbatch, int64_t max_elems, hipStream_t s);

// ---- solve sweeps (solve.hip); workspaces in FrontDesc::W (n x nrhs, ld n)
// y(i, c) = B(perm[i], c) (B complex128, y complex<T>, ld N)
template <class T>
hipError_t launch_permute_in(const void* B, int64_t ldb, void* y, const int64_t* perm, int64_t N, int nrhs,
                             hipStream_t s);
// X(perm[i], c) = x(i, c)
template <class T>
hipError_t launch_permute_out(const void* x, void* X, int64_t ldx, const int64_t* perm, int64_t N, int nrhs,
                              hipStream_t s);
// Forward sweep over the fronts of one level (children done before).
template <class T>
hipError_t launch_forward_level(const FrontDesc* d_fds, int nbatch, int maxn, int maxnu, int maxns, const void* y,
                                int64_t N, int nrhs, hipStream_t s);
// Backward sweep over the fronts of one level (ancestors done before).
// the pivot interchanges of every dense front as one permutation (FrontDesc::pperm), for the sweeps
hipError_t launch_pivot_perm(const FrontDesc* d_fds, int nfront, hipStream_t s);
template <class T>
hipError_t launch_backward_level(const FrontDesc* d_fds, int nbatch, int maxn, int maxnu, int maxns, void* x,
                                 int64_t N, int nrhs, hipStream_t s);

// Gather-only steps of the sweeps (for compressed fronts, whose F11^-1, F12
// and F21 products run as butterfly applications).
template <class T>
hipError_t launch_fwd_gather(const FrontDesc* d_fds, int nbatch, int maxn, const void* y, int64_t N, int nrhs,
                             hipStream_t s);
template <class T>
hipError_t launch_bwd_gather(const FrontDesc* d_fds, int nbatch, int maxnu, const void* x, int64_t N, int nrhs,
                             hipStream_t s);

// ---- GMRES vectors (solve.hip), complex128
// Y = A X, or Y = B - A X when B is not null
hipError_t launch_spmv(const int64_t* rowptr, const int32_t* colind, const void* val, const void* X, int64_t ldx,
                       void* Y, int64_t ldy, const void* B, int64_t ldb, int64_t N, int nrhs, hipStream_t s);
// out[c] = V(:, c)^H W(:, c), or ||W(:, c)||_2 (real part) when norm
hipError_t launch_dots(const void* V, int64_t ldv, const void* Wv, int64_t ldw, int64_t N, int nrhs, void* partial,
                       int nblk, void* out, bool norm, hipStream_t s);
// W(:, c) += sign * a[c] V(:, c)
hipError_t launch_axpy_cols(const void* a, double sign, const void* V, int64_t ldv, void* Wv, int64_t ldw, int64_t N,
                            int nrhs, hipStream_t s);
// V(:, c) = W(:, c) / nrm[c]
hipError_t launch_scale_cols(const void* nrm, const void* Wv, int64_t ldw, void* V, int64_t ldv, int64_t N, int nrhs,
                             hipStream_t s);
// X(:, c) += sum_{k<m} y(k, c) V_k(:, c), V_k at V + k * vstride
hipError_t launch_basis_update(const void* y, int ldy, int m, const void* V, int64_t vstride, int64_t ldv, void* X,
                               int64_t ldx, int64_t N, int nrhs, hipStream_t s);
// slot GMRES of the serving form (per-column arguments; see solve.hip)
hipError_t launch_slot_gather(const void* const* d_src, void* Vcur, int64_t ld, int64_t N, int ncol, hipStream_t s);
hipError_t launch_slot_fix(const int32_t* d_mode, const void* B, int64_t ldb, void* T, int64_t ldt, int64_t N, int ncol,
                           hipStream_t s);
hipError_t launch_axpy_cols_masked(const void* a, double sign, const void* V, int64_t ldv, void* Wv, int64_t ldw,
                                   int64_t N, int nrhs, const int32_t* d_lim, int i0, hipStream_t s);
hipError_t launch_scale_cols_to(const void* nrm, const void* Wv, int64_t ldw, void* const* d_dst, int64_t N, int nrhs,
                                hipStream_t s);
hipError_t launch_basis_update_masked(const void* y, int ldy, const int32_t* d_mc, const void* V, int64_t vstride,
                                      int64_t ldv, void* X, int64_t ldx, int64_t N, int nrhs, hipStream_t s);

// ---- butterfly support (bf.hip)
// Tile shapes of the grouped GEMM (rows x columns of C per 256-thread
// workgroup).  0..4, 6 and 7 stage A and B through LDS; 5 is the skinny shape
// (no LDS, only for tasks with N <= 16 and no transposes).  The 48- and
// 96-row shapes fit the ranks of butterfly blocks (tasks of 33..48 and
// 65..96 rows) that the 32/64/128-row shapes pad by up to a half.  All give
// identical results.
constexpr int GEMM_CFGS = 8;
constexpr int GEMM_CFG_SKINNY = 5;
constexpr int GEMM_CFG_TM[GEMM_CFGS] = {64, 32, 128, 16, 256, 256, 48, 96};
constexpr int GEMM_CFG_TN[GEMM_CFGS] = {64, 128, 32, 256, 16, 16, 128, 64};
inline int64_t gemm_cfg_tiles(int cfg, int M, int N) {
  if (M <= 0 || N <= 0) return 0;
  return (int64_t)((M + GEMM_CFG_TM[cfg] - 1) / GEMM_CFG_TM[cfg]) * ((N + GEMM_CFG_TN[cfg] - 1) / GEMM_CFG_TN[cfg]);
}

// grouped GEMM over ntasks tasks in tile shape cfg; tile_start[i] = first tile
// of task i (tiles counted with gemm_cfg_tiles).  With events given, they take
// the kernel's own start and end timestamps (attached to the dispatch, so the
// time excludes the gaps between dispatches).
template <class T>
hipError_t launch_grouped_gemm(const GTask* d_tasks, const int64_t* d_tile_start, int ntasks, int64_t ntiles,
                               void* const bases[4], int cfg, hipStream_t s, hipEvent_t ev_start = nullptr,
                               hipEvent_t ev_stop = nullptr, bool gram = false);
// truncated column-pivoted QR of every task's q x p block (tol: |R_kk| > tol |R_00|), p <= maxp <=
// CPQR_WIDE_MAXP (the per-column state, 12 bytes a column, sits in dynamic LDS sized by maxp)
template <class T>
hipError_t launch_cpqr_id(const IdTask* d_tasks, int ntasks, double tol, int maxp, hipStream_t s);
// the same decompositions from G = A^H A (IdTask.G) by pivoted Cholesky: the rows of R in
// lds_entries complex entries of dynamic LDS per workgroup where min(maxrank, p) * p fits, else
// in IdTask.R
constexpr int GRAM_LDS_MAX = 4096;
constexpr int GRAM_MAXP = 2048;  // most columns of a Gram ID block
constexpr int CPQR_MAXP = 1024;       // widest Householder ID block before blocks are split into column chunks
constexpr int CPQR_WIDE_MAXP = 8192;  // most columns of a Householder ID block
constexpr int CPQR_MAXQ = 2048;       // most rows of a Householder ID block
constexpr size_t GRAM_LDS_BYTES = 159 * 1024;  // the dynamic LDS of a Gram ID launch at most (one CU's 160 KiB, less the static part)
// dynamic LDS of a Gram ID launch whose blocks have at most maxp columns (maxp a multiple of 16): per-column
// state (pivot search, selection, permutation: 20 bytes; two complex<double> rows: 32 bytes), then the R rows
__host__ __device__ inline size_t gram_aux_bytes(int maxp) { return (size_t)maxp * 52; }
template <class T>
hipError_t launch_gram_id(const IdTask* d_tasks, int ntasks, double tol, int lds_entries, int maxp, hipStream_t s);
// interpolation matrices from the QR results into outs[i] (ld ldo[i]);
// transpose_out writes the rank x p transpose (column ID), conj_out conjugates
template <class T>
hipError_t launch_id_expand(const IdTask* d_tasks, int ntasks, void* const* d_outs, const int64_t* d_ldo,
                            bool transpose_out, bool conj_out, hipStream_t s);
// submatrices of a front (A entries (+) children blocks) or of a dense matrix
template <class T>
hipError_t launch_front_extract(const ExtractTask* d_tasks, int ntasks, int yblocks, const void* values, bool src_single,
                                hipStream_t s);
// entries of butterflies in centre form (BfExtractTask list), written as complex<TO>
template <class TO>
hipError_t launch_bf_extract(const void* d_tasks, int ntasks, int yblocks, hipStream_t s);
// complex Gaussian probes (Philox4x32-10): column c nonzero on rows [gbeg[c/width], gend[c/width])
template <class T>
hipError_t launch_philox_gauss(void* Om, int64_t ld, int64_t n, int ncol, int width, const int32_t* d_gbeg,
                               const int32_t* d_gend, uint64_t seed, uint64_t stream_id, hipStream_t s);
// X A = B per task (tasks: SolveTask array), B overwritten
template <class T>
hipError_t launch_small_solve_right(const void* d_tasks, int ntasks, hipStream_t s);
// in-place inverse of small dense blocks (tasks: InvTask array); *status = 1 on a zero pivot
template <class T>
hipError_t launch_leaf_inverse(const void* d_tasks, int ntasks, int* d_status, hipStream_t s);
// Y(i, :) = X(rows[i], :) or, with scatter, Y(rows[i], :) = X(i, :)
template <class T>
hipError_t launch_gather_rows(const void* X, int64_t ldx, void* Y, int64_t ldy, const int32_t* rows, int nr, int ncol,
                              bool scatter, hipStream_t s);
// Y = a X + b Y (X may be null: Y = b Y)
template <class T>
hipError_t launch_axpby(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol, double a, double b,
                        hipStream_t s);
// y_t = a x_t + b y_t for a batch of blocks (max_entries: the largest m ncol)
// Y (T1) = a X (T2) + b Y + diag E per task (AxpbyTask; X null: zero; E(i, c) = 1 where
// i == c + pad), arithmetic in double
template <class T1, class T2>
hipError_t launch_mix_batch(const AxpbyTask* d_tasks, int ntasks, int64_t max_entries, double a, double b,
                            double diag, hipStream_t s);
// bordered fronts [I I; -I 0] (Y, 2m x 2m) and identities (X, m x m) per task
template <class T>
hipError_t launch_smw_border(const AxpbyTask* d_tasks, int ntasks, int64_t max_n, hipStream_t s);
// Gaussian probe blocks per task (ProbeTask), groups from one pair of row-range arrays
template <class T>
hipError_t launch_philox_gauss_batch(const ProbeTask* d_tasks, int ntasks, int64_t max_entries,
                                     const int32_t* d_gbeg, const int32_t* d_gend, uint64_t seed, hipStream_t s);
template <class T>
hipError_t launch_axpby_batch(const AxpbyTask* d_tasks, int ntasks, int64_t max_entries, double a, double b,
                              hipStream_t s);
// Y(i, j) = v when i == j + off, else 0 (m x ncol block)
template <class T>
hipError_t launch_set_eye(void* Y, int64_t ldy, int64_t m, int ncol, int64_t off, double v, hipStream_t s);
// Y (complex<T1>) = X (complex<T2>)
template <class T1, class T2>
hipError_t launch_convert(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol, hipStream_t s);
// Y (complex<T1>) = a X (complex<T2>) + b Y, arithmetic in FP64 (b = 0 overwrites)
template <class T1, class T2>
hipError_t launch_axpby_mixed(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol, double a,
                              double b, hipStream_t s);

struct SolveTask {
  void* A;
  int64_t lda;
  void* B;
  int64_t ldb;
  int32_t k, r;
};
struct InvTask {
  void* A;
  int64_t lda;
  int32_t n;
  int32_t pad;
};

// B(rows[e], cols[e]) = (vals[2e], vals[2e+1]) for e < nnz (complex128 block, ld ldb)
hipError_t launch_scatter_nz(void* B, int64_t ldb, const int32_t* rows, const int32_t* cols, const double* vals,
                             int64_t nnz, hipStream_t s);

}  // namespace bfmf
