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
hipError_t launch_forward_level(const FrontDesc* d_fds, int nbatch, int maxn, int maxnu, const void* y, int64_t N,
                                int nrhs, hipStream_t s);
// Backward sweep over the fronts of one level (ancestors done before).
template <class T>
hipError_t launch_backward_level(const FrontDesc* d_fds, int nbatch, int maxn, int maxnu, void* x, int64_t N,
                                 int nrhs, hipStream_t s);

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

}  // namespace bfmf
