// Plain-old-data descriptors shared by the host orchestration and the HIP
// kernels.  All pointers are device pointers.
#pragma once
#include <cstdint>

namespace bfmf {

// One dense front F (n x n, column-major, ld = n) of the multifrontal tree.
// F = [F11 F12; F21 F22] with F11 of size ns (the fully-summed variables
// I^s) and F22 of size n - ns (the update variables I^u).
struct FrontDesc {
  void* F;            // complex<T> storage, n*n elements
  int32_t n, ns;
  int32_t nchild;     // 0..2
  int32_t front;      // front id (postorder)
  int64_t sbeg;       // first global (new) index of I^s
  const int32_t* inv[2];   // parent-local -> child-local index or -1 (length n)
  const void* cb[2];       // child contribution block (child F at (ns_c, ns_c))
  int64_t cb_ld[2];        // child leading dimension (child n)
  const int64_t* a_ptr;    // n+1 offsets into a_row / a_vidx, per local column
  const int32_t* a_row;    // local row of each A entry of the column
  const int64_t* a_vidx;   // index of the entry in the CSR value array
  int32_t* piv;            // ns pivots (LAPACK interchange convention, 0-based)
  const int32_t* iu;       // I^u as global new indices (length n - ns)
  void* W;                 // solve workspace (n x nrhs, ld = n)
  const void* cw[2];       // children's solve workspaces (contribution part at row ns_c)
  int64_t cw_ld[2];
};

}  // namespace bfmf
