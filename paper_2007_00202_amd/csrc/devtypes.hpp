// Plain-old-data descriptors shared by the host orchestration and the HIP
// kernels.  All pointers are device pointers.
#pragma once
#include <cstdint>

namespace bfmf {

// operand transformation of the GEMM kernels: none, transpose, conjugate transpose
enum : int32_t { OP_N = 0, OP_T = 1, OP_C = 2 };

// A butterfly expanded to its centre level for entry extraction (Alg. 3 with
// every factor block multiplied once for all rows and columns).  Centre block
// blk = t * nv + v (t: node at level lc of the row tree, v: node at level
// L - lc of the column tree) holds E = (U^L R^{L-1} .. R^{lc}) restricted to
// the block (rows of t x rank, column-major, ld = rows of t) and G = B F
// (rank x columns of v, column-major, ld = rank), so that an entry is
// K(x, y) = E(x, :) G(:, y), one dot product of the block's rank.
struct BfCentreDev {
  const int32_t* tb;     // nt + 1 row boundaries at level lc
  const int32_t* vb;     // nv + 1 column boundaries at level L - lc
  const void* const* E;  // per block
  const void* const* G;  // per block
  const int32_t* rk;     // per block rank
  int32_t nt, nv;
  int32_t single;        // entries complex<float> (else complex<double>)
  int32_t pad;
};

// One node of a contribution block in HOD-BF form (Sec. 4): rows and
// columns [beg, end), children split at mid.  A leaf holds its dense block
// (ld end - beg); an internal node its two off-diagonal butterflies, rows
// [beg, mid) x columns [mid, end) (b12) and the converse (b21), as indices
// into the centre-form array (-1: zero block).
struct HodbfNodeDev {
  int32_t beg, mid, end, left, right, b12, b21, pad;
  const void* leaf;
};
struct HodbfDev {
  const HodbfNodeDev* nodes;  // node 0 is the root
  const BfCentreDev* bfs;
  int32_t single;             // leaf entries complex<float> (else complex<double>)
  int32_t depth;              // longest root-to-leaf path (bounds the descent)
};

// out(i, j) = alpha K(rows[i], cols[j]) (or out += ... when accumulate) for a
// butterfly in centre form; nr x nc (ld ldo), or the transpose when trans.
struct BfExtractTask {
  const BfCentreDev* bf;
  const int32_t* rows;
  const int32_t* cols;
  int32_t nr, nc;
  void* out;
  int64_t ldo;
  int32_t trans, accumulate;
  double alpha;
};

// One dense front F (n x n, column-major, ld = n) of the multifrontal tree.
// F = [F11 F12; F21 F22] with F11 of size ns (the fully-summed variables
// I^s) and F22 of size n - ns (the update variables I^u).
struct FrontDesc {
  void* F;            // complex<T> working storage during the factorization, n*n elements (ld n)
  void* P;            // kept factor after it: [L and U packed; F21'] (n x ns, ld n) ...
  void* F12;          // ... and F12' (ns x nu, ld ld12); both null for compressed fronts
  int64_t ld12;
  int32_t n, ns;
  int32_t nchild;     // 0..2
  int32_t front;      // front id (postorder)
  int32_t f21_unit;   // 1: F21 starts as -I (nu == ns), so its column j is zero below row ns + j until
                      // the panel holding column j is done; the factorization skips those rows
  int32_t pad_;
  int64_t sbeg;       // first global (new) index of I^s
  const int32_t* inv[2];   // parent-local -> child-local index or -1 (length n)
  const void* cb[2];       // child contribution block (child F at (ns_c, ns_c))
  int64_t cb_ld[2];        // child leading dimension (child n)
  const HodbfDev* chb[2];  // when not null: the child's contribution block in HOD-BF form
  const int64_t* a_ptr;    // n+1 offsets into a_row / a_vidx, per local column
  const int32_t* a_row;    // local row of each A entry of the column
  const int64_t* a_vidx;   // index of the entry in the CSR value array
  int32_t* piv;            // ns pivots (LAPACK interchange convention, 0-based)
  int32_t* pperm;          // the interchanges as one permutation: row i of P^T F11 is row pperm[i]
  const int32_t* iu;       // I^u as global new indices (length n - ns)
  void* W;                 // solve workspace (n x nrhs, ld = n)
  const void* cw[2];       // children's solve workspaces (contribution part at row ns_c)
  int64_t cw_ld[2];
};

}  // namespace bfmf

namespace bfmf {

// One product of a grouped (ragged) GEMM: C = beta C + alpha op(A) op(B).
// Operand addresses are element offsets from one of the base pointers the
// launch receives (base[abase] + a_off, ...), so a task list can be reused
// for other input/output buffers with the same layout.  Base index 4 means
// no base: the offset is the operand's device address divided by the
// element size.
struct GTask {
  int64_t a_off, b_off, c_off;
  int64_t lda, ldb, ldc;
  int32_t M, N, K;
  int8_t opA, opB, abase, bbase, cbase, beta;
  int8_t pad[2];
  double alpha_re, alpha_im;
};

// Interpolative decomposition of one block: A is q x p (column-major, lda),
// the transpose of the block whose rows are being selected.  Results: rank,
// pivoted column order (perm, p entries) and T = R11^-1 R12 (rank x (p-rank),
// ld = p) for the interpolation matrix.
struct IdTask {
  void* A;        // q x p workspace, overwritten
  int64_t lda;
  int32_t q, p;
  int32_t maxrank;
  int32_t* rank;  // output
  int32_t* perm;  // output, p entries
  void* T;        // output, maxrank x p (ld maxrank)
  void* G;        // Gram variant: G = A^H A (p x p, ld p), input
  void* R;        // Gram variant: workspace, maxrank x p (row i at R + i p)
};

// Extraction of the dense submatrix F(rows, cols) of a front that is never
// formed (A entries plus the children's contribution blocks), or of a dense
// matrix in device memory.
struct ExtractTask {
  const int32_t* rows;  // front-local row indices
  const int32_t* cols;  // front-local column indices
  int32_t nr, nc;
  void* out;            // nr x nc (ld ldo), or nc x nr (ld ldo) when trans
  int64_t ldo;
  int32_t trans;        // write the transpose
  int32_t pad;
  const void* dense;    // when not null: F is this dense matrix (ld ldd, complex<T>)
  int64_t ldd;
  const FrontDesc* fd;  // otherwise: the front (device descriptor)
};

// One y = a x + b y of a batch (complex<T> blocks m x ncol; x may be null: y = b y)
struct AxpbyTask {
  void* Y;
  const void* X;
  int64_t ldy, ldx, m;
  int32_t ncol, pad;
};

// One block of Gaussian probe columns: Om (n x ncol, ld); column c belongs to
// group g0 + c / width, supported on the rows [gbeg[g], gend[g]) of the
// launch's group arrays; entries from the counter-based generator keyed by
// (seed, stream_id, row, column).
struct ProbeTask {
  void* Om;
  int64_t ld, n;
  int32_t ncol, width, g0, pad;
  uint64_t stream_id;
};

}  // namespace bfmf
