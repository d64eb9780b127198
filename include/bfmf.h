/*
 * bfmf.h -- C ABI of libbfmf, a butterfly-compressed multifrontal solver for
 * complex sparse systems on AMD Instinct MI355X (gfx950).
 *
 * Method: Liu, Ghysels, Claus, Li, "Sparse Approximate Multifrontal
 * Factorization with Butterfly Compression for High Frequency Wave
 * Equations".  The problem statement is: given A in C^{N x N} and b, compute
 * x ~= A^{-1} b (Sec. 2, Alg. 1 and Alg. 5).  The three phases map to:
 *
 *   bfmf_analyze : fill-reducing nested dissection P, separator bisection
 *                  P-hat, assembly tree, index sets I^s / I^u, extend-add maps
 *                  (Alg. 1 steps 1-3, Alg. 5 steps 1-3, Sec. 5.1, Sec. 5.2)
 *   bfmf_factor  : numerical factorization with ID tolerance `tol` and the
 *                  compression threshold n_min (Alg. 5 loop); fronts below
 *                  the threshold use the dense partial LU of Alg. 1
 *   bfmf_solve   : preconditioned restarted GMRES (Alg. 5 last step, Sec. 6)
 *                  with the factorization as preconditioner
 *
 * Conventions
 *   - Every call returns a bfmf_status; no exception crosses the ABI.
 *   - Complex numbers are interleaved (re, im) pairs of doubles at the ABI.
 *     Dense blocks are column-major with an explicit leading dimension.
 *   - Input arrays are borrowed for the duration of the call only and are
 *     copied.  The handle owns all device memory it allocates until
 *     bfmf_destroy.  Pointers returned through views are owned by the handle
 *     and stay valid until the next bfmf_analyze or bfmf_destroy.
 *   - State machine: created -> analyzed -> factored.  A call out of order
 *     returns BFMF_E_STATE.  bfmf_factor may be called again (new tol, new
 *     values through bfmf_set_values) on an analyzed handle.
 *   - A handle is not thread-safe; use one handle per host thread or lock.
 *   - On BFMF_E_DEVICE the handle is unusable; destroy it.
 */
#ifndef BFMF_H
#define BFMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfmf_ctx* bfmf_handle;

typedef enum {
    BFMF_OK = 0,
    BFMF_E_INVAL = -1,    /* bad argument, malformed CSR, NaN/Inf input */
    BFMF_E_NOMEM = -2,    /* device memory (or the handle's HBM budget) exhausted */
    BFMF_E_STATE = -3,    /* call out of order (e.g. solve before factor) */
    BFMF_E_SINGULAR = -4, /* exact zero pivot; see bfmf_stats.singular_front */
    BFMF_E_NOCONV = -5,   /* GMRES hit max_iter; X holds the best iterate */
    BFMF_E_DEVICE = -6    /* HIP runtime error */
} bfmf_status;

enum { BFMF_ORD_GRID = 0, BFMF_ORD_YEE = 1, BFMF_ORD_USER = 2 };
enum { BFMF_C128 = 0, BFMF_C64_MIXED = 1 };
enum { BFMF_HOST = 0, BFMF_DEVICE = 1 };

/* Geometric nested dissection (Sec. 2; planar separators as in Sec. 6).
 * GRID: unknown i sits on node (i % nx, (i / nx) % ny, i / (nx ny)) of an
 *       nx x ny x nz grid; boxes of at most leaf_max nodes are leaves.
 * YEE : unknowns are interior edges of an nx^3 cell grid; coords[3 i + d]
 *       holds the doubled coordinate of edge i along axis d (one odd entry).
 * sep_leaf: leaf size of the recursive separator bisection that defines the
 *       HOD-BF tree of F11 and the permutation P-hat (Sec. 5.1); also the leaf
 *       size of the balanced tree on I^u.
 * parallel_levels (GRID only, default 0): separator variant of the Sec. 6
 *       remark on high frequencies.  The boxes at the top parallel_levels
 *       levels of the tree are cut across the grid's longest axis (while its
 *       extent in the box is at least 3), so those separators are parallel
 *       planes: F12/F21 of their fronts couple well-separated planes.  E_INVAL
 *       if negative, or nonzero with YEE or USER.
 * USER: the caller's ordering and assembly tree (the "given ordering" of the
 *       problem statement, Sec. 2): perm[n] maps new index -> original index;
 *       front f owns the separator [front_ptr[f], front_ptr[f+1]) of the new
 *       numbering (nfronts + 1 entries, front_ptr[0] = 0, strictly increasing,
 *       front_ptr[nfronts] = n); front_parent[f] is its parent, -1 for the
 *       root.  The tree must be in postorder: every parent after its children,
 *       the root last and alone, each subtree a contiguous run of fronts
 *       ending at its root.  Fronts without children are leaves (never
 *       compressed).  Each separator's HOD-BF tree halves its index range
 *       (first half ceil) down to sep_leaf, so the caller orders a separator
 *       the way its bisection should go (P-hat, Sec. 5.1).  E_INVAL when perm
 *       is not a bijection, the tree is not in postorder, or the separator
 *       property fails (an edge of A, or fill, between two fronts neither of
 *       which is an ancestor of the other).  The arrays are copied. */
typedef struct {
    int32_t kind;
    int32_t nx, ny, nz;
    const int32_t* coords;
    int32_t leaf_max; /* default 512 */
    int32_t sep_leaf; /* default 64 */
    int32_t parallel_levels; /* default 0 */
    int32_t nfronts;              /* USER only */
    const int64_t* perm;          /* USER only: [n] */
    const int64_t* front_ptr;     /* USER only: [nfronts + 1] */
    const int32_t* front_parent;  /* USER only: [nfronts] */
} bfmf_ordering;

/* Numerical factorization options (Alg. 5; Sec. 3.1 for alpha and k_nn). */
typedef struct {
    double tol;          /* ID tolerance epsilon (Sec. 6: "ID tolerance") */
    int64_t n_min;       /* compress separator fronts with #I^s >= n_min; <= 0: none */
    int32_t precision;   /* BFMF_C128 or BFMF_C64_MIXED (c64 bulk, FP64 pivots) */
    int32_t batched;     /* 0: one launch per front and op; 1: level-batched launches */
    int32_t samples;     /* random probe columns per block in randomized construction */
    int32_t knn;         /* graph nearest neighbours per row for proxy sampling */
    double alpha;        /* uniform over-sampling factor for proxy sampling */
    uint64_t seed;       /* seed of the device Philox probe generator */
    uint64_t hbm_budget; /* bytes the factorization may use; 0 = all free memory */
    int32_t keep_fronts; /* debug: keep a copy of every assembled dense front, and every
                            factored front whole (no reuse of the level workspaces) */
    int32_t timing;      /* 1: time every kernel class with HIP events (bfmf_get_kernel_stats) */
    int32_t smw_dense;   /* HODBF_invert (Alg. 4): BF_SMW blocks of at most this many rows are
                            inverted densely (FP64 partial LU of the bordered block), larger ones
                            are split into four children butterflies; 0 means 1024, values in
                            1..15 are E_INVAL */
    int32_t id_max_cols; /* widest block given to one interpolative-decomposition kernel
                            (0: the kernels' own limits, 2048 columns for tol >= 1e-4, else
                            1024); wider blocks are decomposed as an ID of the IDs of column
                            chunks (about twice the tolerance), or whole by the Householder
                            kernel (up to 8192 columns and 2048 rows) when every chunk has
                            full rank; a block beyond that gives E_INVAL; values in 1..15 are
                            E_INVAL */
    int32_t compress_cb; /* 1: the contribution block of a compressed front whose parent is
                            compressed too is built as an HOD-BF (tree: balanced bisection of
                            I^u, leaves of at most 64) by entry evaluation of C_nu1 (+) C_nu2 - S
                            (Alg. 5, last step), and the parent reads its entries through
                            extract_HODBF / extract_BF (Alg. 3); such blocks then take no level
                            workspace.  0 (default): they are dense FP64 blocks there.  Other
                            values are E_INVAL */
    int32_t reserved[3];
} bfmf_factor_opts;

/* GMRES options (Sec. 6): restarted GMRES(restart), modified Gram-Schmidt,
 * zero initial guess, left preconditioning; a cycle of a column ends when
 * ||u_i|| <= atol or ||u_i|| / ||u_0|| <= rtol with u_i = M^-1 (A x_i - b).
 * Without true_rtol a column whose cycle ended that way is done.  With
 * true_rtol > 0 the stop is the true residual instead: at the end of every
 * restart cycle each column's ||b - A x|| / ||b|| is computed and the column
 * is done once it is at most true_rtol; a column whose preconditioned test
 * was met while its true residual was still above true_rtol continues with
 * a ten times smaller rtol.  Columns are independent: each has its own
 * Krylov space, and its iterates do not depend on the other columns. */
typedef struct {
    int32_t restart;     /* default 30 */
    int32_t max_iter;    /* default 300 (0 also means 300); negative: direct solve, X = M^-1 B
                            with the approximate factorization and no iteration, the true
                            residual in relres_max, E_NOCONV when it exceeds true_rtol > 0 */
    double rtol, atol;   /* defaults 1e-6, 1e-10 */
    double true_rtol;    /* e.g. 1e-3; 0 disables */
    /* outputs */
    int32_t iters_max;   /* largest iteration count over the columns */
    int32_t graphs;      /* input: 1 (default) replays the preconditioner of the GMRES
                            iterations from a HIP graph captured once per call (same
                            results as 0, which launches every sweep from the host) */
    double relres_max;   /* largest true relative residual over the columns */
    double seconds;      /* wall time of the call */
} bfmf_solve_opts;

/* Read-only view of the symbolic analysis (all arrays owned by the handle). */
typedef struct {
    int64_t n;
    int32_t nfronts;
    int32_t nlevels;
    const int64_t* perm;       /* [n] new index -> original index */
    const int64_t* sbeg;       /* [nfronts] I^s = [sbeg, send) in the new numbering */
    const int64_t* send;
    const int32_t* parent;     /* [nfronts] -1 at the root; fronts are in postorder */
    const int32_t* level;      /* [nfronts] depth, root = 0 */
    const int32_t* child_ptr;  /* [nfronts+1] */
    const int32_t* child_list; /* children, left first */
    const int64_t* iu_ptr;     /* [nfronts+1] */
    const int64_t* iu;         /* sorted I^u of each front (new numbering) */
    const int32_t* map;        /* at iu_ptr[f]: position of I^u_f in concat(I^s_p, I^u_p) */
    const int32_t* sep_ptr;    /* [nfronts+1] node ranges of the bisection trees */
    const int32_t* sep_nodes;  /* 4 ints per node in preorder: beg, end, left, right */
} bfmf_symbolic_view;

/* Counters mirroring the paper's Table "HH" rows plus timings. */
typedef struct {
    int32_t nfronts, compressed_fronts, dense_fronts, nlevels;
    double analyze_seconds, factor_seconds;
    double factor_flops;          /* algorithmic flops of the factorization */
    double factor_bytes;          /* bytes held by the factors */
    double dense_factor_bytes;    /* bytes the same factors take uncompressed */
    int32_t max_rank;
    int32_t singular_front;       /* front of an exact zero pivot, or -1 */
    int32_t singular_index;       /* local pivot index within that front */
    int32_t id_chunked;           /* ID blocks wider than one kernel, done as IDs of sub-IDs */
    double solve_flops_per_rhs;   /* one preconditioner application */
    uint64_t device_bytes_peak;   /* device memory held by the handle */
    double cb_bytes;              /* bytes of the contribution blocks kept in HOD-BF form */
    double cb_dense_bytes;        /* bytes the same blocks take dense (nu^2 entries each) */
    int32_t cb_compressed;        /* contribution blocks built in HOD-BF form (compress_cb) */
    int32_t pad0;
    double workspace_bytes;       /* level workspaces (dense fronts and dense contribution blocks) */
    double reserved[4];
} bfmf_stats;

/* Create a handle on HIP device `device`.  `hip_stream` (hipStream_t) is the
 * stream all work is queued on; NULL uses a stream owned by the handle.
 * device = -1 creates a host-only handle that supports bfmf_analyze,
 * bfmf_get_symbolic and bfmf_get_stats (no device is touched); factor and
 * solve on it return BFMF_E_STATE.  E_DEVICE if the device does not exist. */
bfmf_status bfmf_create(bfmf_handle* h, int32_t device, void* hip_stream);

/* Analyze A (CSR: rowptr[n+1] int64, colind[nnz] int32 sorted per row,
 * values[2 nnz] interleaved complex128 or NULL for pattern only) with the
 * given ordering.  Computes P, P-hat, the assembly tree, I^s, I^u and all
 * extend-add maps on the host and uploads them with the CSR to the device.
 * Errors: E_INVAL for malformed CSR or ordering, E_NOMEM, E_DEVICE. */
bfmf_status bfmf_analyze(bfmf_handle h, int64_t n, const int64_t* rowptr,
                         const int32_t* colind, const double* values,
                         const bfmf_ordering* ord);

/* Replace the numerical values of A (same pattern).  Host array of 2 nnz
 * doubles.  Returns the handle to the analyzed state. */
bfmf_status bfmf_set_values(bfmf_handle h, const double* values);

/* Fill `opts` with the defaults: tol 1e-3, n_min 1024, c128, plain, 64
 * samples, knn 8, alpha 2, seed 0, no budget. */
void bfmf_default_factor_opts(bfmf_factor_opts* opts);
void bfmf_default_solve_opts(bfmf_solve_opts* opts);

/* Numerical factorization (Alg. 5).  Fronts whose separator has at least
 * n_min nodes are compressed (HOD-BF F11 and its inverse, butterfly F12, F21
 * and Schur update); all others use the dense partial LU with pivoting
 * restricted to F11 (Alg. 1).  On E_NOMEM or E_SINGULAR the handle returns
 * to the analyzed state. */
bfmf_status bfmf_factor(bfmf_handle h, const bfmf_factor_opts* opts);

/* Solve A X = B for nrhs columns with GMRES preconditioned by the
 * factorization.  B (ldb >= n) and X (ldx >= n) are interleaved complex128,
 * column-major, in host memory (mem = BFMF_HOST) or device memory
 * (BFMF_DEVICE).  `io` may be NULL (defaults); its output fields are written.
 * Returns E_NOCONV (with the best X) when max_iter is reached. */
bfmf_status bfmf_solve(bfmf_handle h, int64_t nrhs, const double* B, int64_t ldb,
                       double* X, int64_t ldx, int32_t mem, bfmf_solve_opts* io);

/* The direct solve X = M^-1 B (forward then backward sweep through all
 * fronts, the approximate factorization used as a direct solver: Sec. 6,
 * tolerance study) queued on the caller's stream hip_stream (NULL: the
 * handle's) without waiting for it: dB and dX are device pointers
 * (interleaved complex128, column-major, ld >= n), X is valid once the
 * stream has completed the call's work.  The call is ordered after earlier
 * work of the handle and before its later work.  X equals bfmf_solve's with
 * max_iter < 0 bit for bit.  io may be NULL; io->max_iter must be negative
 * (GMRES needs the host at every iteration: E_INVAL otherwise); on return
 * io->iters_max = 0, io->relres_max = -1 (not computed) and io->seconds is
 * the host time of the call.  The first call with a new column count may
 * wait for the device while it sizes its workspaces. */
bfmf_status bfmf_solve_async(bfmf_handle h, int64_t nrhs, const double* dB, int64_t ldb, double* dX, int64_t ldx,
                             void* hip_stream, bfmf_solve_opts* io);

/* Apply the preconditioner once, X = M^-1 B (forward then backward sweep
 * through all fronts), without GMRES.  Same layout rules as bfmf_solve. */
bfmf_status bfmf_apply_preconditioner(bfmf_handle h, int64_t nrhs, const double* B,
                                      int64_t ldb, double* X, int64_t ldx, int32_t mem);

bfmf_status bfmf_get_symbolic(bfmf_handle h, bfmf_symbolic_view* out);
bfmf_status bfmf_get_stats(bfmf_handle h, bfmf_stats* out);

/* Debug access to a dense front after bfmf_factor, copied to host memory:
 *   what = 0: the assembled front F (needs keep_fronts), n x n
 *   what = 1: the factored front [LU F12'; F21' C], n x n; the contribution
 *             block C only with keep_fronts, zeros otherwise (it lives in a
 *             level workspace that later levels reuse)
 *   what = 2: the pivot sequence of F11 (ns int32 values, 0-based, LAPACK
 *             interchange convention), written to out as int32
 * n = #I^s + #I^u of the front; out has leading dimension ld >= n.
 * E_INVAL for compressed fronts or out-of-range arguments. */
bfmf_status bfmf_get_front(bfmf_handle h, int32_t front, int32_t what, void* out, int64_t ld);

/* Debug access to a compressed front after bfmf_factor: Y = B X for one of
 * its blocks, all in the front's local numbering (I^s in P-hat order, then
 * I^u sorted), so that the blocks can be compared with the dense ones:
 *   what = 0: F11 as the HOD-BF built by entry evaluation (Sec. 4.1), ns x ns
 *   what = 1: F11^-1 as built by HODBF_invert (Alg. 4), ns x ns
 *   what = 2: F12 (butterfly, Alg. 2), ns x nu
 *   what = 3: F21 (butterfly, Alg. 2), nu x ns
 *   what = 4: S = F21 F11^-1 F12 by randomized construction (Sec. 3.3), nu x nu
 * X (columns of B x nrhs, ld ldx) and Y (rows of B x nrhs, ld ldy) are host
 * arrays of interleaved complex128, column-major; in the complex64 form X is
 * rounded to complex64 before the product.  E_INVAL if the front is not
 * compressed, for what outside 0..4, for 2..4 on a front with an empty
 * update set, or for bad sizes; E_STATE before bfmf_factor. */
bfmf_status bfmf_apply_front_block(bfmf_handle h, int32_t front, int32_t what, int32_t nrhs, const double* X,
                                   int64_t ldx, double* Y, int64_t ldy);

/* Debug access to the list routing of entry evaluation (Sec. 5): out(i, j)
 * = F(rows[i], cols[j]) of a front that is never formed, F = [A(Is,Is)
 * A(Is,Iu); A(Iu,Is) 0] (+) C_nu1 (+) C_nu2, each request split into its
 * A part and its child parts through the inverse extend-add maps and served
 * by the extraction kernel the compressed fronts use.  Indices are
 * front-local (0 .. n-1: I^s, then I^u); out is a host array of interleaved
 * complex128, column-major, ld ldo >= nrows.  Needs a factorization with
 * keep_fronts (the children's contribution blocks are kept); E_INVAL
 * otherwise or for indices outside the front, E_STATE before bfmf_factor. */
bfmf_status bfmf_extract_front(bfmf_handle h, int32_t front, int32_t nrows, const int32_t* rows, int32_t ncols,
                               const int32_t* cols, double* out, int64_t ldo);

/* Per kernel-class timing, collected with HIP events on the handle's stream
 * while bfmf_factor_opts.timing is set (factor and solve calls accumulate).
 * Classes: 0 assemble (extend-add), 1 panel LU loop (panel, interchanges,
 * triangular solves, rank-32 updates), 2 Schur GEMM C = F22 - F21 F12,
 * 3 forward sweep level, 4 backward sweep level, 5 SpMV, 6 GMRES vector ops,
 * 7 butterfly grouped GEMMs (products of butterflies and the GEMMs of their
 * constructions), 8 interpolative decompositions, 9 entry extraction,
 * 10 copy of the dense fronts' factors out of the level workspace,
 * 11 replays of the captured preconditioner (forward and backward sweeps of
 * the GMRES iterations when bfmf_solve_opts.graphs is set; the sweeps of
 * eager applications count in classes 3, 4 and 7-9).
 * Class 7 times about one launch in eight, chosen quasi-randomly (the
 * fractional parts of i times the golden ratio below 1/8, i = launch index),
 * with the kernel's own start and end timestamps (events attached to the
 * dispatch); the other classes time every launch with events recorded on
 * the stream around it, which also covers the gaps between dispatches.
 * launches counts the timed launches and launches_all every launch of the
 * class; seconds, flops and bytes (algorithmic counts) cover the timed
 * launches.
 * E_INVAL for an unknown class; bfmf_reset_kernel_stats clears all. */
typedef struct {
    char name[32];
    int64_t launches;
    double seconds;
    double flops;
    double bytes;
    int64_t launches_all;
} bfmf_kernel_stat;
enum { BFMF_KERNEL_CLASSES = 12 };
bfmf_status bfmf_get_kernel_stats(bfmf_handle h, int32_t kind, bfmf_kernel_stat* out);
bfmf_status bfmf_reset_kernel_stats(bfmf_handle h);

/* Tile shapes of the grouped GEMM behind every butterfly product (the
 * block-diagonal levels of an apply, Sec. 3, and the products of the
 * constructions).  Rows x columns of C per workgroup:
 *   0: 64 x 64, 1: 32 x 128, 2: 128 x 32, 3: 16 x 256, 4: 256 x 16, 6: 48 x 128,
 *   7: 96 x 64 (A and B staged through LDS), 5: 256 x 16 streaming (only for
 *   tasks with at most 16 columns and no transposes).
 * By default each product phase takes the shape of least predicted time from
 * a table measured on the device on first use (every shape timed on synthetic
 * launches over a grid of task shapes, per precision; a few seconds, once per
 * process and device); a phase whose tasks differ in height is split into one
 * launch per shape when that is predicted at least 5% faster.  All shapes
 * give the same result bit for bit.  bfmf_set_gemm_tile forces one shape for
 * the whole process (-1: back to the measured choice; shape 5 falls back to 0
 * where it does not apply); E_INVAL outside -1..7.
 * bfmf_get_gemm_tile_launches writes the number of launches per shape since
 * the last bfmf_reset_kernel_stats into out[0..7] (n >= 8). */
enum { BFMF_GEMM_TILES = 8 };
bfmf_status bfmf_set_gemm_tile(int32_t cfg);
bfmf_status bfmf_get_gemm_tile_launches(bfmf_handle h, int64_t* out, int32_t n);

/* Butterfly compression of a caller-given dense matrix (Sec. 3), for
 * checking the butterfly kernels on their own.  K: m x n complex128,
 * column-major (ld >= m), host memory, copied.  L: levels of the row and
 * column trees (halving bisection of [0, m) and [0, n)).  method 0: entry
 * evaluation with alpha = 4 uniform proxies per block, at most 2048 below
 * tol 1e-4 (Alg. 2); method 1:
 * randomized products with K and K^H (Sec. 3.3), `samples` probes per tree
 * node (doubled while an ID rank comes within 8 of it).  tol: ID tolerance.
 * E_INVAL for bad sizes, E_DEVICE / E_NOMEM from the runtime. */
typedef struct bfmf_bf bfmf_bf;
bfmf_status bfmf_bf_compress_dense(int32_t device, int32_t m, int32_t n, const double* K, int64_t ldk, int32_t L,
                                   double tol, int32_t method, int32_t samples, uint64_t seed, bfmf_bf** out);
/* Y = K X (adjoint = 0, X n x nrhs, Y m x nrhs) or Y = K^H X (adjoint = 1),
 * host arrays, interleaved complex128, column-major. */
bfmf_status bfmf_bf_apply(bfmf_bf* b, int32_t adjoint, int32_t nrhs, const double* X, int64_t ldx, double* Y,
                          int64_t ldy);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture aside, tight serving loops, harnesses that forbid hipMalloc): the
 * product of bfmf_bf_apply with X (dX, in-columns x nrhs, ld ldx) and Y (dY,
 * ld ldy) in device memory, interleaved complex128, queued on hip_stream
 * (NULL: the butterfly's own stream).  It calls no hipMalloc, hipFree or
 * allocating library routine: its task lists and inter-level workspace live
 * in a fixed device array of 64 MiB per device, held until the process ends.
 * Every launch uses the 64 x 64 tile, so Y equals bfmf_bf_apply's bit for bit.
 * Returns after Y is complete (the stream is synchronized).  Calls that
 * overlap on one device race on the shared array.  E_INVAL for bad sizes or a
 * product that needs more than the fixed array. */
bfmf_status bfmf_bf_apply_noalloc(bfmf_bf* b, int32_t adjoint, int32_t nrhs, const double* dX, int64_t ldx,
                                  double* dY, int64_t ldy, void* hip_stream);
/* A butterfly from caller-given factors (Sec. 3, the factored form
 * K = U^L R^{L-1} .. R^{lc} B^{lc} W^{lc} .. W^1 V^0 with lc = floor(L/2)),
 * over the halving trees of [0, m) and [0, n) (first half ceil) of L levels,
 * 0 <= L <= 12.  Block (l, t, v) pairs node t at level l of the row tree with
 * node v at level L - l of the column tree; blk = t * 2^(L-l) + v.
 *   ranks_left:  (L - lc + 1) x 2^L, row l - lc holds the rank of the left
 *                factor of block (l, t, v) for l = lc..L (at l = L, v = 0 and
 *                blk = t: the columns of U_t);
 *   ranks_right: (lc + 1) x 2^L, row l holds the rank of the right factor of
 *                block (l, t, v) for l = 0..lc (at l = 0, t = 0 and blk = v:
 *                the rows of V_v).
 * Ranks are in 0..4096.  factors (nfactor complex128 entries, interleaved,
 * host memory, copied) holds, each column-major and in this order:
 *   U_t, t ascending:                       |O_t| x rl(L, t)
 *   R of block (l, t, v), l = L-1 .. lc, blk ascending:
 *                (rl(l+1, 2t, v/2) + rl(l+1, 2t+1, v/2)) x rl(l, t, v)
 *   B of block (lc, t, v), blk ascending:  rl(lc, t, v) x rr(lc, t, v)
 *   W of block (l, t, v), l = lc .. 1, blk ascending:
 *                rr(l, t, v) x (rr(l-1, t/2, 2v) + rr(l-1, t/2, 2v+1))
 *   V_v, v ascending:                       rr(0, v) x |S_v|
 * E_INVAL when nfactor differs from the count the ranks imply. */
bfmf_status bfmf_bf_import(int32_t device, int32_t m, int32_t n, int32_t L, const int32_t* ranks_left,
                           const int32_t* ranks_right, const double* factors, int64_t nfactor, bfmf_bf** out);
/* Entries of submatrices K(X_k, Y_k) (extract_BF, Alg. 3) for requests
 * k = 0..nreq-1 with X_k = rows[row_ptr[k] .. row_ptr[k+1]) and Y_k =
 * cols[col_ptr[k] .. col_ptr[k+1]) (host arrays, any order, repeats allowed).
 * out (host, interleaved complex128) receives the blocks one after another,
 * each |X_k| x |Y_k| column-major.  On first use the butterfly is expanded
 * to its centre level (every factor block multiplied once, held by the
 * handle until bfmf_bf_destroy); an entry is then one dot product of its
 * centre block's rank.  E_INVAL for an index outside the matrix. */
bfmf_status bfmf_bf_extract(bfmf_bf* b, int32_t nreq, const int64_t* row_ptr, const int32_t* rows,
                            const int64_t* col_ptr, const int32_t* cols, double* out);
/* levels, largest rank, number of stored complex entries */
bfmf_status bfmf_bf_info(bfmf_bf* b, int32_t* L, int32_t* max_rank, int64_t* entries);
void bfmf_bf_destroy(bfmf_bf* b);

/* ------------------------------------------------------------------ serving
 * Several factored handles stay resident on one device and answer a stream
 * of right-hand-side requests with continuous batching.  Each attached
 * handle gets a worker thread on its own stream and max_batch_rhs column
 * slots; every column of an admitted request takes a slot and runs its own
 * restarted GMRES with the handle's preconditioner (the columns of a slot
 * batch share every launch but not their arithmetic: a request's result is
 * the same bit for bit alone or beside others).  Between two GMRES
 * iterations the worker retires the columns that met the stopping test
 * (solutions go to a result arena until bfmf_server_wait fetches them) and
 * admits queued requests, whole and in arrival order, into the freed slots
 * while their solutions fit the arena; so a request arriving while others
 * are on the device starts at the next iteration.  Models run concurrently.
 * Factors, slot workspaces and the arena are charged against hbm_budget when
 * models are attached (E_NOMEM beyond it).  A handle attached to a server
 * must not be used by the caller afterwards, and must outlive the server.
 * Not for graph capture. */
typedef struct bfmf_server_s* bfmf_server;
typedef struct {
    int32_t max_batch_rhs;   /* column slots per model (default 64); wider requests are refused */
    int32_t reserved0;
    uint64_t hbm_budget;     /* bytes for all models and the arena (0: the device's free memory) */
    uint64_t result_bytes;   /* arena for solutions awaiting bfmf_server_wait (default 4 GiB) */
    bfmf_solve_opts solve;   /* GMRES of every column (default: true_rtol 1e-3; graphs applies) */
} bfmf_server_opts;
typedef struct {
    double t_submit, t_start, t_done;  /* seconds on the server clock: queued, admitted, solution ready */
    int32_t model, nrhs;
    int32_t batch_rhs;                 /* most columns in flight on the model while the request was */
    int32_t batch_requests;            /* most requests in flight on the model while the request was */
    int32_t iters;                     /* GMRES iterations of the request (largest over its columns) */
    int32_t status;                    /* bfmf_status of the request's columns */
    double relres;                     /* largest true relative residual of the request's columns */
} bfmf_request_info;
void bfmf_default_server_opts(bfmf_server_opts* o);
bfmf_status bfmf_server_create(int32_t device, const bfmf_server_opts* o, bfmf_server* out);
/* h: a factored handle on the server's device; model receives its id */
bfmf_status bfmf_server_attach(bfmf_server s, bfmf_handle h, int32_t* model);
/* A request of nrhs columns given as compressed sparse columns: column q has
 * the entries rowind[colptr[q] .. colptr[q+1]) with interleaved complex
 * values (host arrays, copied; duplicates summed).  Never blocks; E_INVAL
 * for bad indices, non-finite values or nrhs > max_batch_rhs. */
bfmf_status bfmf_server_submit(bfmf_server s, int32_t model, int32_t nrhs, const int64_t* colptr,
                               const int64_t* rowind, const double* values, uint64_t* ticket);
/* Blocks until the request is solved; copies its solution (n x nrhs) to X
 * (ld ldx, host or device memory by mem; X == NULL discards it), fills info
 * and releases the request.  Returns the solve's status. */
bfmf_status bfmf_server_wait(bfmf_server s, uint64_t ticket, bfmf_request_info* info, double* X, int64_t ldx,
                             int32_t mem);
double bfmf_server_clock(bfmf_server s);
const char* bfmf_server_last_error(bfmf_server s);
/* stops the workers after the admitted batches; queued requests fail */
void bfmf_server_destroy(bfmf_server s);

/* Number of device allocations (hipMalloc) made by the library in this process
 * so far.  A handle allocates during its first analyze, factor and solve and
 * when later calls need more memory; factoring or solving again with the same
 * sizes and options allocates nothing (a free would synchronize the device). */
int64_t bfmf_device_allocation_count(void);

const char* bfmf_status_str(bfmf_status s);
/* Message of the last failed call on h; with h == NULL, of the last failed
 * call on this thread that returned no handle (bfmf_bf_compress_dense). */
const char* bfmf_last_error(bfmf_handle h);
void bfmf_destroy(bfmf_handle h);

#ifdef __cplusplus
}
#endif
#endif /* BFMF_H */
