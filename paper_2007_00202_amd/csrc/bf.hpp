// Butterfly matrices on the device (paper Sec. 3).
//
// K ~= (U^L R^{L-1} .. R^{lc}) B^{lc} (W^{lc} .. W^1 V^0), lc = floor(L/2),
// over a row tree T_O and a column tree T_S of depth L (complete binary trees
// over contiguous index ranges).  Blocks at level l are indexed
// blk = t * 2^(L-l) + v (t: node at level l of T_O, v: node at level L-l of
// T_S).  Factor storage keeps the two R factors that share a parent column
// node side by side (one matrix per "nu-pair") and the two W factors that share
// a parent row node on top of each other (one matrix per "tau-pair"), so that
// every factor level of a product K x or K^H x is a single grouped GEMM: the
// partial products of sibling blocks are stored stacked and are consumed as
// one operand.
#pragma once
#include <functional>
#include <memory>
#include <vector>

#include "context.hpp"
#include "devtypes.hpp"
#include "kernels/common.hpp"

namespace bfmf {

// ------------------------------------------------------------ device memory
// Growable device buffer addressed by byte offsets (growth copies the content
// and keeps all offsets valid).
struct DevPool {
  DevBuf buf;
  size_t used = 0;
  Budget* budget = nullptr;  // growth charged here when set
  size_t alloc(size_t bytes, hipStream_t s);  // 256-byte aligned byte offset
  char* base() const { return buf.as<char>(); }
  void reset() { used = 0; }
};

// Stack of device temporaries. Chunks are allocated on demand and kept for
// the life of the runtime (freeing device memory synchronizes the device);
// release() rewinds the stack to a mark so the memory is reused.
struct Scratch {
  struct Chunk {
    DevBuf b;
    size_t top = 0;
  };
  std::vector<std::unique_ptr<Chunk>> chunks;
  int cur = -1;  // chunk holding the top of the stack
  size_t chunk_bytes = (size_t)256 << 20;
  Budget* budget = nullptr;  // new chunks charged here when set
  struct Mark {
    int cur;
    size_t top;
  };
  Mark mark() const { return Mark{cur, cur >= 0 ? chunks[cur]->top : 0}; }
  void release(const Mark& m);
  void* take(size_t bytes);
  void clear() {
    chunks.clear();
    cur = -1;
  }
  template <class T>
  T* take_n(size_t n) {
    return (T*)take(n * sizeof(T));
  }
};

// ------------------------------------------------------------------- trees
struct BTree {
  int n = 0, L = 0;
  std::vector<std::vector<int32_t>> b;  // b[l]: 2^l + 1 boundaries
  int beg(int l, int i) const { return b[l][i]; }
  int end(int l, int i) const { return b[l][i + 1]; }
  int size(int l, int i) const { return b[l][i + 1] - b[l][i]; }
};
// Complete tree of depth L over [0, n) following the bisection `nodes`
// (preorder, relative ranges) where it has children, halving (first half
// ceil) elsewhere.
BTree make_tree(int n, int L, const TreeNode* nodes, int nnodes);
int tree_depth(const TreeNode* nodes, int nnodes);

// ------------------------------------------------------------- butterfly
struct Butterfly {
  int m = 0, n = 0, L = 0, lc = 0;
  BTree to, ts;
  std::vector<std::vector<int32_t>> rl, rr;               // ranks (left l in [lc, L], right l in [0, lc])
  std::vector<std::vector<std::vector<int32_t>>> Ob, Sb;  // skeleton positions per level and block
  std::vector<std::vector<int64_t>> offL, offR;           // element offsets in the pool
  std::vector<int64_t> offB;
  int64_t elems = 0;                                       // factor entries
  int nblk() const { return 1 << L; }
  int max_rank() const;
};

// Layout of the per-block partial products of one level: blocks grouped in
// pairs (stacked rows) or alone.
struct VecLayout {
  std::vector<int64_t> grp_off;  // element offset of each group (per rhs block)
  std::vector<int32_t> grp_ld;   // rows of each group
  std::vector<int32_t> grp_of;   // group of each block
  std::vector<int32_t> mem_row;  // row offset of each block in its group
  int64_t rows = 0;              // total rows (elements per rhs column)
};

// One member of a butterfly product: Y(y_off:, :) = alpha op(K) X(x_off:, :) + beta Y
struct BfCall {
  const Butterfly* bf;
  int64_t x_off, y_off;
  double alpha_re, alpha_im;
  int beta;
  // a call with its own input/output: element addresses (address / sizeof element; -1: the plan's
  // shared X / Y), their leading dimensions and its number of columns (0: the plan's)
  int64_t x_abs = -1, y_abs = -1;
  int64_t ldx = 0, ldy = 0;
  int nrhs = 0;
};

// Grouped-GEMM phases of the product of a set of butterflies.
struct BfPlan {
  std::vector<std::vector<GTask>> phase;
  int64_t ws_elems = 0;  // workspace (base 3) in elements of complex<T>
  // right-half-only plans: where each member's level-lc vectors ended up
  std::vector<VecLayout> half_layout;
  std::vector<int64_t> half_off;
};

// adjoint: K^H.  right_half_only: only V and W phases (forward), output left in
// the workspace (used by the randomized construction of the centre blocks).
BfPlan make_plan(const std::vector<BfCall>& calls, bool adjoint, int nrhs, int64_t ldx, int64_t ldy,
                 bool right_half_only = false);

// Runs a plan: bases 0 = factor pool, 1 = X, 2 = Y, 3 = workspace.  lim[i]
// is the number of complex<T> elements addressable from base i; every task's
// operand footprint is checked against it on the host before any launch.
template <class T>
void run_plan(const BfPlan& plan, Context& c, char* pool, const void* X, void* Y, void* ws, hipStream_t s,
              const int64_t lim[4], int kind = K_BF_GEMM);

// Runs a plan with no allocation: every launch in tile shape cfg, the task lists
// copied from host memory to dtasks (at most tasks_cap bytes) and the workspace
// at ws; returns 0 when done (after synchronizing s), else the task-list bytes
// that did not fit (nothing launched).
template <class T>
size_t run_plan_fixed(const BfPlan& plan, char* pool, const void* X, void* Y, void* ws, char* dtasks,
                      size_t tasks_cap, hipStream_t s, const int64_t lim[4], int cfg);

// ------------------------------------------------------------- operators
template <class T>
struct BfRuntime;

// One application of a batch: input X (ld ldx), output Y (ld ldy), nrhs columns.
struct ApplyArg {
  const void* X;
  int64_t ldx;
  void* Y;
  int64_t ldy;
  int nrhs;
};

// Y = alpha op(A) X + beta Y for a linear operator A (m x n), nrhs columns.
template <class T>
struct Op {
  int m = 0, n = 0;
  virtual ~Op() {}
  virtual void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adjoint, double alpha,
                     int beta) = 0;
  // Operators of the same dynamic type and key have the same structure and can be applied together.
  virtual uint64_t key() const { return 0; }
  // ops[i] (all of this dynamic type and key) applied to args[i], independent outputs; the default runs
  // them one after another, the operator types override it with launches shared by the whole batch.
  virtual void apply_many(BfRuntime<T>& rt, const std::vector<Op<T>*>& ops, const std::vector<ApplyArg>& args,
                          bool adjoint, double alpha, int beta) {
    (void)rt;
    for (size_t i = 0; i < ops.size(); ++i)
      ops[i]->apply(args[i].X, args[i].ldx, args[i].Y, args[i].ldy, args[i].nrhs, adjoint, alpha, beta);
  }
};

// Runtime shared by all butterfly work of one factorization.
template <class T>
struct BfRuntime {
  Context* c = nullptr;
  DevPool pool;     // factors of every butterfly and dense leaf
  Scratch scratch;  // temporaries
  uint64_t seed = 0, stream_id = 0;
  int samples = 64;
  int max_samples = 1024;
  int smw_dense = 1024;               // BF_SMW blocks of at most this many rows are inverted densely
  int id_max_cols = 0;                // > 0: blocks wider than this are decomposed as IDs of sub-IDs
  int64_t n_chunked = 0;              // ID blocks decomposed as IDs of sub-IDs
  double tol = 1e-3;
  int max_rank_seen = 0;
  int64_t n_random = 0, n_entry = 0;  // constructions performed
  std::vector<int> sample_hint;       // per log2 size: probes the last randomized construction settled on
  bool batch = true;                  // construct sets of butterflies together (else one at a time)
  hipStream_t s() const { return c->stream; }
  char* pool_base() const { return pool.base(); }
  // single-butterfly product Y = alpha op(K) X + beta Y
  void apply(const Butterfly& bf, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adjoint,
             double alpha, int beta);
  void apply_set(const std::vector<BfCall>& calls, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs,
                 bool adjoint);
  // products of calls that each name their own input and output (x_abs, y_abs, ldx, ldy, nrhs)
  void apply_calls(const std::vector<BfCall>& calls, bool adjoint);
};

// Extraction requests gathered over many blocks (and butterflies, and
// fronts) and served by one launch (two when butterflies are read: the
// butterfly tasks run after the front tasks and may add to their outputs).
struct ExtractBatch {
  std::vector<ExtractTask> tasks;  // rows / cols hold offsets into idx until the launch
  std::vector<BfExtractTask> bf_tasks;
  std::vector<int32_t> idx;
  // out = F(r0 + rows, c0 + cols) of the front fd, or of the dense matrix
  // (ld ldd) when dense is not null; the transpose when trans.
  void add(const FrontDesc* fd, const void* dense, int64_t ldd, const std::vector<int32_t>& rows, int r0,
           const std::vector<int32_t>& cols, int c0, void* out, int64_t ldo, bool trans);
  // out = alpha K(r0 + rows, c0 + cols) of a butterfly in centre form (out += ... when accumulate)
  void add_bf(const BfCentreDev* bf, const std::vector<int32_t>& rows, int r0, const std::vector<int32_t>& cols,
              int c0, void* out, int64_t ldo, bool trans, double alpha, bool accumulate);
};

// ------------------------------------------------------------- centre forms
// Entry extraction from butterflies (Alg. 3): every butterfly of a set is
// expanded to its centre level (E and G of BfCentreDev) by grouped products,
// each factor block multiplied once for all rows and columns, after which an
// entry costs one dot product of its centre block's rank.  Dense square
// blocks of the pool (the leaves of a HOD-BF) are copied beside them.
// Everything goes to `mem` (device memory of at least centre_bytes(spec)
// bytes, kept by the caller while the forms are used): nothing points into
// the factor pool, which moves when it grows.
struct CentreSpec {
  std::vector<const Butterfly*> bfs;
  std::vector<std::pair<int64_t, int>> dense;  // pool element offset and order (ld = order)
};
struct CentreOut {
  const BfCentreDev* bfs = nullptr;  // device array, one descriptor per butterfly
  std::vector<const void*> dense;    // device address of each copied dense block
};
template <class T>
size_t centre_bytes(const CentreSpec& spec);
template <class T>
CentreOut build_centres(BfRuntime<T>& rt, const CentreSpec& spec, char* mem);
// Entries written as complex<TO>; src_single: the dense sources (and the
// contribution blocks) of the batch are complex<float>, else complex<double>.
template <class TO, class T>
void run_extract_to(BfRuntime<T>& rt, ExtractBatch& b, bool src_single);
// front or FP64 dense sources, entries in the runtime's precision
template <class T>
void run_extract(BfRuntime<T>& rt, ExtractBatch& b);

// Source of matrix entries for entry-evaluation construction.
template <class T>
struct EntrySource {
  virtual ~EntrySource() {}
  // queue out(i, j) = K(rows[i], cols[j]) (ld ldo), or the transpose when trans
  virtual void request(ExtractBatch& b, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, void* out,
                       int64_t ldo, bool trans) = 0;
};

// Proxy selection for entry evaluation (Sec. 3.2, Sec. 5.2): for a block with
// the given skeleton/candidate indices, proxies inside node [beg, end).
struct ProxySampler {
  virtual ~ProxySampler() {}
  virtual void columns(const std::vector<int32_t>& rows, int beg, int end, std::vector<int32_t>& out) = 0;
  virtual void rows(const std::vector<int32_t>& cols, int beg, int end, std::vector<int32_t>& out) = 0;
};

// One butterfly K(to, ts) to construct by entry evaluation.
template <class T>
struct EntryJob {
  EntrySource<T>* src;
  ProxySampler* ps;
  BTree to, ts;
  std::unique_ptr<Butterfly> out;
};

// One butterfly to construct from products with the operator op (m x n).
template <class T>
struct RandomJob {
  Op<T>* op = nullptr;
  BTree to, ts;
  std::unique_ptr<Butterfly> out;
  int S = 0;            // probes per tree node of the last attempt
  int max_id_rank = 0;  // largest ID rank of the last attempt
};

// BF_entry_eval (Alg. 2) for a set of butterflies: level k of every
// butterfly is one extraction, one ID and one expansion launch.
template <class T>
void bf_entry_eval_batch(BfRuntime<T>& rt, const std::vector<EntryJob<T>*>& jobs);
template <class T>
std::unique_ptr<Butterfly> bf_entry_eval(BfRuntime<T>& rt, EntrySource<T>& src, ProxySampler& ps, const BTree& to,
                                         const BTree& ts);
// BF_random_matvec (Sec. 3.3): sketches with probes supported on one tree
// node, for a set of butterflies at once (the operator products run one
// after another, the IDs and centre solves of all of them together).
template <class T>
void bf_random_matvec_batch(BfRuntime<T>& rt, const std::vector<RandomJob<T>*>& jobs);
template <class T>
std::unique_ptr<Butterfly> bf_random_matvec(BfRuntime<T>& rt, Op<T>& op, const BTree& to, const BTree& ts);

}  // namespace bfmf
