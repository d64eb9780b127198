// Compressed fronts (paper Alg. 5): HOD-BF F11 and its inverse (Alg. 4 with
// BF_SMW), butterfly F12 / F21 by entry evaluation with graph-distance
// proxies (Alg. 2, Sec. 5.2), the Schur update S by randomized construction
// (Sec. 3.3), the contribution block, and the compressed sweeps.
#include "host_pool.hpp"
#include "compressed.hpp"

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <random>

#include "kernels/kernels.hpp"

namespace bfmf {

namespace {

// copy of a host vector in scratch memory, uploaded through the pinned ring
template <class T, class V>
void* up(BfRuntime<T>& rt, const std::vector<V>& v) {
  void* d = rt.scratch.take(std::max<size_t>(v.size() * sizeof(V), 16));
  rt.c->stage.put(d, v.data(), v.size() * sizeof(V), rt.s());
  return d;
}

// complete tree of depth L over the subtree of node `root` of a preorder list
BTree subtree(const std::vector<TreeNode>& all, int root, int L) {
  const int base = all[root].beg;
  BTree t;
  t.n = all[root].end - base;
  t.L = L;
  struct Cur {
    int b, e, idx;
  };
  std::vector<Cur> cur{{0, t.n, root}};
  for (int l = 0; l <= L; ++l) {
    std::vector<int32_t> bd;
    for (auto& c : cur) bd.push_back(c.b);
    bd.push_back(cur.back().e);
    t.b.push_back(bd);
    if (l == L) break;
    std::vector<Cur> nx;
    for (auto& c : cur) {
      if (c.idx >= 0 && all[c.idx].left >= 0) {
        const int li = all[c.idx].left, ri = all[c.idx].right;
        const int mid = all[li].end - base;
        nx.push_back({c.b, mid, li});
        nx.push_back({mid, c.e, ri});
      } else {
        const int mid = c.b + (c.e - c.b + 1) / 2;
        nx.push_back({c.b, mid, -1});
        nx.push_back({mid, c.e, -1});
      }
    }
    cur.swap(nx);
  }
  return t;
}

int depth_of(const std::vector<TreeNode>& all, int i) {
  if (all[i].left < 0) return 0;
  return 1 + std::max(depth_of(all, all[i].left), depth_of(all, all[i].right));
}

// Entries of the never-formed front: A entries (+) children blocks (Sec. 5,
// list routing: each request is answered from the sparse matrix and from the
// contribution blocks of the children through the extend-add maps).
template <class T>
struct FrontSource : EntrySource<T> {
  const FrontDesc* d_fd;
  int row0, col0;
  FrontSource(const FrontDesc* fd, int r0, int c0) : d_fd(fd), row0(r0), col0(c0) {}
  void request(ExtractBatch& b, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, void* out,
               int64_t ldo, bool trans) override {
    b.add(d_fd, nullptr, 0, rows, row0, cols, col0, out, ldo, trans);
  }
};

// Entries of a contribution block C = (C_nu1 (+) C_nu2)(Iu, Iu) - S that is
// never formed (Alg. 5, last step): the children's part by list routing from
// the front (rows and columns offset by ns), then S by extract_BF of its
// centre form, subtracted in place.  row0 / col0: first I^u-local row and
// column of the block being built.
template <class T>
struct CbSource : EntrySource<T> {
  const FrontDesc* d_fd;
  int ns, row0, col0;
  const BfCentreDev* s;
  CbSource(const FrontDesc* fd, int ns_, int r0, int c0, const BfCentreDev* s_)
      : d_fd(fd), ns(ns_), row0(r0), col0(c0), s(s_) {}
  void request(ExtractBatch& b, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, void* out,
               int64_t ldo, bool trans) override {
    b.add(d_fd, nullptr, 0, rows, ns + row0, cols, ns + col0, out, ldo, trans);
    b.add_bf(s, rows, row0, cols, col0, out, ldo, trans, -1.0, true);
  }
};

// Proxies: alpha |given| uniform samples plus, for every given index, its
// k_nn nearest vertices (breadth-first search in the front's graph, layer by
// layer, ascending index inside a layer) that fall into the node (Sec. 5.2).
struct BfsSampler : ProxySampler {
  const std::vector<std::vector<int32_t>>& near;  // per front-local vertex
  int row0, col0, knn;
  double alpha;
  std::mt19937_64 g;
  BfsSampler(const std::vector<std::vector<int32_t>>& nr, int r0, int c0, int k, double a, uint64_t seed)
      : near(nr), row0(r0), col0(c0), knn(k), alpha(a), g(seed) {}
  void pick(const std::vector<int32_t>& given, int given0, int beg, int end, int node0, std::vector<int32_t>& out) {
    HostTimer ht(HP_SAMPLE);
    out.clear();
    const int n = end - beg;
    if (n <= 0) return;
    const int cap = 2048;
    const int k = std::min(n, std::max(8, (int)(alpha * (double)given.size())));
    // membership marks in a buffer kept between calls (cleared entry by entry afterwards)
    static thread_local std::vector<char> mark;
    if ((int)mark.size() < n) mark.assign(n, 0);
    int cnt = 0;
    // nearest neighbours first
    for (int32_t gi : given) {
      int found = 0;
      for (int32_t v : near[given0 + gi]) {
        const int p = v - node0;
        if (p >= beg && p < end) {
          if (!mark[p - beg] && cnt < cap) {
            mark[p - beg] = 1;
            out.push_back(p);
            ++cnt;
          }
          if (++found >= knn) break;
        }
      }
    }
    // uniform samples
    for (int i = 0; i < k && cnt < std::min(cap, n); ++i) {
      std::uniform_int_distribution<int> d(0, n - 1);
      const int p = d(g);
      if (!mark[p]) {
        mark[p] = 1;
        out.push_back(beg + p);
        ++cnt;
      }
    }
    for (int32_t v : out) mark[v - beg] = 0;
    std::sort(out.begin(), out.end());  // ascending, as the proxy lists are used
  }
  void columns(const std::vector<int32_t>& rows, int beg, int end, std::vector<int32_t>& out) override {
    pick(rows, row0, beg, end, col0, out);
  }
  void rows(const std::vector<int32_t>& cols, int beg, int end, std::vector<int32_t>& out) override {
    pick(cols, col0, beg, end, row0, out);
  }
};

// (I + X) as an operator (X butterfly, dense block, or zero)
template <class T>
struct IPlusX : Op<T> {
  BfRuntime<T>& rt;
  const Butterfly* bf;
  int64_t dense_off;  // element offset in the pool, or -1
  IPlusX(BfRuntime<T>& r, int n_, const Butterfly* b, int64_t doff) : rt(r), bf(b), dense_off(doff) {
    this->m = this->n = n_;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    const int n = this->n;
    if (bf) {
      rt.apply(*bf, X, ldx, Y, ldy, nrhs, adj, alpha, beta);
    } else if (dense_off >= 0) {
      const char* A = rt.pool_base() + dense_off * sizeof(cplx<T>);
      gemm<T>(rt, A, n, adj ? OP_C : OP_N, X, ldx, OP_N, Y, ldy, n, nrhs, n, alpha, 0, beta);
    } else {
      axpby<T>(rt, Y, ldy, X, ldx, n, nrhs, alpha, beta ? 1.0 : 0.0);
      return;
    }
    axpby<T>(rt, Y, ldy, X, ldx, n, nrhs, alpha, 1.0);
  }
  uint64_t key() const override { return bf ? 0 : (dense_off >= 0 ? 1 : 2); }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& all, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    std::vector<AxpbyTask> id;
    for (size_t q = 0; q < all.size(); ++q)
      id.push_back(axt(args[q].Y, args[q].ldy, args[q].X, args[q].ldx, all[q]->n, args[q].nrhs));
    if (bf) {  // Y = alpha K X + beta Y for every item, then Y += alpha X
      std::vector<BfCall> calls;
      for (size_t q = 0; q < all.size(); ++q) {
        BfCall c{static_cast<IPlusX<T>*>(all[q])->bf, 0, 0, alpha, 0.0, beta};
        c.x_abs = eaddr<T>(args[q].X);
        c.y_abs = eaddr<T>(args[q].Y);
        c.ldx = args[q].ldx;
        c.ldy = args[q].ldy;
        c.nrhs = args[q].nrhs;
        calls.push_back(c);
      }
      r.apply_calls(calls, adj);
      axpby_many<T>(r, id, alpha, 1.0);
    } else if (dense_off >= 0) {
      std::vector<GTask> ph;
      for (size_t q = 0; q < all.size(); ++q) {
        auto* o = static_cast<IPlusX<T>*>(all[q]);
        const int n = o->n;
        GTask t = {};
        t.a_off = o->dense_off;
        t.lda = std::max(n, 1);
        t.opA = (int8_t)(adj ? OP_C : OP_N);
        t.abase = 0;
        t.b_off = eaddr<T>(args[q].X);
        t.ldb = std::max<int64_t>(args[q].ldx, 1);
        t.bbase = 4;
        t.c_off = eaddr<T>(args[q].Y);
        t.ldc = std::max<int64_t>(args[q].ldy, 1);
        t.cbase = 4;
        t.M = n;
        t.N = args[q].nrhs;
        t.K = n;
        t.alpha_re = alpha;
        t.beta = (int8_t)beta;
        if (n > 0) ph.push_back(t);
      }
      if (!ph.empty()) {
        BfPlan p;
        p.phase.push_back(ph);
        const int64_t lim[4] = {(int64_t)(r.pool.used / sizeof(cplx<T>)), 0, 0, 0};
        run_plan<T>(p, *r.c, r.pool_base(), nullptr, nullptr, nullptr, r.s(), lim);
      }
      axpby_many<T>(r, id, alpha, 1.0);
    } else {
      axpby_many<T>(r, id, alpha, beta ? 1.0 : 0.0);
    }
  }
};

// A^-1 - I for A = [I + K11, K12; K21, I + K22] from the factored form
// [I 0; -A22i K21 I] diag(A11i, A22i) [I -K12 A22i; 0 I] (Alg. 4, BF_SMW)
template <class T>
struct SmwOp : Op<T> {
  BfRuntime<T>& rt;
  int n1, n2;
  Op<T>*K12, *K21, *A11i, *A22i;
  SmwOp(BfRuntime<T>& r, int a, int b, Op<T>* k12, Op<T>* k21, Op<T>* a11i, Op<T>* a22i)
      : rt(r), n1(a), n2(b), K12(k12), K21(k21), A11i(a11i), A22i(a22i) {
    this->m = this->n = a + b;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    auto mk = rt.scratch.mark();
    const cplx<T>* x = (const cplx<T>*)X;
    cplx<T>* y = (cplx<T>*)Y;
    const int nn = n1 + n2;
    cplx<T>* w = (cplx<T>*)rt.scratch.take((size_t)nn * nrhs * sizeof(cplx<T>));
    cplx<T>* t = (cplx<T>*)rt.scratch.take((size_t)std::max(n1, n2) * nrhs * sizeof(cplx<T>));
    cplx<T>* w1 = w;
    cplx<T>* w2 = w + n1;
    if (!adj) {
      A22i->apply(x + n1, ldx, w2, nn, nrhs, false, 1.0, 0);    // u2 = A22i x2
      K12->apply(w2, nn, t, n1, nrhs, false, 1.0, 0);           // t = K12 u2
      axpby<T>(rt, t, n1, x, ldx, n1, nrhs, 1.0, -1.0);         // t = x1 - K12 u2
      A11i->apply(t, n1, w1, nn, nrhs, false, 1.0, 0);          // w1 = A11i (x1 - K12 u2)
      K21->apply(w1, nn, t, n2, nrhs, false, 1.0, 0);           // t = K21 w1
      A22i->apply(t, n2, w2, nn, nrhs, false, -1.0, 1);         // w2 = u2 - A22i K21 w1
    } else {
      A22i->apply(x + n1, ldx, w2, nn, nrhs, true, 1.0, 0);     // s = A22i^H x2
      K21->apply(w2, nn, t, n1, nrhs, true, 1.0, 0);            // t = K21^H s
      axpby<T>(rt, t, n1, x, ldx, n1, nrhs, 1.0, -1.0);         // t = x1 - K21^H A22i^H x2
      A11i->apply(t, n1, w1, nn, nrhs, true, 1.0, 0);           // w1 = A11i^H t
      K12->apply(w1, nn, t, n2, nrhs, true, 1.0, 0);            // t = K12^H w1
      A22i->apply(x + n1, ldx, w2, nn, nrhs, true, 1.0, 0);     // w2 = A22i^H x2
      A22i->apply(t, n2, w2, nn, nrhs, true, -1.0, 1);          // w2 -= A22i^H K12^H w1
    }
    axpby<T>(rt, w, nn, X, ldx, nn, nrhs, -1.0, 1.0);            // minus the identity
    axpby<T>(rt, Y, ldy, w, nn, nn, nrhs, alpha, beta ? 1.0 : 0.0);
    (void)y;
    rt.scratch.release(mk);
  }
  // the same sequence with each step applied to every item at once
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& all, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    auto mk = r.scratch.mark();
    const size_t nq = all.size();
    std::vector<SmwOp<T>*> o(nq);
    std::vector<cplx<T>*> w(nq), t(nq);
    for (size_t q = 0; q < nq; ++q) {
      o[q] = static_cast<SmwOp<T>*>(all[q]);
      const int nn = o[q]->n1 + o[q]->n2;
      w[q] = (cplx<T>*)r.scratch.take((size_t)nn * args[q].nrhs * sizeof(cplx<T>));
      t[q] = (cplx<T>*)r.scratch.take((size_t)std::max(o[q]->n1, o[q]->n2) * args[q].nrhs * sizeof(cplx<T>));
    }
    auto X = [&](size_t q) { return (const cplx<T>*)args[q].X; };
    auto nn = [&](size_t q) { return (int64_t)(o[q]->n1 + o[q]->n2); };
    // step(op selector, input, input ld, output, output ld, alpha, beta)
    auto step = [&](auto pick, auto in, auto ldi, auto out, auto ldo, double a, int b) {
      std::vector<Op<T>*> ops;
      std::vector<ApplyArg> aa;
      for (size_t q = 0; q < nq; ++q) {
        ops.push_back(pick(q));
        aa.push_back(ApplyArg{in(q), ldi(q), out(q), ldo(q), args[q].nrhs});
      }
      apply_all<T>(r, ops, aa, adj, a, b);
    };
    auto ax = [&](auto y, auto ldy, auto x, auto ldx, auto m, double a, double b) {
      std::vector<AxpbyTask> tk;
      for (size_t q = 0; q < nq; ++q) tk.push_back(axt(y(q), ldy(q), x(q), ldx(q), m(q), args[q].nrhs));
      axpby_many<T>(r, tk, a, b);
    };
    auto n1 = [&](size_t q) { return (int64_t)o[q]->n1; };
    auto n2 = [&](size_t q) { return (int64_t)o[q]->n2; };
    auto w1 = [&](size_t q) { return w[q]; };
    auto w2 = [&](size_t q) { return w[q] + o[q]->n1; };
    auto tt = [&](size_t q) { return t[q]; };
    auto x1 = [&](size_t q) { return X(q); };
    auto x2 = [&](size_t q) { return X(q) + o[q]->n1; };
    auto ldx = [&](size_t q) { return args[q].ldx; };
    auto A11i = [&](size_t q) { return o[q]->A11i; };
    auto A22i = [&](size_t q) { return o[q]->A22i; };
    auto K12 = [&](size_t q) { return o[q]->K12; };
    auto K21 = [&](size_t q) { return o[q]->K21; };
    if (!adj) {
      step(A22i, x2, ldx, w2, nn, 1.0, 0);  // u2 = A22i x2
      step(K12, w2, nn, tt, n1, 1.0, 0);    // t = K12 u2
      ax(tt, n1, x1, ldx, n1, 1.0, -1.0);   // t = x1 - K12 u2
      step(A11i, tt, n1, w1, nn, 1.0, 0);   // w1 = A11i t
      step(K21, w1, nn, tt, n2, 1.0, 0);    // t = K21 w1
      step(A22i, tt, n2, w2, nn, -1.0, 1);  // w2 = u2 - A22i K21 w1
    } else {
      step(A22i, x2, ldx, w2, nn, 1.0, 0);  // s = A22i^H x2
      step(K21, w2, nn, tt, n1, 1.0, 0);    // t = K21^H s
      ax(tt, n1, x1, ldx, n1, 1.0, -1.0);   // t = x1 - K21^H A22i^H x2
      step(A11i, tt, n1, w1, nn, 1.0, 0);   // w1 = A11i^H t
      step(K12, w1, nn, tt, n2, 1.0, 0);    // t = K12^H w1
      step(A22i, x2, ldx, w2, nn, 1.0, 0);  // w2 = A22i^H x2
      step(A22i, tt, n2, w2, nn, -1.0, 1);  // w2 -= A22i^H K12^H w1
    }
    auto wall = [&](size_t q) { return w[q]; };
    auto xall = [&](size_t q) { return X(q); };
    ax(wall, nn, xall, ldx, nn, -1.0, 1.0);  // minus the identity
    auto yall = [&](size_t q) { return (cplx<T>*)args[q].Y; };
    auto ldy = [&](size_t q) { return args[q].ldy; };
    auto wconst = [&](size_t q) { return (const cplx<T>*)w[q]; };
    ax(yall, ldy, wconst, nn, nn, alpha, beta ? 1.0 : 0.0);
    r.scratch.release(mk);
  }
};

// y = D_node^-1 x as an operator on the rows of `node`
template <class T>
struct HodbfInvOp : Op<T> {
  BfRuntime<T>& rt;
  const Hodbf<T>& h;
  int node;
  HodbfInvOp(BfRuntime<T>& r, const Hodbf<T>& hh, int nd) : rt(r), h(hh), node(nd) {
    this->m = this->n = hh.nodes[nd].size();
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    if (alpha == 1.0 && !beta) {
      hodbf_inv_apply<T>(rt, h, node, X, ldx, Y, ldy, nrhs, adj);
      return;
    }
    auto mk = rt.scratch.mark();
    const int n = this->n;
    void* t = rt.scratch.take((size_t)std::max(n, 1) * nrhs * sizeof(cplx<T>));
    hodbf_inv_apply<T>(rt, h, node, X, ldx, t, n, nrhs, adj);
    axpby<T>(rt, Y, ldy, t, n, n, nrhs, alpha, beta ? 1.0 : 0.0);
    rt.scratch.release(mk);
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& all, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    auto mk = r.scratch.mark();
    std::vector<HodbfInvItem<T>> items;
    std::vector<AxpbyTask> fin;
    const bool direct = alpha == 1.0 && !beta;
    for (size_t q = 0; q < all.size(); ++q) {
      auto* o = static_cast<HodbfInvOp<T>*>(all[q]);
      HodbfInvItem<T> it{&o->h, o->node, args[q].X, args[q].ldx, args[q].Y, args[q].ldy, args[q].nrhs};
      if (!direct) {
        const int n = o->n;
        it.Y = r.scratch.take((size_t)std::max(n, 1) * args[q].nrhs * sizeof(cplx<T>));
        it.ldy = std::max(n, 1);
        fin.push_back(axt(args[q].Y, args[q].ldy, it.Y, it.ldy, n, args[q].nrhs));
      }
      items.push_back(it);
    }
    hodbf_inv_apply_many<T>(r, items, adj);
    if (!direct) axpby_many<T>(r, fin, alpha, beta ? 1.0 : 0.0);
    r.scratch.release(mk);
  }
};

struct SmwResult {
  std::unique_ptr<Butterfly> bf;
  int64_t dense_off = -1;
  bool zero = false;
};

}  // namespace

// ------------------------------------------------------------ HOD-BF products
namespace {

// One grouped GEMM over dense diagonal blocks stored in the pool:
// Y(r, :) = op(D_i) X(r, :) (+ Y(r, :) when accumulate) for the row ranges r
// of the blocks; X and Y must not overlap.
template <class T>
void dense_blocks(BfRuntime<T>& rt, const std::vector<std::pair<int64_t, std::pair<int, int>>>& blocks, bool adjoint,
                  const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool accumulate) {
  if (blocks.empty() || nrhs <= 0) return;
  std::vector<GTask> ph;
  int64_t rows = 0;
  for (auto& b : blocks) {
    const int64_t off = b.first;
    const int r0 = b.second.first, n = b.second.second;
    if (n <= 0) continue;
    GTask t = {};
    t.a_off = off;
    t.lda = n;
    t.opA = (int8_t)(adjoint ? OP_C : OP_N);
    t.abase = 0;
    t.b_off = r0;
    t.ldb = ldx;
    t.opB = OP_N;
    t.bbase = 1;
    t.c_off = r0;
    t.ldc = ldy;
    t.cbase = 2;
    t.M = n;
    t.N = nrhs;
    t.K = n;
    t.alpha_re = 1;
    t.beta = (int8_t)(accumulate ? 1 : 0);
    ph.push_back(t);
    rows = std::max<int64_t>(rows, (int64_t)r0 + n);
  }
  if (ph.empty()) return;
  BfPlan p;
  p.phase.push_back(ph);
  const int64_t lim[4] = {(int64_t)(rt.pool.used / sizeof(cplx<T>)), ldx * nrhs, ldy * nrhs, 0};
  if (rows > ldx || rows > ldy) throw Error(BFMF_E_INVAL, "internal: dense block rows beyond the leading dimension");
  run_plan<T>(p, *rt.c, rt.pool_base(), X, Y, nullptr, rt.s(), lim);
}

}  // namespace

template <class T>
void hodbf_apply(BfRuntime<T>& rt, const Hodbf<T>& h, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs) {
  // leaves: y = D x, one grouped GEMM
  std::vector<std::pair<int64_t, std::pair<int, int>>> lb;
  for (const auto& nd : h.nodes)
    if (nd.left < 0) lb.push_back({nd.leaf_off, {nd.beg, nd.size()}});
  dense_blocks<T>(rt, lb, false, X, ldx, Y, ldy, nrhs, false);
  for (int l = h.max_level; l >= 0; --l) {
    std::vector<BfCall> calls;
    for (int i : h.by_level[l]) {
      const auto& nd = h.nodes[i];
      if (nd.left < 0) continue;
      const auto& a = h.nodes[nd.left];
      const auto& b = h.nodes[nd.right];
      calls.push_back(BfCall{nd.b12.get(), b.beg, a.beg, 1.0, 0.0, 1});
      calls.push_back(BfCall{nd.b21.get(), a.beg, b.beg, 1.0, 0.0, 1});
    }
    if (!calls.empty()) rt.apply_set(calls, X, ldx, Y, ldy, nrhs, false);
  }
}

// y = D_node^-1 x (or D_node^-H x) with D^-1 = (I + X_t) diag(D1^-1, D2^-1)
// per internal node t (Alg. 4), for several (tree, node, x, y) at once: the
// leaf inverses of all items in one grouped GEMM, then level by level (the
// absolute level in each tree) the butterfly X_t of every item in place
// (y_t += X_t y_t) and the dense X_t through a copy.  x and y of an item must
// not overlap; different items are independent.
template <class T>
void hodbf_inv_apply_many(BfRuntime<T>& rt, const std::vector<HodbfInvItem<T>>& items, bool adjoint) {
  if (items.empty()) return;
  const size_t nq = items.size();
  struct Sub {
    std::vector<std::vector<int>> lv;
    int base = 0, n = 0, root_level = 0, max_level = -1;
    cplx<T>* tmp = nullptr;
  };
  std::vector<Sub> sub(nq);
  int lo = 1 << 30, hi = -1;
  for (size_t q = 0; q < nq; ++q) {
    const Hodbf<T>& h = *items[q].h;
    const HodbfNode<T>& root = h.nodes[items[q].node];
    Sub& u = sub[q];
    u.base = root.beg;
    u.n = root.size();
    u.root_level = root.level;
    u.lv.assign(h.max_level + 1, {});
    std::vector<int> st{items[q].node};
    while (!st.empty()) {
      const int i = st.back();
      st.pop_back();
      u.lv[h.nodes[i].level].push_back(i);
      u.max_level = std::max(u.max_level, h.nodes[i].level);
      if (h.nodes[i].left >= 0) {
        st.push_back(h.nodes[i].left);
        st.push_back(h.nodes[i].right);
      }
    }
    lo = std::min(lo, u.root_level);
    hi = std::max(hi, u.max_level);
  }
  auto mk = rt.scratch.mark();
  auto tmp_of = [&](size_t q) {
    if (!sub[q].tmp)
      sub[q].tmp = (cplx<T>*)rt.scratch.take((size_t)std::max(sub[q].n, 1) * items[q].nrhs * sizeof(cplx<T>));
    return sub[q].tmp;
  };
  // dense blocks D (pool offset, rows r0..r0+nb of the item): Y = op(D) S (+ Y)
  struct DenseBlock {
    size_t q;
    int64_t off;
    int r0, nb;
  };
  auto run_dense = [&](const std::vector<DenseBlock>& bl, bool from_tmp, bool accumulate) {
    std::vector<GTask> ph;
    for (auto& b : bl) {
      if (b.nb <= 0) continue;
      const HodbfInvItem<T>& it = items[b.q];
      GTask t = {};
      t.a_off = b.off;
      t.lda = b.nb;
      t.opA = (int8_t)(adjoint ? OP_C : OP_N);
      t.abase = 0;
      t.b_off = from_tmp ? eaddr<T>(sub[b.q].tmp) + b.r0 : eaddr<T>(it.X) + b.r0;
      t.ldb = from_tmp ? std::max(sub[b.q].n, 1) : it.ldx;
      t.bbase = 4;
      t.c_off = eaddr<T>(it.Y) + b.r0;
      t.ldc = it.ldy;
      t.cbase = 4;
      t.M = b.nb;
      t.N = it.nrhs;
      t.K = b.nb;
      t.alpha_re = 1;
      t.beta = (int8_t)(accumulate ? 1 : 0);
      ph.push_back(t);
    }
    if (ph.empty()) return;
    BfPlan p;
    p.phase.push_back(ph);
    const int64_t lim[4] = {(int64_t)(rt.pool.used / sizeof(cplx<T>)), 0, 0, 0};
    run_plan<T>(p, *rt.c, rt.pool_base(), nullptr, nullptr, nullptr, rt.s(), lim);
  };
  std::vector<DenseBlock> leaves;
  for (size_t q = 0; q < nq; ++q)
    for (auto& lvl : sub[q].lv)
      for (int i : lvl) {
        const auto& nd = items[q].h->nodes[i];
        if (nd.left < 0) leaves.push_back(DenseBlock{q, nd.inv_off, nd.beg - sub[q].base, nd.size()});
      }
  auto copy_all = [&](const std::vector<size_t>& qs, bool x_to_y) {  // y = x, or tmp = y
    std::vector<AxpbyTask> tk;
    for (size_t q : qs) {
      const HodbfInvItem<T>& it = items[q];
      if (x_to_y)
        tk.push_back(axt(it.Y, it.ldy, it.X, it.ldx, sub[q].n, it.nrhs));
      else
        tk.push_back(axt(tmp_of(q), std::max(sub[q].n, 1), it.Y, it.ldy, sub[q].n, it.nrhs));
    }
    axpby_many<T>(rt, tk, 1.0, 0.0);
  };
  auto level_update = [&](int l) {  // y_t += X_t^(H) y_t for the internal nodes of level l of every item
    std::vector<BfCall> calls;
    std::vector<DenseBlock> dense;
    std::vector<size_t> need_copy;
    for (size_t q = 0; q < nq; ++q) {
      if (l < sub[q].root_level || l > sub[q].max_level) continue;
      const HodbfInvItem<T>& it = items[q];
      bool copied = false;
      for (int i : sub[q].lv[l]) {
        const auto& nd = it.h->nodes[i];
        if (nd.left < 0 || nd.x_zero) continue;
        const int r0 = nd.beg - sub[q].base;
        if (nd.x_dense) {
          if (!copied) need_copy.push_back(q);
          copied = true;
          dense.push_back(DenseBlock{q, nd.inv_off, r0, nd.size()});
        } else {
          // in place: the first phase of a product reads y before its last phase writes it
          BfCall c{nd.x.get(), r0, r0, 1.0, 0.0, 1};
          c.x_abs = c.y_abs = eaddr<T>(it.Y);
          c.ldx = c.ldy = it.ldy;
          c.nrhs = it.nrhs;
          calls.push_back(c);
        }
      }
    }
    if (!dense.empty()) {
      copy_all(need_copy, false);
      run_dense(dense, true, true);
    }
    rt.apply_calls(calls, adjoint);
  };
  std::vector<size_t> all(nq);
  for (size_t q = 0; q < nq; ++q) all[q] = q;
  if (!adjoint) {
    run_dense(leaves, false, false);
    for (int l = hi; l >= lo; --l) level_update(l);
  } else {
    copy_all(all, true);
    for (int l = lo; l <= hi; ++l) level_update(l);
    copy_all(all, false);
    run_dense(leaves, true, false);
  }
  rt.scratch.release(mk);
}

template <class T>
void hodbf_inv_apply(BfRuntime<T>& rt, const Hodbf<T>& h, int node, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     int nrhs, bool adjoint) {
  hodbf_inv_apply_many<T>(rt, {HodbfInvItem<T>{&h, node, X, ldx, Y, ldy, nrhs}}, adjoint);
}

template void hodbf_apply<double>(BfRuntime<double>&, const Hodbf<double>&, const void*, int64_t, void*, int64_t, int);
template void hodbf_inv_apply<double>(BfRuntime<double>&, const Hodbf<double>&, int, const void*, int64_t, void*,
                                      int64_t, int, bool);
template void hodbf_apply<float>(BfRuntime<float>&, const Hodbf<float>&, const void*, int64_t, void*, int64_t, int);
template void hodbf_inv_apply<float>(BfRuntime<float>&, const Hodbf<float>&, int, const void*, int64_t, void*,
                                     int64_t, int, bool);
template void hodbf_inv_apply_many<double>(BfRuntime<double>&, const std::vector<HodbfInvItem<double>>&, bool);
template void hodbf_inv_apply_many<float>(BfRuntime<float>&, const std::vector<HodbfInvItem<float>>&, bool);

// ------------------------------------------------------------ BF_SMW
namespace {

template <class T>
struct SmwJob {
  const std::vector<TreeNode>* nodes = nullptr;
  int node = 0;
  Op<T>*K11 = nullptr, *K12 = nullptr, *K21 = nullptr, *K22 = nullptr;  // null blocks are zero
  Op<T>* Kfull = nullptr;
  SmwResult res;
};

// Dense base case for a set of blocks: M = I + K, X = M^-1 - I, where M^-1 is
// the Schur complement of the bordered front [M I; -I 0] (partial LU with
// pivoting inside M, the same kernels as the dense fronts, all blocks in one
// batched launch sequence).
template <class T>
void smw_dense_batch(BfRuntime<T>& rt, const std::vector<SmwJob<T>*>& jobs, int* d_status) {
  if (jobs.empty()) return;
  hipStream_t s = rt.s();
  auto mk = rt.scratch.mark();
  const size_t nj = jobs.size();
  std::vector<int> hn(nj), hns(nj);
  std::vector<int64_t> eoff(nj);
  for (size_t i = 0; i < nj; ++i) {  // every pool allocation first (the pool may move)
    const TreeNode& nd = (*jobs[i]->nodes)[jobs[i]->node];
    hns[i] = nd.end - nd.beg;
    hn[i] = 2 * hns[i];
    eoff[i] = (int64_t)(rt.pool.alloc((size_t)hns[i] * hns[i] * sizeof(cplx<T>), s) / sizeof(cplx<T>));
  }
  std::vector<FrontDesc> fds(nj);
  std::vector<cplx<double>*> Fs(nj);  // the bordered fronts, factored in FP64
  std::vector<cplx<T>*> Fw(nj);        // the same in the working precision, before the LU
  std::vector<AxpbyTask> border(nj), widen, finish(nj);
  std::vector<Op<T>*> kops(nj);
  std::vector<ApplyArg> kargs(nj);
  int64_t maxn = 0;
  for (size_t i = 0; i < nj; ++i) {
    const int n = hns[i], N2 = hn[i];
    maxn = std::max<int64_t>(maxn, n);
    cplx<T>* F = (cplx<T>*)rt.scratch.take((size_t)N2 * N2 * sizeof(cplx<T>));
    cplx<T>* I = (cplx<T>*)rt.scratch.take((size_t)n * n * sizeof(cplx<T>));
    int32_t* piv = (int32_t*)rt.scratch.take((size_t)n * sizeof(int32_t));
    border[i] = AxpbyTask{F, I, N2, n, n, n, 0};  // F = [I I; -I 0], I = identity
    kops[i] = jobs[i]->Kfull;
    kargs[i] = ApplyArg{I, n, F, N2, n};  // F11 += K
    cplx<double>* F64 = (cplx<double>*)F;
    if (sizeof(T) != 8) {  // pivot blocks in FP64
      F64 = (cplx<double>*)rt.scratch.take((size_t)N2 * N2 * sizeof(cplx<double>));
      widen.push_back(AxpbyTask{F64, F, N2, N2, N2, N2, 0});
    }
    FrontDesc& fd = fds[i];
    std::memset(&fd, 0, sizeof(fd));
    fd.F = F64;
    fd.n = N2;
    fd.ns = n;
    fd.front = -1;
    fd.f21_unit = 1;  // the bordered front [M I; -I 0]
    fd.piv = piv;
    Fs[i] = F64;
    Fw[i] = F;
  }
  ochk(launch_smw_border<T>((const AxpbyTask*)up(rt, border), (int)nj, maxn, s), "border");
  apply_all<T>(rt, kops, kargs, false, 1.0, 1);
  if (!widen.empty())
    ochk(launch_mix_batch<double, T>((const AxpbyTask*)up(rt, widen), (int)widen.size(), 4 * maxn * maxn, 1.0, 0.0,
                                     0.0, s),
         "border to FP64");
  const FrontDesc* d_fd = (const FrontDesc*)up(rt, fds);
  ochk(launch_partial_lu<double>(d_fd, (int)nj, hn.data(), hns.data(), d_status, s), "smw dense lu");
  ochk(launch_schur<double>(d_fd, (int)nj, hn.data(), hns.data(), s), "smw dense schur");
  for (size_t i = 0; i < nj; ++i) {
    const int n = hns[i], N2 = hn[i];
    cplx<T>* X = (cplx<T>*)(rt.pool_base() + eoff[i] * sizeof(cplx<T>));
    finish[i] = AxpbyTask{X, Fs[i] + n + (size_t)n * N2, n, N2, n, n, 0};  // X = M^-1 - I
    jobs[i]->res.dense_off = eoff[i];
  }
  ochk(launch_mix_batch<T, double>((const AxpbyTask*)up(rt, finish), (int)nj, maxn * maxn, 1.0, 0.0, -1.0, s),
       "M^-1 - I");
  rt.scratch.release(mk);
}

// BF_SMW (Alg. 4) for a set of nodes: X with (I + K)^-1 = I + X, K given by
// its 2 x 2 blocks over the node's children.  Every stage of the recursion
// (X22 of all nodes, then the S11 constructions, then X11, then X) is one
// batch.
template <class T>
void smw_batch(BfRuntime<T>& rt, const std::vector<SmwJob<T>*>& jobs, int* d_status) {
  if (jobs.empty()) return;
  if (!rt.batch && jobs.size() > 1) {
    for (auto* j : jobs) smw_batch<T>(rt, {j}, d_status);
    return;
  }
  std::vector<SmwJob<T>*> dense, rec;
  for (auto* j : jobs) {
    const TreeNode& nd = (*j->nodes)[j->node];
    const bool base = depth_of(*j->nodes, j->node) == 0 || nd.end - nd.beg <= rt.smw_dense;
    (base ? dense : rec).push_back(j);
  }
  smw_dense_batch<T>(rt, dense, d_status);
  if (rec.empty()) return;
  struct Rec {
    int c1 = -1, c2 = -1, n1 = 0, n2 = 0, d = 0;
    std::vector<std::unique_ptr<Op<T>>> keep;
    SmwJob<T> sub22, sub11;
    std::unique_ptr<IPlusX<T>> A22i, A11i;
    std::unique_ptr<ProductOp<T>> a22k21, k12a22k21;
    std::unique_ptr<SumOp<T>> s11op;
    std::unique_ptr<BfOp<T>> s11b;
    std::unique_ptr<SmwOp<T>> aop;
    RandomJob<T> s11job, xjob;
    Op<T>* view(BfRuntime<T>& r, Op<T>* op, int r0, int c0, int m, int n) {
      keep.push_back(std::make_unique<SubOp<T>>(r, op, r0, c0, m, n));
      return keep.back().get();
    }
  };
  std::vector<std::unique_ptr<Rec>> R;
  // children blocks of a general operator come from views of it
  auto split = [&](Rec& r, SmwJob<T>& sub, Op<T>* K, int child) {
    const auto& nodes = *sub.nodes;
    sub.node = child;
    sub.Kfull = K;
    const int cl = nodes[child].left;
    if (cl >= 0) {
      const int n = nodes[child].end - nodes[child].beg;
      const int m1 = nodes[cl].end - nodes[cl].beg, m2 = n - m1;
      sub.K11 = r.view(rt, K, 0, 0, m1, m1);
      sub.K12 = r.view(rt, K, 0, m1, m1, m2);
      sub.K21 = r.view(rt, K, m1, 0, m2, m1);
      sub.K22 = r.view(rt, K, m1, m1, m2, m2);
    }
  };
  // X22: (I + K22)^-1 = I + X22
  std::vector<SmwJob<T>*> sub;
  for (auto* j : rec) {
    auto r = std::make_unique<Rec>();
    const auto& nodes = *j->nodes;
    const TreeNode& nd = nodes[j->node];
    r->c1 = nd.left;
    r->c2 = nd.right;
    r->n1 = nodes[r->c1].end - nodes[r->c1].beg;
    r->n2 = (nd.end - nd.beg) - r->n1;
    r->d = depth_of(nodes, j->node);
    r->sub22.nodes = r->sub11.nodes = j->nodes;
    if (j->K22) {
      split(*r, r->sub22, j->K22, r->c2);
      sub.push_back(&r->sub22);
    } else {
      r->sub22.res.zero = true;
    }
    R.push_back(std::move(r));
  }
  smw_batch<T>(rt, sub, d_status);
  // S11 = K11 - K12 A22i K21 over T1 x T1: children butterflies of L - 2 levels
  std::vector<RandomJob<T>*> rj;
  for (size_t i = 0; i < rec.size(); ++i) {
    Rec& r = *R[i];
    SmwJob<T>& j = *rec[i];
    r.A22i = std::make_unique<IPlusX<T>>(rt, r.n2, r.sub22.res.bf.get(), r.sub22.res.zero ? -1 : r.sub22.res.dense_off);
    r.a22k21 = std::make_unique<ProductOp<T>>(rt, r.A22i.get(), j.K21);
    r.k12a22k21 = std::make_unique<ProductOp<T>>(rt, j.K12, r.a22k21.get());
    r.s11op = std::make_unique<SumOp<T>>(rt, r.n1, r.n1);
    if (j.K11) r.s11op->add(j.K11, 1.0);
    r.s11op->add(r.k12a22k21.get(), -1.0);
    r.s11job.op = r.s11op.get();
    r.s11job.to = r.s11job.ts = subtree(*j.nodes, r.c1, std::max(0, r.d - 2));
    rj.push_back(&r.s11job);
  }
  bf_random_matvec_batch<T>(rt, rj);
  // X11 from S11
  sub.clear();
  for (size_t i = 0; i < rec.size(); ++i) {
    Rec& r = *R[i];
    r.s11b = std::make_unique<BfOp<T>>(rt, r.s11job.out.get());
    split(r, r.sub11, r.s11b.get(), r.c1);
    sub.push_back(&r.sub11);
  }
  smw_batch<T>(rt, sub, d_status);
  // X = [I + K11, K12; K21, I + K22]^-1 - I by randomized construction
  rj.clear();
  for (size_t i = 0; i < rec.size(); ++i) {
    Rec& r = *R[i];
    SmwJob<T>& j = *rec[i];
    r.A11i = std::make_unique<IPlusX<T>>(rt, r.n1, r.sub11.res.bf.get(), r.sub11.res.zero ? -1 : r.sub11.res.dense_off);
    r.aop = std::make_unique<SmwOp<T>>(rt, r.n1, r.n2, j.K12, j.K21, r.A11i.get(), r.A22i.get());
    r.xjob.op = r.aop.get();
    r.xjob.to = r.xjob.ts = subtree(*j.nodes, j.node, r.d);
    rj.push_back(&r.xjob);
  }
  bf_random_matvec_batch<T>(rt, rj);
  for (size_t i = 0; i < rec.size(); ++i) rec[i]->res.bf = std::move(R[i]->xjob.out);
}

}  // namespace

// ------------------------------------------------------------ front driver
template <class T>
struct CompState {
  BfRuntime<T> rt;
  std::vector<std::unique_ptr<CompressedFront<T>>> fronts;  // by front id (null if dense)
  DevBuf status;                                            // singular leaf or SMW block (int[4])
  // centre forms and descriptors of the contribution blocks in HOD-BF form, one buffer per
  // factor_level call, tagged with the tree depth of its fronts; released once the level above
  // their parents' has started (the parents are then factored)
  struct CbBuf {
    int depth;
    DevBuf buf;
  };
  std::vector<std::unique_ptr<CbBuf>> cbufs;
  uint64_t cbuf_held = 0, cbuf_peak = 0;
  double cb_bytes = 0, cb_dense_bytes = 0;
  int cb_count = 0;
  Budget* budget = nullptr;
};

template struct CompState<double>;
template struct CompState<float>;

// The compressed-front state of a handle, in the precision of the last
// factorization: complex128 throughout, or complex64 butterflies with FP64
// pivot blocks, decompositions, contribution blocks and solve vectors.
struct CompHolder {
  bool single = false;
  std::unique_ptr<CompState<double>> d;
  std::unique_ptr<CompState<float>> f;
};

void* comp_state_create(Context& c) {
  (void)c;
  return new CompHolder();
}

void comp_state_destroy(void* p) { delete (CompHolder*)p; }

template <class T>
static void reset_state(CompState<T>& st, Context& c, int nfronts) {
  st.fronts.clear();
  st.fronts.resize(nfronts);
  st.cbufs.clear();
  st.cbuf_held = st.cbuf_peak = 0;
  st.cb_bytes = st.cb_dense_bytes = 0;
  st.cb_count = 0;
  st.budget = &c.fbudget;
  st.rt.c = &c;
  st.rt.pool.reset();
  // buffers kept from an earlier factorization count against this one's budget; beyond it they are
  // released and grown again under the budget
  uint64_t held = st.rt.pool.buf.bytes;
  for (auto& ch : st.rt.scratch.chunks) held += ch->b.bytes;
  if (held > c.fbudget.limit) {
    st.rt.pool.buf.release();
    st.rt.scratch.clear();
    held = 0;
  }
  c.fbudget.held = held;
  st.rt.pool.budget = &c.fbudget;
  st.rt.scratch.budget = &c.fbudget;
  st.rt.tol = c.fopts.tol;
  st.rt.samples = c.fopts.samples > 0 ? c.fopts.samples : 64;
  st.rt.seed = c.fopts.seed;
  st.rt.stream_id = 0;
  st.rt.max_rank_seen = 0;
  st.rt.n_chunked = 0;
  st.rt.sample_hint.clear();
  st.rt.batch = c.fopts.batched != 0;
  // measured on the 100^3 workload: a dense base of 1024 rows beats 128, 256, 512 and 2048
  st.rt.smw_dense = c.fopts.smw_dense > 0 ? c.fopts.smw_dense : 1024;
  st.rt.id_max_cols = c.fopts.id_max_cols;
  if (!st.status.p) {
    HIPCHK(dev_malloc((void**)&st.status.p, 16));
    st.status.bytes = 16;
  }
}

void comp_state_reset(void* p, Context& c, int nfronts) {
  auto* h = (CompHolder*)p;
  h->single = c.fopts.precision == BFMF_C64_MIXED;
  if (h->single) {
    h->d.reset();  // release the other precision's pools
    if (!h->f) h->f = std::make_unique<CompState<float>>();
    reset_state(*h->f, c, nfronts);
  } else {
    h->f.reset();
    if (!h->d) h->d = std::make_unique<CompState<double>>();
    reset_state(*h->d, c, nfronts);
  }
}

// nearest-vertex lists by breadth-first search in the graph of A restricted
// to the front (front-local indices); `limit` restricts the search to [0, limit)
static void bfs_lists(const Context& c, int f, int limit, int K, std::vector<std::vector<int32_t>>& out) {
  const Symbolic& s = c.sym;
  const int ns = (int)s.ns(f), nu = (int)s.nu(f), n = ns + nu;
  const int64_t b = s.sbeg[f], e = s.send[f];
  const int64_t* iu = s.iu.data() + s.iu_ptr[f];
  auto local = [&](int64_t g) -> int {
    if (g >= b && g < e) return (int)(g - b);
    const int64_t* it = std::lower_bound(iu, iu + nu, g);
    if (it == iu + nu || *it != g) return -1;
    return ns + (int)(it - iu);
  };
  std::vector<std::vector<int32_t>> adj(n);
  for (int i = 0; i < n; ++i) {
    const int64_t gi = i < ns ? b + i : iu[i - ns];
    const int64_t o = s.perm[gi];
    for (int64_t t = c.rowptr[o]; t < c.rowptr[o + 1]; ++t) {
      const int j = local(s.iperm[c.colind[t]]);
      if (j >= 0 && j != i && j < limit && i < limit) adj[i].push_back(j);
    }
    std::sort(adj[i].begin(), adj[i].end());
  }
  out.assign(n, {});
  std::vector<int> seen(n, -1);
  std::vector<int32_t> layer, next;
  for (int i = 0; i < std::min(n, limit); ++i) {
    auto& lst = out[i];
    seen[i] = i;
    layer.assign(1, i);
    while (!layer.empty() && (int)lst.size() < K) {
      next.clear();
      for (int u : layer)
        for (int v : adj[u])
          if (seen[v] != i) {
            seen[v] = i;
            next.push_back(v);
          }
      std::sort(next.begin(), next.end());
      for (int v : next) {
        if ((int)lst.size() >= K) break;
        lst.push_back(v);
      }
      layer.swap(next);
    }
  }
}

namespace {

// Work of one compressed front while its level is being factored.
template <class T>
struct FrontWork {
  int f = -1;
  const FrontDesc* d_fd = nullptr;
  void* cb = nullptr;
  std::unique_ptr<CompressedFront<T>> cf;
  std::vector<TreeNode> nodes;  // separator bisection (P-hat), preorder
  std::vector<TreeNode> unodes;  // balanced tree over I^u
  std::vector<std::vector<int32_t>> near11, nearall;
  uint64_t seed = 0;
  std::vector<std::unique_ptr<EntrySource<T>>> srcs;
  std::vector<std::unique_ptr<ProxySampler>> samplers;
};

}  // namespace

// HOD-BF structure over a preorder bisection tree (node 0 the root)
template <class T>
static void hodbf_from_tree(Hodbf<T>& h, const std::vector<TreeNode>& nodes, int n) {
  h.n = n;
  h.nodes.clear();
  h.nodes.resize(nodes.size());
  h.max_level = 0;
  std::vector<std::pair<int, int>> stck{{0, 0}};
  while (!stck.empty() && !nodes.empty()) {
    auto [i, l] = stck.back();
    stck.pop_back();
    auto& hn = h.nodes[i];
    hn.beg = nodes[i].beg;
    hn.end = nodes[i].end;
    hn.left = nodes[i].left;
    hn.right = nodes[i].right;
    hn.level = l;
    hn.depth = depth_of(nodes, i);
    h.max_level = std::max(h.max_level, l);
    if (hn.left >= 0) {
      stck.push_back({hn.left, l + 1});
      stck.push_back({hn.right, l + 1});
    }
  }
  h.by_level.assign(h.max_level + 1, {});
  for (int i = 0; i < (int)h.nodes.size(); ++i) h.by_level[h.nodes[i].level].push_back(i);
}

// Contribution blocks in HOD-BF form (Alg. 5, last step) for the fronts Wc
// of one level at tree depth `depth`: C = (C_nu1 (+) C_nu2)(Iu, Iu) - S by
// HODBF_entry_eval over the balanced tree of I^u (dense leaves, then every
// off-diagonal block by Alg. 2, all fronts' blocks of a step together), each
// request answered by list routing from the children (dense, or HOD-BF
// through extract_HODBF) and by extract_BF of S.  Then the centre forms of
// every block of C and its device descriptor, read by the parent's
// extractions, in a buffer kept until the parent's level has been factored.
template <class T>
static void build_cb_hodbf(CompState<T>* st, Context& c, const std::vector<FrontWork<T>*>& Wc, int depth,
                           double alpha, int knn) {
  BfRuntime<T>& rt = st->rt;
  hipStream_t s = rt.s();
  const size_t esz = sizeof(cplx<T>);
  if (Wc.empty()) return;
  // centre buffers of fronts whose parents have been factored (two levels deeper or more)
  if (!c.fopts.keep_fronts) {
    for (auto& b : st->cbufs)
      if (b && b->depth >= depth + 2) {
        st->cbuf_held -= b->buf.bytes;
        st->budget->held -= std::min<uint64_t>(st->budget->held, b->buf.bytes);
        b.reset();
      }
    st->cbufs.erase(std::remove(st->cbufs.begin(), st->cbufs.end(), nullptr), st->cbufs.end());
  }
  auto mk = rt.scratch.mark();
  // S of every front in centre form (temporary)
  CentreSpec sspec;
  for (auto* w : Wc) sspec.bfs.push_back(w->cf->s.get());
  char* smem = (char*)rt.scratch.take(centre_bytes<T>(sspec));
  const CentreOut scen = build_centres<T>(rt, sspec, smem);
  // the HOD-BF trees and dense leaves: C(leaf, leaf), every pool allocation first
  for (auto* w : Wc) {
    Hodbf<T>& h = w->cf->cbh;
    hodbf_from_tree<T>(h, w->unodes, w->cf->nu);
    for (auto& nd : h.nodes)
      if (nd.left < 0)
        nd.leaf_off = (int64_t)(rt.pool.alloc((size_t)nd.size() * nd.size() * esz, s) / esz);
  }
  {
    ExtractBatch eb;
    for (size_t k = 0; k < Wc.size(); ++k) {
      FrontWork<T>& w = *Wc[k];
      for (auto& nd : w.cf->cbh.nodes)
        if (nd.left < 0 && nd.size() > 0) {
          std::vector<int32_t> r(nd.size());
          for (int q = 0; q < nd.size(); ++q) r[q] = nd.beg + q;
          void* out = rt.pool_base() + nd.leaf_off * esz;
          eb.add(w.d_fd, nullptr, 0, r, w.cf->ns, r, w.cf->ns, out, nd.size(), false);
          eb.add_bf(scen.bfs + k, r, 0, r, 0, out, nd.size(), false, -1.0, true);
        }
    }
    run_extract<T>(rt, eb);
  }
  // off-diagonal butterflies (Alg. 2)
  {
    std::vector<std::unique_ptr<EntryJob<T>>> jobs;
    std::vector<std::pair<HodbfNode<T>*, int>> dest;
    for (size_t k = 0; k < Wc.size(); ++k) {
      FrontWork<T>& w = *Wc[k];
      const auto& nodes = w.unodes;
      for (int i = 0; i < (int)nodes.size(); ++i) {
        if (nodes[i].left < 0) continue;
        const int a = nodes[i].left, b = nodes[i].right;
        const int L = std::min(depth_of(nodes, a), depth_of(nodes, b));
        BTree ta = subtree(nodes, a, L), tb = subtree(nodes, b, L);
        for (int side = 0; side < 2; ++side) {
          const int r = side ? b : a, cc = side ? a : b;
          w.srcs.push_back(std::make_unique<CbSource<T>>(w.d_fd, w.cf->ns, nodes[r].beg, nodes[cc].beg, scen.bfs + k));
          w.samplers.push_back(std::make_unique<BfsSampler>(w.nearall, w.cf->ns + nodes[r].beg,
                                                            w.cf->ns + nodes[cc].beg, knn, alpha,
                                                            w.seed + 9001 + 2 * i + side));
          jobs.push_back(std::make_unique<EntryJob<T>>(
              EntryJob<T>{w.srcs.back().get(), w.samplers.back().get(), side ? tb : ta, side ? ta : tb, nullptr}));
          dest.push_back({&w.cf->cbh.nodes[i], side});
        }
      }
    }
    std::vector<EntryJob<T>*> jp;
    for (auto& j : jobs) jp.push_back(j.get());
    bf_entry_eval_batch<T>(rt, jp);
    for (size_t k = 0; k < jobs.size(); ++k)
      (dest[k].second ? dest[k].first->b21 : dest[k].first->b12) = std::move(jobs[k]->out);
  }
  rt.scratch.release(mk);  // S's centre form is no longer read (stream order)
  // centre forms of C and the descriptors, in one buffer
  CentreSpec spec;
  std::vector<std::vector<int>> b12(Wc.size()), b21(Wc.size()), leaf(Wc.size());
  for (size_t k = 0; k < Wc.size(); ++k) {
    const Hodbf<T>& h = Wc[k]->cf->cbh;
    b12[k].assign(h.nodes.size(), -1);
    b21[k].assign(h.nodes.size(), -1);
    leaf[k].assign(h.nodes.size(), -1);
    for (int i = 0; i < (int)h.nodes.size(); ++i) {
      const auto& nd = h.nodes[i];
      if (nd.left < 0) {
        leaf[k][i] = (int)spec.dense.size();
        spec.dense.push_back({nd.leaf_off, nd.size()});
        continue;
      }
      if (nd.b12) {
        b12[k][i] = (int)spec.bfs.size();
        spec.bfs.push_back(nd.b12.get());
      }
      if (nd.b21) {
        b21[k][i] = (int)spec.bfs.size();
        spec.bfs.push_back(nd.b21.get());
      }
    }
  }
  const size_t cbytes = (centre_bytes<T>(spec) + 63) & ~(size_t)63;
  size_t dbytes = 0;
  for (auto* w : Wc) dbytes += w->cf->cbh.nodes.size() * sizeof(HodbfNodeDev) + sizeof(HodbfDev) + 128;
  const size_t total = cbytes + dbytes;
  if (!st->budget->fits(total))
    throw Error(BFMF_E_NOMEM, "contribution-block centre forms of " + std::to_string(total) +
                                  " bytes exceed the HBM budget");
  auto cb = std::make_unique<typename CompState<T>::CbBuf>();
  cb->depth = depth;
  HIPCHK(dev_malloc(&cb->buf.p, total));
  cb->buf.bytes = total;
  st->budget->held += total;
  st->cbuf_held += total;
  st->cbuf_peak = std::max(st->cbuf_peak, st->cbuf_held);
  char* mem = (char*)cb->buf.p;
  const CentreOut cen = build_centres<T>(rt, spec, mem);
  std::vector<char> hd(dbytes, 0);
  size_t off = 0;
  for (size_t k = 0; k < Wc.size(); ++k) {
    CompressedFront<T>& cf = *Wc[k]->cf;
    const Hodbf<T>& h = cf.cbh;
    const size_t node_off = off;
    for (int i = 0; i < (int)h.nodes.size(); ++i) {
      const auto& nd = h.nodes[i];
      HodbfNodeDev d;
      std::memset(&d, 0, sizeof(d));
      d.beg = nd.beg;
      d.end = nd.end;
      d.left = nd.left;
      d.right = nd.right;
      d.mid = nd.left >= 0 ? h.nodes[nd.left].end : nd.end;
      d.b12 = b12[k][i];
      d.b21 = b21[k][i];
      d.leaf = nd.left < 0 ? cen.dense[leaf[k][i]] : nullptr;
      if (off + sizeof(d) > dbytes) throw Error(BFMF_E_INVAL, "internal: contribution-block descriptors overflow");
      std::memcpy(hd.data() + off, &d, sizeof(d));
      off += sizeof(d);
    }
    HodbfDev hdv;
    std::memset(&hdv, 0, sizeof(hdv));
    hdv.nodes = (const HodbfNodeDev*)(mem + cbytes + node_off);
    hdv.bfs = cen.bfs;
    hdv.single = sizeof(T) == 4 ? 1 : 0;
    hdv.depth = h.nodes.empty() ? 0 : h.nodes[0].depth;
    off = (off + 63) & ~(size_t)63;
    if (off + sizeof(hdv) > dbytes) throw Error(BFMF_E_INVAL, "internal: contribution-block descriptors overflow");
    std::memcpy(hd.data() + off, &hdv, sizeof(hdv));
    cf.cb_dev = (const HodbfDev*)(mem + cbytes + off);
    off += sizeof(hdv);
    off = (off + 63) & ~(size_t)63;
    // pool entries of the block and what it would take dense
    int64_t e = 0;
    for (const auto& nd : h.nodes) {
      if (nd.left < 0) e += (int64_t)nd.size() * nd.size();
      if (nd.b12) e += nd.b12->elems;
      if (nd.b21) e += nd.b21->elems;
    }
    st->cb_bytes += (double)e * esz;
    st->cb_dense_bytes += (double)cf.nu * cf.nu * sizeof(cplx<double>);
    st->cb_count += 1;
  }
  rt.c->stage.put(mem + cbytes, hd.data(), off, s);
  st->cbufs.push_back(std::move(cb));
}

// Compressed factorization (Alg. 5) of the fronts `fr` of one level of the
// assembly tree: d_fds[i] is the device descriptor of fr[i], cbs[i] receives
// its contribution block (nu x nu, ld nu).  With batching every phase runs
// over all fronts of the level at once.
template <class T>
static void factor_level(CompState<T>* st, Context& c, const std::vector<int>& fr,
                         const std::vector<const FrontDesc*>& d_fds, const std::vector<void*>& cbs) {
  BfRuntime<T>& rt = st->rt;
  if (fr.empty()) return;
  if (!rt.batch && fr.size() > 1) {
    for (size_t i = 0; i < fr.size(); ++i) factor_level<T>(st, c, {fr[i]}, {d_fds[i]}, {cbs[i]});
    return;
  }
  const Symbolic& sy = c.sym;
  hipStream_t s = rt.s();
  int* d_status = (int*)st->status.p;
  ochk(hipMemsetAsync(d_status, 0, 16, s), "status");
  auto clock = [] { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); };
  double tph[6] = {clock(), 0, 0, 0, 0, 0};
  const int64_t r0 = rt.n_random, e0 = rt.n_entry;
  const double alpha = c.fopts.alpha > 0 ? c.fopts.alpha : 2.0;
  const int knn = c.fopts.knn;
  std::vector<std::unique_ptr<FrontWork<T>>> W;
  for (size_t k = 0; k < fr.size(); ++k) {
    auto w = std::make_unique<FrontWork<T>>();
    const int f = fr[k];
    w->f = f;
    w->d_fd = d_fds[k];
    w->cb = cbs[k];
    w->cf = std::make_unique<CompressedFront<T>>();
    w->cf->front = f;
    w->cf->ns = (int)sy.ns(f);
    w->cf->nu = (int)sy.nu(f);
    // HOD-BF tree of F11: the separator bisection (P-hat), Sec. 5.1
    w->nodes.assign(sy.sep_nodes.begin() + sy.sep_ptr[f], sy.sep_nodes.begin() + sy.sep_ptr[f + 1]);
    Hodbf<T>& h = w->cf->f11;
    h.n = w->cf->ns;
    h.nodes.resize(w->nodes.size());
    std::vector<std::pair<int, int>> stck{{0, 0}};
    while (!stck.empty()) {
      auto [i, l] = stck.back();
      stck.pop_back();
      auto& hn = h.nodes[i];
      hn.beg = w->nodes[i].beg;
      hn.end = w->nodes[i].end;
      hn.left = w->nodes[i].left;
      hn.right = w->nodes[i].right;
      hn.level = l;
      hn.depth = depth_of(w->nodes, i);
      h.max_level = std::max(h.max_level, l);
      if (hn.left >= 0) {
        stck.push_back({hn.left, l + 1});
        stck.push_back({hn.right, l + 1});
      }
    }
    h.by_level.assign(h.max_level + 1, {});
    for (int i = 0; i < (int)h.nodes.size(); ++i) h.by_level[h.nodes[i].level].push_back(i);
    w->seed = c.fopts.seed * 1000003ull + (uint64_t)f;
    W.push_back(std::move(w));
  }
  // nearest-vertex lists of every front (host work, two independent lists per front) on the
  // host thread pool
  HostPool::get().parallel_for(2 * W.size(), [&](size_t t) {
    FrontWork<T>& w = *W[t / 2];
    if (t % 2 == 0)
      bfs_lists(c, w.f, w.cf->ns, 32, w.near11);
    else
      bfs_lists(c, w.f, w.cf->ns + w.cf->nu, 32, w.nearall);
  });
  // leaves D = F11(leaf, leaf): every pool allocation first, then one extraction
  {
    for (auto& w : W)
      for (auto& nd : w->cf->f11.nodes)
        if (nd.left < 0) nd.leaf_off = (int64_t)(rt.pool.alloc((size_t)nd.size() * nd.size() * sizeof(cplx<T>), s) /
                                                 sizeof(cplx<T>));
    ExtractBatch eb;
    for (auto& w : W)
      for (auto& nd : w->cf->f11.nodes)
        if (nd.left < 0) {
          std::vector<int32_t> r(nd.size());
          for (int k = 0; k < nd.size(); ++k) r[k] = nd.beg + k;
          eb.add(w->d_fd, nullptr, 0, r, 0, r, 0, rt.pool_base() + nd.leaf_off * sizeof(cplx<T>), std::max(1, nd.size()),
                 false);
        }
    run_extract<T>(rt, eb);
  }
  // off-diagonal butterflies of F11 (Alg. 2 on F11 = A(Is,Is) (+) C_nu1 (+) C_nu2)
  {
    std::vector<std::unique_ptr<EntryJob<T>>> jobs;
    std::vector<std::pair<HodbfNode<T>*, int>> dest;
    for (auto& w : W) {
      auto& nodes = w->nodes;
      for (int i = 0; i < (int)nodes.size(); ++i) {
        if (nodes[i].left < 0) continue;
        const int a = nodes[i].left, b = nodes[i].right;
        const int L = std::min(depth_of(nodes, a), depth_of(nodes, b));
        BTree ta = subtree(nodes, a, L), tb = subtree(nodes, b, L);
        for (int side = 0; side < 2; ++side) {
          const int r = side ? b : a, cc = side ? a : b;
          w->srcs.push_back(std::make_unique<FrontSource<T>>(w->d_fd, nodes[r].beg, nodes[cc].beg));
          w->samplers.push_back(
              std::make_unique<BfsSampler>(w->near11, nodes[r].beg, nodes[cc].beg, knn, alpha, w->seed + 2 * i + side));
          jobs.push_back(std::make_unique<EntryJob<T>>(
              EntryJob<T>{w->srcs.back().get(), w->samplers.back().get(), side ? tb : ta, side ? ta : tb, nullptr}));
          dest.push_back({&w->cf->f11.nodes[i], side});
        }
      }
    }
    std::vector<EntryJob<T>*> jp;
    for (auto& j : jobs) jp.push_back(j.get());
    bf_entry_eval_batch<T>(rt, jp);
    for (size_t k = 0; k < jobs.size(); ++k) (dest[k].second ? dest[k].first->b21 : dest[k].first->b12) = std::move(jobs[k]->out);
  }
  tph[1] = clock();
  // HODBF_invert (Alg. 4): leaf inverses, then the internal nodes by height
  {
    for (auto& w : W)
      for (auto& nd : w->cf->f11.nodes)
        if (nd.left < 0) nd.inv_off = (int64_t)(rt.pool.alloc((size_t)nd.size() * nd.size() * sizeof(cplx<T>), s) /
                                                sizeof(cplx<T>));
    std::vector<InvTask> it;
    auto mk = rt.scratch.mark();
    std::vector<AxpbyTask> cp;  // copies / conversions of all leaves in one launch
    int64_t maxe = 0;
    if (sizeof(T) == 8) {  // invert the leaves in place of a copy
      for (auto& w : W)
        for (auto& nd : w->cf->f11.nodes)
          if (nd.left < 0) {
            cp.push_back(AxpbyTask{rt.pool_base() + nd.inv_off * sizeof(cplx<T>),
                                   rt.pool_base() + nd.leaf_off * sizeof(cplx<T>), std::max(nd.size(), 1),
                                   std::max(nd.size(), 1), nd.size(), nd.size(), 0});
            maxe = std::max<int64_t>(maxe, (int64_t)nd.size() * nd.size());
            it.push_back(InvTask{rt.pool_base() + nd.inv_off * sizeof(cplx<T>), std::max(nd.size(), 1), nd.size(), 0});
          }
      if (!cp.empty())
        ochk(launch_mix_batch<double, double>((const AxpbyTask*)up(rt, cp), (int)cp.size(), maxe, 1.0, 0.0, 0.0, s),
             "leaf copy");
      void* d_it = up(rt, it);
      ochk(launch_leaf_inverse<double>(d_it, (int)it.size(), d_status, s), "leaf inverse");
    } else {  // pivot blocks in FP64: extract the leaves again in FP64, invert, store in complex64
      ExtractBatch eb;
      std::vector<std::pair<void*, HodbfNode<T>*>> tmp;
      for (auto& w : W)
        for (auto& nd : w->cf->f11.nodes)
          if (nd.left < 0) {
            void* d = rt.scratch.take((size_t)std::max(nd.size(), 1) * nd.size() * sizeof(cplx<double>));
            std::vector<int32_t> r(nd.size());
            for (int k = 0; k < nd.size(); ++k) r[k] = nd.beg + k;
            eb.add(w->d_fd, nullptr, 0, r, 0, r, 0, d, std::max(1, nd.size()), false);
            it.push_back(InvTask{d, std::max(nd.size(), 1), nd.size(), 0});
            tmp.push_back({d, &nd});
          }
      run_extract_to<double>(rt, eb, false);
      void* d_it = up(rt, it);
      ochk(launch_leaf_inverse<double>(d_it, (int)it.size(), d_status, s), "leaf inverse");
      for (auto& t : tmp) {
        const int sz = t.second->size();
        cp.push_back(AxpbyTask{rt.pool_base() + t.second->inv_off * sizeof(cplx<T>), t.first, std::max(sz, 1),
                               std::max(sz, 1), sz, sz, 0});
        maxe = std::max<int64_t>(maxe, (int64_t)sz * sz);
      }
      if (!cp.empty())
        ochk(launch_mix_batch<T, double>((const AxpbyTask*)up(rt, cp), (int)cp.size(), maxe, 1.0, 0.0, 0.0, s),
             "leaf convert");
    }
    rt.scratch.release(mk);
  }
  int H = 0;
  for (auto& w : W)
    for (auto& nd : w->cf->f11.nodes) H = std::max(H, nd.depth);
  for (int hgt = 1; hgt <= H; ++hgt) {
    struct NodeWork {
      HodbfNode<T>* nd;
      std::unique_ptr<HodbfInvOp<T>> d1, d2;
      std::unique_ptr<BfOp<T>> b12, b21, k12, k21;
      std::unique_ptr<ProductOp<T>> p1, p2;
      std::unique_ptr<Block2Op<T>> kfull;
      RandomJob<T> j1, j2;
      SmwJob<T> smw;
    };
    std::vector<std::unique_ptr<NodeWork>> nw;
    std::vector<RandomJob<T>*> rj;
    for (auto& w : W) {
      Hodbf<T>& h = w->cf->f11;
      for (int i = 0; i < (int)h.nodes.size(); ++i) {
        HodbfNode<T>& nd = h.nodes[i];
        if (nd.left < 0 || nd.depth != hgt) continue;
        auto x = std::make_unique<NodeWork>();
        x->nd = &nd;
        // B1' = D1^-1 B12, B2' = D2^-1 B21 by randomized construction
        x->d1 = std::make_unique<HodbfInvOp<T>>(rt, h, nd.left);
        x->d2 = std::make_unique<HodbfInvOp<T>>(rt, h, nd.right);
        x->b12 = std::make_unique<BfOp<T>>(rt, nd.b12.get());
        x->b21 = std::make_unique<BfOp<T>>(rt, nd.b21.get());
        x->p1 = std::make_unique<ProductOp<T>>(rt, x->d1.get(), x->b12.get());
        x->p2 = std::make_unique<ProductOp<T>>(rt, x->d2.get(), x->b21.get());
        x->j1.op = x->p1.get();
        x->j1.to = nd.b12->to;
        x->j1.ts = nd.b12->ts;
        x->j2.op = x->p2.get();
        x->j2.to = nd.b21->to;
        x->j2.ts = nd.b21->ts;
        x->smw.nodes = &w->nodes;
        x->smw.node = i;
        rj.push_back(&x->j1);
        rj.push_back(&x->j2);
        nw.push_back(std::move(x));
      }
    }
    bf_random_matvec_batch<T>(rt, rj);
    // [I B1'; B2' I]^-1 = I + X (BF_SMW with zero diagonal blocks)
    std::vector<SmwJob<T>*> sj;
    for (auto& x : nw) {
      const int na = x->j1.to.n, nb = x->j2.to.n;
      x->k12 = std::make_unique<BfOp<T>>(rt, x->j1.out.get());
      x->k21 = std::make_unique<BfOp<T>>(rt, x->j2.out.get());
      x->kfull = std::make_unique<Block2Op<T>>(rt, na + nb, na + nb, na, na, nullptr, x->k12.get(), x->k21.get(), nullptr);
      x->smw.K12 = x->k12.get();
      x->smw.K21 = x->k21.get();
      x->smw.Kfull = x->kfull.get();
      sj.push_back(&x->smw);
    }
    smw_batch<T>(rt, sj, d_status);
    for (auto& x : nw) {
      SmwResult& r = x->smw.res;
      x->nd->x = std::move(r.bf);
      x->nd->x_dense = r.dense_off >= 0;
      if (x->nd->x_dense) x->nd->inv_off = r.dense_off;
      x->nd->x_zero = r.zero;
    }
  }
  tph[2] = clock();
  // F12 and F21 (Alg. 2), trees: separator bisection x balanced tree on I^u
  {
    std::vector<std::unique_ptr<EntryJob<T>>> jobs;
    std::vector<std::pair<CompressedFront<T>*, int>> dest;
    for (auto& w : W) {
      const int ns = w->cf->ns, nu = w->cf->nu;
      if (nu == 0) continue;
      w->unodes = balanced_tree(nu, 64);
      const int L = std::min(depth_of(w->nodes, 0), depth_of(w->unodes, 0));
      BTree ts_ = subtree(w->nodes, 0, L), tu = subtree(w->unodes, 0, L);
      for (int side = 0; side < 2; ++side) {
        const int r = side ? ns : 0, cc = side ? 0 : ns;
        w->srcs.push_back(std::make_unique<FrontSource<T>>(w->d_fd, r, cc));
        w->samplers.push_back(
            std::make_unique<BfsSampler>(w->nearall, r, cc, knn, alpha, w->seed + (side ? 8888 : 7777)));
        jobs.push_back(std::make_unique<EntryJob<T>>(
            EntryJob<T>{w->srcs.back().get(), w->samplers.back().get(), side ? tu : ts_, side ? ts_ : tu, nullptr}));
        dest.push_back({w->cf.get(), side});
      }
    }
    std::vector<EntryJob<T>*> jp;
    for (auto& j : jobs) jp.push_back(j.get());
    bf_entry_eval_batch<T>(rt, jp);
    for (size_t k = 0; k < jobs.size(); ++k) (dest[k].second ? dest[k].first->f21 : dest[k].first->f12) = std::move(jobs[k]->out);
  }
  tph[3] = clock();
  // S = F21 F11^-1 F12 (Sec. 3.3)
  {
    struct SWork {
      std::unique_ptr<HodbfInvOp<T>> f11i;
      std::unique_ptr<BfOp<T>> f12, f21;
      std::unique_ptr<ProductOp<T>> p1, p2;
      RandomJob<T> j;
    };
    std::vector<std::unique_ptr<SWork>> sw;
    std::vector<RandomJob<T>*> rj;
    std::vector<CompressedFront<T>*> dest;
    for (auto& w : W) {
      if (w->cf->nu == 0) continue;
      auto x = std::make_unique<SWork>();
      x->f11i = std::make_unique<HodbfInvOp<T>>(rt, w->cf->f11, 0);
      x->f12 = std::make_unique<BfOp<T>>(rt, w->cf->f12.get());
      x->f21 = std::make_unique<BfOp<T>>(rt, w->cf->f21.get());
      x->p1 = std::make_unique<ProductOp<T>>(rt, x->f11i.get(), x->f12.get());
      x->p2 = std::make_unique<ProductOp<T>>(rt, x->f21.get(), x->p1.get());
      x->j.op = x->p2.get();
      x->j.to = x->j.ts = subtree(w->unodes, 0, depth_of(w->unodes, 0));
      rj.push_back(&x->j);
      dest.push_back(w->cf.get());
      sw.push_back(std::move(x));
    }
    bf_random_matvec_batch<T>(rt, rj);
    for (size_t k = 0; k < sw.size(); ++k) dest[k]->s = std::move(sw[k]->j.out);
  }
  tph[4] = clock();
  // C = (C_nu1 (+) C_nu2)(Iu, Iu) - S: in HOD-BF form where the parent is compressed and
  // compress_cb is set, else dense FP64 in the level workspace (S applied to identity columns)
  std::vector<FrontWork<T>*> Wd, Wc;
  for (auto& w : W)
    if (w->cf->nu > 0) (c.cbcomp.size() > (size_t)w->f && c.cbcomp[w->f] ? Wc : Wd).push_back(w.get());
  build_cb_hodbf<T>(st, c, Wc, c.sym.level[fr[0]], alpha, knn);
  {
    ExtractBatch eb;
    int maxnu = 0;
    for (auto* w : Wd) {
      const int ns = w->cf->ns, nu = w->cf->nu;
      if (nu == 0) continue;
      maxnu = std::max(maxnu, nu);
      std::vector<int32_t> r(nu);
      for (int k = 0; k < nu; ++k) r[k] = k;
      eb.add(w->d_fd, nullptr, 0, r, ns, r, ns, w->cb, nu, false);
    }
    run_extract_to<double>(rt, eb, false);  // C_nu1 (+) C_nu2 on I^u x I^u, FP64
    // S applied to identity columns in chunks of 1024, chunk c0 of every front in one product
    const int chunk = 1024;
    auto mk = rt.scratch.mark();
    std::vector<cplx<T>*> I(Wd.size(), nullptr), St(Wd.size(), nullptr);
    for (size_t k = 0; k < Wd.size(); ++k) {
      const int nu = Wd[k]->cf->nu;
      if (nu == 0) continue;
      I[k] = (cplx<T>*)rt.scratch.take((size_t)nu * std::min(chunk, nu) * sizeof(cplx<T>));
      if (sizeof(T) != 8) St[k] = (cplx<T>*)rt.scratch.take((size_t)nu * std::min(chunk, nu) * sizeof(cplx<T>));
    }
    const int64_t esz = (int64_t)sizeof(cplx<T>);
    for (int c0 = 0; c0 < maxnu; c0 += chunk) {
      std::vector<AxpbyTask> eye, upd;
      std::vector<BfCall> calls;
      int64_t maxe = 0;
      for (size_t k = 0; k < Wd.size(); ++k) {
        const int nu = Wd[k]->cf->nu;
        if (nu <= c0) continue;
        const int wd = std::min(chunk, nu - c0);
        maxe = std::max<int64_t>(maxe, (int64_t)nu * wd);
        eye.push_back(AxpbyTask{I[k], nullptr, nu, nu, nu, wd, c0});  // I(i, c) = 1 where i == c0 + c
        cplx<double>* cbc = (cplx<double>*)Wd[k]->cb + (size_t)c0 * nu;  // contribution blocks stay FP64
        BfCall cl;
        cl.bf = Wd[k]->cf->s.get();
        cl.x_off = cl.y_off = 0;
        cl.alpha_im = 0;
        cl.x_abs = (int64_t)((uintptr_t)I[k] / esz);
        cl.ldx = cl.ldy = nu;
        cl.nrhs = wd;
        if (sizeof(T) == 8) {  // C -= S I
          cl.alpha_re = -1.0;
          cl.beta = 1;
          cl.y_abs = (int64_t)((uintptr_t)cbc / esz);
        } else {  // St = S I, then C -= St in FP64
          cl.alpha_re = 1.0;
          cl.beta = 0;
          cl.y_abs = (int64_t)((uintptr_t)St[k] / esz);
          upd.push_back(AxpbyTask{cbc, St[k], nu, nu, nu, wd, 0});
        }
        calls.push_back(cl);
      }
      ochk(launch_mix_batch<T, T>((const AxpbyTask*)up(rt, eye), (int)eye.size(), maxe, 0.0, 0.0, 1.0, s), "eye");
      if (rt.batch) {
        rt.apply_calls(calls, false);
      } else {  // the plain form: one front after another
        for (const BfCall& cl : calls) rt.apply_calls({cl}, false);
      }
      if (!upd.empty())
        ochk(launch_mix_batch<double, T>((const AxpbyTask*)up(rt, upd), (int)upd.size(), maxe, -1.0, 1.0, 0.0, s),
             "cb update");
    }
    rt.scratch.release(mk);
  }
  int hst[4] = {0, 0, 0, 0};
  ochk(hipMemcpyAsync(hst, d_status, 16, hipMemcpyDeviceToHost, s), "status");
  rt.c->stage.sync(s);
  if (hst[0]) throw Error(BFMF_E_SINGULAR, "singular HOD-BF leaf or inversion block in a compressed front");
  tph[5] = clock();
  if (c.verbose) {
    int nsmax = 0, numax = 0;
    for (auto& w : W) {
      nsmax = std::max(nsmax, w->cf->ns);
      numax = std::max(numax, w->cf->nu);
    }
    fprintf(stderr,
            "[bfmf] %zu compressed front(s), ns <= %d, nu <= %d: F11 %.3fs inv %.3fs F12/F21 %.3fs S %.3fs C %.3fs; "
            "constructions random %lld entry %lld; max rank %d\n",
            W.size(), nsmax, numax, tph[1] - tph[0], tph[2] - tph[1], tph[3] - tph[2], tph[4] - tph[3],
            tph[5] - tph[4], (long long)(rt.n_random - r0), (long long)(rt.n_entry - e0), rt.max_rank_seen);
  }
  for (auto& w : W) st->fronts[w->f] = std::move(w->cf);
}

// ------------------------------------------------------------ sweeps
// forward: W(0:ns) <- F11^-1 W(0:ns); W(ns:n) -= F21 W(0:ns).  W is FP64; in
// the complex64 form the front's part goes through complex64 copies.
template <class T>
static void forward_front(CompState<T>& st, int f, void* W, int n, int nrhs) {
  BfRuntime<T>& rt = st.rt;
  CompressedFront<T>& cf = *st.fronts[f];
  cplx<double>* w = (cplx<double>*)W;
  hipStream_t s = rt.s();
  auto mk = rt.scratch.mark();
  cplx<T>* z = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
  if (sizeof(T) == 8) {
    hodbf_inv_apply<T>(rt, cf.f11, 0, w, n, z, cf.ns, nrhs, false);
    ochk(launch_axpby<double>(w, n, z, cf.ns, cf.ns, nrhs, 1.0, 0.0, s), "copy");
    if (cf.nu > 0) rt.apply(*cf.f21, w, n, w + cf.ns, n, nrhs, false, -1.0, 1);
  } else {
    cplx<T>* ws = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
    ochk(launch_convert<T, double>(ws, cf.ns, w, n, cf.ns, nrhs, s), "to c64");
    hodbf_inv_apply<T>(rt, cf.f11, 0, ws, cf.ns, z, cf.ns, nrhs, false);
    ochk(launch_convert<double, T>(w, n, z, cf.ns, cf.ns, nrhs, s), "to c128");
    if (cf.nu > 0) {
      cplx<T>* t = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.nu, 1) * nrhs * sizeof(cplx<T>));
      rt.apply(*cf.f21, z, cf.ns, t, cf.nu, nrhs, false, 1.0, 0);
      ochk(launch_axpby_mixed<double, T>(w + cf.ns, n, t, cf.nu, cf.nu, nrhs, -1.0, 1.0, s), "update");
    }
  }
  rt.scratch.release(mk);
}

// backward: W(0:ns) -= F11^-1 F12 W(ns:n)   (W(ns:n) already holds x(I^u))
template <class T>
static void backward_front(CompState<T>& st, int f, void* W, int n, int nrhs) {
  BfRuntime<T>& rt = st.rt;
  CompressedFront<T>& cf = *st.fronts[f];
  cplx<double>* w = (cplx<double>*)W;
  if (cf.nu == 0) return;
  hipStream_t s = rt.s();
  auto mk = rt.scratch.mark();
  cplx<T>* t = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
  cplx<T>* t2 = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
  if (sizeof(T) == 8) {
    rt.apply(*cf.f12, w + cf.ns, n, t, cf.ns, nrhs, false, 1.0, 0);
  } else {
    cplx<T>* u = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.nu, 1) * nrhs * sizeof(cplx<T>));
    ochk(launch_convert<T, double>(u, cf.nu, w + cf.ns, n, cf.nu, nrhs, s), "to c64");
    rt.apply(*cf.f12, u, cf.nu, t, cf.ns, nrhs, false, 1.0, 0);
  }
  hodbf_inv_apply<T>(rt, cf.f11, 0, t, cf.ns, t2, cf.ns, nrhs, false);
  ochk(launch_axpby_mixed<double, T>(w, n, t2, cf.ns, cf.ns, nrhs, -1.0, 1.0, s), "update");
  rt.scratch.release(mk);
}

// The same sweeps for all compressed fronts of a level at once (batched form):
// the F11^-1 products of every front in one HOD-BF inverse application, the
// F21 / F12 products in one butterfly plan, conversions and updates in single
// launches.  Same arithmetic as the per-front sweeps, so the same result.
template <class T>
static void forward_level(CompState<T>& st, const std::vector<int>& fs, const std::vector<void*>& Ws,
                          const std::vector<int>& ns_, int nrhs) {
  BfRuntime<T>& rt = st.rt;
  hipStream_t s = rt.s();
  auto mk = rt.scratch.mark();
  const int64_t esz = (int64_t)sizeof(cplx<T>);
  std::vector<HodbfInvItem<T>> inv;
  std::vector<AxpbyTask> to_low, back, upd;
  std::vector<BfCall> calls;
  int64_t maxe = 0;
  for (size_t k = 0; k < fs.size(); ++k) {
    CompressedFront<T>& cf = *st.fronts[fs[k]];
    cplx<double>* w = (cplx<double>*)Ws[k];
    const int n = ns_[k];
    maxe = std::max<int64_t>(maxe, (int64_t)std::max(cf.ns, cf.nu) * nrhs);
    cplx<T>* z = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
    const void* x = w;
    int64_t ldx = n;
    if (sizeof(T) != 8) {
      cplx<T>* wl = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
      to_low.push_back(AxpbyTask{wl, w, cf.ns, n, cf.ns, nrhs, 0});
      x = wl;
      ldx = cf.ns;
    }
    inv.push_back(HodbfInvItem<T>{&cf.f11, 0, x, ldx, z, cf.ns, nrhs});
    back.push_back(AxpbyTask{w, z, n, cf.ns, cf.ns, nrhs, 0});  // W(0:ns) = F11^-1 W(0:ns)
    if (cf.nu > 0) {
      BfCall cl;
      cl.bf = cf.f21.get();
      cl.x_off = cl.y_off = 0;
      cl.alpha_im = 0;
      cl.nrhs = nrhs;
      if (sizeof(T) == 8) {  // W(ns:n) -= F21 W(0:ns) in place
        cl.alpha_re = -1.0;
        cl.beta = 1;
        cl.x_abs = (int64_t)((uintptr_t)w / esz);
        cl.ldx = n;
        cl.y_abs = (int64_t)((uintptr_t)(w + cf.ns) / esz);
        cl.ldy = n;
      } else {  // t = F21 z, then W(ns:n) -= t in FP64
        cplx<T>* t = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.nu, 1) * nrhs * sizeof(cplx<T>));
        cl.alpha_re = 1.0;
        cl.beta = 0;
        cl.x_abs = (int64_t)((uintptr_t)z / esz);
        cl.ldx = cf.ns;
        cl.y_abs = (int64_t)((uintptr_t)t / esz);
        cl.ldy = cf.nu;
        upd.push_back(AxpbyTask{w + cf.ns, t, n, cf.nu, cf.nu, nrhs, 0});
      }
      calls.push_back(cl);
    }
  }
  if (!to_low.empty())
    ochk(launch_mix_batch<T, double>((const AxpbyTask*)up(rt, to_low), (int)to_low.size(), maxe, 1.0, 0.0, 0.0, s),
         "to c64");
  hodbf_inv_apply_many<T>(rt, inv, false);
  ochk(launch_mix_batch<double, T>((const AxpbyTask*)up(rt, back), (int)back.size(), maxe, 1.0, 0.0, 0.0, s),
       "copy back");
  if (!calls.empty()) rt.apply_calls(calls, false);
  if (!upd.empty())
    ochk(launch_mix_batch<double, T>((const AxpbyTask*)up(rt, upd), (int)upd.size(), maxe, -1.0, 1.0, 0.0, s),
         "update");
  rt.scratch.release(mk);
}

template <class T>
static void backward_level(CompState<T>& st, const std::vector<int>& fs, const std::vector<void*>& Ws,
                           const std::vector<int>& ns_, int nrhs) {
  BfRuntime<T>& rt = st.rt;
  hipStream_t s = rt.s();
  auto mk = rt.scratch.mark();
  const int64_t esz = (int64_t)sizeof(cplx<T>);
  std::vector<HodbfInvItem<T>> inv;
  std::vector<AxpbyTask> to_low, upd;
  std::vector<BfCall> calls;
  int64_t maxe = 0;
  for (size_t k = 0; k < fs.size(); ++k) {
    CompressedFront<T>& cf = *st.fronts[fs[k]];
    if (cf.nu == 0) continue;
    cplx<double>* w = (cplx<double>*)Ws[k];
    const int n = ns_[k];
    maxe = std::max<int64_t>(maxe, (int64_t)std::max(cf.ns, cf.nu) * nrhs);
    cplx<T>* t = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
    cplx<T>* t2 = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
    BfCall cl;
    cl.bf = cf.f12.get();
    cl.x_off = cl.y_off = 0;
    cl.alpha_re = 1.0;
    cl.alpha_im = 0;
    cl.beta = 0;
    cl.nrhs = nrhs;
    cl.y_abs = (int64_t)((uintptr_t)t / esz);
    cl.ldy = cf.ns;
    if (sizeof(T) == 8) {  // t = F12 W(ns:n)
      cl.x_abs = (int64_t)((uintptr_t)(w + cf.ns) / esz);
      cl.ldx = n;
    } else {  // u = W(ns:n) in complex64, t = F12 u
      cplx<T>* u = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.nu, 1) * nrhs * sizeof(cplx<T>));
      to_low.push_back(AxpbyTask{u, w + cf.ns, cf.nu, n, cf.nu, nrhs, 0});
      cl.x_abs = (int64_t)((uintptr_t)u / esz);
      cl.ldx = cf.nu;
    }
    calls.push_back(cl);
    inv.push_back(HodbfInvItem<T>{&cf.f11, 0, t, cf.ns, t2, cf.ns, nrhs});
    upd.push_back(AxpbyTask{w, t2, n, cf.ns, cf.ns, nrhs, 0});  // W(0:ns) -= F11^-1 t
  }
  if (calls.empty()) {
    rt.scratch.release(mk);
    return;
  }
  if (!to_low.empty())
    ochk(launch_mix_batch<T, double>((const AxpbyTask*)up(rt, to_low), (int)to_low.size(), maxe, 1.0, 0.0, 0.0, s),
         "to c64");
  rt.apply_calls(calls, false);
  hodbf_inv_apply_many<T>(rt, inv, false);
  ochk(launch_mix_batch<double, T>((const AxpbyTask*)up(rt, upd), (int)upd.size(), maxe, -1.0, 1.0, 0.0, s),
       "update");
  rt.scratch.release(mk);
}

void factor_compressed_level(void* state, Context& c, const std::vector<int>& fronts,
                             const std::vector<const FrontDesc*>& d_fds, const std::vector<void*>& cbs) {
  auto* h = (CompHolder*)state;
  if (h->single)
    factor_level<float>(h->f.get(), c, fronts, d_fds, cbs);
  else
    factor_level<double>(h->d.get(), c, fronts, d_fds, cbs);
}

void forward_compressed(void* state, Context& c, int f, void* W, int n, int nrhs) {
  auto* h = (CompHolder*)state;
  (void)c;
  if (h->single)
    forward_front<float>(*h->f, f, W, n, nrhs);
  else
    forward_front<double>(*h->d, f, W, n, nrhs);
}

void backward_compressed(void* state, Context& c, int f, void* W, int n, int nrhs) {
  auto* h = (CompHolder*)state;
  (void)c;
  if (h->single)
    backward_front<float>(*h->f, f, W, n, nrhs);
  else
    backward_front<double>(*h->d, f, W, n, nrhs);
}

void forward_compressed_level(void* state, Context& c, const std::vector<int>& fs, const std::vector<void*>& Ws,
                              const std::vector<int>& ns, int nrhs) {
  auto* h = (CompHolder*)state;
  (void)c;
  if (h->single)
    forward_level<float>(*h->f, fs, Ws, ns, nrhs);
  else
    forward_level<double>(*h->d, fs, Ws, ns, nrhs);
}

void backward_compressed_level(void* state, Context& c, const std::vector<int>& fs, const std::vector<void*>& Ws,
                               const std::vector<int>& ns, int nrhs) {
  auto* h = (CompHolder*)state;
  (void)c;
  if (h->single)
    backward_level<float>(*h->f, fs, Ws, ns, nrhs);
  else
    backward_level<double>(*h->d, fs, Ws, ns, nrhs);
}

// Y = B X for one block of a compressed front (debug access): 0 F11, 1 F11^-1,
// 2 F12, 3 F21, 4 S.  X and Y are host arrays of interleaved complex128.
template <class T>
static void apply_block(CompState<T>& st, int f, int what, int nrhs, const double* X, int64_t ldx, double* Y,
                        int64_t ldy) {
  BfRuntime<T>& rt = st.rt;
  if (f < 0 || f >= (int)st.fronts.size() || !st.fronts[f]) throw Error(BFMF_E_INVAL, "front is not compressed");
  CompressedFront<T>& cf = *st.fronts[f];
  const int ns = cf.ns, nu = cf.nu;
  const int rows = (what <= 2) ? ns : nu, cols = (what == 0 || what == 1 || what == 3) ? ns : nu;
  if (what < 0 || what > 5) throw Error(BFMF_E_INVAL, "apply_front_block: bad 'what'");
  if (what >= 2 && nu == 0) throw Error(BFMF_E_INVAL, "apply_front_block: the front has no update set");
  if (what == 5 && !cf.cb_dev)
    throw Error(BFMF_E_INVAL, "apply_front_block: the contribution block is not in HOD-BF form");
  if (nrhs <= 0 || ldx < cols || ldy < rows || !X || !Y) throw Error(BFMF_E_INVAL, "apply_front_block: bad arguments");
  hipStream_t s = rt.s();
  std::vector<cplx<T>> hx((size_t)cols * nrhs), hy((size_t)rows * nrhs);
  for (int j = 0; j < nrhs; ++j)
    for (int i = 0; i < cols; ++i) {
      const double* p = X + 2 * ((size_t)j * ldx + i);
      hx[(size_t)j * cols + i] = cplx<T>{(T)p[0], (T)p[1]};
    }
  auto mk = rt.scratch.mark();
  cplx<T>* dx = (cplx<T>*)rt.scratch.take(hx.size() * sizeof(cplx<T>));
  cplx<T>* dy = (cplx<T>*)rt.scratch.take(hy.size() * sizeof(cplx<T>));
  ochk(hipMemcpyAsync(dx, hx.data(), hx.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s), "upload");
  switch (what) {
    case 0: hodbf_apply<T>(rt, cf.f11, dx, cols, dy, rows, nrhs); break;
    case 1: hodbf_inv_apply<T>(rt, cf.f11, 0, dx, cols, dy, rows, nrhs, false); break;
    case 2: rt.apply(*cf.f12, dx, cols, dy, rows, nrhs, false, 1.0, 0); break;
    case 3: rt.apply(*cf.f21, dx, cols, dy, rows, nrhs, false, 1.0, 0); break;
    case 5: hodbf_apply<T>(rt, cf.cbh, dx, cols, dy, rows, nrhs); break;
    default: rt.apply(*cf.s, dx, cols, dy, rows, nrhs, false, 1.0, 0); break;
  }
  ochk(hipMemcpyAsync(hy.data(), dy, hy.size() * sizeof(cplx<T>), hipMemcpyDeviceToHost, s), "download");
  ochk(hipStreamSynchronize(s), "sync");
  rt.scratch.release(mk);
  for (int j = 0; j < nrhs; ++j)
    for (int i = 0; i < rows; ++i) {
      double* p = Y + 2 * ((size_t)j * ldy + i);
      p[0] = (double)hy[(size_t)j * rows + i].re;
      p[1] = (double)hy[(size_t)j * rows + i].im;
    }
}

// Entries of the never-formed front f (A entries (+) the children's contribution blocks, the list
// routing of the compressed fronts' entry evaluation): out(i, j) = F(rows[i], cols[j]), host arrays.
void extract_front_entries(Context& c, int f, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols,
                           double* out, int64_t ldo) {
  BfRuntime<double> rt;
  rt.c = &c;
  const size_t nr = rows.size(), nc = cols.size();
  void* d_out = rt.scratch.take(std::max<size_t>(nr * nc, 1) * sizeof(cplx<double>));
  const FrontDesc* dfd = c.d_fds.as<FrontDesc>() + c.desc_index[f];
  ExtractBatch eb;
  eb.add(dfd, nullptr, 0, rows, 0, cols, 0, d_out, (int64_t)std::max<size_t>(nr, 1), false);
  run_extract_to<double, double>(rt, eb, false);
  std::vector<cplx<double>> h(nr * nc);
  ochk(hipMemcpyAsync(h.data(), d_out, nr * nc * sizeof(cplx<double>), hipMemcpyDeviceToHost, c.stream), "download");
  ochk(hipStreamSynchronize(c.stream), "sync");
  for (size_t j = 0; j < nc; ++j)
    for (size_t i = 0; i < nr; ++i) {
      out[2 * (i + j * ldo)] = h[i + j * nr].re;
      out[2 * (i + j * ldo) + 1] = h[i + j * nr].im;
    }
}

void comp_apply_block(void* state, int f, int what, int nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy) {
  auto* h = (CompHolder*)state;
  if (!h) throw Error(BFMF_E_INVAL, "no compressed fronts");
  if (h->single)
    apply_block<float>(*h->f, f, what, nrhs, X, ldx, Y, ldy);
  else
    apply_block<double>(*h->d, f, what, nrhs, X, ldx, Y, ldy);
}

template <class T>
static uint64_t state_bytes(const CompState<T>& st) {
  uint64_t b = st.rt.pool.buf.bytes + st.status.bytes + st.cbuf_held;
  for (auto& ch : st.rt.scratch.chunks) b += ch->b.bytes;
  return b;
}

uint64_t comp_state_bytes(void* state) {
  auto* h = (CompHolder*)state;
  if (!h) return 0;
  return (h->d ? state_bytes(*h->d) : 0) + (h->f ? state_bytes(*h->f) : 0);
}

void compressed_stats(void* state, double& bytes, int& maxrank, int& chunked) {
  auto* h = (CompHolder*)state;
  // the factors: the pool less the contribution blocks kept in it
  if (h->single) {
    bytes = (double)h->f->rt.pool.used - h->f->cb_bytes;
    maxrank = h->f->rt.max_rank_seen;
    chunked = (int)h->f->rt.n_chunked;
  } else {
    bytes = (double)h->d->rt.pool.used - h->d->cb_bytes;
    maxrank = h->d->rt.max_rank_seen;
    chunked = (int)h->d->rt.n_chunked;
  }
}

void compressed_cb_stats(void* state, double& bytes, double& dense_bytes, int& count, uint64_t& centre_peak) {
  auto* h = (CompHolder*)state;
  bytes = dense_bytes = 0;
  count = 0;
  centre_peak = 0;
  if (!h) return;
  auto get = [&](auto& st) {
    bytes = st.cb_bytes;
    dense_bytes = st.cb_dense_bytes;
    count = st.cb_count;
    centre_peak = st.cbuf_peak;
  };
  if (h->single && h->f) get(*h->f);
  if (!h->single && h->d) get(*h->d);
}

uint64_t comp_centre_held(void* state) {
  auto* h = (CompHolder*)state;
  if (!h) return 0;
  if (h->single) return h->f ? h->f->cbuf_held : 0;
  return h->d ? h->d->cbuf_held : 0;
}

const HodbfDev* comp_cb_dev(void* state, int f) {
  auto* h = (CompHolder*)state;
  if (!h) return nullptr;
  if (h->single) {
    if (!h->f || f < 0 || f >= (int)h->f->fronts.size() || !h->f->fronts[f]) return nullptr;
    return h->f->fronts[f]->cb_dev;
  }
  if (!h->d || f < 0 || f >= (int)h->d->fronts.size() || !h->d->fronts[f]) return nullptr;
  return h->d->fronts[f]->cb_dev;
}

}  // namespace bfmf
