// Compressed fronts (paper Alg. 5): HOD-BF F11 and its inverse (Alg. 4 with
// BF_SMW), butterfly F12 / F21 by entry evaluation with graph-distance
// proxies (Alg. 2, Sec. 5.2), the Schur update S by randomized construction
// (Sec. 3.3), the contribution block, and the compressed sweeps.
#include "compressed.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <random>

#include "kernels/kernels.hpp"

namespace bfmf {

namespace {

template <class V>
void* up(Scratch& sc, const std::vector<V>& v, hipStream_t s) {
  void* d = sc.take(std::max<size_t>(v.size() * sizeof(V), 16));
  if (!v.empty()) ochk(hipMemcpyAsync(d, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, s), "upload");
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
  BfRuntime<T>& rt;
  const FrontDesc* d_fd;
  const void* values;
  int row0, col0;
  FrontSource(BfRuntime<T>& r, const FrontDesc* fd, const void* vals, int r0, int c0)
      : rt(r), d_fd(fd), values(vals), row0(r0), col0(c0) {}
  void extract(const std::vector<const std::vector<int32_t>*>& rows, const std::vector<const std::vector<int32_t>*>& cols,
               const std::vector<void*>& outs, const std::vector<int64_t>& ldo, bool trans) override {
    const size_t nb = rows.size();
    std::vector<int32_t> idx;
    std::vector<int64_t> ro(nb), co(nb);
    for (size_t i = 0; i < nb; ++i) {
      ro[i] = (int64_t)idx.size();
      for (int32_t r : *rows[i]) idx.push_back(row0 + r);
      co[i] = (int64_t)idx.size();
      for (int32_t c : *cols[i]) idx.push_back(col0 + c);
    }
    auto mk = rt.scratch.mark();
    int32_t* d_idx = (int32_t*)up(rt.scratch, idx, rt.s());
    std::vector<ExtractTask> tk(nb);
    for (size_t i = 0; i < nb; ++i) {
      ExtractTask& e = tk[i];
      std::memset(&e, 0, sizeof(e));
      e.rows = d_idx + ro[i];
      e.cols = d_idx + co[i];
      e.nr = (int32_t)rows[i]->size();
      e.nc = (int32_t)cols[i]->size();
      e.out = outs[i];
      e.ldo = ldo[i];
      e.trans = trans ? 1 : 0;
    }
    ExtractTask* d_tk = (ExtractTask*)up(rt.scratch, tk, rt.s());
    ochk(launch_front_extract<T>(d_tk, (int)nb, 8, d_fd, values, sizeof(T) == 4, rt.s()), "front extract");
    ochk(hipStreamSynchronize(rt.s()), "front extract");
    rt.scratch.release(mk);
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
    out.clear();
    const int n = end - beg;
    if (n <= 0) return;
    const int cap = 2048;
    const int k = std::min(n, std::max(8, (int)(alpha * (double)given.size())));
    std::vector<char> mark(n, 0);
    int cnt = 0;
    // nearest neighbours first
    for (int32_t gi : given) {
      int found = 0;
      for (int32_t v : near[given0 + gi]) {
        const int p = v - node0;
        if (p >= beg && p < end) {
          if (!mark[p - beg] && cnt < cap) {
            mark[p - beg] = 1;
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
        ++cnt;
      }
    }
    for (int i = 0; i < n; ++i)
      if (mark[i]) out.push_back(beg + i);
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
};

// blocks up to this size are inverted densely inside BF_SMW
constexpr int kSmwDense = 512;

struct SmwResult {
  std::unique_ptr<Butterfly> bf;
  int64_t dense_off = -1;
  bool zero = false;
};

}  // namespace

// ------------------------------------------------------------ HOD-BF products
template <class T>
void hodbf_apply(BfRuntime<T>& rt, const Hodbf<T>& h, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs) {
  const char* pool = rt.pool_base();
  // leaves: y = D x
  for (const auto& nd : h.nodes)
    if (nd.left < 0)
      gemm<T>(rt, pool + nd.leaf_off * sizeof(cplx<T>), nd.size(), OP_N, (const cplx<T>*)X + nd.beg, ldx, OP_N,
              (cplx<T>*)Y + nd.beg, ldy, nd.size(), nrhs, nd.size(), 1.0, 0, 0);
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

template <class T>
void hodbf_inv_apply(BfRuntime<T>& rt, const Hodbf<T>& h, int node, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     int nrhs, bool adjoint) {
  const HodbfNode<T>& root = h.nodes[node];
  const int base = root.beg, n = root.size();
  // nodes of the subtree grouped by level
  std::vector<std::vector<int>> lv(h.max_level + 1);
  std::vector<int> st{node};
  while (!st.empty()) {
    int i = st.back();
    st.pop_back();
    lv[h.nodes[i].level].push_back(i);
    if (h.nodes[i].left >= 0) {
      st.push_back(h.nodes[i].left);
      st.push_back(h.nodes[i].right);
    }
  }
  const char* pool = rt.pool_base();
  cplx<T>* y = (cplx<T>*)Y;
  const cplx<T>* x = (const cplx<T>*)X;
  auto mk = rt.scratch.mark();
  cplx<T>* tmp = (cplx<T>*)rt.scratch.take((size_t)std::max(n, 1) * nrhs * sizeof(cplx<T>));
  auto leaves = [&](const cplx<T>* src, int64_t lds) {
    for (int l = 0; l <= h.max_level; ++l)
      for (int i : lv[l]) {
        const auto& nd = h.nodes[i];
        if (nd.left >= 0) continue;
        gemm<T>(rt, pool + nd.inv_off * sizeof(cplx<T>), nd.size(), adjoint ? OP_C : OP_N, src + (nd.beg - base), lds,
                OP_N, y + (nd.beg - base), ldy, nd.size(), nrhs, nd.size(), 1.0, 0, 0);
      }
  };
  auto level_update = [&](int l) {  // y_t += X_t^(H) y_t for internal nodes of level l
    std::vector<BfCall> calls;
    for (int i : lv[l]) {
      const auto& nd = h.nodes[i];
      if (nd.left < 0 || nd.x_zero) continue;
      if (nd.x_dense) {
        gemm<T>(rt, pool + nd.inv_off * sizeof(cplx<T>), nd.size(), adjoint ? OP_C : OP_N, y + (nd.beg - base), ldy,
                OP_N, tmp + (nd.beg - base), n, nd.size(), nrhs, nd.size(), 1.0, 0, 0);
      } else {
        calls.push_back(BfCall{nd.x.get(), nd.beg - base, nd.beg - base, 1.0, 0.0, 0});
      }
    }
    if (!calls.empty()) rt.apply_set(calls, y, ldy, tmp, n, nrhs, adjoint);
    for (int i : lv[l]) {
      const auto& nd = h.nodes[i];
      if (nd.left < 0 || nd.x_zero) continue;
      axpby<T>(rt, y + (nd.beg - base), ldy, tmp + (nd.beg - base), n, nd.size(), nrhs, 1.0, 1.0);
    }
  };
  if (!adjoint) {
    leaves(x, ldx);
    for (int l = h.max_level; l >= root.level; --l) level_update(l);
  } else {
    axpby<T>(rt, y, ldy, x, ldx, n, nrhs, 1.0, 0.0);
    for (int l = root.level; l <= h.max_level; ++l) level_update(l);
    // leaves: y_leaf = Dinv^H y_leaf (through tmp)
    axpby<T>(rt, tmp, n, y, ldy, n, nrhs, 1.0, 0.0);
    leaves(tmp, n);
  }
  rt.scratch.release(mk);
}

template void hodbf_apply<double>(BfRuntime<double>&, const Hodbf<double>&, const void*, int64_t, void*, int64_t, int);
template void hodbf_inv_apply<double>(BfRuntime<double>&, const Hodbf<double>&, int, const void*, int64_t, void*,
                                      int64_t, int, bool);

// ------------------------------------------------------------ BF_SMW
namespace {

template <class T>
SmwResult bf_smw(BfRuntime<T>& rt, const std::vector<TreeNode>& nodes, int node, Op<T>* K11, Op<T>* K12, Op<T>* K21,
                 Op<T>* K22, Op<T>* Kfull) {
  SmwResult res;
  const TreeNode& nd = nodes[node];
  const int n = nd.end - nd.beg;
  const int d = depth_of(nodes, node);
  hipStream_t s = rt.s();
  if (d == 0 || n <= kSmwDense) {
    // dense: M = I + K, X = M^-1 - I.  M^-1 is the Schur complement of the
    // bordered front [M I; -I 0] (partial LU with pivoting inside M).
    const size_t off = rt.pool.alloc((size_t)n * n * sizeof(cplx<T>), s);
    const int64_t eoff = (int64_t)(off / sizeof(cplx<T>));
    auto mk = rt.scratch.mark();
    const int N2 = 2 * n;
    cplx<T>* F = (cplx<T>*)rt.scratch.take((size_t)N2 * N2 * sizeof(cplx<T>));
    std::vector<cplx<T>> border((size_t)N2 * N2, cplx<T>{0, 0});
    for (int i = 0; i < n; ++i) {
      border[(size_t)i * N2 + i] = cplx<T>{1, 0};                  // M = I + K: identity part
      border[(size_t)(n + i) * N2 + i] = cplx<T>{1, 0};            // F12 = I
      border[(size_t)i * N2 + n + i] = cplx<T>{-1, 0};             // F21 = -I
    }
    ochk(hipMemcpyAsync(F, border.data(), border.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s), "border");
    // a separate identity (F12 is overwritten by the factorization)
    cplx<T>* I = (cplx<T>*)rt.scratch.take((size_t)n * n * sizeof(cplx<T>));
    ochk(launch_axpby<T>(I, n, F + (size_t)n * N2, N2, n, n, 1.0, 0.0, s), "identity");
    Kfull->apply(I, n, F, N2, n, false, 1.0, 1);                  // F11 = I + K
    int32_t* piv = (int32_t*)rt.scratch.take((size_t)n * sizeof(int32_t));
    int* dst = (int*)rt.scratch.take(16);
    ochk(hipMemsetAsync(dst, 0, 16, s), "status");
    FrontDesc fd;
    std::memset(&fd, 0, sizeof(fd));
    fd.F = F;
    fd.n = N2;
    fd.ns = n;
    fd.front = -1;
    fd.piv = piv;
    void* d_fd = up(rt.scratch, std::vector<FrontDesc>{fd}, s);
    const int hn = N2, hns = n;
    ochk(launch_partial_lu<T>((const FrontDesc*)d_fd, 1, &hn, &hns, dst, s), "smw dense lu");
    ochk(launch_schur<T>((const FrontDesc*)d_fd, 1, &hn, &hns, s), "smw dense schur");
    cplx<T>* X = (cplx<T>*)(rt.pool_base() + off);
    cplx<T>* C = F + n + (size_t)n * N2;  // M^-1
    ochk(launch_axpby<T>(X, n, C, N2, n, n, 1.0, 0.0, s), "copy");
    ochk(launch_axpby<T>(X, n, I, n, n, n, -1.0, 1.0, s), "minus identity");
    int hst[3] = {0, 0, 0};
    ochk(hipMemcpyAsync(hst, dst, 12, hipMemcpyDeviceToHost, s), "status");
    ochk(hipStreamSynchronize(s), "smw dense");
    rt.scratch.release(mk);
    if (hst[0]) throw Error(BFMF_E_SINGULAR, "singular block in the HOD-BF inversion");
    res.dense_off = eoff;
    return res;
  }
  const int c1 = nd.left, c2 = nd.right;
  const int n1 = nodes[c1].end - nodes[c1].beg, n2 = n - n1;
  std::vector<std::unique_ptr<Op<T>>> keep;
  auto sub = [&](Op<T>* op, int r0, int cc0, int m, int nn) -> Op<T>* {
    keep.push_back(std::make_unique<SubOp<T>>(rt, op, r0, cc0, m, nn));
    return keep.back().get();
  };
  // children blocks of a general butterfly come from views of the full operator
  Op<T>* k11 = K11;
  Op<T>* k12 = K12;
  Op<T>* k21 = K21;
  Op<T>* k22 = K22;
  // X22: (I + K22)^-1 = I + X22
  SmwResult x22;
  if (k22) {
    // recursive call on the children of c2 uses views of K22
    const int c21 = nodes[c2].left;
    if (c21 >= 0) {
      const int m1 = nodes[c21].end - nodes[c21].beg, m2 = n2 - m1;
      x22 = bf_smw<T>(rt, nodes, c2, sub(k22, 0, 0, m1, m1), sub(k22, 0, m1, m1, m2), sub(k22, m1, 0, m2, m1),
                      sub(k22, m1, m1, m2, m2), k22);
    } else {
      x22 = bf_smw<T>(rt, nodes, c2, nullptr, nullptr, nullptr, nullptr, k22);
    }
  } else {
    x22.zero = true;
  }
  IPlusX<T> A22i(rt, n2, x22.bf.get(), x22.zero ? -1 : x22.dense_off);
  // S11 = K11 - K12 A22i K21 over T1 x T1
  ProductOp<T> a22k21(rt, &A22i, k21);
  ProductOp<T> k12a22k21(rt, k12, &a22k21);
  SumOp<T> s11op(rt, n1, n1);
  if (k11) s11op.add(k11, 1.0);
  s11op.add(&k12a22k21, -1.0);
  const int L11 = std::max(0, d - 2);  // children butterflies of L - 2 levels (Alg. 4)
  BTree t1 = subtree(nodes, c1, L11);
  auto s11 = bf_random_matvec<T>(rt, s11op, t1, t1);
  BfOp<T> s11b(rt, s11.get());
  SmwResult x11;
  const int c11 = nodes[c1].left;
  if (c11 >= 0) {
    const int m1 = nodes[c11].end - nodes[c11].beg, m2 = n1 - m1;
    x11 = bf_smw<T>(rt, nodes, c1, sub(&s11b, 0, 0, m1, m1), sub(&s11b, 0, m1, m1, m2), sub(&s11b, m1, 0, m2, m1),
                    sub(&s11b, m1, m1, m2, m2), &s11b);
  } else {
    x11 = bf_smw<T>(rt, nodes, c1, nullptr, nullptr, nullptr, nullptr, &s11b);
  }
  IPlusX<T> A11i(rt, n1, x11.bf.get(), x11.zero ? -1 : x11.dense_off);
  SmwOp<T> aop(rt, n1, n2, k12, k21, &A11i, &A22i);
  BTree tt = subtree(nodes, node, d);
  res.bf = bf_random_matvec<T>(rt, aop, tt, tt);
  return res;
}

}  // namespace

// ------------------------------------------------------------ front driver
template <class T>
struct CompState {
  BfRuntime<T> rt;
  std::vector<std::unique_ptr<CompressedFront<T>>> fronts;  // by front id (null if dense)
};

template struct CompState<double>;

void* comp_state_create(Context& c) {
  auto* st = new CompState<double>();
  st->rt.c = &c;
  return st;
}

void comp_state_destroy(void* p) { delete (CompState<double>*)p; }

void comp_state_reset(void* p, Context& c, int nfronts) {
  auto* st = (CompState<double>*)p;
  st->fronts.clear();
  st->fronts.resize(nfronts);
  st->rt.c = &c;
  st->rt.pool.reset();
  st->rt.tol = c.fopts.tol;
  st->rt.samples = c.fopts.samples > 0 ? c.fopts.samples : 64;
  st->rt.seed = c.fopts.seed;
  st->rt.stream_id = 0;
  st->rt.max_rank_seen = 0;
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

// Compressed factorization of front f (its descriptor at d_fd on the device).
// The contribution block goes to `cb` (nu x nu, ld nu).
void factor_compressed_front(void* state, Context& c, int f, const FrontDesc* d_fd, void* cb) {
  typedef double T;
  auto* st = (CompState<T>*)state;
  BfRuntime<T>& rt = st->rt;
  const Symbolic& sy = c.sym;
  auto cf = std::make_unique<CompressedFront<T>>();
  cf->front = f;
  cf->ns = (int)sy.ns(f);
  cf->nu = (int)sy.nu(f);
  const int ns = cf->ns, nu = cf->nu;
  hipStream_t s = rt.s();
  auto clock = [] { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); };
  double tph[6] = {clock(), 0, 0, 0, 0, 0};
  const int64_t r0 = rt.n_random, e0 = rt.n_entry;
  // HOD-BF tree of F11: the separator bisection (P-hat), Sec. 5.1
  std::vector<TreeNode> nodes(sy.sep_nodes.begin() + sy.sep_ptr[f], sy.sep_nodes.begin() + sy.sep_ptr[f + 1]);
  Hodbf<T>& h = cf->f11;
  h.n = ns;
  h.nodes.resize(nodes.size());
  {
    std::vector<std::pair<int, int>> stck{{0, 0}};
    while (!stck.empty()) {
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
  std::vector<std::vector<int32_t>> near11, nearall;
  bfs_lists(c, f, ns, 32, near11);
  bfs_lists(c, f, ns + nu, 32, nearall);
  const uint64_t seed = c.fopts.seed * 1000003ull + (uint64_t)f;
  const double alpha = c.fopts.alpha > 0 ? c.fopts.alpha : 2.0;
  const int knn = c.fopts.knn;
  // leaves D = F11(leaf, leaf)
  {
    std::vector<std::vector<int32_t>> idx;
    std::vector<int> leaves;
    for (int i = 0; i < (int)h.nodes.size(); ++i)
      if (h.nodes[i].left < 0) {
        leaves.push_back(i);
        const size_t off = rt.pool.alloc((size_t)h.nodes[i].size() * h.nodes[i].size() * sizeof(cplx<T>), s);
        h.nodes[i].leaf_off = (int64_t)(off / sizeof(cplx<T>));
        std::vector<int32_t> r(h.nodes[i].size());
        for (int k = 0; k < h.nodes[i].size(); ++k) r[k] = h.nodes[i].beg + k;
        idx.push_back(r);
      }
    std::vector<const std::vector<int32_t>*> pr;
    std::vector<void*> outs;
    std::vector<int64_t> ldo;
    for (size_t k = 0; k < leaves.size(); ++k) {
      pr.push_back(&idx[k]);
      outs.push_back(rt.pool_base() + h.nodes[leaves[k]].leaf_off * sizeof(cplx<T>));
      ldo.push_back(std::max(1, h.nodes[leaves[k]].size()));
    }
    FrontSource<T> src(rt, d_fd, c.d_values.p, 0, 0);
    src.extract(pr, pr, outs, ldo, false);
  }
  // off-diagonal butterflies (Alg. 2 on F11 = A(Is,Is) (+) C_nu1 (+) C_nu2)
  for (int i = 0; i < (int)h.nodes.size(); ++i) {
    auto& nd = h.nodes[i];
    if (nd.left < 0) continue;
    const int a = nd.left, b = nd.right;
    const int L = std::min(depth_of(nodes, a), depth_of(nodes, b));
    BTree ta = subtree(nodes, a, L), tb = subtree(nodes, b, L);
    {
      FrontSource<T> src(rt, d_fd, c.d_values.p, nodes[a].beg, nodes[b].beg);
      BfsSampler ps(near11, nodes[a].beg, nodes[b].beg, knn, alpha, seed + 2 * i);
      nd.b12 = bf_entry_eval<T>(rt, src, ps, ta, tb);
    }
    {
      FrontSource<T> src(rt, d_fd, c.d_values.p, nodes[b].beg, nodes[a].beg);
      BfsSampler ps(near11, nodes[b].beg, nodes[a].beg, knn, alpha, seed + 2 * i + 1);
      nd.b21 = bf_entry_eval<T>(rt, src, ps, tb, ta);
    }
  }
  tph[1] = clock();
  // HODBF_invert (Alg. 4): leaves, then every internal node bottom-up
  {
    std::vector<InvTask> it;
    for (auto& nd : h.nodes)
      if (nd.left < 0) {
        const size_t off = rt.pool.alloc((size_t)nd.size() * nd.size() * sizeof(cplx<T>), s);
        nd.inv_off = (int64_t)(off / sizeof(cplx<T>));
      }
    for (auto& nd : h.nodes)
      if (nd.left < 0) {
        ochk(hipMemcpyAsync(rt.pool_base() + nd.inv_off * sizeof(cplx<T>), rt.pool_base() + nd.leaf_off * sizeof(cplx<T>),
                            (size_t)nd.size() * nd.size() * sizeof(cplx<T>), hipMemcpyDeviceToDevice, s),
             "leaf copy");
        it.push_back(InvTask{rt.pool_base() + nd.inv_off * sizeof(cplx<T>), std::max(nd.size(), 1), nd.size(), 0});
      }
    auto mk = rt.scratch.mark();
    void* d_it = up(rt.scratch, it, s);
    int* d_st = (int*)rt.scratch.take(16);
    ochk(hipMemsetAsync(d_st, 0, 16, s), "status");
    ochk(launch_leaf_inverse<T>(d_it, (int)it.size(), d_st, s), "leaf inverse");
    int hst = 0;
    ochk(hipMemcpyAsync(&hst, d_st, 4, hipMemcpyDeviceToHost, s), "status");
    ochk(hipStreamSynchronize(s), "leaf inverse");
    rt.scratch.release(mk);
    if (hst) throw Error(BFMF_E_SINGULAR, "singular HOD-BF leaf in compressed front " + std::to_string(f));
  }
  for (int l = h.max_level; l >= 0; --l)
    for (int i : h.by_level[l]) {
      auto& nd = h.nodes[i];
      if (nd.left < 0) continue;
      const int a = nd.left, b = nd.right;
      const int na = h.nodes[a].size(), nb = h.nodes[b].size();
      // B1' = D1^-1 B12, B2' = D2^-1 B21 by randomized construction
      HodbfInvOp<T> d1(rt, h, a), d2(rt, h, b);
      BfOp<T> b12(rt, nd.b12.get()), b21(rt, nd.b21.get());
      ProductOp<T> p1(rt, &d1, &b12), p2(rt, &d2, &b21);
      auto b1p = bf_random_matvec<T>(rt, p1, nd.b12->to, nd.b12->ts);
      auto b2p = bf_random_matvec<T>(rt, p2, nd.b21->to, nd.b21->ts);
      BfOp<T> k12(rt, b1p.get()), k21(rt, b2p.get());
      // [I B1'; B2' I]^-1 = I + X (BF_SMW with zero diagonal blocks)
      Block2Op<T> kfull(rt, na + nb, na + nb, na, na, nullptr, &k12, &k21, nullptr);
      SmwResult r = bf_smw<T>(rt, nodes, i, nullptr, &k12, &k21, nullptr, &kfull);
      nd.x = std::move(r.bf);
      nd.x_dense = r.dense_off >= 0;
      if (nd.x_dense) nd.inv_off = r.dense_off;
      nd.x_zero = r.zero;
    }
  tph[2] = clock();
  if (nu > 0) {
    // F12 and F21 (Alg. 2), trees: separator bisection x balanced tree on I^u
    const int leaf = 64;
    std::vector<TreeNode> unodes = balanced_tree(nu, leaf);
    const int Ls = depth_of(nodes, 0), Lu = depth_of(unodes, 0);
    const int L = std::min(Ls, Lu);
    BTree ts_ = subtree(nodes, 0, L), tu = subtree(unodes, 0, L);
    {
      FrontSource<T> src(rt, d_fd, c.d_values.p, 0, ns);
      BfsSampler ps(nearall, 0, ns, knn, alpha, seed + 7777);
      cf->f12 = bf_entry_eval<T>(rt, src, ps, ts_, tu);
    }
    {
      FrontSource<T> src(rt, d_fd, c.d_values.p, ns, 0);
      BfsSampler ps(nearall, ns, 0, knn, alpha, seed + 8888);
      cf->f21 = bf_entry_eval<T>(rt, src, ps, tu, ts_);
    }
    tph[3] = clock();
    // S = F21 F11^-1 F12 (Sec. 3.3)
    HodbfInvOp<T> f11i(rt, h, 0);
    BfOp<T> f12(rt, cf->f12.get()), f21(rt, cf->f21.get());
    ProductOp<T> p1(rt, &f11i, &f12), p2(rt, &f21, &p1);
    BTree tuu = subtree(unodes, 0, Lu);
    cf->s = bf_random_matvec<T>(rt, p2, tuu, tuu);
    tph[4] = clock();
    // C = (C_nu1 (+) C_nu2)(Iu, Iu) - S
    {
      std::vector<int32_t> r(nu);
      for (int k = 0; k < nu; ++k) r[k] = k;
      FrontSource<T> src(rt, d_fd, c.d_values.p, ns, ns);
      src.extract({&r}, {&r}, {cb}, {std::max(nu, 1)}, false);
      const int chunk = 1024;
      auto mk = rt.scratch.mark();
      cplx<T>* I = (cplx<T>*)rt.scratch.take((size_t)nu * chunk * sizeof(cplx<T>));
      for (int c0 = 0; c0 < nu; c0 += chunk) {
        const int w = std::min(chunk, nu - c0);
        std::vector<cplx<T>> eye((size_t)nu * w, cplx<T>{0, 0});
        for (int k = 0; k < w; ++k) eye[(size_t)k * nu + c0 + k] = cplx<T>{1, 0};
        ochk(hipMemcpyAsync(I, eye.data(), eye.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s), "eye");
        rt.apply(*cf->s, I, nu, (cplx<T>*)cb + (size_t)c0 * nu, nu, w, false, -1.0, 1);
      }
      ochk(hipStreamSynchronize(s), "cb");
      rt.scratch.release(mk);
    }
  }
  tph[5] = clock();
  if (c.verbose) {
    const double t3 = tph[3] > 0 ? tph[3] : tph[2], t4 = tph[4] > 0 ? tph[4] : t3;
    fprintf(stderr,
            "[bfmf] front %d ns %d nu %d: F11 %.3fs inv %.3fs F12/F21 %.3fs S %.3fs C %.3fs; constructions "
            "random %lld entry %lld; max rank %d\n",
            f, ns, nu, tph[1] - tph[0], tph[2] - tph[1], t3 - tph[2], t4 - t3, tph[5] - t4,
            (long long)(rt.n_random - r0), (long long)(rt.n_entry - e0), rt.max_rank_seen);
  }
  st->fronts[f] = std::move(cf);
}

// ------------------------------------------------------------ sweeps
// forward: W(0:ns) <- F11^-1 W(0:ns); W(ns:n) -= F21 W(0:ns)
void forward_compressed(void* state, Context& c, int f, void* W, int n, int nrhs) {
  typedef double T;
  auto* st = (CompState<T>*)state;
  BfRuntime<T>& rt = st->rt;
  CompressedFront<T>& cf = *st->fronts[f];
  cplx<T>* w = (cplx<T>*)W;
  auto mk = rt.scratch.mark();
  cplx<T>* z = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
  hodbf_inv_apply<T>(rt, cf.f11, 0, w, n, z, cf.ns, nrhs, false);
  axpby<T>(rt, w, n, z, cf.ns, cf.ns, nrhs, 1.0, 0.0);
  if (cf.nu > 0) rt.apply(*cf.f21, w, n, w + cf.ns, n, nrhs, false, -1.0, 1);
  ochk(hipStreamSynchronize(rt.s()), "forward compressed");
  rt.scratch.release(mk);
  (void)c;
}

// backward: W(0:ns) -= F11^-1 F12 W(ns:n)   (W(ns:n) already holds x(I^u))
void backward_compressed(void* state, Context& c, int f, void* W, int n, int nrhs) {
  typedef double T;
  auto* st = (CompState<T>*)state;
  BfRuntime<T>& rt = st->rt;
  CompressedFront<T>& cf = *st->fronts[f];
  cplx<T>* w = (cplx<T>*)W;
  if (cf.nu == 0) return;
  auto mk = rt.scratch.mark();
  cplx<T>* t = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
  cplx<T>* t2 = (cplx<T>*)rt.scratch.take((size_t)std::max(cf.ns, 1) * nrhs * sizeof(cplx<T>));
  rt.apply(*cf.f12, w + cf.ns, n, t, cf.ns, nrhs, false, 1.0, 0);
  hodbf_inv_apply<T>(rt, cf.f11, 0, t, cf.ns, t2, cf.ns, nrhs, false);
  axpby<T>(rt, w, n, t2, cf.ns, cf.ns, nrhs, -1.0, 1.0);
  ochk(hipStreamSynchronize(rt.s()), "backward compressed");
  rt.scratch.release(mk);
  (void)c;
}

void compressed_stats(void* state, double& bytes, int& maxrank) {
  auto* st = (CompState<double>*)state;
  bytes = (double)st->rt.pool.used;
  maxrank = st->rt.max_rank_seen;
}

}  // namespace bfmf
