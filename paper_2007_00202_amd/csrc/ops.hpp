// Linear operators on device vectors used by the randomized constructions
// and the HOD-BF inversion (paper Sec. 3.3, Sec. 4.2): dense blocks,
// butterflies, and products / sums / block arrangements of operators.
#pragma once
#include <memory>
#include <typeinfo>
#include <utility>
#include <vector>

#include "bf.hpp"
#include "kernels/kernels.hpp"

namespace bfmf {

inline void ochk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(BFMF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// C = beta C + alpha op(A) op(B) as a one-task grouped GEMM
template <class T>
void gemm(BfRuntime<T>& rt, const void* A, int64_t lda, int opA, const void* B, int64_t ldb, int opB, void* C,
          int64_t ldc, int M, int N, int K, double are, double aim, int beta) {
  if (M <= 0 || N <= 0) return;
  GTask t = {};
  t.lda = std::max<int64_t>(lda, 1);
  t.ldb = std::max<int64_t>(ldb, 1);
  t.ldc = std::max<int64_t>(ldc, 1);
  t.opA = (int8_t)opA;
  t.opB = (int8_t)opB;
  t.abase = 0;
  t.bbase = 1;
  t.cbase = 2;
  t.M = M;
  t.N = N;
  t.K = K;
  t.alpha_re = are;
  t.alpha_im = aim;
  t.beta = (int8_t)beta;
  BfPlan p;
  p.phase.push_back({t});
  // extents of the operands as given (the caller owns these buffers)
  const int64_t la = opA == OP_N ? (int64_t)(M - 1) + (int64_t)(K - 1) * t.lda + 1 : (int64_t)(K - 1) + (int64_t)(M - 1) * t.lda + 1;
  const int64_t lb = opB == OP_N ? (int64_t)(K - 1) + (int64_t)(N - 1) * t.ldb + 1 : (int64_t)(N - 1) + (int64_t)(K - 1) * t.ldb + 1;
  const int64_t lim[4] = {K > 0 ? la : 1, K > 0 ? lb : 1, (int64_t)(M - 1) + (int64_t)(N - 1) * t.ldc + 1, 0};
  run_plan<T>(p, *rt.c, (char*)const_cast<void*>(A), B, C, nullptr, rt.s(), lim);
}

// y = alpha x + beta y on m x nrhs blocks
template <class T>
void axpby(BfRuntime<T>& rt, void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int nrhs, double a, double b) {
  ochk(launch_axpby<T>(Y, ldy, X, ldx, m, nrhs, a, b, rt.s()), "axpby");
}

// element address of a device pointer (operands addressed without a base, GTask base 4)
template <class T>
inline int64_t eaddr(const void* p) {
  return (int64_t)((uintptr_t)p / sizeof(cplx<T>));
}

// y_t = a x_t + b y_t for a batch of blocks, one launch
template <class T>
void axpby_many(BfRuntime<T>& rt, const std::vector<AxpbyTask>& t, double a, double b) {
  if (t.empty()) return;
  int64_t mx = 0;
  for (auto& x : t) mx = std::max<int64_t>(mx, x.m * x.ncol);
  auto mk = rt.scratch.mark();
  void* d = rt.scratch.take(t.size() * sizeof(AxpbyTask));
  rt.c->stage.put(d, t.data(), t.size() * sizeof(AxpbyTask), rt.s());
  ochk(launch_axpby_batch<T>((const AxpbyTask*)d, (int)t.size(), mx, a, b, rt.s()), "axpby batch");
  rt.scratch.release(mk);
}

inline AxpbyTask axt(void* Y, int64_t ldy, const void* X, int64_t ldx, int64_t m, int ncol) {
  return AxpbyTask{Y, X, ldy, ldx, m, ncol, 0};
}

// Applies ops[i] to args[i] (independent outputs): operators of one dynamic type and structure key
// go through that type's batched application; one at a time in the plain form.
template <class T>
void apply_all(BfRuntime<T>& rt, const std::vector<Op<T>*>& ops, const std::vector<ApplyArg>& args, bool adj,
               double alpha, int beta) {
  if (ops.empty()) return;
  if (!rt.batch || ops.size() == 1) {
    for (size_t i = 0; i < ops.size(); ++i)
      ops[i]->apply(args[i].X, args[i].ldx, args[i].Y, args[i].ldy, args[i].nrhs, adj, alpha, beta);
    return;
  }
  std::vector<std::pair<std::pair<size_t, uint64_t>, std::vector<size_t>>> groups;
  for (size_t i = 0; i < ops.size(); ++i) {
    const std::pair<size_t, uint64_t> k{typeid(*ops[i]).hash_code(), ops[i]->key()};
    size_t g = 0;
    while (g < groups.size() && groups[g].first != k) ++g;
    if (g == groups.size()) groups.push_back({k, {}});
    groups[g].second.push_back(i);
  }
  for (auto& g : groups) {
    std::vector<Op<T>*> o;
    std::vector<ApplyArg> a;
    for (size_t i : g.second) {
      o.push_back(ops[i]);
      a.push_back(args[i]);
    }
    if (o.size() == 1)
      o[0]->apply(a[0].X, a[0].ldx, a[0].Y, a[0].ldy, a[0].nrhs, adj, alpha, beta);
    else
      o[0]->apply_many(rt, o, a, adj, alpha, beta);
  }
}

// Y = alpha op(A) X + beta Y with A dense (m x n, ld) on the device
template <class T>
struct DenseOp : Op<T> {
  BfRuntime<T>& rt;
  const void* A;
  int64_t lda;
  DenseOp(BfRuntime<T>& r, const void* a, int64_t ld, int m_, int n_) : rt(r), A(a), lda(ld) {
    this->m = m_;
    this->n = n_;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    if (!adj)
      gemm<T>(rt, A, lda, OP_N, X, ldx, OP_N, Y, ldy, this->m, nrhs, this->n, alpha, 0, beta);
    else
      gemm<T>(rt, A, lda, OP_C, X, ldx, OP_N, Y, ldy, this->n, nrhs, this->m, alpha, 0, beta);
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& ops, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    std::vector<GTask> ph;
    for (size_t i = 0; i < ops.size(); ++i) {
      auto* o = static_cast<DenseOp<T>*>(ops[i]);
      GTask t = {};
      t.a_off = eaddr<T>(o->A);
      t.lda = std::max<int64_t>(o->lda, 1);
      t.opA = (int8_t)(adj ? OP_C : OP_N);
      t.abase = 4;
      t.b_off = eaddr<T>(args[i].X);
      t.ldb = std::max<int64_t>(args[i].ldx, 1);
      t.opB = OP_N;
      t.bbase = 4;
      t.c_off = eaddr<T>(args[i].Y);
      t.ldc = std::max<int64_t>(args[i].ldy, 1);
      t.cbase = 4;
      t.M = adj ? o->n : o->m;
      t.N = args[i].nrhs;
      t.K = adj ? o->m : o->n;
      t.alpha_re = alpha;
      t.beta = (int8_t)beta;
      if (t.M > 0 && t.N > 0) ph.push_back(t);
    }
    if (ph.empty()) return;
    BfPlan p;
    p.phase.push_back(ph);
    const int64_t lim[4] = {0, 0, 0, 0};
    run_plan<T>(p, *r.c, nullptr, nullptr, nullptr, nullptr, r.s(), lim);
  }
};

template <class T>
struct BfOp : Op<T> {
  BfRuntime<T>& rt;
  const Butterfly* bf;
  BfOp(BfRuntime<T>& r, const Butterfly* b) : rt(r), bf(b) {
    this->m = b->m;
    this->n = b->n;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    rt.apply(*bf, X, ldx, Y, ldy, nrhs, adj, alpha, beta);
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& ops, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    std::vector<BfCall> calls;
    for (size_t i = 0; i < ops.size(); ++i) {
      BfCall c{static_cast<BfOp<T>*>(ops[i])->bf, 0, 0, alpha, 0.0, beta};
      c.x_abs = eaddr<T>(args[i].X);
      c.y_abs = eaddr<T>(args[i].Y);
      c.ldx = args[i].ldx;
      c.ldy = args[i].ldy;
      c.nrhs = args[i].nrhs;
      if (c.nrhs > 0) calls.push_back(c);
    }
    r.apply_calls(calls, adj);
  }
};

// Y = alpha (A B) X + beta Y
template <class T>
struct ProductOp : Op<T> {
  BfRuntime<T>& rt;
  Op<T>*A, *B;
  ProductOp(BfRuntime<T>& r, Op<T>* a, Op<T>* b) : rt(r), A(a), B(b) {
    this->m = a->m;
    this->n = b->n;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    auto mk = rt.scratch.mark();
    const int k = A->n;
    void* tmp = rt.scratch.take((size_t)std::max(k, 1) * nrhs * sizeof(cplx<T>));
    if (!adj) {
      B->apply(X, ldx, tmp, std::max(k, 1), nrhs, false, 1.0, 0);
      A->apply(tmp, std::max(k, 1), Y, ldy, nrhs, false, alpha, beta);
    } else {
      A->apply(X, ldx, tmp, std::max(k, 1), nrhs, true, 1.0, 0);
      B->apply(tmp, std::max(k, 1), Y, ldy, nrhs, true, alpha, beta);
    }
    rt.scratch.release(mk);
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& ops, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    auto mk = r.scratch.mark();
    std::vector<Op<T>*> As, Bs;
    std::vector<ApplyArg> a1, a2;
    for (size_t i = 0; i < ops.size(); ++i) {
      auto* o = static_cast<ProductOp<T>*>(ops[i]);
      const int k = o->A->n;
      void* tmp = r.scratch.take((size_t)std::max(k, 1) * args[i].nrhs * sizeof(cplx<T>));
      As.push_back(o->A);
      Bs.push_back(o->B);
      a1.push_back(ApplyArg{args[i].X, args[i].ldx, tmp, std::max(k, 1), args[i].nrhs});
      a2.push_back(ApplyArg{tmp, std::max(k, 1), args[i].Y, args[i].ldy, args[i].nrhs});
    }
    if (!adj) {
      apply_all<T>(r, Bs, a1, false, 1.0, 0);
      apply_all<T>(r, As, a2, false, alpha, beta);
    } else {
      apply_all<T>(r, As, a1, true, 1.0, 0);
      apply_all<T>(r, Bs, a2, true, alpha, beta);
    }
    r.scratch.release(mk);
  }
};

// Y = alpha (sum_i c_i A_i) X + beta Y  (real coefficients, identity when A_i is null)
template <class T>
struct SumOp : Op<T> {
  BfRuntime<T>& rt;
  std::vector<Op<T>*> ops;
  std::vector<double> coef;
  SumOp(BfRuntime<T>& r, int m_, int n_) : rt(r) {
    this->m = m_;
    this->n = n_;
  }
  void add(Op<T>* op, double c) {
    ops.push_back(op);
    coef.push_back(c);
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    const int rows = adj ? this->n : this->m;
    bool first = true;
    for (size_t i = 0; i < ops.size(); ++i) {
      const int b = (first && !beta) ? 0 : 1;
      if (ops[i]) {
        ops[i]->apply(X, ldx, Y, ldy, nrhs, adj, alpha * coef[i], b);
      } else {  // identity
        axpby<T>(rt, Y, ldy, X, ldx, rows, nrhs, alpha * coef[i], b ? 1.0 : 0.0);
      }
      first = false;
    }
    if (ops.empty() && !beta) axpby<T>(rt, Y, ldy, nullptr, 0, rows, nrhs, 0.0, 0.0);
  }
  uint64_t key() const override {  // number of terms, which are identities, their coefficients
    uint64_t k = ops.size();
    for (size_t i = 0; i < ops.size(); ++i) {
      k = k * 1000003u + (ops[i] ? 1u : 2u);
      k = k * 1000003u + (uint64_t)(int64_t)(coef[i] * 1024.0);
    }
    return k;
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& all, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    auto* o0 = static_cast<SumOp<T>*>(all[0]);
    const size_t nt = o0->ops.size();
    for (size_t t = 0; t < nt; ++t) {
      const int b = (t == 0 && !beta) ? 0 : 1;
      const double a = alpha * o0->coef[t];
      if (o0->ops[t]) {
        std::vector<Op<T>*> o;
        for (auto* x : all) o.push_back(static_cast<SumOp<T>*>(x)->ops[t]);
        apply_all<T>(r, o, args, adj, a, b);
      } else {
        std::vector<AxpbyTask> tk;
        for (size_t i = 0; i < all.size(); ++i)
          tk.push_back(axt(args[i].Y, args[i].ldy, args[i].X, args[i].ldx, adj ? all[i]->n : all[i]->m, args[i].nrhs));
        axpby_many<T>(r, tk, a, b ? 1.0 : 0.0);
      }
    }
    if (nt == 0 && !beta) {
      std::vector<AxpbyTask> tk;
      for (size_t i = 0; i < all.size(); ++i)
        tk.push_back(axt(args[i].Y, args[i].ldy, nullptr, 0, adj ? all[i]->n : all[i]->m, args[i].nrhs));
      axpby_many<T>(r, tk, 0.0, 0.0);
    }
  }
};

// [A11 A12; A21 A22] with row split m1 and column split n1 (null blocks are zero)
template <class T>
struct Block2Op : Op<T> {
  BfRuntime<T>& rt;
  Op<T>* A[2][2];
  int m1, n1;
  Block2Op(BfRuntime<T>& r, int m_, int n_, int m1_, int n1_, Op<T>* a11, Op<T>* a12, Op<T>* a21, Op<T>* a22)
      : rt(r), m1(m1_), n1(n1_) {
    this->m = m_;
    this->n = n_;
    A[0][0] = a11;
    A[0][1] = a12;
    A[1][0] = a21;
    A[1][1] = a22;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    const cplx<T>* x = (const cplx<T>*)X;
    cplx<T>* y = (cplx<T>*)Y;
    const int rs[2] = {0, adj ? n1 : m1}, re[2] = {adj ? n1 : m1, adj ? this->n : this->m};
    const int cs[2] = {0, adj ? m1 : n1};
    for (int i = 0; i < 2; ++i) {
      bool first = true;
      for (int j = 0; j < 2; ++j) {
        Op<T>* op = adj ? A[j][i] : A[i][j];
        if (!op) continue;
        const int b = (first && !beta) ? 0 : 1;
        op->apply(x + cs[j], ldx, y + rs[i], ldy, nrhs, adj, alpha, b);
        first = false;
      }
      if (first && !beta) axpby<T>(rt, y + rs[i], ldy, nullptr, 0, re[i] - rs[i], nrhs, 0.0, 0.0);
    }
  }
  uint64_t key() const override {
    return (A[0][0] ? 1u : 0u) | (A[0][1] ? 2u : 0u) | (A[1][0] ? 4u : 0u) | (A[1][1] ? 8u : 0u);
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& all, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    auto* o0 = static_cast<Block2Op<T>*>(all[0]);
    for (int i = 0; i < 2; ++i) {
      bool first = true;
      for (int j = 0; j < 2; ++j) {
        if (!(adj ? o0->A[j][i] : o0->A[i][j])) continue;
        const int b = (first && !beta) ? 0 : 1;
        std::vector<Op<T>*> o;
        std::vector<ApplyArg> a;
        for (size_t q = 0; q < all.size(); ++q) {
          auto* p = static_cast<Block2Op<T>*>(all[q]);
          const int rs = i == 0 ? 0 : (adj ? p->n1 : p->m1), cs = j == 0 ? 0 : (adj ? p->m1 : p->n1);
          o.push_back(adj ? p->A[j][i] : p->A[i][j]);
          a.push_back(ApplyArg{(const cplx<T>*)args[q].X + cs, args[q].ldx, (cplx<T>*)args[q].Y + rs, args[q].ldy,
                               args[q].nrhs});
        }
        apply_all<T>(r, o, a, adj, alpha, b);
        first = false;
      }
      if (first && !beta) {
        std::vector<AxpbyTask> tk;
        for (size_t q = 0; q < all.size(); ++q) {
          auto* p = static_cast<Block2Op<T>*>(all[q]);
          const int rs = i == 0 ? 0 : (adj ? p->n1 : p->m1);
          const int re = i == 0 ? (adj ? p->n1 : p->m1) : (adj ? p->n : p->m);
          tk.push_back(axt((cplx<T>*)args[q].Y + rs, args[q].ldy, nullptr, 0, re - rs, args[q].nrhs));
        }
        axpby_many<T>(r, tk, 0.0, 0.0);
      }
    }
  }
};

// View of rows [r0, r0+m) x cols [c0, c0+n) of another operator
template <class T>
struct SubOp : Op<T> {
  BfRuntime<T>& rt;
  Op<T>* P;
  int r0, c0;
  SubOp(BfRuntime<T>& r, Op<T>* p, int r0_, int c0_, int m_, int n_) : rt(r), P(p), r0(r0_), c0(c0_) {
    this->m = m_;
    this->n = n_;
  }
  void apply(const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adj, double alpha, int beta) override {
    auto mk = rt.scratch.mark();
    const int pin = adj ? P->m : P->n, pout = adj ? P->n : P->m;
    const int in0 = adj ? r0 : c0, out0 = adj ? c0 : r0;
    const int nin = adj ? this->m : this->n, nout = adj ? this->n : this->m;
    cplx<T>* xin = (cplx<T>*)rt.scratch.take((size_t)std::max(pin, 1) * nrhs * sizeof(cplx<T>));
    cplx<T>* yout = (cplx<T>*)rt.scratch.take((size_t)std::max(pout, 1) * nrhs * sizeof(cplx<T>));
    axpby<T>(rt, xin, std::max(pin, 1), nullptr, 0, pin, nrhs, 0.0, 0.0);
    axpby<T>(rt, xin + in0, std::max(pin, 1), X, ldx, nin, nrhs, 1.0, 0.0);
    P->apply(xin, std::max(pin, 1), yout, std::max(pout, 1), nrhs, adj, 1.0, 0);
    axpby<T>(rt, Y, ldy, yout + out0, std::max(pout, 1), nout, nrhs, alpha, beta ? 1.0 : 0.0);
    rt.scratch.release(mk);
  }
  void apply_many(BfRuntime<T>& r, const std::vector<Op<T>*>& all, const std::vector<ApplyArg>& args, bool adj,
                  double alpha, int beta) override {
    auto mk = r.scratch.mark();
    std::vector<AxpbyTask> zero, in, out;
    std::vector<Op<T>*> o;
    std::vector<ApplyArg> a;
    for (size_t q = 0; q < all.size(); ++q) {
      auto* p = static_cast<SubOp<T>*>(all[q]);
      const int nrhs = args[q].nrhs;
      const int pin = adj ? p->P->m : p->P->n, pout = adj ? p->P->n : p->P->m;
      const int in0 = adj ? p->r0 : p->c0, out0 = adj ? p->c0 : p->r0;
      const int nin = adj ? p->m : p->n, nout = adj ? p->n : p->m;
      cplx<T>* xin = (cplx<T>*)r.scratch.take((size_t)std::max(pin, 1) * nrhs * sizeof(cplx<T>));
      cplx<T>* yout = (cplx<T>*)r.scratch.take((size_t)std::max(pout, 1) * nrhs * sizeof(cplx<T>));
      zero.push_back(axt(xin, std::max(pin, 1), nullptr, 0, pin, nrhs));
      in.push_back(axt(xin + in0, std::max(pin, 1), args[q].X, args[q].ldx, nin, nrhs));
      o.push_back(p->P);
      a.push_back(ApplyArg{xin, std::max(pin, 1), yout, std::max(pout, 1), nrhs});
      out.push_back(axt(args[q].Y, args[q].ldy, yout + out0, std::max(pout, 1), nout, nrhs));
    }
    axpby_many<T>(r, zero, 0.0, 0.0);
    axpby_many<T>(r, in, 1.0, 0.0);
    apply_all<T>(r, o, a, adj, 1.0, 0);
    axpby_many<T>(r, out, alpha, beta ? 1.0 : 0.0);
    r.scratch.release(mk);
  }
};

}  // namespace bfmf
