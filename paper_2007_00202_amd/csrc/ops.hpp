// Linear operators on device vectors used by the randomized constructions
// and the HOD-BF inversion (paper Sec. 3.3, Sec. 4.2): dense blocks,
// butterflies, and products / sums / block arrangements of operators.
#pragma once
#include <memory>
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
};

}  // namespace bfmf
