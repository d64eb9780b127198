// Compressed fronts (paper Alg. 5, Sec. 4 and Sec. 5): a front whose
// separator has at least n_min unknowns is never formed.
//   F11       HOD-BF over the separator bisection tree: dense leaves and two
//             butterflies per internal node, built by entry evaluation
//   F11^-1    HODBF_invert (Alg. 4): D^-1 = (I + X) diag(D1^-1, D2^-1) per
//             node, X from BF_SMW with randomized constructions
//   F12, F21  single butterflies by entry evaluation
//   S         F21 F11^-1 F12 by randomized construction
//   C         contribution block C_nu1 (+) C_nu2 - S on I^u x I^u
// The forward sweep applies F11^-1 then F21, the backward sweep F12 then F11^-1.
#pragma once
#include <memory>
#include <vector>

#include "bf.hpp"
#include "ops.hpp"

namespace bfmf {

template <class T>
struct HodbfNode {
  int beg = 0, end = 0, left = -1, right = -1, depth = 0, level = 0;
  int64_t leaf_off = -1;                 // dense leaf D (size x size) in the pool
  std::unique_ptr<Butterfly> b12, b21;   // F(T1, T2), F(T2, T1)
  // inverse
  int64_t inv_off = -1;                  // leaf: D^-1; small internal node: dense X
  std::unique_ptr<Butterfly> x;          // internal node: X with D^-1 = (I + X) diag(...)
  bool x_dense = false;
  bool x_zero = false;
  int size() const { return end - beg; }
};

template <class T>
struct Hodbf {
  int n = 0;
  std::vector<HodbfNode<T>> nodes;  // preorder, node 0 = root
  std::vector<std::vector<int>> by_level;
  int max_level = 0;
};

template <class T>
struct CompressedFront {
  int front = -1;
  int ns = 0, nu = 0;
  Hodbf<T> f11;
  std::unique_ptr<Butterfly> f12, f21, s;
  int64_t cb_off = -1;  // dense contribution block nu x nu (byte offset in the front arena)
  double flops = 0;
  // contribution block in HOD-BF form (when the parent is compressed and compress_cb is set):
  // leaves and butterflies in the pool, its device descriptor (centre forms, kept until the
  // parent's level has been factored) for the parent's entry extraction
  Hodbf<T> cbh;
  const HodbfDev* cb_dev = nullptr;
};

// y = alpha F11 x + beta y (the HOD-BF itself)
template <class T>
void hodbf_apply(BfRuntime<T>& rt, const Hodbf<T>& h, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs);
// y = D_node^-1 x for the subtree of `node` (x, y: rows of that node only)
template <class T>
void hodbf_inv_apply(BfRuntime<T>& rt, const Hodbf<T>& h, int node, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     int nrhs, bool adjoint);

// one (tree, node, x, y) of a batched inverse product
template <class T>
struct HodbfInvItem {
  const Hodbf<T>* h;
  int node;
  const void* X;
  int64_t ldx;
  void* Y;
  int64_t ldy;
  int nrhs;
};
template <class T>
void hodbf_inv_apply_many(BfRuntime<T>& rt, const std::vector<HodbfInvItem<T>>& items, bool adjoint);

}  // namespace bfmf
