// Butterfly format, products and construction (paper Sec. 3).  See bf.hpp.
#include "bf.hpp"
#include "host_pool.hpp"
#include "ops.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>

#include "kernels/kernels.hpp"

namespace bfmf {

namespace {
void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(BFMF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
void dev_alloc(DevBuf& b, size_t bytes) {
  b.release();
  if (bytes == 0) bytes = 256;
  if (dev_malloc((void**)&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    throw Error(BFMF_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (butterfly)");
  }
  b.bytes = bytes;
}
// copy of a host vector in scratch memory, uploaded through the pinned ring
template <class R, class V>
void* upload_tmp(R& rt, const std::vector<V>& v) {
  void* d = rt.scratch.take(std::max<size_t>(v.size() * sizeof(V), 16));
  rt.c->stage.put(d, v.data(), v.size() * sizeof(V), rt.s());
  return d;
}
// Several host arrays in one scratch allocation, staged with one copy (a copy call costs the host
// about as much as a launch).  Parts are 256-byte aligned; part(i) gives a part's device address
// before the copy (so that other parts can point into it); the sources are read at commit().
template <class R>
struct PackedUpload {
  R& rt;
  std::vector<std::pair<const void*, size_t>> src;
  std::vector<size_t> off;
  size_t total = 0;
  char* base = nullptr;
  explicit PackedUpload(R& r) : rt(r) {}
  int add(const void* p, size_t bytes) {
    off.push_back(total);
    src.push_back({p, bytes});
    total = (total + bytes + 255) & ~(size_t)255;
    return (int)off.size() - 1;
  }
  char* part(int i) {
    if (!base) base = (char*)rt.scratch.take(std::max<size_t>(total, 16));
    return base + off[i];
  }
  void commit() {
    if (!base) base = (char*)rt.scratch.take(std::max<size_t>(total, 16));
    std::vector<char> h(std::max<size_t>(total, 1));
    for (size_t i = 0; i < src.size(); ++i)
      if (src[i].second) std::memcpy(h.data() + off[i], src[i].first, src[i].second);
    rt.c->stage.put(base, h.data(), total, rt.s());
  }
};
}  // namespace

// ------------------------------------------------------------ device memory
size_t DevPool::alloc(size_t bytes, hipStream_t s) {
  const size_t off = (used + 255) & ~(size_t)255;
  const size_t need = off + std::max<size_t>(bytes, 1);
  if (need > buf.bytes) {
    size_t cap = std::max<size_t>(need, buf.bytes * 2);
    cap = std::max<size_t>(cap, (size_t)64 << 20);
    if (budget && !budget->fits(cap)) {  // the old buffer is held while the content is copied
      cap = std::max<size_t>(need, (size_t)1 << 20);
      if (!budget->fits(cap))
        throw Error(BFMF_E_NOMEM, "butterfly pool growth to " + std::to_string(cap) +
                                      " bytes exceeds the HBM budget");
    }
    DevBuf nb;
    dev_alloc(nb, cap);
    if (budget) budget->held += cap - buf.bytes;
    if (used) chk(hipMemcpyAsync(nb.p, buf.p, used, hipMemcpyDeviceToDevice, s), "pool grow");
    chk(hipStreamSynchronize(s), "pool grow");
    std::swap(buf.p, nb.p);
    std::swap(buf.bytes, nb.bytes);
  }
  used = need;
  return off;
}

void Scratch::release(const Mark& m) {
  cur = m.cur;
  if (cur >= 0) chunks[cur]->top = m.top;
}

void* Scratch::take(size_t bytes) {
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
  if (cur < 0 || chunks[cur]->top + bytes > chunks[cur]->b.bytes) {
    // next chunk: the chunks above the top hold nothing, so any of them that is large enough is
    // moved to the next position; only when none is, a new chunk is inserted there (never freed:
    // freeing device memory synchronizes the device)
    const size_t next = (size_t)(cur + 1);
    size_t fit = next;
    while (fit < chunks.size() && chunks[fit]->b.bytes < bytes) ++fit;
    if (fit < chunks.size()) {
      std::swap(chunks[next], chunks[fit]);
    } else {
      auto ch = std::make_unique<Chunk>();
      const size_t cb = std::max(bytes, chunk_bytes);
      if (budget && !budget->fits(cb))
        throw Error(BFMF_E_NOMEM, "scratch chunk of " + std::to_string(cb) + " bytes exceeds the HBM budget");
      dev_alloc(ch->b, cb);
      if (budget) budget->held += cb;
      chunks.insert(chunks.begin() + next, std::move(ch));
    }
    cur = (int)next;
    chunks[cur]->top = 0;
  }
  Chunk& c = *chunks[cur];
  void* p = c.b.as<char>() + c.top;
  c.top += bytes;
  return p;
}

// ------------------------------------------------------------------- trees
int tree_depth(const TreeNode* nodes, int nnodes) {
  if (!nodes || nnodes == 0) return 0;
  std::function<int(int)> d = [&](int i) -> int {
    if (nodes[i].left < 0) return 0;
    return 1 + std::max(d(nodes[i].left), d(nodes[i].right));
  };
  return d(0);
}

BTree make_tree(int n, int L, const TreeNode* nodes, int nnodes) {
  BTree t;
  t.n = n;
  t.L = L;
  struct Cur {
    int b, e, idx;
  };
  std::vector<Cur> cur{{0, n, (nodes && nnodes) ? 0 : -1}};
  for (int l = 0; l <= L; ++l) {
    std::vector<int32_t> bd;
    for (auto& c : cur) bd.push_back(c.b);
    bd.push_back(cur.back().e);
    t.b.push_back(bd);
    if (l == L) break;
    std::vector<Cur> nx;
    for (auto& c : cur) {
      if (c.idx >= 0 && nodes[c.idx].left >= 0) {
        const int li = nodes[c.idx].left, ri = nodes[c.idx].right;
        const int mid = nodes[li].end - nodes[0].beg;
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

int Butterfly::max_rank() const {
  int r = 0;
  for (auto& v : rl)
    for (int x : v) r = std::max(r, x);
  for (auto& v : rr)
    for (int x : v) r = std::max(r, x);
  return r;
}

// ------------------------------------------------------------- layouts
namespace {

// pairing: 0 single, 1 nu-siblings (blk ^ 1), 2 tau-siblings (t ^ 1, same v)
VecLayout layout(const std::vector<int32_t>& r, int L, int l, int pairing, int nrhs) {
  VecLayout lay;
  const int nb = 1 << L;
  lay.grp_of.assign(nb, -1);
  lay.mem_row.assign(nb, 0);
  const int vs = 1 << (L - l);  // column nodes at this level
  int64_t off = 0;
  auto add_group = [&](std::initializer_list<int> members) {
    int g = (int)lay.grp_off.size();
    int rows = 0;
    for (int b : members) {
      lay.grp_of[b] = g;
      lay.mem_row[b] = rows;
      rows += r[b];
    }
    lay.grp_off.push_back(off);
    lay.grp_ld.push_back(rows);
    off += (int64_t)rows * nrhs;
  };
  if (pairing == 1 && L - l >= 1) {
    for (int b = 0; b < nb; b += 2) add_group({b, b + 1});
  } else if (pairing == 2 && l >= 1) {
    for (int t2 = 0; t2 < (1 << (l - 1)); ++t2)
      for (int v = 0; v < vs; ++v) add_group({(2 * t2) * vs + v, (2 * t2 + 1) * vs + v});
  } else {
    for (int b = 0; b < nb; ++b) add_group({b});
  }
  lay.rows = off / std::max(nrhs, 1);
  return lay;
}

GTask task(int64_t a_off, int64_t lda, int opA, int abase, int64_t b_off, int64_t ldb, int bbase, int64_t c_off,
           int64_t ldc, int cbase, int M, int N, int K, double are, double aim, int beta) {
  GTask t;
  std::memset(&t, 0, sizeof(t));
  t.a_off = a_off;
  t.lda = std::max<int64_t>(lda, 1);
  t.opA = (int8_t)opA;
  t.opB = OP_N;
  t.abase = (int8_t)abase;
  t.b_off = b_off;
  t.ldb = std::max<int64_t>(ldb, 1);
  t.bbase = (int8_t)bbase;
  t.c_off = c_off;
  t.ldc = std::max<int64_t>(ldc, 1);
  t.cbase = (int8_t)cbase;
  t.M = M;
  t.N = N;
  t.K = K;
  t.alpha_re = are;
  t.alpha_im = aim;
  t.beta = (int8_t)beta;
  return t;
}

}  // namespace

BfPlan make_plan(const std::vector<BfCall>& calls, bool adjoint, int nrhs, int64_t ldx, int64_t ldy,
                 bool right_half_only) {
  HostTimer ht(HP_PLAN);
  BfPlan plan;
  int64_t ws = 0;
  size_t maxph = 0;
  for (auto& cl : calls) maxph = std::max<size_t>(maxph, (size_t)cl.bf->L + 3);
  plan.phase.assign(maxph, {});
  for (auto& cl : calls) {
    const Butterfly& bf = *cl.bf;
    const int L = bf.L, lc = bf.lc, nb = 1 << L;
    // this call's input and output: shared buffers (bases 1, 2) or its own (base 4, absolute)
    const int nr = cl.nrhs > 0 ? cl.nrhs : nrhs;
    const int xb = cl.x_abs >= 0 ? 4 : 1, yb = cl.y_abs >= 0 ? 4 : 2;
    const int64_t xo = (cl.x_abs >= 0 ? cl.x_abs : 0) + cl.x_off, yo = (cl.y_abs >= 0 ? cl.y_abs : 0) + cl.y_off;
    const int64_t lx = cl.ldx > 0 ? cl.ldx : ldx, ly = cl.ldy > 0 ? cl.ldy : ldy;
    // two ping-pong regions sized for the largest level
    int64_t maxrows = 0;
    for (int l = lc; l <= L; ++l) maxrows = std::max<int64_t>(maxrows, std::accumulate(bf.rl[l].begin(), bf.rl[l].end(), (int64_t)0));
    for (int l = 0; l <= lc; ++l) maxrows = std::max<int64_t>(maxrows, std::accumulate(bf.rr[l].begin(), bf.rr[l].end(), (int64_t)0));
    const int64_t region = maxrows * nr;
    const int64_t w0 = ws, w1 = ws + region;
    ws += 2 * region;
    int ph = 0;
    bool in0 = true;  // the current input lives in region 0
    auto W = [&](bool r0) { return r0 ? w0 : w1; };
    if (!adjoint) {
      // V: t_0 = Vt X(S_v)
      VecLayout out = layout(bf.rr[0], L, 0, 1, nr);
      for (int v = 0; v < nb; ++v) {
        const int M = bf.rr[0][v];
        if (M == 0) continue;
        plan.phase[ph].push_back(task(bf.offR[0][v], M, OP_N, 0, xo + bf.ts.beg(L, v), lx, xb,
                                      W(true) + out.grp_off[out.grp_of[v]] + out.mem_row[v], out.grp_ld[out.grp_of[v]], 3,
                                      M, nr, bf.ts.size(L, v), 1, 0, 0));
      }
      ++ph;
      VecLayout in = out;
      in0 = true;
      for (int l = 1; l <= lc; ++l) {
        VecLayout o = layout(bf.rr[l], L, l, 1, nr);
        const int vs = 1 << (L - l);
        for (int t = 0; t < (1 << l); ++t)
          for (int v = 0; v < vs; ++v) {
            const int blk = t * vs + v;
            const int M = bf.rr[l][blk];
            if (M == 0) continue;
            const int t2 = t / 2;
            const int a = (2 * t2) * vs + v, b = (2 * t2 + 1) * vs + v;
            const int q = t2 * vs + v;  // tau-pair id
            const int wrows = bf.rr[l][a] + bf.rr[l][b];
            const int row_off = (t & 1) ? bf.rr[l][a] : 0;
            const int ia = t2 * (2 * vs) + 2 * v;  // input nu-pair members at level l-1
            const int K = bf.rr[l - 1][ia] + bf.rr[l - 1][ia + 1];
            const int gi = in.grp_of[ia];
            plan.phase[ph].push_back(task(bf.offR[l][q] + row_off, wrows, OP_N, 0, W(in0) + in.grp_off[gi], in.grp_ld[gi],
                                          3, W(!in0) + o.grp_off[o.grp_of[blk]] + o.mem_row[blk],
                                          o.grp_ld[o.grp_of[blk]], 3, M, nr, K, 1, 0, 0));
          }
        ++ph;
        in = o;
        in0 = !in0;
      }
      if (right_half_only) {
        plan.half_layout.push_back(in);
        plan.half_off.push_back(W(in0));
        continue;
      }
      // B: s_lc = B t_lc
      {
        VecLayout o = layout(bf.rl[lc], L, lc, 1, nr);
        for (int blk = 0; blk < nb; ++blk) {
          const int M = bf.rl[lc][blk], K = bf.rr[lc][blk];
          if (M == 0) continue;
          const int gi = in.grp_of[blk];
          plan.phase[ph].push_back(task(bf.offB[blk], M, OP_N, 0, W(in0) + in.grp_off[gi] + in.mem_row[blk],
                                        in.grp_ld[gi], 3, W(!in0) + o.grp_off[o.grp_of[blk]] + o.mem_row[blk],
                                        o.grp_ld[o.grp_of[blk]], 3, M, nr, K, 1, 0, 0));
        }
        ++ph;
        in = o;
        in0 = !in0;
      }
      // R: s_{l+1} from nu-pairs of s_l
      for (int l = lc; l < L; ++l) {
        VecLayout o = layout(bf.rl[l + 1], L, l + 1, 1, nr);
        const int vs1 = 1 << (L - l - 1);  // column nodes at level l+1
        for (int t1 = 0; t1 < (1 << (l + 1)); ++t1)
          for (int v1 = 0; v1 < vs1; ++v1) {
            const int blk1 = t1 * vs1 + v1;
            const int M = bf.rl[l + 1][blk1];
            if (M == 0) continue;
            const int pt = t1 / 2;
            const int pair = pt * vs1 + v1;  // nu-pair id at level l (members 2 pair, 2 pair + 1)
            const int top = bf.rl[l + 1][(2 * pt) * vs1 + v1];
            const int rrows = top + bf.rl[l + 1][(2 * pt + 1) * vs1 + v1];
            const int row_off = (t1 & 1) ? top : 0;
            const int K = bf.rl[l][2 * pair] + bf.rl[l][2 * pair + 1];
            const int gi = in.grp_of[2 * pair];
            plan.phase[ph].push_back(task(bf.offL[l][pair] + row_off, rrows, OP_N, 0, W(in0) + in.grp_off[gi],
                                          in.grp_ld[gi], 3, W(!in0) + o.grp_off[o.grp_of[blk1]] + o.mem_row[blk1],
                                          o.grp_ld[o.grp_of[blk1]], 3, M, nr, K, 1, 0, 0));
          }
        ++ph;
        in = o;
        in0 = !in0;
      }
      // U: Y(O_t) = alpha U s_L + beta Y
      for (int t = 0; t < nb; ++t) {
        const int M = bf.to.size(L, t), K = bf.rl[L][t];
        if (M == 0) continue;
        const int gi = in.grp_of[t];
        plan.phase[ph].push_back(task(bf.offL[L][t], M, OP_N, 0, W(in0) + in.grp_off[gi] + in.mem_row[t],
                                      in.grp_ld[gi], 3, yo + bf.to.beg(L, t), ly, yb, M, nr, K, cl.alpha_re,
                                      cl.alpha_im, cl.beta));
      }
    } else {
      // U^H: s_L = U^H X(O_t), tau-paired
      VecLayout out = layout(bf.rl[L], L, L, 2, nr);
      for (int t = 0; t < nb; ++t) {
        const int M = bf.rl[L][t];
        if (M == 0) continue;
        plan.phase[ph].push_back(task(bf.offL[L][t], bf.to.size(L, t), OP_C, 0, xo + bf.to.beg(L, t), lx, xb,
                                      W(true) + out.grp_off[out.grp_of[t]] + out.mem_row[t], out.grp_ld[out.grp_of[t]],
                                      3, M, nr, bf.to.size(L, t), 1, 0, 0));
      }
      ++ph;
      VecLayout in = out;
      in0 = true;
      for (int l = L - 1; l >= lc; --l) {
        VecLayout o = layout(bf.rl[l], L, l, 2, nr);
        const int vs = 1 << (L - l), vs1 = vs / 2;
        for (int t = 0; t < (1 << l); ++t)
          for (int v = 0; v < vs; ++v) {
            const int blk = t * vs + v;
            const int M = bf.rl[l][blk];
            if (M == 0) continue;
            const int pair = blk / 2;  // nu-pair holding the combined R
            const int a1 = (2 * t) * vs1 + v / 2, b1 = (2 * t + 1) * vs1 + v / 2;
            const int rrows = bf.rl[l + 1][a1] + bf.rl[l + 1][b1];
            const int col_off = (blk & 1) ? bf.rl[l][blk - 1] : 0;
            const int gi = in.grp_of[a1];
            plan.phase[ph].push_back(task(bf.offL[l][pair] + (int64_t)col_off * rrows, rrows, OP_C, 0,
                                          W(in0) + in.grp_off[gi], in.grp_ld[gi], 3,
                                          W(!in0) + o.grp_off[o.grp_of[blk]] + o.mem_row[blk], o.grp_ld[o.grp_of[blk]],
                                          3, M, nr, rrows, 1, 0, 0));
          }
        ++ph;
        in = o;
        in0 = !in0;
      }
      {  // B^H
        VecLayout o = layout(bf.rr[lc], L, lc, 2, nr);
        for (int blk = 0; blk < nb; ++blk) {
          const int M = bf.rr[lc][blk], K = bf.rl[lc][blk];
          if (M == 0) continue;
          const int gi = in.grp_of[blk];
          plan.phase[ph].push_back(task(bf.offB[blk], std::max(K, 1), OP_C, 0, W(in0) + in.grp_off[gi] + in.mem_row[blk],
                                        in.grp_ld[gi], 3, W(!in0) + o.grp_off[o.grp_of[blk]] + o.mem_row[blk],
                                        o.grp_ld[o.grp_of[blk]], 3, M, nr, K, 1, 0, 0));
        }
        ++ph;
        in = o;
        in0 = !in0;
      }
      for (int l = lc; l >= 1; --l) {  // W^H: t_{l-1} from tau-pairs of t_l
        VecLayout o = layout(bf.rr[l - 1], L, l - 1, 2, nr);
        const int vs = 1 << (L - l), vs0 = 2 * vs;  // column nodes at levels l and l-1
        for (int t0 = 0; t0 < (1 << (l - 1)); ++t0)
          for (int v0 = 0; v0 < vs0; ++v0) {
            const int blk0 = t0 * vs0 + v0;
            const int M = bf.rr[l - 1][blk0];
            if (M == 0) continue;
            const int v = v0 / 2;
            const int q = t0 * vs + v;  // tau-pair at level l: (2 t0, v), (2 t0 + 1, v)
            const int a = (2 * t0) * vs + v, b = (2 * t0 + 1) * vs + v;
            const int wrows = bf.rr[l][a] + bf.rr[l][b];
            const int c1 = bf.rr[l - 1][t0 * vs0 + 2 * v];
            const int col_off = (v0 & 1) ? c1 : 0;
            const int gi = in.grp_of[a];
            plan.phase[ph].push_back(task(bf.offR[l][q] + (int64_t)col_off * std::max(wrows, 1), wrows, OP_C, 0,
                                          W(in0) + in.grp_off[gi], in.grp_ld[gi], 3,
                                          W(!in0) + o.grp_off[o.grp_of[blk0]] + o.mem_row[blk0],
                                          o.grp_ld[o.grp_of[blk0]], 3, M, nr, wrows, 1, 0, 0));
          }
        ++ph;
        in = o;
        in0 = !in0;
      }
      for (int v = 0; v < nb; ++v) {  // V^H: Y(S_v) = alpha conj(V) t_0 + beta Y
        const int M = bf.ts.size(L, v), K = bf.rr[0][v];
        if (M == 0) continue;
        const int gi = in.grp_of[v];
        plan.phase[ph].push_back(task(bf.offR[0][v], std::max(K, 1), OP_C, 0, W(in0) + in.grp_off[gi] + in.mem_row[v],
                                      in.grp_ld[gi], 3, yo + bf.ts.beg(L, v), ly, yb, M, nr, K, cl.alpha_re,
                                      cl.alpha_im, cl.beta));
      }
    }
  }
  plan.ws_elems = ws;
  return plan;
}

namespace {
// largest element index touched by an operand stored rows x cols (ld), or -1
int64_t footprint(int64_t off, int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return -1;
  return off + (rows - 1) + (cols - 1) * ld;
}

// every task's operands inside the buffers of its bases (lim[b] elements from base b; base 4 is
// absolute and built only from allocations sized for the task)
void check_plan(const BfPlan& plan, void* const bases[4], const int64_t lim[4]) {
  for (auto& ph : plan.phase)
    for (const GTask& t : ph) {
      const int64_t fa = t.opA == OP_N ? footprint(t.a_off, t.M, t.K, t.lda) : footprint(t.a_off, t.K, t.M, t.lda);
      const int64_t fb = t.opB == OP_N ? footprint(t.b_off, t.K, t.N, t.ldb) : footprint(t.b_off, t.N, t.K, t.ldb);
      const int64_t fc = footprint(t.c_off, t.M, t.N, t.ldc);
      auto out_of = [&](int b, int64_t off, int64_t f) {
        if (f < 0) return false;
        if (b == 4) return off <= 0;
        return off < 0 || f >= lim[b] || !bases[b];
      };
      bool bad = t.abase < 0 || t.abase > 4 || t.bbase < 0 || t.bbase > 4 || t.cbase < 0 || t.cbase > 4;
      bad = bad || out_of(t.abase, t.a_off, fa) || out_of(t.bbase, t.b_off, fb) || out_of(t.cbase, t.c_off, fc);
      if (bad)
        throw Error(BFMF_E_INVAL, "internal: butterfly product task outside its buffers (M " + std::to_string(t.M) +
                                      " N " + std::to_string(t.N) + " K " + std::to_string(t.K) + ")");
    }
}
}  // namespace

template <class T>
void run_plan(const BfPlan& plan, Context& c, char* pool, const void* X, void* Y, void* ws, hipStream_t s,
              const int64_t lim[4], int kind) {
  HostTimer ht_run(HP_RUN);
  void* bases[4] = {pool, const_cast<void*>(X), Y, ws};
  check_plan(plan, bases, lim);
  // launches in phase order: a phase in one tile shape from the autotuned table, or split into
  // one launch per shape when its tasks differ in height (all shapes give the same result, and
  // the tasks of a phase are independent, so neither the split nor the order changes it)
  struct Launch {
    const GTask* t;
    size_t n;
    int cfg;
  };
  std::deque<std::vector<GTask>> groups;  // split phases' tasks (a deque keeps them in place)
  std::vector<Launch> launches;
  {
    std::vector<int> task_cfg;
    for (auto& ph : plan.phase) {
      if (ph.empty()) continue;
      const int cfg = choose_gemm_cfg_split<T>(c.device, s, ph, task_cfg);
      if (cfg >= 0) {
        launches.push_back(Launch{ph.data(), ph.size(), cfg});
        continue;
      }
      for (int q = 0; q < GEMM_CFGS; ++q) {
        std::vector<GTask> grp;
        for (size_t i = 0; i < ph.size(); ++i)
          if (task_cfg[i] == q) grp.push_back(ph[i]);
        if (grp.empty()) continue;
        groups.push_back(std::move(grp));
        launches.push_back(Launch{groups.back().data(), groups.back().size(), q});
      }
    }
  }
  // one upload for all launches: per launch its tasks then its tile starts
  std::vector<char> blob;
  std::vector<size_t> toff, soff;
  std::vector<int64_t> ntiles;
  for (const Launch& ln : launches) {
    const int cfg = ln.cfg;
    if (c.verbose && kind == K_BF_GEMM) {
      const double tm = GEMM_CFG_TM[cfg], tn = GEMM_CFG_TN[cfg];
      for (size_t i = 0; i < ln.n; ++i) {
        const GTask& t = ln.t[i];
        const double M = t.M, N = t.N, K = t.K;
        const double Mp = std::ceil(M / tm) * tm, Np = std::ceil(N / tn) * tn, Kp = std::ceil(K / 16.0) * 16.0;
        double* pd = c.timer.pad;
        pd[0] += M * N * K;
        pd[1] += Mp * N * K;
        pd[2] += M * Np * K;
        pd[3] += M * N * Kp;
        pd[4] += Mp * Np * Kp;
        c.timer.mhist[std::min(19, (t.M + 15) / 16)] += M * N * K;
        c.timer.nhist[std::min(19, (t.N + 15) / 16)] += M * N * K;
      }
    }
    std::vector<int64_t> start(ln.n);
    int64_t tiles = 0;
    for (size_t i = 0; i < ln.n; ++i) {
      start[i] = tiles;
      tiles += gemm_cfg_tiles(cfg, ln.t[i].M, ln.t[i].N);
    }
    if (tiles >= ((int64_t)1 << 31)) throw Error(BFMF_E_INVAL, "internal: grouped GEMM launch with 2^31 tiles");
    size_t o = (blob.size() + 15) & ~(size_t)15;
    blob.resize(o + ln.n * sizeof(GTask) + start.size() * sizeof(int64_t));
    if (ln.n) std::memcpy(blob.data() + o, ln.t, ln.n * sizeof(GTask));
    if (!start.empty()) std::memcpy(blob.data() + o + ln.n * sizeof(GTask), start.data(), start.size() * sizeof(int64_t));
    toff.push_back(o);
    soff.push_back(o + ln.n * sizeof(GTask));
    ntiles.push_back(tiles);
  }
  if (blob.empty()) return;
  // the task blob lives in the stream-ordered staging area of the context
  if (c.g_tmp_plan.bytes < blob.size()) dev_alloc(c.g_tmp_plan, std::max<size_t>(blob.size() * 2, (size_t)1 << 20));
  char* d = c.g_tmp_plan.as<char>();
  c.stage.put(d, blob.data(), blob.size(), s);
  for (size_t k = 0; k < launches.size(); ++k) {
    const Launch& ln = launches[k];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int tk = c.timer.want(kind) ? c.timer.begin_ext(&e0, &e1) : -1;
    {
      HostTimer ht(HP_LAUNCH);
      chk(launch_grouped_gemm<T>((const GTask*)(d + toff[k]), (const int64_t*)(d + soff[k]), (int)ln.n, ntiles[k],
                                 bases, ln.cfg, s, e0, e1, kind == K_ID),
          "grouped gemm");
    }
    c.gemm_cfg_launches[ln.cfg] += 1;
    if (tk >= 0) {
      double fl = 0, by = 0;
      int mm = 0, mn = 0, mk = 0;
      for (size_t i = 0; i < ln.n; ++i) {
        const GTask& t = ln.t[i];
        const double M = t.M, N = t.N, K = t.K;
        fl += 8.0 * M * N * K;
        by += sizeof(cplx<T>) * (M * K + K * N + M * N * (t.beta ? 2.0 : 1.0));
        mm = std::max(mm, t.M);
        mn = std::max(mn, t.N);
        mk = std::max(mk, t.K);
      }
      c.timer.set_shape(tk, (int)ln.n, mm, mn, mk);
      c.timer.end_ext(tk, kind, fl, by);
    }
  }
  // no synchronisation: the next plan's upload is ordered after these launches on the stream
}

template void run_plan<double>(const BfPlan&, Context&, char*, const void*, void*, void*, hipStream_t,
                               const int64_t[4], int);
template void run_plan<float>(const BfPlan&, Context&, char*, const void*, void*, void*, hipStream_t,
                              const int64_t[4], int);

// The task lists of a plan with every launch in tile shape cfg: per phase its tasks, then its tile
// starts, each phase at a 16-byte boundary.
static void plan_blob(const BfPlan& plan, int cfg, std::vector<char>& blob, std::vector<size_t>& toff,
                      std::vector<size_t>& soff, std::vector<int64_t>& ntiles) {
  blob.clear();
  for (auto& ph : plan.phase) {
    std::vector<int64_t> start(ph.size());
    int64_t tiles = 0;
    for (size_t i = 0; i < ph.size(); ++i) {
      start[i] = tiles;
      tiles += gemm_cfg_tiles(cfg, ph[i].M, ph[i].N);
    }
    if (tiles >= ((int64_t)1 << 31)) throw Error(BFMF_E_INVAL, "internal: grouped GEMM launch with 2^31 tiles");
    size_t o = (blob.size() + 15) & ~(size_t)15;
    blob.resize(o + ph.size() * sizeof(GTask) + start.size() * sizeof(int64_t));
    if (!ph.empty()) std::memcpy(blob.data() + o, ph.data(), ph.size() * sizeof(GTask));
    if (!start.empty())
      std::memcpy(blob.data() + o + ph.size() * sizeof(GTask), start.data(), start.size() * sizeof(int64_t));
    toff.push_back(o);
    soff.push_back(o + ph.size() * sizeof(GTask));
    ntiles.push_back(tiles);
  }
}

template <class T>
size_t run_plan_fixed(const BfPlan& plan, char* pool, const void* X, void* Y, void* ws, char* dtasks,
                      size_t tasks_cap, hipStream_t s, const int64_t lim[4], int cfg) {
  void* bases[4] = {pool, const_cast<void*>(X), Y, ws};
  check_plan(plan, bases, lim);
  std::vector<char> blob;
  std::vector<size_t> toff, soff;
  std::vector<int64_t> ntiles;
  plan_blob(plan, cfg, blob, toff, soff, ntiles);
  if (blob.size() > tasks_cap) return blob.size();
  if (blob.empty()) return 0;
  chk(hipMemcpyAsync(dtasks, blob.data(), blob.size(), hipMemcpyHostToDevice, s), "task upload");
  for (size_t k = 0; k < plan.phase.size(); ++k) {
    if (plan.phase[k].empty()) continue;
    chk(launch_grouped_gemm<T>((const GTask*)(dtasks + toff[k]), (const int64_t*)(dtasks + soff[k]),
                               (int)plan.phase[k].size(), ntiles[k], bases, cfg, s, nullptr, nullptr),
        "grouped gemm");
  }
  // the host copy of the task lists must outlive the upload
  chk(hipStreamSynchronize(s), "sync");
  return 0;
}

template size_t run_plan_fixed<double>(const BfPlan&, char*, const void*, void*, void*, char*, size_t, hipStream_t,
                                       const int64_t[4], int);

template <class T>
void BfRuntime<T>::apply(const Butterfly& bf, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, bool adjoint,
                         double alpha, int beta) {
  apply_set({BfCall{&bf, 0, 0, alpha, 0.0, beta}}, X, ldx, Y, ldy, nrhs, adjoint);
}

template <class T>
void BfRuntime<T>::apply_set(const std::vector<BfCall>& calls, const void* X, int64_t ldx, void* Y, int64_t ldy,
                             int nrhs, bool adjoint) {
  BfPlan plan = make_plan(calls, adjoint, nrhs, ldx, ldy);
  auto mk = scratch.mark();
  void* ws = scratch.take(std::max<int64_t>(plan.ws_elems, 1) * sizeof(cplx<T>));
  int64_t rows_in = 0, rows_out = 0;
  for (auto& cl : calls) {
    rows_in = std::max<int64_t>(rows_in, cl.x_off + (adjoint ? cl.bf->m : cl.bf->n));
    rows_out = std::max<int64_t>(rows_out, cl.y_off + (adjoint ? cl.bf->n : cl.bf->m));
  }
  if (rows_in > ldx || rows_out > ldy) throw Error(BFMF_E_INVAL, "internal: butterfly product leading dimension");
  const int64_t lim[4] = {(int64_t)(pool.used / sizeof(cplx<T>)), ldx * nrhs, ldy * nrhs, std::max<int64_t>(plan.ws_elems, 1)};
  run_plan<T>(plan, *c, pool_base(), X, Y, ws, s(), lim);
  scratch.release(mk);
}

template <class T>
void BfRuntime<T>::apply_calls(const std::vector<BfCall>& calls, bool adjoint) {
  if (calls.empty()) return;
  for (auto& cl : calls) {
    const int64_t rows_in = cl.x_off + (adjoint ? cl.bf->m : cl.bf->n);
    const int64_t rows_out = cl.y_off + (adjoint ? cl.bf->n : cl.bf->m);
    if (cl.x_abs < 0 || cl.y_abs < 0 || cl.nrhs <= 0 || rows_in > cl.ldx || rows_out > cl.ldy)
      throw Error(BFMF_E_INVAL, "internal: butterfly call without its own buffers");
  }
  BfPlan plan = make_plan(calls, adjoint, 1, 1, 1);
  auto mk = scratch.mark();
  void* ws = scratch.take(std::max<int64_t>(plan.ws_elems, 1) * sizeof(cplx<T>));
  const int64_t lim[4] = {(int64_t)(pool.used / sizeof(cplx<T>)), 0, 0, std::max<int64_t>(plan.ws_elems, 1)};
  run_plan<T>(plan, *c, pool_base(), nullptr, nullptr, ws, s(), lim);
  scratch.release(mk);
}

template struct BfRuntime<double>;
template struct BfRuntime<float>;

// ------------------------------------------------------------ extraction
void ExtractBatch::add(const FrontDesc* fd, const void* dense, int64_t ldd, const std::vector<int32_t>& rows, int r0,
                       const std::vector<int32_t>& cols, int c0, void* out, int64_t ldo, bool trans) {
  if (rows.empty() || cols.empty()) return;
  ExtractTask e;
  std::memset(&e, 0, sizeof(e));
  e.rows = (const int32_t*)(intptr_t)idx.size();  // offsets into idx until the launch
  for (int32_t r : rows) idx.push_back(r0 + r);
  e.cols = (const int32_t*)(intptr_t)idx.size();
  for (int32_t c : cols) idx.push_back(c0 + c);
  e.nr = (int32_t)rows.size();
  e.nc = (int32_t)cols.size();
  e.out = out;
  e.ldo = std::max<int64_t>(ldo, 1);
  e.trans = trans ? 1 : 0;
  e.dense = dense;
  e.ldd = ldd;
  e.fd = fd;
  tasks.push_back(e);
}

void ExtractBatch::add_bf(const BfCentreDev* bf, const std::vector<int32_t>& rows, int r0,
                          const std::vector<int32_t>& cols, int c0, void* out, int64_t ldo, bool trans, double alpha,
                          bool accumulate) {
  if (rows.empty() || cols.empty()) return;
  BfExtractTask e;
  std::memset(&e, 0, sizeof(e));
  e.bf = bf;
  e.rows = (const int32_t*)(intptr_t)idx.size();
  for (int32_t r : rows) idx.push_back(r0 + r);
  e.cols = (const int32_t*)(intptr_t)idx.size();
  for (int32_t c : cols) idx.push_back(c0 + c);
  e.nr = (int32_t)rows.size();
  e.nc = (int32_t)cols.size();
  e.out = out;
  e.ldo = std::max<int64_t>(ldo, 1);
  e.trans = trans ? 1 : 0;
  e.accumulate = accumulate ? 1 : 0;
  e.alpha = alpha;
  bf_tasks.push_back(e);
}

template <class TO, class T>
void run_extract_to(BfRuntime<T>& rt, ExtractBatch& b, bool src_single) {
  HostTimer ht(HP_EXTRACT);
  if (b.tasks.empty() && b.bf_tasks.empty()) {
    b.idx.clear();
    return;
  }
  PackedUpload<BfRuntime<T>> pk(rt);  // index lists and tasks in one copy
  const int pi = pk.add(b.idx.data(), b.idx.size() * sizeof(int32_t));
  const int pt = pk.add(b.tasks.data(), b.tasks.size() * sizeof(ExtractTask));
  const int pb = pk.add(b.bf_tasks.data(), b.bf_tasks.size() * sizeof(BfExtractTask));
  int32_t* d_idx = (int32_t*)pk.part(pi);
  int64_t maxe = 0, maxb = 0;
  for (auto& e : b.tasks) {
    e.rows = d_idx + (intptr_t)e.rows;
    e.cols = d_idx + (intptr_t)e.cols;
    maxe = std::max<int64_t>(maxe, (int64_t)e.nr * e.nc);
  }
  for (auto& e : b.bf_tasks) {
    e.rows = d_idx + (intptr_t)e.rows;
    e.cols = d_idx + (intptr_t)e.cols;
    maxb = std::max<int64_t>(maxb, (int64_t)e.nr * e.nc);
  }
  ExtractTask* d_t = (ExtractTask*)pk.part(pt);
  void* d_b = pk.part(pb);
  pk.commit();
  KernelTimer& tm = rt.c->timer;
  const int tk = tm.want(K_EXTRACT) ? tm.begin(rt.s()) : -1;
  if (!b.tasks.empty()) {
    const int yb = (int)std::min<int64_t>(32, std::max<int64_t>(1, (maxe + 2047) / 2048));
    chk(launch_front_extract<TO>(d_t, (int)b.tasks.size(), yb, rt.c->d_values.p, src_single, rt.s()), "extract");
  }
  if (!b.bf_tasks.empty()) {  // after the front tasks: they may add to the same outputs
    const int yb = (int)std::min<int64_t>(32, std::max<int64_t>(1, (maxb + 2047) / 2048));
    chk(launch_bf_extract<TO>(d_b, (int)b.bf_tasks.size(), yb, rt.s()), "butterfly extract");
  }
  if (tk >= 0) {
    double by = 0;  // every output entry written once, plus its row and column index
    for (auto& e : b.tasks) by += (double)e.nr * e.nc * sizeof(cplx<TO>) + 4.0 * (e.nr + e.nc);
    for (auto& e : b.bf_tasks) by += (double)e.nr * e.nc * sizeof(cplx<TO>) + 4.0 * (e.nr + e.nc);
    tm.end(tk, rt.s(), K_EXTRACT, 0, by);
  }
  b.tasks.clear();
  b.bf_tasks.clear();
  b.idx.clear();
}

template <class T>
void run_extract(BfRuntime<T>& rt, ExtractBatch& b) {
  run_extract_to<T, T>(rt, b, false);
}

template void run_extract<double>(BfRuntime<double>&, ExtractBatch&);
template void run_extract<float>(BfRuntime<float>&, ExtractBatch&);
template void run_extract_to<double, double>(BfRuntime<double>&, ExtractBatch&, bool);
template void run_extract_to<double, float>(BfRuntime<float>&, ExtractBatch&, bool);
template void run_extract_to<float, float>(BfRuntime<float>&, ExtractBatch&, bool);

// ------------------------------------------------------------ centre forms
namespace {

// Placement of the centre forms of a set in one device buffer: per butterfly
// E and G of every centre block, then the copied dense blocks, then the
// descriptor arrays and the descriptors.
struct CentreLayout {
  std::vector<std::vector<size_t>> e, g;  // byte offsets per butterfly and centre block
  std::vector<size_t> dense;
  std::vector<size_t> tb, vb, rk, ep, gp;  // descriptor arrays per butterfly
  size_t descs = 0, total = 0;
};

template <class T>
CentreLayout centre_layout(const CentreSpec& spec) {
  const size_t esz = sizeof(cplx<T>);
  CentreLayout lay;
  size_t off = 0;
  auto take = [&](size_t bytes, size_t align) {
    off = (off + align - 1) / align * align;
    const size_t o = off;
    off += bytes;
    return o;
  };
  for (const Butterfly* bf : spec.bfs) {
    const int L = bf->L, lc = bf->lc, nt = 1 << lc, nv = 1 << (L - lc);
    std::vector<size_t> eo(nt * nv), go(nt * nv);
    for (int t = 0; t < nt; ++t)
      for (int v = 0; v < nv; ++v) {
        const int blk = t * nv + v, r = bf->rl[lc][blk];
        eo[blk] = take((size_t)bf->to.size(lc, t) * r * esz, 64);
        go[blk] = take((size_t)r * bf->ts.size(L - lc, v) * esz, 64);
      }
    lay.e.push_back(std::move(eo));
    lay.g.push_back(std::move(go));
  }
  for (auto& d : spec.dense) lay.dense.push_back(take((size_t)d.second * d.second * esz, 64));
  for (const Butterfly* bf : spec.bfs) {
    const int L = bf->L, lc = bf->lc, nt = 1 << lc, nv = 1 << (L - lc);
    lay.tb.push_back(take((size_t)(nt + 1) * 4, 8));
    lay.vb.push_back(take((size_t)(nv + 1) * 4, 8));
    lay.rk.push_back(take((size_t)nt * nv * 4, 8));
    lay.ep.push_back(take((size_t)nt * nv * sizeof(void*), 8));
    lay.gp.push_back(take((size_t)nt * nv * sizeof(void*), 8));
  }
  lay.descs = take(spec.bfs.size() * sizeof(BfCentreDev), 64);
  lay.total = std::max<size_t>(off, 64);
  return lay;
}

}  // namespace

template <class T>
size_t centre_bytes(const CentreSpec& spec) {
  return centre_layout<T>(spec).total;
}

// E of level l from E of level l + 1 (left factors, leaves to centre):
//   E_l(t, v) = [E_{l+1}(2t, v/2) R_top ; E_{l+1}(2t+1, v/2) R_bottom]
// with R the block's columns of its nu-pair matrix, split after the first
// child's rank; G = B F_lc with F of level l from level l - 1 (right factors):
//   F_l(t, v) = [W_1 F_{l-1}(t/2, 2v), W_2 F_{l-1}(t/2, 2v+1)]
// with W the block's rows of its tau-pair matrix, split after the first
// child's rank.  One grouped launch per level step for every butterfly.
template <class T>
CentreOut build_centres(BfRuntime<T>& rt, const CentreSpec& spec, char* mem) {
  const size_t esz = sizeof(cplx<T>);
  const CentreLayout lay = centre_layout<T>(spec);
  CentreOut out;
  hipStream_t s = rt.s();
  char* pool = rt.pool_base();
  auto mk = rt.scratch.mark();
  auto abs_off = [&](const void* p) { return (int64_t)((uintptr_t)p / esz); };
  BfPlan plan;
  std::vector<AxpbyTask> copies;  // U of a butterfly with lc == L, and the dense blocks
  int64_t maxcopy = 0;
  auto phase = [&](int k) -> std::vector<GTask>& {
    if ((int)plan.phase.size() <= k) plan.phase.resize(k + 1);
    return plan.phase[k];
  };
  auto gt = [](int64_t a_off, int64_t lda, int abase, int64_t b_off, int64_t ldb, int bbase, int64_t c_off,
               int64_t ldc, int M, int N, int K) {
    GTask t;
    std::memset(&t, 0, sizeof(t));
    t.a_off = a_off;
    t.lda = std::max<int64_t>(lda, 1);
    t.opA = OP_N;
    t.opB = OP_N;
    t.abase = (int8_t)abase;
    t.b_off = b_off;
    t.ldb = std::max<int64_t>(ldb, 1);
    t.bbase = (int8_t)bbase;
    t.c_off = c_off;
    t.ldc = std::max<int64_t>(ldc, 1);
    t.cbase = 4;
    t.M = M;
    t.N = N;
    t.K = K;
    t.alpha_re = 1.0;
    return t;
  };
  for (size_t b = 0; b < spec.bfs.size(); ++b) {
    const Butterfly& bf = *spec.bfs[b];
    const int L = bf.L, lc = bf.lc;
    // left side: E(l) per block as (address, is-pool-offset); level L is U in the pool
    std::vector<int64_t> eaddr(1 << L);  // element offset (pool) or absolute element address
    std::vector<int> ebase(1 << L, 0);
    for (int t = 0; t < (1 << L); ++t) eaddr[t] = bf.offL[L][t];
    if (lc == L) {
      for (int t = 0; t < (1 << L); ++t) {
        const int rows = bf.to.size(L, t), r = bf.rl[L][t];
        if (rows == 0 || r == 0) continue;
        copies.push_back(AxpbyTask{mem + lay.e[b][t], pool + bf.offL[L][t] * esz, rows, rows, rows, r, 0});
        maxcopy = std::max<int64_t>(maxcopy, (int64_t)rows * r);
      }
    }
    for (int l = L - 1; l >= lc; --l) {
      const int vs = 1 << (L - l), vs1 = vs / 2, step = L - 1 - l;
      std::vector<int64_t> naddr(1 << L, 0);
      for (int t = 0; t < (1 << l); ++t)
        for (int v = 0; v < vs; ++v) {
          const int blk = t * vs + v, r = bf.rl[l][blk];
          const int mt = bf.to.size(l, t), m1 = bf.to.size(l + 1, 2 * t), m2 = bf.to.size(l + 1, 2 * t + 1);
          char* dst = l == lc ? mem + lay.e[b][blk] : (char*)rt.scratch.take((size_t)mt * r * esz);
          naddr[blk] = abs_off(dst);
          if (r == 0 || mt == 0) continue;
          const int pair = blk / 2, col_off = (blk & 1) ? bf.rl[l][blk - 1] : 0;
          const int a1 = (2 * t) * vs1 + v / 2, b1 = (2 * t + 1) * vs1 + v / 2;
          const int top = bf.rl[l + 1][a1], rrows = top + bf.rl[l + 1][b1];
          const int64_t roff = bf.offL[l][pair] + (int64_t)col_off * rrows;
          const int ab = l + 1 == L ? 0 : 4;
          if (m1 > 0)
            phase(step).push_back(gt(eaddr[a1], m1, ab, roff, rrows, 0, naddr[blk], mt, m1, r, top));
          if (m2 > 0)
            phase(step).push_back(
                gt(eaddr[b1], m2, ab, roff + top, rrows, 0, naddr[blk] + m1, mt, m2, r, rrows - top));
        }
      eaddr.swap(naddr);
    }
    // right side: F(0) = Vt in the pool, then F(1..lc), then G = B F(lc)
    std::vector<int64_t> faddr(1 << L);
    for (int v = 0; v < (1 << L); ++v) faddr[v] = bf.offR[0][v];
    for (int l = 1; l <= lc; ++l) {
      const int vs = 1 << (L - l), step = l - 1;
      std::vector<int64_t> naddr(1 << L, 0);
      for (int t = 0; t < (1 << l); ++t)
        for (int v = 0; v < vs; ++v) {
          const int blk = t * vs + v, M = bf.rr[l][blk];
          const int n1 = bf.ts.size(L - l + 1, 2 * v), n2 = bf.ts.size(L - l + 1, 2 * v + 1);
          char* dst = (char*)rt.scratch.take((size_t)M * (n1 + n2) * esz);
          naddr[blk] = abs_off(dst);
          if (M == 0 || n1 + n2 == 0) continue;
          const int t2 = t / 2, q = t2 * vs + v;
          const int a = (2 * t2) * vs + v, bb = (2 * t2 + 1) * vs + v;
          const int wrows = bf.rr[l][a] + bf.rr[l][bb], row_off = (t & 1) ? bf.rr[l][a] : 0;
          const int ia = t2 * (2 * vs) + 2 * v;
          const int c1 = bf.rr[l - 1][ia], c2 = bf.rr[l - 1][ia + 1];
          const int64_t woff = bf.offR[l][q] + row_off;
          const int fb = l - 1 == 0 ? 0 : 4;
          if (n1 > 0) phase(step).push_back(gt(woff, wrows, 0, faddr[ia], c1, fb, naddr[blk], M, M, n1, c1));
          if (n2 > 0)
            phase(step).push_back(gt(woff + (int64_t)c1 * wrows, wrows, 0, faddr[ia + 1], c2, fb,
                                     naddr[blk] + (int64_t)n1 * M, M, M, n2, c2));
        }
      faddr.swap(naddr);
    }
    {
      const int nt = 1 << lc, nv = 1 << (L - lc), fb = lc == 0 ? 0 : 4;
      for (int t = 0; t < nt; ++t)
        for (int v = 0; v < nv; ++v) {
          const int blk = t * nv + v, M = bf.rl[lc][blk], K = bf.rr[lc][blk], N = bf.ts.size(L - lc, v);
          if (M == 0 || N == 0) continue;
          phase(lc).push_back(
              gt(bf.offB[blk], std::max(M, 1), 0, faddr[blk], std::max(K, 1), fb, abs_off(mem + lay.g[b][blk]), M, M, N, K));
        }
    }
  }
  for (size_t d = 0; d < spec.dense.size(); ++d) {
    const int n = spec.dense[d].second;
    out.dense.push_back(mem + lay.dense[d]);
    if (n == 0) continue;
    copies.push_back(AxpbyTask{mem + lay.dense[d], pool + spec.dense[d].first * esz, n, n, n, n, 0});
    maxcopy = std::max<int64_t>(maxcopy, (int64_t)n * n);
  }
  const int64_t lim[4] = {(int64_t)(rt.pool.used / esz), 0, 0, 0};
  run_plan<T>(plan, *rt.c, pool, nullptr, nullptr, nullptr, s, lim, K_BF_GEMM);
  if (!copies.empty())
    chk(launch_mix_batch<T, T>((const AxpbyTask*)upload_tmp(rt, copies), (int)copies.size(), maxcopy, 1.0, 0.0, 0.0,
                               s),
        "centre copies");
  // descriptors
  std::vector<char> h(lay.total, 0);
  const size_t dlo = lay.tb.empty() ? lay.descs : lay.tb[0];
  std::vector<BfCentreDev> descs(spec.bfs.size());
  for (size_t b = 0; b < spec.bfs.size(); ++b) {
    const Butterfly& bf = *spec.bfs[b];
    const int L = bf.L, lc = bf.lc, nt = 1 << lc, nv = 1 << (L - lc);
    std::memcpy(h.data() + lay.tb[b], bf.to.b[lc].data(), (size_t)(nt + 1) * 4);
    std::memcpy(h.data() + lay.vb[b], bf.ts.b[L - lc].data(), (size_t)(nv + 1) * 4);
    std::memcpy(h.data() + lay.rk[b], bf.rl[lc].data(), (size_t)nt * nv * 4);
    for (int blk = 0; blk < nt * nv; ++blk) {
      const void* e = mem + lay.e[b][blk];
      const void* g = mem + lay.g[b][blk];
      std::memcpy(h.data() + lay.ep[b] + blk * sizeof(void*), &e, sizeof(void*));
      std::memcpy(h.data() + lay.gp[b] + blk * sizeof(void*), &g, sizeof(void*));
    }
    BfCentreDev& d = descs[b];
    std::memset(&d, 0, sizeof(d));
    d.tb = (const int32_t*)(mem + lay.tb[b]);
    d.vb = (const int32_t*)(mem + lay.vb[b]);
    d.rk = (const int32_t*)(mem + lay.rk[b]);
    d.E = (const void* const*)(mem + lay.ep[b]);
    d.G = (const void* const*)(mem + lay.gp[b]);
    d.nt = nt;
    d.nv = nv;
    d.single = sizeof(T) == 4 ? 1 : 0;
  }
  if (!descs.empty()) std::memcpy(h.data() + lay.descs, descs.data(), descs.size() * sizeof(BfCentreDev));
  if (lay.total > dlo) rt.c->stage.put(mem + dlo, h.data() + dlo, lay.total - dlo, s);
  out.bfs = (const BfCentreDev*)(mem + lay.descs);
  // the intermediate levels are reused once the launches above have run (stream order)
  rt.scratch.release(mk);
  return out;
}

template size_t centre_bytes<double>(const CentreSpec&);
template size_t centre_bytes<float>(const CentreSpec&);
template CentreOut build_centres<double>(BfRuntime<double>&, const CentreSpec&, char*);
template CentreOut build_centres<float>(BfRuntime<float>&, const CentreSpec&, char*);

// ------------------------------------------------------------ construction
namespace {

// Interpolative decompositions of a list of blocks in one launch, in FP64
// whatever the runtime's precision: the blocks A_i are complex<double>; the
// expansion writes the interpolation matrices in the runtime's precision.
template <class T>
struct IdLevel {
  BfRuntime<T>& rt;
  explicit IdLevel(BfRuntime<T>& r) : rt(r) {}
  // widest block one ID kernel takes (the kernels' limits, or a smaller forced one)
  int max_cols() const {
    const int lim = rt.tol >= 1e-4 ? GRAM_MAXP : CPQR_MAXP;
    return rt.id_max_cols > 0 ? std::min(rt.id_max_cols, lim) : lim;
  }
  // blocks: A_i (q_i x p_i) already in device memory; returns ranks and perms.  Blocks wider than
  // max_cols() are decomposed as an ID of sub-IDs: IDs of column chunks, then the ID of the chunks'
  // skeleton columns, the interpolation matrices composed by one product per chunk.
  void run(const std::vector<void*>& A, const std::vector<int>& q, const std::vector<int>& p, std::vector<int>& rank,
           std::vector<std::vector<int32_t>>& perm) {
    const int lim = max_cols();
    bool wide = false;
    for (int pi : p) wide |= pi > lim;
    if (!wide) {
      run_direct(A, q, p, rank, perm);
      return;
    }
    run_chunked(A, q, p, rank, perm, lim);
  }

  void run_chunked(const std::vector<void*>& A, const std::vector<int>& q, const std::vector<int>& p,
                   std::vector<int>& rank, std::vector<std::vector<int32_t>>& perm, int lim);

  // householder: the Householder kernel whatever the tolerance (the Gram kernel's column limit is lower)
  void run_direct(const std::vector<void*>& A, const std::vector<int>& q, const std::vector<int>& p,
                  std::vector<int>& rank, std::vector<std::vector<int32_t>>& perm, bool householder = false) {
    const size_t nb = A.size();
    hipStream_t s = rt.s();
    std::vector<IdTask> tasks(nb);
    int64_t tot_perm = 0;
    for (size_t i = 0; i < nb; ++i) tot_perm += p[i];
    int32_t* d_rank = rt.scratch.template take_n<int32_t>(std::max<size_t>(nb, 1));
    int32_t* d_perm = rt.scratch.template take_n<int32_t>(std::max<int64_t>(tot_perm, 1));
    int64_t po = 0;
    // Gram variant for tolerances where eps p / tol^2 is negligible
    const bool gram = !householder && rt.tol >= 1e-4;
    for (size_t i = 0; i < nb; ++i) {
      // the Gram kernel takes up to GRAM_MAXP columns and any number of rows (it sees A^H A); the
      // Householder kernel up to CPQR_WIDE_MAXP columns and CPQR_MAXQ rows (run() splits blocks wider
      // than CPQR_MAXP into column chunks and sends a whole block only when its chunks have full rank)
      if (p[i] > (gram ? GRAM_MAXP : CPQR_WIDE_MAXP) || (!gram && q[i] > CPQR_MAXQ))
        throw Error(BFMF_E_INVAL, "ID block too large (" + std::to_string(q[i]) + " x " + std::to_string(p[i]) + ")");
      const int maxrank = std::max(1, std::min(p[i], q[i]));
      void* Tb = rt.scratch.take((size_t)maxrank * std::max(p[i], 1) * sizeof(cplx<double>));
      tasks[i] = IdTask{A[i], std::max(q[i], 1), q[i], p[i], maxrank, d_rank + i, d_perm + po, Tb, nullptr, nullptr};
      po += p[i];
    }
    // Gram variant (FP64): G_i = A_i^H A_i in one grouped GEMM
    if (gram) {
      std::vector<GTask> gt;
      for (size_t i = 0; i < nb; ++i) {
        const int pp = std::max(p[i], 1);
        tasks[i].G = rt.scratch.take((size_t)pp * pp * sizeof(cplx<double>));
        tasks[i].R = rt.scratch.take((size_t)tasks[i].maxrank * pp * sizeof(cplx<double>));
        if (p[i] <= 0) continue;
        GTask t = {};
        t.a_off = (int64_t)((uintptr_t)A[i] / sizeof(cplx<double>));
        t.lda = std::max(q[i], 1);
        t.opA = OP_C;
        t.abase = 4;
        t.b_off = t.a_off;
        t.ldb = t.lda;
        t.opB = OP_N;
        t.bbase = 4;
        t.c_off = (int64_t)((uintptr_t)tasks[i].G / sizeof(cplx<double>));
        t.ldc = p[i];
        t.cbase = 4;
        t.M = p[i];
        t.N = p[i];
        t.K = q[i];
        t.alpha_re = 1;
        t.beta = 0;
        gt.push_back(t);
      }
      if (!gt.empty()) {
        BfPlan gp;
        gp.phase.push_back(gt);
        const int64_t lim[4] = {0, 0, 0, 0};
        run_plan<double>(gp, *rt.c, nullptr, nullptr, nullptr, nullptr, s, lim, K_ID);
      }
    }
    IdTask* dt = (IdTask*)upload_tmp(rt, tasks);
    const bool vb = rt.c->verbose;
    if (vb) rt.c->stage.sync(s);
    const auto t_id0 = std::chrono::steady_clock::now();
    KernelTimer& tm = rt.c->timer;
    const int tk = tm.want(K_ID) ? tm.begin(s) : -1;
    int maxp = 16;
    for (const IdTask& t : tasks) maxp = std::max(maxp, (t.p + 15) / 16 * 16);
    // the largest R (kmax x p) that fits the LDS left beside the per-column state sizes the launch's LDS
    const int64_t lds_cap = std::min<int64_t>(GRAM_LDS_MAX, (int64_t)(GRAM_LDS_BYTES - gram_aux_bytes(maxp)) / 16);
    int lds_entries = 0;
    for (const IdTask& t : tasks) {
      const int64_t e = (int64_t)std::min(t.maxrank, t.p) * t.p;
      if (e <= lds_cap) lds_entries = std::max<int>(lds_entries, (int)e);
    }
    if (gram)
      chk(launch_gram_id<double>(dt, (int)nb, rt.tol, lds_entries, maxp, s), "gram id");
    else
      chk(launch_cpqr_id<double>(dt, (int)nb, rt.tol, maxp, s), "cpqr");
    if (tk >= 0) {
      double fl = 0, by = 0;  // pivoted QR of q x p truncated at rank k ~ min(p, q): 8 q p k flops, A read and written
      for (size_t i = 0; i < nb; ++i) {
        const double qq = q[i], pp = p[i], kk = std::min(q[i], p[i]);
        fl += 8.0 * qq * pp * kk;
        by += 2.0 * sizeof(cplx<double>) * qq * pp;
      }
      tm.end(tk, s, K_ID, fl, by);
    }
    rank.assign(nb, 0);
    std::vector<int32_t> hp(std::max<int64_t>(tot_perm, 1));
    chk(hipMemcpyAsync(rank.data(), d_rank, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s), "rank");
    chk(hipMemcpyAsync(hp.data(), d_perm, std::max<int64_t>(tot_perm, 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s),
        "perm");
    rt.c->stage.sync(s);
    if (vb) {  // one line per ID launch: blocks, largest q, p and rank, wall time of launch + wait
      int mq = 0, mp = 0, mr = 0;
      double work = 0;
      for (size_t i = 0; i < nb; ++i) {
        mq = std::max(mq, q[i]);
        mp = std::max(mp, p[i]);
        mr = std::max(mr, rank[i]);
        work = std::max(work, (double)q[i] * p[i] * rank[i]);
      }
      const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t_id0).count();
      fprintf(stderr, "[bfmf-id] blocks %zu maxq %d maxp %d maxrank %d maxqpk %.3g us %.1f\n", nb, mq, mp, mr, work, us);
    }
    perm.assign(nb, {});
    po = 0;
    for (size_t i = 0; i < nb; ++i) {
      if (rank[i] < 0) throw Error(BFMF_E_INVAL, "ID block refused by the kernel");
      perm[i].assign(hp.begin() + po, hp.begin() + po + p[i]);
      po += p[i];
    }
    d_tasks = dt;
    ntasks = (int)nb;
    htasks = tasks;
  }
  // expand the interpolation matrices into outs (device, ld per block)
  void expand(const std::vector<void*>& outs, const std::vector<int64_t>& ldo, bool transpose, bool conj) {
    if (ntasks == 0) return;
    PackedUpload<BfRuntime<T>> pk(rt);  // both arrays in one copy
    const int po = pk.add(outs.data(), outs.size() * sizeof(void*));
    const int pl = pk.add(ldo.data(), ldo.size() * sizeof(int64_t));
    void** d_outs = (void**)pk.part(po);
    int64_t* d_ldo = (int64_t*)pk.part(pl);
    pk.commit();
    chk(launch_id_expand<T>(d_tasks, ntasks, d_outs, d_ldo, transpose, conj, rt.s()), "id expand");
  }
  IdTask* d_tasks = nullptr;
  int ntasks = 0;
  std::vector<IdTask> htasks;  // host copy of the tasks behind d_tasks
};

// ID of sub-IDs for blocks wider than one kernel takes.  A block's columns are split into chunks of
// at most lim; chunk c gives A(:, c) ~= A(:, J_c) Z_c.  The chunks' skeleton columns, side by side,
// form A2 = A(:, J_1 .. J_m), whose ID A2 ~= A(:, J) Z2 (again chunked if A2 is still too wide)
// gives the block's skeleton J and, per chunk, Z(:, c) = Z2(:, J_c part) Z_c: one grouped product.
// The interpolation error is that of the two levels of IDs added (about twice the tolerance).
template <class T>
void IdLevel<T>::run_chunked(const std::vector<void*>& A, const std::vector<int>& q, const std::vector<int>& p,
                             std::vector<int>& rank, std::vector<std::vector<int32_t>>& perm, int lim) {
  const size_t nb = A.size();
  hipStream_t s = rt.s();
  const size_t esz = sizeof(cplx<double>);
  // stage 1: narrow blocks as they are, wide blocks as chunks, all in one launch
  std::vector<void*> A1;
  std::vector<int> q1, p1;
  std::vector<int> first(nb), nchunk(nb, 1);
  std::vector<std::vector<int>> cbeg(nb);
  for (size_t i = 0; i < nb; ++i) {
    first[i] = (int)A1.size();
    if (p[i] <= lim) {
      A1.push_back(A[i]);
      q1.push_back(q[i]);
      p1.push_back(p[i]);
      cbeg[i] = {0, p[i]};
      continue;
    }
    // chunks of near-equal width w <= lim (their number can fall below ceil(p / lim): count them)
    const int m = (p[i] + lim - 1) / lim, w = (p[i] + m - 1) / m;
    ++rt.n_chunked;
    for (int c0 = 0; c0 < p[i]; c0 += w) {
      const int pc = std::min(w, p[i] - c0);
      A1.push_back((char*)A[i] + (size_t)c0 * std::max(q[i], 1) * esz);
      q1.push_back(q[i]);
      p1.push_back(pc);
      cbeg[i].push_back(c0);
    }
    nchunk[i] = (int)cbeg[i].size();
    cbeg[i].push_back(p[i]);
  }
  // the Householder kernel overwrites its blocks: keep the wide blocks' columns for the second stage
  std::vector<const cplx<double>*> src(nb);
  {
    std::vector<AxpbyTask> cp;
    for (size_t i = 0; i < nb; ++i) {
      src[i] = (const cplx<double>*)A[i];
      if (nchunk[i] == 1 || rt.tol >= 1e-4) continue;
      const int qq = std::max(q[i], 1);
      cplx<double>* keep = (cplx<double>*)rt.scratch.take((size_t)qq * std::max(p[i], 1) * esz);
      cp.push_back(AxpbyTask{keep, A[i], qq, qq, q[i], p[i], 0});
      src[i] = keep;
    }
    int64_t maxe = 0;
    for (const AxpbyTask& t : cp) maxe = std::max<int64_t>(maxe, t.m * t.ncol);
    if (!cp.empty())
      chk(launch_axpby_batch<double>((const AxpbyTask*)upload_tmp(rt, cp), (int)cp.size(), maxe, 1.0, 0.0, s),
          "keep wide blocks");
  }
  std::vector<int> r1;
  std::vector<std::vector<int32_t>> perm1;
  run_direct(A1, q1, p1, r1, perm1);
  const std::vector<IdTask> t1 = htasks;
  IdTask* d_t1 = d_tasks;
  std::vector<IdTask> out(nb);
  rank.assign(nb, 0);
  perm.assign(nb, {});
  std::vector<AxpbyTask> gather;  // column copies, run together per phase
  for (size_t i = 0; i < nb; ++i) {
    if (nchunk[i] == 1) {
      out[i] = t1[first[i]];
      rank[i] = r1[first[i]];
      perm[i] = perm1[first[i]];
      continue;
    }
    // the chunks' skeleton columns side by side
    std::vector<int32_t> Jall;
    std::vector<int> soff;
    for (int c = 0; c < nchunk[i]; ++c) {
      const int k = first[i] + c;
      soff.push_back((int)Jall.size());
      for (int t = 0; t < r1[k]; ++t) Jall.push_back(cbeg[i][c] + perm1[k][t]);
    }
    soff.push_back((int)Jall.size());
    const int ns = (int)Jall.size(), qq = std::max(q[i], 1);
    // every chunk of full rank: a second stage would be as wide as the block (no progress), so the
    // whole block is decomposed directly instead: by the runtime's own kernel where it fits (the cap
    // was forced lower), else by the Householder kernel up to its wide limit, on a copy in the Gram
    // case (the Householder kernel overwrites its block, the Gram kernel leaves it as it was)
    if (ns >= p[i]) {
      const bool gram = rt.tol >= 1e-4;
      const bool wide = p[i] > (gram ? GRAM_MAXP : CPQR_MAXP);
      if (wide && (p[i] > CPQR_WIDE_MAXP || q[i] > CPQR_MAXQ))
        throw Error(BFMF_E_INVAL, "ID block of " + std::to_string(q[i]) + " x " + std::to_string(p[i]) +
                                      ": its column chunks of at most " + std::to_string(lim) +
                                      " have full rank, and the block is larger than one decomposition kernel"
                                      " takes");
      void* blk = (void*)src[i];
      if (wide && gram) {
        blk = rt.scratch.take((size_t)qq * std::max(p[i], 1) * esz);
        const AxpbyTask cp{blk, src[i], qq, qq, q[i], p[i], 0};
        chk(launch_axpby_batch<double>((const AxpbyTask*)upload_tmp(rt, std::vector<AxpbyTask>{cp}), 1,
                                       (int64_t)q[i] * p[i], 1.0, 0.0, s),
            "copy the wide block");
      }
      IdLevel<T> whole(rt);
      std::vector<int> rw;
      std::vector<std::vector<int32_t>> pw;
      whole.run_direct({blk}, {q[i]}, {p[i]}, rw, pw, wide);
      out[i] = whole.htasks[0];
      rank[i] = rw[0];
      perm[i] = pw[0];
      continue;
    }
    cplx<double>* A2 = (cplx<double>*)rt.scratch.take((size_t)std::max(ns, 1) * qq * esz);
    gather.clear();
    for (int t = 0; t < ns; ++t)
      gather.push_back(AxpbyTask{A2 + (size_t)t * qq, src[i] + (size_t)Jall[t] * qq, qq, qq, q[i], 1, 0});
    if (!gather.empty())
      chk(launch_axpby_batch<double>((const AxpbyTask*)upload_tmp(rt, gather), (int)gather.size(), q[i], 1.0, 0.0, s),
          "gather skeleton columns");
    IdLevel<T> sub(rt);
    std::vector<int> r2;
    std::vector<std::vector<int32_t>> perm2;
    sub.run({(void*)A2}, {q[i]}, {ns}, r2, perm2);
    const int r = r2[0];
    // dense interpolation matrices: Z2 (r x ns) and Z_c (r_c x p_c), written transposed by the expansion
    cplx<double>* Z2 = (cplx<double>*)rt.scratch.take((size_t)std::max(r, 1) * std::max(ns, 1) * esz);
    std::vector<void*> zo{Z2};
    std::vector<int64_t> zl{std::max(r, 1)};
    {
      PackedUpload<BfRuntime<T>> pk(rt);
      const int po = pk.add(zo.data(), sizeof(void*)), pl = pk.add(zl.data(), sizeof(int64_t));
      void** d_o = (void**)pk.part(po);
      int64_t* d_l = (int64_t*)pk.part(pl);
      pk.commit();
      if (r > 0) chk(launch_id_expand<double>(sub.d_tasks, 1, d_o, d_l, true, false, s), "expand Z2");
    }
    std::vector<cplx<double>*> Zc(nchunk[i]);
    {
      std::vector<void*> co;
      std::vector<int64_t> cl;
      for (int c = 0; c < nchunk[i]; ++c) {
        const int k = first[i] + c;
        Zc[c] = (cplx<double>*)rt.scratch.take((size_t)std::max(r1[k], 1) * std::max(p1[k], 1) * esz);
        co.push_back(Zc[c]);
        cl.push_back(std::max(r1[k], 1));
      }
      PackedUpload<BfRuntime<T>> pk(rt);
      const int po = pk.add(co.data(), co.size() * sizeof(void*)), pl = pk.add(cl.data(), cl.size() * sizeof(int64_t));
      void** d_o = (void**)pk.part(po);
      int64_t* d_l = (int64_t*)pk.part(pl);
      pk.commit();
      chk(launch_id_expand<double>(d_t1 + first[i], nchunk[i], d_o, d_l, true, false, s), "expand Z_c");
    }
    // Z (r x p) = per chunk Z2(:, soff_c .. soff_c + r_c) Z_c
    const int maxrank = std::max(1, std::min(p[i], q[i]));
    cplx<double>* Z = (cplx<double>*)rt.scratch.take((size_t)std::max(r, 1) * std::max(p[i], 1) * esz);
    std::vector<GTask> gt;
    for (int c = 0; c < nchunk[i]; ++c) {
      const int k = first[i] + c, rc = r1[k], pc = p1[k];
      if (r == 0 || pc == 0) continue;
      GTask g = {};
      g.a_off = (int64_t)((uintptr_t)(Z2 + (size_t)soff[c] * std::max(r, 1)) / esz);
      g.lda = std::max(r, 1);
      g.opA = OP_N;
      g.abase = 4;
      g.b_off = (int64_t)((uintptr_t)Zc[c] / esz);
      g.ldb = std::max(rc, 1);
      g.opB = OP_N;
      g.bbase = 4;
      g.c_off = (int64_t)((uintptr_t)(Z + (size_t)cbeg[i][c] * std::max(r, 1)) / esz);
      g.ldc = std::max(r, 1);
      g.cbase = 4;
      g.M = r;
      g.N = pc;
      g.K = rc;
      g.alpha_re = 1;
      g.beta = 0;
      if (rc == 0) {  // no skeleton in the chunk: its columns interpolate to zero
        gather.clear();
        gather.push_back(AxpbyTask{Z + (size_t)cbeg[i][c] * r, nullptr, r, r, r, pc, 0});
        chk(launch_axpby_batch<double>((const AxpbyTask*)upload_tmp(rt, gather), 1, (int64_t)r * pc, 0.0, 0.0, s),
            "zero chunk");
        continue;
      }
      gt.push_back(g);
    }
    if (!gt.empty()) {
      BfPlan gp;
      gp.phase.push_back(gt);
      const int64_t lim4[4] = {0, 0, 0, 0};
      run_plan<double>(gp, *rt.c, nullptr, nullptr, nullptr, nullptr, s, lim4, K_ID);
    }
    // the block's ID: skeleton J (in the order of the second ID), then the other columns ascending;
    // T = Z(:, other columns)
    std::vector<int32_t> pm;
    std::vector<char> isk(p[i], 0);
    for (int t = 0; t < r; ++t) {
      pm.push_back(Jall[perm2[0][t]]);
      isk[Jall[perm2[0][t]]] = 1;
    }
    for (int j = 0; j < p[i]; ++j)
      if (!isk[j]) pm.push_back(j);
    cplx<double>* Tb = (cplx<double>*)rt.scratch.take((size_t)maxrank * std::max(p[i], 1) * esz);
    gather.clear();
    for (int c = 0; c + r < p[i]; ++c)
      if (r > 0) gather.push_back(AxpbyTask{Tb + (size_t)c * maxrank, Z + (size_t)pm[r + c] * r, maxrank, r, r, 1, 0});
    if (!gather.empty())
      chk(launch_axpby_batch<double>((const AxpbyTask*)upload_tmp(rt, gather), (int)gather.size(), r, 1.0, 0.0, s),
          "interpolation columns");
    int32_t* d_rk = rt.scratch.template take_n<int32_t>(1);
    int32_t* d_pm = (int32_t*)upload_tmp(rt, pm);
    const std::vector<int32_t> rk{r};
    rt.c->stage.put(d_rk, rk.data(), sizeof(int32_t), s);
    out[i] = IdTask{A[i], qq, q[i], p[i], maxrank, d_rk, d_pm, Tb, nullptr, nullptr};
    rank[i] = r;
    perm[i] = pm;
  }
  htasks = out;
  d_tasks = (IdTask*)upload_tmp(rt, out);
  ntasks = (int)nb;
}

template <class T>
struct FactorAlloc {
  BfRuntime<T>& rt;
  Butterfly& bf;
  int64_t alloc(int64_t elems) {
    const size_t off = rt.pool.alloc((size_t)std::max<int64_t>(elems, 1) * sizeof(cplx<T>), rt.s());
    bf.elems += elems;
    return (int64_t)(off / sizeof(cplx<T>));
  }
};

void init_bf(Butterfly& bf, const BTree& to, const BTree& ts) {
  if (to.L != ts.L) throw Error(BFMF_E_INVAL, "butterfly trees of different depth");
  bf.to = to;
  bf.ts = ts;
  bf.m = to.n;
  bf.n = ts.n;
  bf.L = to.L;
  bf.lc = bf.L / 2;
  const int nb = 1 << bf.L;
  bf.rl.assign(bf.L + 1, {});
  bf.rr.assign(bf.L + 1, {});
  bf.Ob.assign(bf.L + 1, {});
  bf.Sb.assign(bf.L + 1, {});
  bf.offL.assign(bf.L + 1, {});
  bf.offR.assign(bf.L + 1, {});
  for (int l = bf.lc; l <= bf.L; ++l) {
    bf.rl[l].assign(nb, 0);
    bf.Ob[l].assign(nb, {});
  }
  for (int l = 0; l <= bf.lc; ++l) {
    bf.rr[l].assign(nb, 0);
    bf.Sb[l].assign(nb, {});
  }
  bf.offB.assign(nb, 0);
}

// candidate rows of left block (l, t, v)
std::vector<int32_t> left_rows(const Butterfly& bf, int l, int t, int v) {
  std::vector<int32_t> rows;
  if (l == bf.L) {
    for (int i = bf.to.beg(l, t); i < bf.to.end(l, t); ++i) rows.push_back(i);
  } else {
    const int vs1 = 1 << (bf.L - l - 1);
    const auto& a = bf.Ob[l + 1][(2 * t) * vs1 + v / 2];
    const auto& b = bf.Ob[l + 1][(2 * t + 1) * vs1 + v / 2];
    rows = a;
    rows.insert(rows.end(), b.begin(), b.end());
  }
  return rows;
}

std::vector<int32_t> right_cols(const Butterfly& bf, int l, int t, int v) {
  std::vector<int32_t> cols;
  if (l == 0) {
    for (int j = bf.ts.beg(bf.L, v); j < bf.ts.end(bf.L, v); ++j) cols.push_back(j);
  } else {
    const int vs0 = 1 << (bf.L - l + 1);
    const auto& a = bf.Sb[l - 1][(t / 2) * vs0 + 2 * v];
    const auto& b = bf.Sb[l - 1][(t / 2) * vs0 + 2 * v + 1];
    cols = a;
    cols.insert(cols.end(), b.begin(), b.end());
  }
  return cols;
}

// allocate level storage after the ranks of level l (left side) are known
template <class T>
void alloc_left(FactorAlloc<T>& fa, Butterfly& bf, int l) {
  const int nb = 1 << bf.L;
  if (l == bf.L) {
    bf.offL[l].assign(nb, 0);
    for (int t = 0; t < nb; ++t) bf.offL[l][t] = fa.alloc((int64_t)bf.to.size(l, t) * bf.rl[l][t]);
  } else {
    const int vs1 = 1 << (bf.L - l - 1);
    bf.offL[l].assign(nb / 2, 0);
    for (int pr = 0; pr < nb / 2; ++pr) {
      const int t = pr / vs1, v1 = pr % vs1;
      const int rows = bf.rl[l + 1][(2 * t) * vs1 + v1] + bf.rl[l + 1][(2 * t + 1) * vs1 + v1];
      bf.offL[l][pr] = fa.alloc((int64_t)rows * (bf.rl[l][2 * pr] + bf.rl[l][2 * pr + 1]));
    }
  }
}

// destinations of the interpolation matrices of left level l (appended)
template <class T>
void left_outs(BfRuntime<T>& rt, Butterfly& bf, int l, std::vector<void*>& outs, std::vector<int64_t>& ldo) {
  const int nb = 1 << bf.L;
  char* base = rt.pool_base();
  for (int blk = 0; blk < nb; ++blk) {
    if (l == bf.L) {
      outs.push_back(base + bf.offL[l][blk] * sizeof(cplx<T>));
      ldo.push_back(std::max(1, bf.to.size(l, blk)));
    } else {
      const int vs1 = 1 << (bf.L - l - 1);
      const int pr = blk / 2, t = pr / vs1, v1 = pr % vs1;
      const int rows = bf.rl[l + 1][(2 * t) * vs1 + v1] + bf.rl[l + 1][(2 * t + 1) * vs1 + v1];
      const int col_off = (blk & 1) ? bf.rl[l][blk - 1] : 0;
      outs.push_back(base + (bf.offL[l][pr] + (int64_t)col_off * rows) * sizeof(cplx<T>));
      ldo.push_back(std::max(rows, 1));
    }
  }
}

template <class T>
void alloc_right(FactorAlloc<T>& fa, Butterfly& bf, int l) {
  const int nb = 1 << bf.L;
  if (l == 0) {
    bf.offR[0].assign(nb, 0);
    for (int v = 0; v < nb; ++v) bf.offR[0][v] = fa.alloc((int64_t)bf.rr[0][v] * bf.ts.size(bf.L, v));
  } else {
    const int vs = 1 << (bf.L - l), vs0 = 2 * vs;
    bf.offR[l].assign(nb / 2, 0);
    for (int t2 = 0; t2 < (1 << (l - 1)); ++t2)
      for (int v = 0; v < vs; ++v) {
        const int q = t2 * vs + v;
        const int a = (2 * t2) * vs + v, b = (2 * t2 + 1) * vs + v;
        const int cols = bf.rr[l - 1][t2 * vs0 + 2 * v] + bf.rr[l - 1][t2 * vs0 + 2 * v + 1];
        bf.offR[l][q] = fa.alloc((int64_t)(bf.rr[l][a] + bf.rr[l][b]) * cols);
      }
  }
}

// destinations of the interpolation matrices of right level l (appended)
template <class T>
void right_outs(BfRuntime<T>& rt, Butterfly& bf, int l, std::vector<void*>& outs, std::vector<int64_t>& ldo) {
  const int nb = 1 << bf.L;
  char* base = rt.pool_base();
  const int vs = 1 << (bf.L - l);
  for (int blk = 0; blk < nb; ++blk) {
    if (l == 0) {
      outs.push_back(base + bf.offR[0][blk] * sizeof(cplx<T>));
      ldo.push_back(std::max(1, bf.rr[0][blk]));
    } else {
      const int t = blk / vs, v = blk % vs, t2 = t / 2;
      const int q = t2 * vs + v;
      const int a = (2 * t2) * vs + v, b = (2 * t2 + 1) * vs + v;
      const int rows = bf.rr[l][a] + bf.rr[l][b];
      const int row_off = (t & 1) ? bf.rr[l][a] : 0;
      outs.push_back(base + (bf.offR[l][q] + row_off) * sizeof(cplx<T>));
      ldo.push_back(std::max(rows, 1));
    }
  }
}

// One block of a construction step: its butterfly, position and candidates.
struct StepBlock {
  Butterfly* bf;
  int blk, level;
  std::vector<int32_t> cand;  // candidate rows (left) or columns (right)
};

// After the IDs of one step: record ranks and skeletons, allocate the level,
// and expand the interpolation matrices of every block in one launch.
template <class T>
void finish_step(BfRuntime<T>& rt, IdLevel<T>& idl, std::vector<StepBlock>& blocks, const std::vector<int>& rank,
                 const std::vector<std::vector<int32_t>>& perm, const std::vector<Butterfly*>& act,
                 const std::vector<int>& act_level, bool left, bool conj) {
  for (size_t b = 0; b < blocks.size(); ++b) {
    Butterfly& bf = *blocks[b].bf;
    const int blk = blocks[b].blk;
    const int l = blocks[b].level;
    auto& r = left ? bf.rl[l][blk] : bf.rr[l][blk];
    auto& sk = left ? bf.Ob[l][blk] : bf.Sb[l][blk];
    r = rank[b];
    sk.clear();
    for (int k = 0; k < rank[b]; ++k) sk.push_back(blocks[b].cand[perm[b][k]]);
  }
  // every allocation first: the pool may move while it grows
  for (size_t a = 0; a < act.size(); ++a) {
    FactorAlloc<T> fa{rt, *act[a]};
    if (left)
      alloc_left(fa, *act[a], act_level[a]);
    else
      alloc_right(fa, *act[a], act_level[a]);
  }
  std::vector<void*> outs;
  std::vector<int64_t> ldo;
  for (size_t a = 0; a < act.size(); ++a) {
    if (left)
      left_outs(rt, *act[a], act_level[a], outs, ldo);
    else
      right_outs(rt, *act[a], act_level[a], outs, ldo);
  }
  idl.expand(outs, ldo, !left, conj);
}

}  // namespace

// ----------------------------------------------------------- Alg. 2
// one construction step of one job: its blocks (candidates) and their proxies
struct JobStep {
  int l = -1;
  std::vector<StepBlock> blocks;
  std::vector<std::vector<int32_t>> prox;
};

template <class T>
void bf_entry_eval_batch(BfRuntime<T>& rt, const std::vector<EntryJob<T>*>& jobs) {
  if (jobs.empty()) return;
  HostTimer ht(HP_ENTRY);
  auto mk = rt.scratch.mark();
  for (auto* j : jobs) {
    j->out = std::make_unique<Butterfly>();
    init_bf(*j->out, j->to, j->ts);
    ++rt.n_entry;
  }
  // left to middle: row IDs of K(rows, proxy columns); step k works on level L - k of every butterfly
  for (int k = 0;; ++k) {
    auto smk = rt.scratch.mark();
    ExtractBatch eb;
    std::vector<StepBlock> blocks;
    std::vector<void*> A;
    std::vector<int> q, p;
    std::vector<Butterfly*> act;
    std::vector<int> act_level;
    // candidates and proxy columns of every block, in parallel over the jobs (a job's sampler stays on
    // one thread and runs in block order, so the proxies do not depend on the threads)
    std::vector<JobStep> js(jobs.size());
    HostPool::get().parallel_for(jobs.size(), [&](size_t ji) {
      Butterfly& bf = *jobs[ji]->out;
      const int L = bf.L, l = L - k;
      JobStep& st = js[ji];
      st.l = l < bf.lc ? -1 : l;
      if (st.l < 0) return;
      const int vs = 1 << (L - l);
      st.blocks.reserve(1 << L);
      st.prox.resize(1 << L);
      for (int blk = 0; blk < (1 << L); ++blk) {
        const int t = blk / vs, v = blk % vs;
        st.blocks.push_back(StepBlock{&bf, blk, l, left_rows(bf, l, t, v)});
        jobs[ji]->ps->columns(st.blocks.back().cand, bf.ts.beg(L - l, v), bf.ts.end(L - l, v), st.prox[blk]);
      }
    });
    for (size_t ji = 0; ji < jobs.size(); ++ji) {
      auto* j = jobs[ji];
      JobStep& st = js[ji];
      if (st.l < 0) continue;
      act.push_back(j->out.get());
      act_level.push_back(st.l);
      for (size_t blk = 0; blk < st.blocks.size(); ++blk) {
        StepBlock& sb = st.blocks[blk];
        const std::vector<int32_t>& cols = st.prox[blk];
        const int pp = (int)sb.cand.size(), qq = (int)cols.size();
        void* a = rt.scratch.take((size_t)std::max(pp * qq, 1) * sizeof(cplx<double>));
        j->src->request(eb, sb.cand, cols, a, std::max(qq, 1), true);  // A = K(rows, cols)^T, q x p
        A.push_back(a);
        q.push_back(qq);
        p.push_back(pp);
        blocks.push_back(std::move(sb));
      }
    }
    if (act.empty()) break;
    run_extract_to<double>(rt, eb, false);
    IdLevel<T> idl(rt);
    std::vector<int> rank;
    std::vector<std::vector<int32_t>> perm;
    idl.run(A, q, p, rank, perm);
    finish_step(rt, idl, blocks, rank, perm, act, act_level, true, false);
    rt.scratch.release(smk);
  }
  // right to middle: column IDs of K(proxy rows, cols); step k works on level k
  for (int k = 0;; ++k) {
    auto smk = rt.scratch.mark();
    ExtractBatch eb;
    std::vector<StepBlock> blocks;
    std::vector<void*> A;
    std::vector<int> q, p;
    std::vector<Butterfly*> act;
    std::vector<int> act_level;
    std::vector<JobStep> js(jobs.size());
    HostPool::get().parallel_for(jobs.size(), [&](size_t ji) {
      Butterfly& bf = *jobs[ji]->out;
      const int L = bf.L, l = k;
      JobStep& st = js[ji];
      st.l = l > bf.lc ? -1 : l;
      if (st.l < 0) return;
      const int vs = 1 << (L - l);
      st.blocks.reserve(1 << L);
      st.prox.resize(1 << L);
      for (int blk = 0; blk < (1 << L); ++blk) {
        const int t = blk / vs, v = blk % vs;
        st.blocks.push_back(StepBlock{&bf, blk, l, right_cols(bf, l, t, v)});
        jobs[ji]->ps->rows(st.blocks.back().cand, bf.to.beg(l, t), bf.to.end(l, t), st.prox[blk]);
      }
    });
    for (size_t ji = 0; ji < jobs.size(); ++ji) {
      auto* j = jobs[ji];
      JobStep& st = js[ji];
      if (st.l < 0) continue;
      act.push_back(j->out.get());
      act_level.push_back(st.l);
      for (size_t blk = 0; blk < st.blocks.size(); ++blk) {
        StepBlock& sb = st.blocks[blk];
        const std::vector<int32_t>& rows = st.prox[blk];
        const int pp = (int)sb.cand.size(), qq = (int)rows.size();
        void* a = rt.scratch.take((size_t)std::max(pp * qq, 1) * sizeof(cplx<double>));
        j->src->request(eb, rows, sb.cand, a, std::max(qq, 1), false);  // A = K(rows, cols), q x p
        A.push_back(a);
        q.push_back(qq);
        p.push_back(pp);
        blocks.push_back(std::move(sb));
      }
    }
    if (act.empty()) break;
    run_extract_to<double>(rt, eb, false);
    IdLevel<T> idl(rt);
    std::vector<int> rank;
    std::vector<std::vector<int32_t>> perm;
    idl.run(A, q, p, rank, perm);
    finish_step(rt, idl, blocks, rank, perm, act, act_level, false, false);
    rt.scratch.release(smk);
  }
  // centre: B = K(Obar, Sbar); every allocation first (the pool may move)
  for (auto* j : jobs) {
    Butterfly& bf = *j->out;
    FactorAlloc<T> fa{rt, bf};
    for (int blk = 0; blk < (1 << bf.L); ++blk) bf.offB[blk] = fa.alloc((int64_t)bf.rl[bf.lc][blk] * bf.rr[bf.lc][blk]);
  }
  ExtractBatch eb;
  for (auto* j : jobs) {
    Butterfly& bf = *j->out;
    for (int blk = 0; blk < (1 << bf.L); ++blk)
      j->src->request(eb, bf.Ob[bf.lc][blk], bf.Sb[bf.lc][blk], rt.pool_base() + bf.offB[blk] * sizeof(cplx<T>),
                      std::max(1, bf.rl[bf.lc][blk]), false);
  }
  run_extract(rt, eb);
  rt.scratch.release(mk);
  for (auto* j : jobs) rt.max_rank_seen = std::max(rt.max_rank_seen, j->out->max_rank());
}

template <class T>
std::unique_ptr<Butterfly> bf_entry_eval(BfRuntime<T>& rt, EntrySource<T>& src, ProxySampler& ps, const BTree& to,
                                         const BTree& ts) {
  EntryJob<T> j{&src, &ps, to, ts, nullptr};
  bf_entry_eval_batch<T>(rt, {&j});
  return std::move(j.out);
}

// ----------------------------------------------------------- Sec. 3.3
namespace {

template <class T>
struct Sketch {
  int ncl = 0, ncr = 0;
  std::vector<int> lcol0, rcol0;
  void *Om = nullptr, *Y = nullptr, *Ps = nullptr, *Z = nullptr;
};

// One attempt of the randomized construction for every job at its sample count.
template <class T>
void random_once_batch(BfRuntime<T>& rt, const std::vector<RandomJob<T>*>& jobs) {
  hipStream_t s = rt.s();
  auto mk = rt.scratch.mark();
  const size_t nj = jobs.size();
  std::vector<Sketch<T>> sk(nj);
  // probes and sketches: Y = K Omega (column groups of left levels), Z = K^H Psi (row groups of right levels);
  // the probe blocks of every job are drawn in one launch (each keeps its own generator stream)
  std::vector<ProbeTask> ptasks;
  std::vector<int32_t> gbeg, gend;
  int64_t pmax = 0;
  for (size_t ji = 0; ji < nj; ++ji) {
    RandomJob<T>& j = *jobs[ji];
    j.out = std::make_unique<Butterfly>();
    Butterfly& bf = *j.out;
    init_bf(bf, j.to, j.ts);
    const int L = bf.L, lc = bf.lc, S = j.S, m = j.to.n, n = j.ts.n;
    Sketch<T>& w = sk[ji];
    std::vector<int32_t> gb, ge, hb, he;
    w.lcol0.assign(L + 1, 0);
    for (int l = L; l >= lc; --l) {
      w.lcol0[l] = (int)gb.size() * S;
      for (int v = 0; v < (1 << (L - l)); ++v) {
        gb.push_back(j.ts.beg(L - l, v));
        ge.push_back(j.ts.end(L - l, v));
      }
    }
    w.ncl = (int)gb.size() * S;
    w.rcol0.assign(lc + 1, 0);
    for (int l = 0; l <= lc; ++l) {
      w.rcol0[l] = (int)hb.size() * S;
      for (int t = 0; t < (1 << l); ++t) {
        hb.push_back(j.to.beg(l, t));
        he.push_back(j.to.end(l, t));
      }
    }
    w.ncr = (int)hb.size() * S;
    w.Om = rt.scratch.take((size_t)std::max(n, 1) * w.ncl * sizeof(cplx<T>));
    w.Y = rt.scratch.take((size_t)std::max(m, 1) * w.ncl * sizeof(cplx<T>));
    w.Ps = rt.scratch.take((size_t)std::max(m, 1) * w.ncr * sizeof(cplx<T>));
    w.Z = rt.scratch.take((size_t)std::max(n, 1) * w.ncr * sizeof(cplx<T>));
    ProbeTask po{w.Om, std::max(n, 1), n, w.ncl, S, (int32_t)gbeg.size(), 0, rt.stream_id++};
    gbeg.insert(gbeg.end(), gb.begin(), gb.end());
    gend.insert(gend.end(), ge.begin(), ge.end());
    ProbeTask pp{w.Ps, std::max(m, 1), m, w.ncr, S, (int32_t)gbeg.size(), 0, rt.stream_id++};
    gbeg.insert(gbeg.end(), hb.begin(), hb.end());
    gend.insert(gend.end(), he.begin(), he.end());
    for (const ProbeTask& p : {po, pp})
      if (p.n > 0 && p.ncol > 0) {
        ptasks.push_back(p);
        pmax = std::max<int64_t>(pmax, p.n * p.ncol);
      }
    j.max_id_rank = 0;
  }
  if (!ptasks.empty()) {
    PackedUpload<BfRuntime<T>> pk(rt);  // the three arrays in one copy
    const int p0 = pk.add(gbeg.data(), gbeg.size() * sizeof(int32_t));
    const int p1 = pk.add(gend.data(), gend.size() * sizeof(int32_t));
    const int p2 = pk.add(ptasks.data(), ptasks.size() * sizeof(ProbeTask));
    const int32_t* d_gb = (const int32_t*)pk.part(p0);
    const int32_t* d_ge = (const int32_t*)pk.part(p1);
    const ProbeTask* d_pt = (const ProbeTask*)pk.part(p2);
    pk.commit();
    chk(launch_philox_gauss_batch<T>(d_pt, (int)ptasks.size(), pmax, d_gb, d_ge, rt.seed, s), "probes");
  }
  // the sketches of every job: operators of one structure are applied together (apply_all)
  {
    std::vector<Op<T>*> ops;
    std::vector<ApplyArg> fw, bw;
    for (size_t ji = 0; ji < nj; ++ji) {
      RandomJob<T>& j = *jobs[ji];
      const int m = j.to.n, n = j.ts.n;
      ops.push_back(j.op);
      fw.push_back(ApplyArg{sk[ji].Om, std::max(n, 1), sk[ji].Y, std::max(m, 1), sk[ji].ncl});
      bw.push_back(ApplyArg{sk[ji].Ps, std::max(m, 1), sk[ji].Z, std::max(n, 1), sk[ji].ncr});
    }
    apply_all<T>(rt, ops, fw, false, 1.0, 0);
    apply_all<T>(rt, ops, bw, true, 1.0, 0);
  }
  // left: row IDs of the sketch rows; step k works on level L - k of every butterfly
  for (int k = 0;; ++k) {
    auto smk = rt.scratch.mark();
    ExtractBatch eb;
    std::vector<StepBlock> blocks;
    std::vector<void*> A;
    std::vector<int> q, p;
    std::vector<Butterfly*> act;
    std::vector<int> act_level;
    std::vector<RandomJob<T>*> owner;
    for (size_t ji = 0; ji < nj; ++ji) {
      RandomJob<T>& j = *jobs[ji];
      Butterfly& bf = *j.out;
      const int L = bf.L, l = L - k, S = j.S;
      if (l < bf.lc) continue;
      act.push_back(&bf);
      act_level.push_back(l);
      const int vs = 1 << (L - l);
      for (int blk = 0; blk < (1 << L); ++blk) {
        const int t = blk / vs, v = blk % vs;
        StepBlock sb{&bf, blk, l, left_rows(bf, l, t, v)};
        std::vector<int32_t> grp(S);
        for (int kk = 0; kk < S; ++kk) grp[kk] = sk[ji].lcol0[l] + v * S + kk;
        const int pp = (int)sb.cand.size();
        void* a = rt.scratch.take((size_t)std::max(pp * S, 1) * sizeof(cplx<double>));
        eb.add(nullptr, sk[ji].Y, std::max(j.to.n, 1), sb.cand, 0, grp, 0, a, S, true);  // A = Y(rows, group)^T
        A.push_back(a);
        q.push_back(S);
        p.push_back(pp);
        owner.push_back(&j);
        blocks.push_back(std::move(sb));
      }
    }
    if (act.empty()) break;
    run_extract_to<double>(rt, eb, sizeof(T) == 4);  // sketch rows, to FP64 for the ID
    IdLevel<T> idl(rt);
    std::vector<int> rank;
    std::vector<std::vector<int32_t>> perm;
    idl.run(A, q, p, rank, perm);
    for (size_t b = 0; b < blocks.size(); ++b) owner[b]->max_id_rank = std::max(owner[b]->max_id_rank, rank[b]);
    finish_step(rt, idl, blocks, rank, perm, act, act_level, true, false);
    rt.scratch.release(smk);
  }
  // right: column IDs through K^H sketches (row IDs of the Z rows); step k works on level k
  for (int k = 0;; ++k) {
    auto smk = rt.scratch.mark();
    ExtractBatch eb;
    std::vector<StepBlock> blocks;
    std::vector<void*> A;
    std::vector<int> q, p;
    std::vector<Butterfly*> act;
    std::vector<int> act_level;
    std::vector<RandomJob<T>*> owner;
    for (size_t ji = 0; ji < nj; ++ji) {
      RandomJob<T>& j = *jobs[ji];
      Butterfly& bf = *j.out;
      const int L = bf.L, l = k, S = j.S;
      if (l > bf.lc) continue;
      act.push_back(&bf);
      act_level.push_back(l);
      const int vs = 1 << (L - l);
      for (int blk = 0; blk < (1 << L); ++blk) {
        const int t = blk / vs, v = blk % vs;
        StepBlock sb{&bf, blk, l, right_cols(bf, l, t, v)};
        std::vector<int32_t> grp(S);
        for (int kk = 0; kk < S; ++kk) grp[kk] = sk[ji].rcol0[l] + t * S + kk;
        const int pp = (int)sb.cand.size();
        void* a = rt.scratch.take((size_t)std::max(pp * S, 1) * sizeof(cplx<double>));
        eb.add(nullptr, sk[ji].Z, std::max(j.ts.n, 1), sb.cand, 0, grp, 0, a, S, true);  // A = Z(cols, group)^T
        A.push_back(a);
        q.push_back(S);
        p.push_back(pp);
        owner.push_back(&j);
        blocks.push_back(std::move(sb));
      }
    }
    if (act.empty()) break;
    run_extract_to<double>(rt, eb, sizeof(T) == 4);
    IdLevel<T> idl(rt);
    std::vector<int> rank;
    std::vector<std::vector<int32_t>> perm;
    idl.run(A, q, p, rank, perm);
    for (size_t b = 0; b < blocks.size(); ++b) owner[b]->max_id_rank = std::max(owner[b]->max_id_rank, rank[b]);
    finish_step(rt, idl, blocks, rank, perm, act, act_level, false, true);  // Vt = U_c^H
    rt.scratch.release(smk);
  }
  // centre: B G = Yc with G = (right half) Omega_lc and Yc = Y(Obar, group);
  // normal equations B (G G^H) = Yc G^H, solved per block
  struct Centre {
    BfPlan hp;
    int64_t ws_off = 0, cw = 0;
    std::vector<int64_t> m1_off, yc_off;
  };
  std::vector<Centre> ce(nj);
  int64_t total = 0;
  for (size_t ji = 0; ji < nj; ++ji) {
    RandomJob<T>& j = *jobs[ji];
    Butterfly& bf = *j.out;
    const int L = bf.L, lc = bf.lc, nb = 1 << L, S = j.S, n = j.ts.n;
    const int ncol = (1 << (L - lc)) * S;
    Centre& c = ce[ji];
    c.hp = make_plan({BfCall{&bf, 0, 0, 1.0, 0.0, 0}}, false, ncol, std::max(n, 1), 1, true);
    // workspace of the job: [half plan | M1 blocks | Yc blocks]
    int64_t cw = std::max<int64_t>(c.hp.ws_elems, 1);
    c.m1_off.assign(nb, 0);
    c.yc_off.assign(nb, 0);
    for (int blk = 0; blk < nb; ++blk) {
      c.m1_off[blk] = cw;
      cw += (int64_t)std::max(bf.rr[lc][blk] * bf.rr[lc][blk], 1);
    }
    for (int blk = 0; blk < nb; ++blk) {
      c.yc_off[blk] = cw;
      cw += (int64_t)std::max(bf.rl[lc][blk] * S, 1);
    }
    c.ws_off = total;
    c.cw = cw;
    total += (cw + 15) & ~(int64_t)15;
  }
  cplx<T>* ws = (cplx<T>*)rt.scratch.take((size_t)std::max<int64_t>(total, 1) * sizeof(cplx<T>));
  ExtractBatch eb;
  for (size_t ji = 0; ji < nj; ++ji) {
    RandomJob<T>& j = *jobs[ji];
    Butterfly& bf = *j.out;
    const int L = bf.L, lc = bf.lc, nb = 1 << L, S = j.S, m = j.to.n, n = j.ts.n;
    const int ncol = (1 << (L - lc)) * S;
    Centre& c = ce[ji];
    const void* Olc = (const char*)sk[ji].Om + (size_t)sk[ji].lcol0[lc] * std::max(n, 1) * sizeof(cplx<T>);
    const int64_t lim[4] = {(int64_t)(rt.pool.used / sizeof(cplx<T>)), (int64_t)std::max(n, 1) * ncol, 0, c.cw};
    run_plan<T>(c.hp, *rt.c, rt.pool_base(), Olc, nullptr, ws + c.ws_off, s, lim);
    std::vector<int32_t> grp(S);
    for (int kk = 0; kk < S; ++kk) grp[kk] = kk;
    const int vs = 1 << (L - lc);
    for (int blk = 0; blk < nb; ++blk) {
      const int v = blk % vs, r = bf.rl[lc][blk];
      if (r == 0) continue;
      const void* Ysrc = (const char*)sk[ji].Y + (size_t)(sk[ji].lcol0[lc] + v * S) * std::max(m, 1) * sizeof(cplx<T>);
      eb.add(nullptr, Ysrc, std::max(m, 1), bf.Ob[lc][blk], 0, grp, 0, ws + c.ws_off + c.yc_off[blk], r, false);
    }
  }
  run_extract_to<T>(rt, eb, sizeof(T) == 4);
  // every allocation first: the pool may move while it grows
  for (size_t ji = 0; ji < nj; ++ji) {
    Butterfly& bf = *jobs[ji]->out;
    FactorAlloc<T> fa{rt, bf};
    for (int blk = 0; blk < (1 << bf.L); ++blk) bf.offB[blk] = fa.alloc((int64_t)bf.rl[bf.lc][blk] * bf.rr[bf.lc][blk]);
  }
  std::vector<GTask> gt;
  std::vector<SolveTask> st;
  for (size_t ji = 0; ji < nj; ++ji) {
    RandomJob<T>& j = *jobs[ji];
    Butterfly& bf = *j.out;
    const int L = bf.L, lc = bf.lc, nb = 1 << L, S = j.S;
    Centre& c = ce[ji];
    const VecLayout& hl = c.hp.half_layout[0];
    const int64_t hoff = c.hp.half_off[0];
    const int vs = 1 << (L - lc);
    for (int blk = 0; blk < nb; ++blk) {
      const int v = blk % vs;
      const int r = bf.rl[lc][blk], rp = bf.rr[lc][blk];
      if (r == 0 || rp == 0) continue;
      const int gi = hl.grp_of[blk];
      const int64_t g_off = c.ws_off + hoff + hl.grp_off[gi] + hl.mem_row[blk] + (int64_t)v * S * hl.grp_ld[gi];
      const int64_t g_ld = std::max<int64_t>(hl.grp_ld[gi], 1);
      GTask t1 = {};  // M1 = G G^H (rp x rp)
      t1.a_off = g_off; t1.lda = g_ld; t1.opA = OP_N; t1.abase = 3;
      t1.b_off = g_off; t1.ldb = g_ld; t1.opB = OP_C; t1.bbase = 3;
      t1.c_off = c.ws_off + c.m1_off[blk]; t1.ldc = rp; t1.cbase = 3;
      t1.M = rp; t1.N = rp; t1.K = S; t1.alpha_re = 1; t1.beta = 0;
      gt.push_back(t1);
      GTask t2 = {};  // B = Yc G^H (r x rp), into the factor pool
      t2.a_off = c.ws_off + c.yc_off[blk]; t2.lda = r; t2.opA = OP_N; t2.abase = 3;
      t2.b_off = g_off; t2.ldb = g_ld; t2.opB = OP_C; t2.bbase = 3;
      t2.c_off = bf.offB[blk]; t2.ldc = r; t2.cbase = 0;
      t2.M = r; t2.N = rp; t2.K = S; t2.alpha_re = 1; t2.beta = 0;
      gt.push_back(t2);
      st.push_back(SolveTask{ws + c.ws_off + c.m1_off[blk], rp, rt.pool_base() + bf.offB[blk] * sizeof(cplx<T>), r, rp, r});
    }
  }
  if (!gt.empty()) {
    BfPlan gp;
    gp.phase.push_back(gt);
    const int64_t lim[4] = {(int64_t)(rt.pool.used / sizeof(cplx<T>)), 0, 0, std::max<int64_t>(total, 1)};
    run_plan<T>(gp, *rt.c, rt.pool_base(), nullptr, nullptr, ws, s, lim);
    void* d_st = upload_tmp(rt, st);
    chk(launch_small_solve_right<T>(d_st, (int)st.size(), s), "lsq");
  }
  rt.scratch.release(mk);
}

int size_bucket(int m, int n) {
  int b = 0;
  for (int x = std::max(std::max(m, n), 1); x > 1; x >>= 1) ++b;
  return b;
}

}  // namespace

template <class T>
void bf_random_matvec_batch(BfRuntime<T>& rt, const std::vector<RandomJob<T>*>& jobs) {
  HostTimer ht(HP_RANDOM);
  std::vector<RandomJob<T>*> pending;
  for (auto* j : jobs) {
    const int b = size_bucket(j->to.n, j->ts.n);
    // start at the sample count the last construction of this size settled on
    const int hint = b < (int)rt.sample_hint.size() ? rt.sample_hint[b] : 0;
    j->S = std::max({8, rt.samples, hint});
    ++rt.n_random;
    pending.push_back(j);
  }
  while (!pending.empty()) {
    const size_t pool_mark = rt.pool.used;
    random_once_batch<T>(rt, pending);
    std::vector<RandomJob<T>*> again;
    for (auto* j : pending) {
      if (j->max_id_rank >= j->S - 8 && j->S < rt.max_samples) {
        again.push_back(j);
        continue;
      }
      const int b = size_bucket(j->to.n, j->ts.n);
      if (b >= (int)rt.sample_hint.size()) rt.sample_hint.resize(b + 1, 0);
      rt.sample_hint[b] = j->S;
      rt.max_rank_seen = std::max(rt.max_rank_seen, j->out->max_rank());
    }
    if (again.size() == pending.size()) rt.pool.used = pool_mark;  // every attempt of this pass is discarded
    for (auto* j : again) {
      j->out.reset();
      j->S *= 2;
    }
    pending.swap(again);
  }
}

template <class T>
std::unique_ptr<Butterfly> bf_random_matvec(BfRuntime<T>& rt, Op<T>& op, const BTree& to, const BTree& ts) {
  RandomJob<T> j;
  j.op = &op;
  j.to = to;
  j.ts = ts;
  bf_random_matvec_batch<T>(rt, {&j});
  return std::move(j.out);
}

#define BF_INST(T)                                                                                                  \
  template void bf_entry_eval_batch<T>(BfRuntime<T>&, const std::vector<EntryJob<T>*>&);                            \
  template std::unique_ptr<Butterfly> bf_entry_eval<T>(BfRuntime<T>&, EntrySource<T>&, ProxySampler&, const BTree&, \
                                                       const BTree&);                                               \
  template void bf_random_matvec_batch<T>(BfRuntime<T>&, const std::vector<RandomJob<T>*>&);                        \
  template std::unique_ptr<Butterfly> bf_random_matvec<T>(BfRuntime<T>&, Op<T>&, const BTree&, const BTree&);
BF_INST(double)
BF_INST(float)

}  // namespace bfmf
