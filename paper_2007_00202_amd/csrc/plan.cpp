// Device plan of the dense fronts: inverse extend-add maps,
// per-front lists of the A entries each front assembles, level schedule.
//
// Entry A(i, j) (new numbering) is assembled in the front tau whose I^s
// contains min(i, j); the other index then lies in I^s_tau or I^u_tau (Sec. 2,
// the blocks A(I^s,I^s), A(I^s,I^u), A(I^u,I^s) of the front).
#include <algorithm>
#include <cstring>

#include "context.hpp"

namespace bfmf {

namespace {
template <class T>
void upload(DevBuf& b, const std::vector<T>& v) {
  b.release();
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  HIPCHK(dev_malloc((void**)&b.p, bytes));
  b.bytes = bytes;
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}
}  // namespace

void build_plan(Context& c) {
  Symbolic& s = c.sym;
  const int32_t nf = s.nfronts();
  c.fp.assign(nf, FrontPlan());
  int64_t aptr = 0, piv = 0, iu = 0, woff = 0;
  for (int32_t f = 0; f < nf; ++f) {
    FrontPlan& p = c.fp[f];
    p.ns = (int32_t)s.ns(f);
    p.nu = (int32_t)s.nu(f);
    p.n = p.ns + p.nu;
    p.nchild = s.child_ptr[f + 1] - s.child_ptr[f];
    if (p.nchild > 2) throw Error(BFMF_E_INVAL, "assembly tree node with more than two children");
    for (int k = 0; k < p.nchild; ++k) p.child[k] = s.child_list[s.child_ptr[f] + k];
    p.aptr_off = aptr;
    aptr += p.n + 1;
    p.piv_off = piv;
    piv += p.ns;
    p.iu_off = iu;
    iu += p.nu;
    p.w_off = woff;
    woff += p.n;
  }
  c.sum_n = woff;

  // inverse maps: parent-local -> child-local (or -1)
  c.h_inv.clear();
  for (int32_t f = 0; f < nf; ++f) {
    FrontPlan& p = c.fp[f];
    for (int k = 0; k < p.nchild; ++k) {
      const int32_t ch = p.child[k];
      p.inv_off[k] = (int64_t)c.h_inv.size();
      c.h_inv.resize(c.h_inv.size() + p.n, -1);
      int32_t* inv = c.h_inv.data() + p.inv_off[k];
      for (int64_t t = s.iu_ptr[ch]; t < s.iu_ptr[ch + 1]; ++t) inv[s.map[t]] = (int32_t)(t - s.iu_ptr[ch]);
    }
  }

  // A entries per front, sorted by (local column, local row)
  c.h_aptr.assign(aptr, 0);
  c.h_arow.clear();
  c.h_avidx.clear();
  c.h_arow.reserve(c.nnz);
  c.h_avidx.reserve(c.nnz);
  struct Ent {
    int32_t col, row;
    int64_t vidx;
  };
  std::vector<Ent> ents;
  for (int32_t f = 0; f < nf; ++f) {
    FrontPlan& p = c.fp[f];
    const int64_t b = s.sbeg[f], e = s.send[f];
    const int64_t* iuf = s.iu.data() + s.iu_ptr[f];
    auto local = [&](int64_t g) -> int32_t {
      if (g >= b && g < e) return (int32_t)(g - b);
      const int64_t* it = std::lower_bound(iuf, iuf + p.nu, g);
      if (it == iuf + p.nu || *it != g) return -1;
      return (int32_t)(p.ns + (it - iuf));
    };
    ents.clear();
    for (int64_t i = b; i < e; ++i) {
      const int64_t o = s.perm[i];
      for (int64_t t = c.rowptr[o]; t < c.rowptr[o + 1]; ++t) {
        const int64_t j = s.iperm[c.colind[t]];
        if (j < b) continue;  // assembled in a descendant front
        const int32_t lj = local(j);
        if (lj < 0) throw Error(BFMF_E_INVAL, "matrix entry outside its front (pattern not symmetric?)");
        ents.push_back(Ent{lj, (int32_t)(i - b), t});
      }
    }
    for (int32_t k = 0; k < p.nu; ++k) {
      const int64_t o = s.perm[iuf[k]];
      for (int64_t t = c.rowptr[o]; t < c.rowptr[o + 1]; ++t) {
        const int64_t j = s.iperm[c.colind[t]];
        if (j >= b && j < e) ents.push_back(Ent{(int32_t)(j - b), p.ns + k, t});
      }
    }
    std::sort(ents.begin(), ents.end(),
              [](const Ent& x, const Ent& y) { return x.col != y.col ? x.col < y.col : x.row < y.row; });
    int64_t* ap = c.h_aptr.data() + p.aptr_off;
    const int64_t base = (int64_t)c.h_arow.size();
    size_t q = 0;
    for (int32_t j = 0; j <= p.n; ++j) {
      ap[j] = base + (int64_t)q;
      if (j == p.n) break;
      while (q < ents.size() && ents[q].col == j) {
        c.h_arow.push_back(ents[q].row);
        c.h_avidx.push_back(ents[q].vidx);
        ++q;
      }
    }
  }

  // level schedule, deepest level first; postorder inside a level
  c.level_ptr.assign(s.nlevels + 1, 0);
  c.level_fronts.clear();
  for (int32_t L = s.nlevels - 1; L >= 0; --L) {
    for (int32_t f = 0; f < nf; ++f)
      if (s.level[f] == L) c.level_fronts.push_back(f);
    c.level_ptr[s.nlevels - L] = (int32_t)c.level_fronts.size();
  }
  c.desc_index.assign(nf, -1);
  for (size_t k = 0; k < c.level_fronts.size(); ++k) c.desc_index[c.level_fronts[k]] = (int32_t)k;
}

void upload_values(Context& c) { upload(c.d_values, c.values); }

void upload_plan(Context& c) {
  Symbolic& s = c.sym;
  upload(c.d_rowptr, c.rowptr);
  upload(c.d_colind, c.colind);
  upload_values(c);
  upload(c.d_perm, s.perm);
  upload(c.d_aptr, c.h_aptr);
  upload(c.d_arow, c.h_arow);
  upload(c.d_avidx, c.h_avidx);
  upload(c.d_inv, c.h_inv);
  std::vector<int32_t> iu32(s.iu.size());
  for (size_t k = 0; k < s.iu.size(); ++k) iu32[k] = (int32_t)s.iu[k];
  upload(c.d_iu32, iu32);
  int64_t npiv = 0;
  for (auto& p : c.fp) npiv += p.ns;
  c.d_piv.release();
  HIPCHK(dev_malloc((void**)&c.d_piv.p, std::max<int64_t>(npiv, 4) * sizeof(int32_t)));
  c.d_piv.bytes = std::max<int64_t>(npiv, 4) * sizeof(int32_t);
  c.d_pperm.release();
  HIPCHK(dev_malloc((void**)&c.d_pperm.p, std::max<int64_t>(npiv, 4) * sizeof(int32_t)));
  c.d_pperm.bytes = std::max<int64_t>(npiv, 4) * sizeof(int32_t);
  c.d_status.release();
  HIPCHK(dev_malloc((void**)&c.d_status.p, 16));
  c.d_status.bytes = 16;
}

thread_local HostProf* g_hprof = nullptr;

void Staging::put(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  HostTimer ht(HP_PUT);
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (arena) {  // graph capture: a region of its own for every copy
    if (arena_head + need > arena_cap) throw Error(BFMF_E_NOMEM, "graph capture: task-list arena full");
    char* h = arena + arena_head;
    std::memcpy(h, src, bytes);
    arena_head += need;
    HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
    return;
  }
  put_bytes += need;
  if (head + need > cap) {
    sync(s);  // every earlier copy out of the ring has completed
    if (need > cap) {
      if (host) (void)hipHostFree(host);
      host = nullptr;
      cap = std::max(need, (size_t)64 << 20);
      if (hipHostMalloc((void**)&host, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        host = nullptr;
        cap = 0;
        throw Error(BFMF_E_NOMEM, "pinned host allocation of " + std::to_string(need) + " bytes failed");
      }
    }
  }
  char* h = host + head;
  std::memcpy(h, src, bytes);
  head += need;
  HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
}

void Staging::sync(hipStream_t s) {
  HostTimer ht(HP_SYNC);
  HIPCHK(hipStreamSynchronize(s));
  head = 0;
}

Staging::~Staging() {
  if (host) (void)hipHostFree(host);
}

void PrecGraph::release() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (host) (void)hipHostFree(host);
  exec = nullptr;
  graph = nullptr;
  host = nullptr;
  host_cap = 0;
  in = nullptr;
  out = nullptr;
  nrhs = 0;
}

Context::~Context() {
  pgraph.release();  // the stream has been synchronised by the handle's destruction
  if (comp) comp_state_destroy(comp);
  comp = nullptr;
}

uint64_t Context::device_bytes() const {
  uint64_t t = 0;
  for (const DevBuf* b : {&d_rowptr, &d_colind, &d_values, &d_perm, &d_aptr, &d_arow, &d_avidx, &d_inv, &d_iu32,
                          &d_piv, &d_pperm, &d_status, &d_fds, &d_work, &d_fac, &d_kept, &d_W, &d_y, &d_x, &g_B, &g_X, &g_V, &g_w, &g_tmp_scatter,
                          &g_r, &g_scal, &g_part, &g_tmp})
    t += b->bytes;
  t += stage.cap;  // pinned host ring (counted with the handle's memory)
  if (comp) t += comp_state_bytes(comp);
  return t;
}

}  // namespace bfmf
