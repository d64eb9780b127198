// C ABI for butterflies of caller-given dense matrices: compression by entry
// evaluation (Alg. 2) or by randomized products (Sec. 3.3), products K X and
// K^H X, and decompression.  Used to check the butterfly kernels in isolation.
#include <cstring>
#include <limits>
#include <mutex>
#include <random>

#include "bf.hpp"
#include "ops.hpp"

using namespace bfmf;

struct bfmf_bf {
  Context ctx;
  BfRuntime<double> rt;
  DevBuf K;
  std::unique_ptr<Butterfly> bf;
  std::string err;
  DevBuf centre;  // centre form for entry extraction, built on first use
  const BfCentreDev* centre_dev = nullptr;
};

namespace bfmf {
thread_local std::string g_thread_error;
}

// Scratch of bfmf_bf_apply_noalloc: the product's task lists, then its
// inter-level workspace.  Each device holds its own copy for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the name itself is a host-side stand-in).
#define BFMF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) char scratch[BFMF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `device` (the current device), looked up once per device
char* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(BFMF_E_INVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    ochk(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    if (!p) throw Error(BFMF_E_DEVICE, "scratch address is null");
    g_scratch_ptr[device] = (char*)p;
  }
  return g_scratch_ptr[device];
}

}  // namespace

namespace {

struct DenseSource : EntrySource<double> {
  const void* K;
  int64_t ldk;
  DenseSource(const void* k, int64_t ld) : K(k), ldk(ld) {}
  void request(ExtractBatch& b, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, void* out,
               int64_t ldo, bool trans) override {
    b.add(nullptr, K, ldk, rows, 0, cols, 0, out, ldo, trans);
  }
};

// alpha * |given| uniform proxies (without replacement) inside the node, at most cap
struct UniformSampler : ProxySampler {
  std::mt19937_64 g;
  double alpha;
  int cap;
  UniformSampler(uint64_t seed, double a, int c) : g(seed), alpha(a), cap(c) {}
  void pick(size_t given, int beg, int end, std::vector<int32_t>& out) {
    out.clear();
    const int n = end - beg;
    const int k = std::min({n, cap, std::max(8, (int)(alpha * (double)given))});
    std::vector<int32_t> all(n);
    for (int i = 0; i < n; ++i) all[i] = beg + i;
    for (int i = 0; i < k; ++i) {
      std::uniform_int_distribution<int> d(i, n - 1);
      std::swap(all[i], all[d(g)]);
    }
    out.assign(all.begin(), all.begin() + k);
    std::sort(out.begin(), out.end());
  }
  void columns(const std::vector<int32_t>& rows, int beg, int end, std::vector<int32_t>& out) override {
    pick(rows.size(), beg, end, out);
  }
  void rows(const std::vector<int32_t>& cols, int beg, int end, std::vector<int32_t>& out) override {
    pick(cols.size(), beg, end, out);
  }
};

}  // namespace

namespace {

// a handle with its own stream on `device`
bfmf_bf* new_handle(int32_t device) {
  bfmf_bf* b = new (std::nothrow) bfmf_bf();
  if (!b) return nullptr;
  if (hipSetDevice(device) != hipSuccess) {
    delete b;
    return nullptr;
  }
  b->ctx.device = device;
  return b;
}

}  // namespace

extern "C" {

bfmf_status bfmf_bf_import(int32_t device, int32_t m, int32_t n, int32_t L, const int32_t* ranks_left,
                           const int32_t* ranks_right, const double* factors, int64_t nfactor, bfmf_bf** out) {
  if (!out) return BFMF_E_INVAL;
  *out = nullptr;
  if (m <= 0 || n <= 0 || L < 0 || L > 12 || !ranks_left || !ranks_right || !factors || nfactor < 0)
    return BFMF_E_INVAL;
  const int lc = L / 2, nb = 1 << L;
  for (int64_t i = 0; i < (int64_t)(L - lc + 1) * nb; ++i)
    if (ranks_left[i] < 0 || ranks_left[i] > 4096) return BFMF_E_INVAL;
  for (int64_t i = 0; i < (int64_t)(lc + 1) * nb; ++i)
    if (ranks_right[i] < 0 || ranks_right[i] > 4096) return BFMF_E_INVAL;
  bfmf_bf* b = nullptr;
  try {
    auto bf = std::make_unique<Butterfly>();
    Butterfly& B = *bf;
    B.to = make_tree(m, L, nullptr, 0);
    B.ts = make_tree(n, L, nullptr, 0);
    B.m = m;
    B.n = n;
    B.L = L;
    B.lc = lc;
    B.rl.assign(L + 1, {});
    B.rr.assign(L + 1, {});
    B.offL.assign(L + 1, {});
    B.offR.assign(L + 1, {});
    B.Ob.assign(L + 1, {});
    B.Sb.assign(L + 1, {});
    for (int l = lc; l <= L; ++l) B.rl[l].assign(ranks_left + (size_t)(l - lc) * nb, ranks_left + (size_t)(l - lc + 1) * nb);
    for (int l = 0; l <= lc; ++l) B.rr[l].assign(ranks_right + (size_t)l * nb, ranks_right + (size_t)(l + 1) * nb);
    // the caller's order (one matrix per block) and the pool's (pairs side by side or stacked)
    std::vector<double> pool;
    int64_t in = 0;  // complex entries of the input read so far
    auto need = [&](int64_t cnt) {
      if (in + cnt > nfactor) throw Error(BFMF_E_INVAL, "import: fewer factor entries than the ranks require");
    };
    auto put = [&](int64_t src, int64_t cnt) {  // appends cnt entries of the input at src to the pool image
      pool.insert(pool.end(), factors + 2 * src, factors + 2 * (src + cnt));
    };
    B.offL[L].assign(nb, 0);
    for (int t = 0; t < nb; ++t) {  // U_t
      const int64_t cnt = (int64_t)B.to.size(L, t) * B.rl[L][t];
      need(cnt);
      B.offL[L][t] = (int64_t)pool.size() / 2;
      put(in, cnt);
      in += cnt;
    }
    for (int l = L - 1; l >= lc; --l) {  // R of every block; a nu-pair side by side
      const int vs = 1 << (L - l), vs1 = vs / 2;
      B.offL[l].assign(nb / 2, 0);
      for (int pr = 0; pr < nb / 2; ++pr) {
        const int t = (2 * pr) / vs, v = (2 * pr) % vs;
        const int rows = B.rl[l + 1][(2 * t) * vs1 + v / 2] + B.rl[l + 1][(2 * t + 1) * vs1 + v / 2];
        const int64_t c0 = (int64_t)rows * B.rl[l][2 * pr], c1 = (int64_t)rows * B.rl[l][2 * pr + 1];
        need(c0 + c1);
        B.offL[l][pr] = (int64_t)pool.size() / 2;
        put(in, c0 + c1);  // the two blocks follow each other in the input too
        in += c0 + c1;
      }
    }
    B.offB.assign(nb, 0);
    for (int blk = 0; blk < nb; ++blk) {
      const int64_t cnt = (int64_t)B.rl[lc][blk] * B.rr[lc][blk];
      need(cnt);
      B.offB[blk] = (int64_t)pool.size() / 2;
      put(in, cnt);
      in += cnt;
    }
    for (int l = lc; l >= 1; --l) {  // W of every block; a tau-pair stacked
      const int vs = 1 << (L - l), vs0 = 2 * vs;
      B.offR[l].assign(nb / 2, 0);
      std::vector<int64_t> blk_in(nb);
      for (int blk = 0; blk < nb; ++blk) {
        const int t = blk / vs, v = blk % vs;
        const int cols = B.rr[l - 1][(t / 2) * vs0 + 2 * v] + B.rr[l - 1][(t / 2) * vs0 + 2 * v + 1];
        const int64_t cnt = (int64_t)B.rr[l][blk] * cols;
        need(cnt);
        blk_in[blk] = in;
        in += cnt;
      }
      for (int t2 = 0; t2 < (1 << (l - 1)); ++t2)
        for (int v = 0; v < vs; ++v) {
          const int q = t2 * vs + v, a = (2 * t2) * vs + v, bb = (2 * t2 + 1) * vs + v;
          const int ra = B.rr[l][a], rb = B.rr[l][bb];
          const int cols = B.rr[l - 1][t2 * vs0 + 2 * v] + B.rr[l - 1][t2 * vs0 + 2 * v + 1];
          B.offR[l][q] = (int64_t)pool.size() / 2;
          for (int c = 0; c < cols; ++c) {
            put(blk_in[a] + (int64_t)c * ra, ra);
            put(blk_in[bb] + (int64_t)c * rb, rb);
          }
        }
    }
    B.offR[0].assign(nb, 0);
    for (int v = 0; v < nb; ++v) {  // V_v
      const int64_t cnt = (int64_t)B.rr[0][v] * B.ts.size(L, v);
      need(cnt);
      B.offR[0][v] = (int64_t)pool.size() / 2;
      put(in, cnt);
      in += cnt;
    }
    if (in != nfactor) throw Error(BFMF_E_INVAL, "import: more factor entries than the ranks require");
    B.elems = in;
    b = new_handle(device);
    if (!b) return BFMF_E_DEVICE;
    ochk(hipStreamCreateWithFlags(&b->ctx.stream, hipStreamNonBlocking), "stream");
    b->ctx.own_stream = true;
    b->rt.c = &b->ctx;
    (void)scratch_address(device);
    const size_t off = b->rt.pool.alloc(std::max<size_t>(pool.size() * sizeof(double), 16), b->ctx.stream);
    for (auto& v : B.offL)
      for (auto& o : v) o += (int64_t)(off / 16);
    for (auto& v : B.offR)
      for (auto& o : v) o += (int64_t)(off / 16);
    for (auto& o : B.offB) o += (int64_t)(off / 16);
    if (!pool.empty())
      ochk(hipMemcpy(b->rt.pool_base() + off, pool.data(), pool.size() * sizeof(double), hipMemcpyHostToDevice),
           "upload");
    b->bf = std::move(bf);
  } catch (const Error& e) {
    g_thread_error = e.msg;
    delete b;
    return e.status;
  }
  *out = b;
  return BFMF_OK;
}

bfmf_status bfmf_bf_extract(bfmf_bf* b, int32_t nreq, const int64_t* row_ptr, const int32_t* rows,
                            const int64_t* col_ptr, const int32_t* cols, double* out) {
  if (!b || nreq < 0 || (nreq > 0 && (!row_ptr || !col_ptr || !out))) return BFMF_E_INVAL;
  if (nreq > 0 && ((row_ptr[nreq] > 0 && !rows) || (col_ptr[nreq] > 0 && !cols))) return BFMF_E_INVAL;
  const Butterfly& B = *b->bf;
  int64_t total = 0;
  for (int32_t k = 0; k < nreq; ++k) {
    const int64_t nr = row_ptr[k + 1] - row_ptr[k], nc = col_ptr[k + 1] - col_ptr[k];
    if (row_ptr[k] < 0 || col_ptr[k] < 0 || nr < 0 || nc < 0 || nr > INT32_MAX || nc > INT32_MAX)
      return BFMF_E_INVAL;
    for (int64_t i = row_ptr[k]; i < row_ptr[k + 1]; ++i)
      if (rows[i] < 0 || rows[i] >= B.m) return BFMF_E_INVAL;
    for (int64_t j = col_ptr[k]; j < col_ptr[k + 1]; ++j)
      if (cols[j] < 0 || cols[j] >= B.n) return BFMF_E_INVAL;
    total += nr * nc;
  }
  if (total == 0) return BFMF_OK;
  try {
    ochk(hipSetDevice(b->ctx.device), "set device");
    if (!b->centre_dev) {
      CentreSpec spec;
      spec.bfs.push_back(b->bf.get());
      const size_t bytes = centre_bytes<double>(spec);
      ochk(dev_malloc((void**)&b->centre.p, bytes), "centre form");
      b->centre.bytes = bytes;
      b->centre_dev = build_centres<double>(b->rt, spec, b->centre.as<char>()).bfs;
    }
    auto mk = b->rt.scratch.mark();
    char* dout = (char*)b->rt.scratch.take((size_t)total * 16);
    ExtractBatch eb;
    int64_t pos = 0;
    for (int32_t k = 0; k < nreq; ++k) {
      std::vector<int32_t> r(rows + row_ptr[k], rows + row_ptr[k + 1]), c(cols + col_ptr[k], cols + col_ptr[k + 1]);
      eb.add_bf(b->centre_dev, r, 0, c, 0, dout + pos * 16, std::max<int64_t>((int64_t)r.size(), 1), false, 1.0, false);
      pos += (int64_t)r.size() * (int64_t)c.size();
    }
    run_extract<double>(b->rt, eb);
    ochk(hipMemcpyAsync(out, dout, (size_t)total * 16, hipMemcpyDeviceToHost, b->ctx.stream), "download");
    b->ctx.stage.sync(b->ctx.stream);
    b->rt.scratch.release(mk);
  } catch (const Error& e) {
    b->err = e.msg;
    g_thread_error = e.msg;
    return e.status;
  }
  return BFMF_OK;
}

bfmf_status bfmf_bf_compress_dense(int32_t device, int32_t m, int32_t n, const double* K, int64_t ldk, int32_t L,
                                   double tol, int32_t method, int32_t samples, uint64_t seed, bfmf_bf** out) {
  if (!out || !K || m <= 0 || n <= 0 || ldk < m || L < 0 || L > 16 || !(tol > 0)) return BFMF_E_INVAL;
  *out = nullptr;
  bfmf_bf* b = new (std::nothrow) bfmf_bf();
  if (!b) return BFMF_E_NOMEM;
  try {
    if (hipSetDevice(device) != hipSuccess) throw Error(BFMF_E_DEVICE, "set device");
    b->ctx.device = device;
    (void)scratch_address(device);  // set-up of the allocation-free product on this device
    ochk(hipStreamCreateWithFlags(&b->ctx.stream, hipStreamNonBlocking), "stream");
    b->ctx.own_stream = true;
    b->rt.c = &b->ctx;
    b->rt.tol = tol;
    b->rt.seed = seed;
    b->rt.samples = samples > 0 ? samples : 64;
    const size_t bytes = (size_t)m * n * 16;
    ochk(dev_malloc((void**)&b->K.p, bytes), "malloc");
    b->K.bytes = bytes;
    ochk(hipMemcpy2D(b->K.p, (size_t)m * 16, K, (size_t)ldk * 16, (size_t)m * 16, n, hipMemcpyHostToDevice), "upload");
    BTree to = make_tree(m, L, nullptr, 0), ts = make_tree(n, L, nullptr, 0);
    if (method == 0) {
      DenseSource src(b->K.p, m);
      // proxies are the rows of the ID blocks: below tol 1e-4 the Householder kernel takes at most
      // CPQR_MAXQ of them (the Gram kernel any number)
      UniformSampler ps(seed ^ 0x9e3779b97f4a7c15ull, 4.0, tol < 1e-4 ? CPQR_MAXQ : std::numeric_limits<int>::max());
      b->bf = bf_entry_eval<double>(b->rt, src, ps, to, ts);
    } else {
      DenseOp<double> op(b->rt, b->K.p, m, m, n);
      b->bf = bf_random_matvec<double>(b->rt, op, to, ts);
    }
    b->ctx.stage.sync(b->ctx.stream);
  } catch (const Error& e) {
    g_thread_error = e.msg;
    bfmf_status st = e.status;
    delete b;
    return st;
  }
  *out = b;
  return BFMF_OK;
}

bfmf_status bfmf_bf_apply(bfmf_bf* b, int32_t adjoint, int32_t nrhs, const double* X, int64_t ldx, double* Y,
                          int64_t ldy) {
  if (!b || !X || !Y || nrhs <= 0) return BFMF_E_INVAL;
  const int nin = adjoint ? b->bf->m : b->bf->n, nout = adjoint ? b->bf->n : b->bf->m;
  if (ldx < nin || ldy < nout) return BFMF_E_INVAL;
  try {
    ochk(hipSetDevice(b->ctx.device), "set device");
    auto mk = b->rt.scratch.mark();
    void* dx = b->rt.scratch.take((size_t)nin * nrhs * 16);
    void* dy = b->rt.scratch.take((size_t)nout * nrhs * 16);
    ochk(hipMemcpy2DAsync(dx, (size_t)nin * 16, X, (size_t)ldx * 16, (size_t)nin * 16, nrhs, hipMemcpyHostToDevice,
                          b->ctx.stream),
         "upload");
    b->rt.apply(*b->bf, dx, nin, dy, nout, nrhs, adjoint != 0, 1.0, 0);
    ochk(hipMemcpy2DAsync(Y, (size_t)ldy * 16, dy, (size_t)nout * 16, (size_t)nout * 16, nrhs, hipMemcpyDeviceToHost,
                          b->ctx.stream),
         "download");
    b->ctx.stage.sync(b->ctx.stream);
    b->rt.scratch.release(mk);
  } catch (const Error& e) {
    b->err = e.msg;
    return e.status;
  }
  return BFMF_OK;
}

bfmf_status bfmf_bf_apply_noalloc(bfmf_bf* b, int32_t adjoint, int32_t nrhs, const double* dX, int64_t ldx,
                                  double* dY, int64_t ldy, void* hip_stream) {
  if (!b || !dX || !dY || nrhs <= 0) return BFMF_E_INVAL;
  const int nin = adjoint ? b->bf->m : b->bf->n, nout = adjoint ? b->bf->n : b->bf->m;
  if (ldx < nin || ldy < nout) return BFMF_E_INVAL;
  try {
    ochk(hipSetDevice(b->ctx.device), "set device");
    char* base = scratch_address(b->ctx.device);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : b->ctx.stream;
    BfPlan plan = make_plan({BfCall{b->bf.get(), 0, 0, 1.0, 0.0, 0}}, adjoint != 0, nrhs, ldx, ldy);
    const size_t ws_bytes = (size_t)std::max<int64_t>(plan.ws_elems, 1) * 16;
    if (ws_bytes > BFMF_NOALLOC_SCRATCH_BYTES)
      throw Error(BFMF_E_INVAL, "apply_noalloc: the product needs " + std::to_string(ws_bytes) +
                                    " bytes of workspace, more than the fixed scratch of " +
                                    std::to_string(BFMF_NOALLOC_SCRATCH_BYTES));
    // workspace first (256-byte aligned at the start of the array), task lists after it
    const size_t ws_span = (ws_bytes + 255) & ~(size_t)255;
    const int64_t lim[4] = {(int64_t)(b->rt.pool.used / 16), ldx * nrhs, ldy * nrhs, std::max<int64_t>(plan.ws_elems, 1)};
    const size_t need = run_plan_fixed<double>(plan, b->rt.pool_base(), dX, dY, base, base + ws_span,
                                               BFMF_NOALLOC_SCRATCH_BYTES - ws_span, s, lim, 0);
    if (need)
      throw Error(BFMF_E_INVAL, "apply_noalloc: the product needs " + std::to_string(ws_span + need) +
                                    " bytes of scratch, more than the fixed " +
                                    std::to_string(BFMF_NOALLOC_SCRATCH_BYTES));
  } catch (const Error& e) {
    b->err = e.msg;
    g_thread_error = e.msg;
    return e.status;
  }
  return BFMF_OK;
}

bfmf_status bfmf_bf_info(bfmf_bf* b, int32_t* L, int32_t* max_rank, int64_t* entries) {
  if (!b) return BFMF_E_INVAL;
  if (L) *L = b->bf->L;
  if (max_rank) *max_rank = b->bf->max_rank();
  if (entries) *entries = b->bf->elems;
  return BFMF_OK;
}

void bfmf_bf_destroy(bfmf_bf* b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx.device);
  if (b->ctx.stream) (void)hipStreamSynchronize(b->ctx.stream);  // queued work still uses the buffers
  b->bf.reset();
  b->centre.release();
  b->rt.scratch.clear();
  b->rt.pool.buf.release();
  b->K.release();
  if (b->ctx.stream) {
    (void)hipStreamDestroy(b->ctx.stream);
    b->ctx.stream = nullptr;
  }
  delete b;
}

}  // extern "C"
