// Serving: several factorizations resident in HBM answer a stream of
// right-hand-side requests with continuous batching.  Each attached model has
// a worker thread on its handle's stream and max_batch_rhs column slots; every
// column of an admitted request takes a slot and runs its own restarted GMRES
// (SlotGmres): between two iterations the worker retires the columns that
// finished (their solutions go to the result arena) and admits queued
// requests into the freed slots, so a request that arrives while others are
// on the device starts at the next iteration instead of waiting for a batch.
// Models run at the same time on their own streams.  All device memory
// (factors, slot workspaces, result arena) is charged against one HBM budget
// when models are attached.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "context.hpp"
#include "kernels/kernels.hpp"

using namespace bfmf;

namespace {

// First-fit allocator over one device allocation (offsets in bytes).
struct Arena {
  DevBuf buf;
  std::map<size_t, size_t> free_;  // offset -> size
  size_t used = 0;
  void init(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) return;
    if (dev_malloc((void**)&buf.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      buf.p = nullptr;
      throw Error(BFMF_E_NOMEM, "server: result arena of " + std::to_string(bytes) + " bytes");
    }
    buf.bytes = bytes;
    free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {  // merge with the next block
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {  // and with the previous one
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  uint64_t ticket = 0;
  int model = 0, nrhs = 0;
  int64_t n = 0;                     // rows of the model
  std::vector<int32_t> row, col;     // nonzeros of the right-hand sides (sorted, merged)
  std::vector<double> val;           // interleaved complex
  size_t x_off = 0, x_bytes = 0;     // solution columns in the arena
  bool admitted = false, done = false;
  int cols_done = 0;                 // columns retired so far
  bool all_ok = true;                // every retired column met the stopping test
  bfmf_request_info info{};
};

struct SlotRef {  // the request column a slot holds
  Request* r = nullptr;
  int col = 0;
};

struct Model {
  bfmf_handle h = nullptr;
  int id = 0;
  int64_t n = 0;
  std::deque<Request*> queue;
  DevBuf B, X;                        // slot right-hand sides and solutions (n x max_batch)
  DevBuf nz;                          // nonzeros of the admitted columns on the device
  SlotGmres sg;                       // the slots' GMRES state
  std::vector<SlotRef> slot;
  std::thread worker;
  uint64_t charged = 0;               // bytes charged against the budget
};

}  // namespace

struct bfmf_server_s {
  bfmf_server_opts opts{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;        // workers: new requests or arena space; callers: completions
  bool stop = false;
  std::vector<std::unique_ptr<Model>> models;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  Arena arena;
  uint64_t budget = 0, charged = 0;
  hipStream_t copy_stream = nullptr;  // fetches of results
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::string err;
  double clock() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

// device bytes of one model's batch: B and X blocks, GMRES(m) basis and
// vectors, sweep workspaces, per column
uint64_t batch_bytes(const Context& c, int nrhs, int m) {
  const uint64_t col = 16ull * (uint64_t)c.n;
  return (uint64_t)nrhs * (col * (2 + (m + 1) + 3 + 2) + 16ull * (uint64_t)c.sum_n) + 64ull * (m + 2) * nrhs;
}

// Loads the columns of newly admitted requests into their slots: B(:, q) = the column, X(:, q) = 0.
void load_columns(Model& m, const std::vector<int>& slots) {
  Context& c = *m.h;
  const int64_t n = m.n;
  std::vector<int32_t> rows, colidx;
  std::vector<double> vals;
  std::vector<AxpbyTask> zero;
  for (int q : slots) {
    const SlotRef& ref = m.slot[q];
    const Request* r = ref.r;
    for (size_t k = 0; k < r->row.size(); ++k) {
      if (r->col[k] != ref.col) continue;
      rows.push_back(r->row[k]);
      colidx.push_back(q);
      vals.push_back(r->val[2 * k]);
      vals.push_back(r->val[2 * k + 1]);
    }
    zero.push_back(AxpbyTask{m.B.as<char>() + (size_t)q * n * 16, nullptr, n, n, n, 1, 0});
    zero.push_back(AxpbyTask{m.X.as<char>() + (size_t)q * n * 16, nullptr, n, n, n, 1, 0});
  }
  const size_t nnz = rows.size();
  const size_t tasks_bytes = (zero.size() * sizeof(AxpbyTask) + 255) & ~(size_t)255;
  const size_t need = tasks_bytes + std::max<size_t>(nnz, 1) * (2 * sizeof(int32_t) + 2 * sizeof(double)) + 256;
  if (m.nz.bytes < need) {
    m.nz.release();
    HIPCHK(dev_malloc((void**)&m.nz.p, need * 2));
    m.nz.bytes = need * 2;
  }
  AxpbyTask* d_zero = m.nz.as<AxpbyTask>();
  int32_t* d_rows = (int32_t*)(m.nz.as<char>() + tasks_bytes);
  int32_t* d_cols = d_rows + std::max<size_t>(nnz, 1);
  double* d_vals = (double*)(d_cols + std::max<size_t>(nnz, 1));  // 2 M int32 before it: 8-byte aligned
  c.stage.put(d_zero, zero.data(), zero.size() * sizeof(AxpbyTask), c.stream);
  HIPCHK(launch_axpby_batch<double>(d_zero, (int)zero.size(), n, 0.0, 0.0, c.stream));  // B, X columns = 0
  if (nnz) {
    c.stage.put(d_rows, rows.data(), nnz * sizeof(int32_t), c.stream);
    c.stage.put(d_cols, colidx.data(), nnz * sizeof(int32_t), c.stream);
    c.stage.put(d_vals, vals.data(), nnz * 2 * sizeof(double), c.stream);
    HIPCHK(launch_scatter_nz(m.B.p, n, d_rows, d_cols, d_vals, (int64_t)nnz, c.stream));
  }
}

void worker_main(bfmf_server_s* s, Model* m) {
  (void)hipSetDevice(s->device);
  Context& c = *m->h;
  const int nslot = s->opts.max_batch_rhs;
  std::vector<int> fin;
  for (;;) {
    std::vector<int> fresh;  // slots loaded in this admission pass
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // admit whole requests of this model in arrival order while their columns find free slots and their
      // solutions fit the arena
      auto admit = [&]() {
        int nfree = 0;
        for (const SlotRef& r : m->slot) nfree += r.r == nullptr;
        while (!m->queue.empty() && !s->stop) {
          Request* r = m->queue.front();
          if (r->nrhs > nfree) break;
          size_t off = 0;
          if (!s->arena.alloc(r->x_bytes, off)) break;
          r->x_off = off;
          r->admitted = true;
          r->info.t_start = s->clock();
          m->queue.pop_front();
          int col = 0;
          for (int q = 0; q < nslot && col < r->nrhs; ++q)
            if (!m->slot[q].r) {
              m->slot[q] = SlotRef{r, col++};
              fresh.push_back(q);
            }
          nfree -= r->nrhs;
        }
        return !fresh.empty();
      };
      if (m->sg.busy()) {
        admit();
      } else {
        s->cv.wait(lk, [&] { return admit() || s->stop; });
        if (fresh.empty()) {  // stopped with nothing in flight: requests that can no longer be admitted fail
          for (Request* r : m->queue) {
            r->info.status = BFMF_E_STATE;
            r->done = true;
          }
          m->queue.clear();
          lk.unlock();
          s->cv.notify_all();
          return;
        }
      }
      // occupancy of this pass, for the requests' reports
      int busy_cols = 0;
      std::vector<Request*> in;
      for (const SlotRef& r : m->slot)
        if (r.r) {
          ++busy_cols;
          if (std::find(in.begin(), in.end(), r.r) == in.end()) in.push_back(r.r);
        }
      for (int q : fresh) {
        Request* r = m->slot[q].r;
        r->info.batch_rhs = std::max<int32_t>(r->info.batch_rhs, busy_cols);
        r->info.batch_requests = std::max<int32_t>(r->info.batch_requests, (int32_t)in.size());
      }
      for (Request* r : in) {  // requests already in flight see the new neighbours too
        r->info.batch_rhs = std::max<int32_t>(r->info.batch_rhs, busy_cols);
        r->info.batch_requests = std::max<int32_t>(r->info.batch_requests, (int32_t)in.size());
      }
    }
    bfmf_status st = BFMF_OK;
    std::string msg;
    try {
      if (!fresh.empty()) {
        load_columns(*m, fresh);
        for (int q : fresh) m->sg.admit(q);
      }
      m->sg.step(fin);
      for (int q : fin) {  // the column's solution to its request's place in the arena
        const SlotRef& ref = m->slot[q];
        HIPCHK(hipMemcpyAsync(s->arena.buf.as<char>() + ref.r->x_off + (size_t)ref.col * m->n * 16,
                              m->X.as<char>() + (size_t)q * m->n * 16, (size_t)m->n * 16, hipMemcpyDeviceToDevice,
                              c.stream));
      }
      if (!fin.empty()) HIPCHK(hipStreamSynchronize(c.stream));
    } catch (const Error& e) {
      st = e.status;
      msg = e.msg;
    } catch (const std::exception& e) {
      st = BFMF_E_DEVICE;
      msg = e.what();
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      const double t = s->clock();
      if (st != BFMF_OK) {  // every request in flight fails
        s->err = msg;
        for (int q = 0; q < nslot; ++q) {
          Request* r = m->slot[q].r;
          if (r && !r->done) {
            r->info.status = st;
            r->info.t_done = t;
            r->done = true;
          }
          m->slot[q] = SlotRef{};
          m->sg.mode[q] = SlotGmres::IDLE;
        }
      } else {
        for (int q : fin) {
          Request* r = m->slot[q].r;
          r->info.iters = std::max<int32_t>(r->info.iters, m->sg.iters[q]);
          r->info.relres = std::max(r->info.relres, m->sg.relres[q]);
          r->all_ok = r->all_ok && m->sg.ok[q];
          m->slot[q] = SlotRef{};
          if (++r->cols_done == r->nrhs) {
            r->info.status = r->all_ok ? BFMF_OK : BFMF_E_NOCONV;
            r->info.t_done = t;
            r->done = true;
          }
        }
      }
    }
    if (st != BFMF_OK || !fin.empty()) s->cv.notify_all();
  }
}

}  // namespace

extern "C" {

void bfmf_default_server_opts(bfmf_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_batch_rhs = 64;
  o->result_bytes = 4ull << 30;
  bfmf_default_solve_opts(&o->solve);
  o->solve.true_rtol = 1e-3;
}

bfmf_status bfmf_server_create(int32_t device, const bfmf_server_opts* o, bfmf_server* out) {
  if (!out || device < 0) return BFMF_E_INVAL;
  *out = nullptr;
  auto* s = new (std::nothrow) bfmf_server_s();
  if (!s) return BFMF_E_NOMEM;
  if (o)
    s->opts = *o;
  else
    bfmf_default_server_opts(&s->opts);
  if (s->opts.max_batch_rhs <= 0) s->opts.max_batch_rhs = 64;
  s->device = device;
  try {
    HIPCHK(hipSetDevice(device));
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    s->budget = s->opts.hbm_budget ? s->opts.hbm_budget : (uint64_t)free_b;
    if (s->opts.result_bytes > s->budget) throw Error(BFMF_E_NOMEM, "server: result arena exceeds the HBM budget");
    s->arena.init(s->opts.result_bytes);
    s->charged = s->opts.result_bytes;
    HIPCHK(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
  } catch (const Error& e) {
    g_thread_error = e.msg;
    delete s;
    return e.status;
  }
  *out = s;
  return BFMF_OK;
}

bfmf_status bfmf_server_attach(bfmf_server s, bfmf_handle h, int32_t* model) {
  if (!s || !h) return BFMF_E_INVAL;
  try {
    if (h->state != State::Factored) throw Error(BFMF_E_STATE, "server: attach a factored handle");
    if (h->device != s->device) throw Error(BFMF_E_INVAL, "server: handle on another device");
    HIPCHK(hipSetDevice(s->device));
    auto m = std::make_unique<Model>();
    m->h = h;
    m->n = h->n;
    const int mb = s->opts.max_batch_rhs;
    const int restart = s->opts.solve.restart > 0 ? s->opts.solve.restart : 30;
    const uint64_t need = h->device_bytes() + batch_bytes(*h, mb, restart);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->charged + need > s->budget)
        throw Error(BFMF_E_NOMEM, "server: model needs " + std::to_string(need) + " bytes, " +
                                      std::to_string(s->budget - s->charged) + " left in the HBM budget");
      s->charged += need;
    }
    m->charged = need;
    try {  // every batch buffer now, so that no request waits for an allocation
      const size_t blk = (size_t)h->n * mb * 16;
      HIPCHK(dev_malloc((void**)&m->B.p, blk));
      m->B.bytes = blk;
      HIPCHK(dev_malloc((void**)&m->X.p, blk));
      m->X.bytes = blk;
      m->slot.assign(mb, SlotRef{});
      m->sg.init(*h, mb, s->opts.solve, m->B.p, m->X.p);
      HIPCHK(hipStreamSynchronize(h->stream));
    } catch (...) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->charged -= need;
      throw;
    }
    Model* mp = m.get();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      mp->id = (int)s->models.size();
      s->models.push_back(std::move(m));
    }
    mp->worker = std::thread(worker_main, s, mp);
    if (model) *model = mp->id;
  } catch (const Error& e) {
    s->err = e.msg;
    return e.status;
  }
  return BFMF_OK;
}

bfmf_status bfmf_server_submit(bfmf_server s, int32_t model, int32_t nrhs, const int64_t* colptr, const int64_t* rowind,
                               const double* values, uint64_t* ticket) {
  if (!s || !colptr || nrhs <= 0 || !ticket) return BFMF_E_INVAL;
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return BFMF_E_NOMEM;
  int64_t n = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (model < 0 || model >= (int)s->models.size() || s->stop) return BFMF_E_INVAL;
    n = s->models[model]->n;
  }
  if (nrhs > s->opts.max_batch_rhs) {
    s->err = "server: request wider than the batch";
    return BFMF_E_INVAL;
  }
  r->model = model;
  r->nrhs = nrhs;
  r->n = n;
  r->x_bytes = (size_t)n * nrhs * 16;
  if (r->x_bytes > s->arena.buf.bytes) {
    s->err = "server: request larger than the result arena";
    return BFMF_E_NOMEM;
  }
  // nonzeros per column, sorted by row with duplicates summed
  for (int q = 0; q < nrhs; ++q) {
    const int64_t b = colptr[q], e = colptr[q + 1];
    if (e < b || (e > b && (!rowind || !values))) return BFMF_E_INVAL;
    std::vector<std::pair<int64_t, int64_t>> ent;
    for (int64_t k = b; k < e; ++k) {
      if (rowind[k] < 0 || rowind[k] >= n) return BFMF_E_INVAL;
      if (!std::isfinite(values[2 * k]) || !std::isfinite(values[2 * k + 1])) return BFMF_E_INVAL;
      ent.push_back({rowind[k], k});
    }
    std::sort(ent.begin(), ent.end());
    for (size_t k = 0; k < ent.size(); ++k) {
      if (k > 0 && ent[k].first == ent[k - 1].first) {
        r->val[r->val.size() - 2] += values[2 * ent[k].second];
        r->val[r->val.size() - 1] += values[2 * ent[k].second + 1];
        continue;
      }
      r->row.push_back((int32_t)ent[k].first);
      r->col.push_back(q);
      r->val.push_back(values[2 * ent[k].second]);
      r->val.push_back(values[2 * ent[k].second + 1]);
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->info.t_submit = s->clock();
    r->info.model = model;
    r->info.nrhs = nrhs;
    *ticket = r->ticket;
    s->models[model]->queue.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
  }
  s->cv.notify_all();
  return BFMF_OK;
}

bfmf_status bfmf_server_wait(bfmf_server s, uint64_t ticket, bfmf_request_info* info, double* X, int64_t ldx,
                             int32_t mem) {
  if (!s) return BFMF_E_INVAL;
  Request* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return BFMF_E_INVAL;
    r = it->second.get();
    s->cv.wait(lk, [&] { return r->done; });
  }
  bfmf_status st = BFMF_OK;
  if (X && r->info.status == BFMF_OK) {
    const int64_t n = r->n;
    if (ldx < n || (mem != BFMF_HOST && mem != BFMF_DEVICE)) {
      st = BFMF_E_INVAL;
    } else {
      const hipError_t e = hipMemcpy2DAsync(X, (size_t)ldx * 16, s->arena.buf.as<char>() + r->x_off, (size_t)n * 16,
                                            (size_t)n * 16, r->nrhs,
                                            mem == BFMF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                            s->copy_stream);
      const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(s->copy_stream) : e;
      if (e2 != hipSuccess) st = BFMF_E_DEVICE;
    }
  }
  if (info) *info = r->info;
  const bfmf_status solve_st = (bfmf_status)r->info.status;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->admitted) s->arena.release(r->x_off, r->x_bytes);
    s->reqs.erase(ticket);
  }
  s->cv.notify_all();  // arena space for waiting workers
  return st != BFMF_OK ? st : solve_st;
}

double bfmf_server_clock(bfmf_server s) { return s ? s->clock() : 0.0; }

const char* bfmf_server_last_error(bfmf_server s) { return s ? s->err.c_str() : "null server"; }

void bfmf_server_destroy(bfmf_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& m : s->models)
    if (m->worker.joinable()) m->worker.join();
  (void)hipSetDevice(s->device);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  delete s;
}

}  // extern "C"
