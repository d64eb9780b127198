// extern "C" entry points of libbfmf (declared in include/bfmf.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "context.hpp"
#include "kernels/kernels.hpp"

using namespace bfmf;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class F>
bfmf_status guarded(bfmf_handle h, F&& fn) {
  if (!h) return BFMF_E_INVAL;
  try {
    if (h->device >= 0) HIPCHK(hipSetDevice(h->device));
    fn();
    return BFMF_OK;
  } catch (const Error& e) {
    h->last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    h->last_error = "host allocation failed";
    return BFMF_E_NOMEM;
  } catch (const std::exception& e) {
    h->last_error = e.what();
    return BFMF_E_INVAL;
  }
}

bool finite_values(const double* v, int64_t cnt) {
  for (int64_t i = 0; i < cnt; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

extern "C" {

bfmf_status bfmf_create(bfmf_handle* h, int32_t device, void* hip_stream) {
  if (!h) return BFMF_E_INVAL;
  *h = nullptr;
  if (device == -1) {  // host-only handle: analysis without a device
    bfmf_ctx* c = new (std::nothrow) bfmf_ctx();
    if (!c) return BFMF_E_NOMEM;
    c->device = -1;
    bfmf_default_factor_opts(&c->fopts);
    *h = c;
    return BFMF_OK;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BFMF_E_DEVICE;
  bfmf_ctx* c = new (std::nothrow) bfmf_ctx();
  if (!c) return BFMF_E_NOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return BFMF_E_DEVICE;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return BFMF_E_DEVICE;
    }
    c->own_stream = true;
  }
  bfmf_default_factor_opts(&c->fopts);
  c->verbose = getenv("BFMF_VERBOSE") != nullptr;
  c->stats.singular_front = -1;
  c->stats.singular_index = -1;
  *h = c;
  return BFMF_OK;
}

void bfmf_default_factor_opts(bfmf_factor_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-3;
  o->n_min = 1024;
  o->precision = BFMF_C128;
  o->batched = 0;
  o->samples = 64;
  o->knn = 8;
  o->alpha = 2.0;
  o->seed = 0;
  o->hbm_budget = 0;
}

void bfmf_default_solve_opts(bfmf_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->restart = 30;
  o->max_iter = 300;
  o->rtol = 1e-6;
  o->atol = 1e-10;
  o->true_rtol = 0;
  o->graphs = 1;
}

bfmf_status bfmf_analyze(bfmf_handle h, int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const double* values, const bfmf_ordering* ord) {
  return guarded(h, [&] {
    if (n <= 0 || !rowptr || !colind || !ord) throw Error(BFMF_E_INVAL, "analyze: null argument or n <= 0");
    if (rowptr[0] != 0) throw Error(BFMF_E_INVAL, "analyze: rowptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
      if (rowptr[i + 1] < rowptr[i]) throw Error(BFMF_E_INVAL, "analyze: rowptr not non-decreasing");
    const int64_t nnz = rowptr[n];
    for (int64_t i = 0; i < n; ++i)
      for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
        if (colind[t] < 0 || colind[t] >= n) throw Error(BFMF_E_INVAL, "analyze: column index out of range");
        if (t > rowptr[i] && colind[t] <= colind[t - 1])
          throw Error(BFMF_E_INVAL, "analyze: column indices not strictly increasing within a row");
      }
    if (values && !finite_values(values, 2 * nnz)) throw Error(BFMF_E_INVAL, "analyze: non-finite matrix value");
    const double t0 = now_s();
    h->state = State::Created;
    h->n = n;
    h->nnz = nnz;
    h->rowptr.assign(rowptr, rowptr + n + 1);
    h->colind.assign(colind, colind + nnz);
    if (values)
      h->values.assign(values, values + 2 * nnz);
    else
      h->values.assign(2 * nnz, 0.0);
    std::string err;
    const int32_t leaf = ord->leaf_max > 0 ? ord->leaf_max : 512;
    const int32_t sl = ord->sep_leaf > 0 ? ord->sep_leaf : 64;
    bool ok;
    if (ord->kind == BFMF_ORD_GRID) {
      if ((int64_t)ord->nx * ord->ny * ord->nz != n) throw Error(BFMF_E_INVAL, "analyze: nx*ny*nz != n");
      ok = nd_grid(ord->nx, ord->ny, ord->nz, leaf, sl, ord->parallel_levels, h->sym, err);
    } else if (ord->kind == BFMF_ORD_YEE) {
      if (ord->parallel_levels != 0) throw Error(BFMF_E_INVAL, "analyze: parallel_levels applies to GRID orderings");
      ok = nd_yee(ord->nx, n, ord->coords, leaf, sl, h->sym, err);
    } else if (ord->kind == BFMF_ORD_USER) {
      if (ord->parallel_levels != 0) throw Error(BFMF_E_INVAL, "analyze: parallel_levels applies to GRID orderings");
      ok = nd_user(n, ord->perm, ord->nfronts, ord->front_ptr, ord->front_parent, sl, h->sym, err);
    } else {
      throw Error(BFMF_E_INVAL, "analyze: unknown ordering kind");
    }
    if (!ok) throw Error(BFMF_E_INVAL, err);
    if (!symbolic_phase(n, rowptr, colind, h->sym, err)) throw Error(BFMF_E_INVAL, err);
    build_plan(*h);
    if (h->device >= 0) upload_plan(*h);
    h->d_work.release();
    h->d_fac.release();
    h->d_kept.release();
    h->analyze_seconds = now_s() - t0;
    h->stats.analyze_seconds = h->analyze_seconds;
    h->state = State::Analyzed;
  });
}

bfmf_status bfmf_set_values(bfmf_handle h, const double* values) {
  return guarded(h, [&] {
    if (h->state == State::Created) throw Error(BFMF_E_STATE, "set_values before analyze");
    if (!values) throw Error(BFMF_E_INVAL, "set_values: null values");
    if (!finite_values(values, 2 * h->nnz)) throw Error(BFMF_E_INVAL, "set_values: non-finite matrix value");
    h->values.assign(values, values + 2 * h->nnz);
    if (h->device >= 0) upload_values(*h);
    h->state = State::Analyzed;
  });
}

bfmf_status bfmf_factor(bfmf_handle h, const bfmf_factor_opts* opts) {
  return guarded(h, [&] {
    if (h->state == State::Created) throw Error(BFMF_E_STATE, "factor before analyze");
    if (h->device < 0) throw Error(BFMF_E_STATE, "factor on a host-only handle");
    bfmf_factor_opts o;
    if (opts)
      o = *opts;
    else
      bfmf_default_factor_opts(&o);
    if (!(o.tol > 0) || o.samples < 0 || o.knn < 0 || o.alpha < 0 || o.smw_dense < 0 ||
        (o.smw_dense > 0 && o.smw_dense < 16) || o.id_max_cols < 0 || (o.id_max_cols > 0 && o.id_max_cols < 16) ||
        (o.compress_cb != 0 && o.compress_cb != 1))
      throw Error(BFMF_E_INVAL, "factor: bad options");
    if (o.precision != BFMF_C128 && o.precision != BFMF_C64_MIXED)
      throw Error(BFMF_E_INVAL, "factor: unknown precision");
    h->fopts = o;
    h->timer.enabled = o.timing != 0;
    h->state = State::Analyzed;
    try {
      factor_dense(*h);
    } catch (...) {
      // back to the analyzed state: no factor memory is kept (the next factorization allocates again)
      (void)hipStreamSynchronize(h->stream);
      if (h->comp) {
        comp_state_destroy(h->comp);
        h->comp = nullptr;
      }
      h->d_work.release();
      h->d_fac.release();
      h->d_kept.release();
      throw;
    }
    // the centre forms of contribution blocks in HOD-BF form are released level by level: add
    // the most they held at once beyond what they hold now
    uint64_t centre_peak = 0;
    if (h->comp) {
      double b0 = 0, b1 = 0;
      int n0 = 0;
      compressed_cb_stats(h->comp, b0, b1, n0, centre_peak);
    }
    const uint64_t now_b = h->device_bytes();
    h->stats.device_bytes_peak = now_b + centre_peak - std::min<uint64_t>(centre_peak, comp_centre_held(h->comp));
    h->state = State::Factored;
  });
}

static bfmf_status solve_common(bfmf_handle h, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                                int32_t mem, bfmf_solve_opts* io, bool precond_only) {
  return guarded(h, [&] {
    if (h->state != State::Factored) throw Error(BFMF_E_STATE, "solve before factor");
    if (nrhs <= 0 || !B || !X || ldb < h->n || ldx < h->n) throw Error(BFMF_E_INVAL, "solve: bad arguments");
    if (mem != BFMF_HOST && mem != BFMF_DEVICE) throw Error(BFMF_E_INVAL, "solve: bad memory kind");
    bfmf_solve_opts o;
    if (io)
      o = *io;
    else
      bfmf_default_solve_opts(&o);
    if (o.restart <= 0) o.restart = 30;
    if (o.max_iter == 0) o.max_iter = 300;  // negative: direct solve
    const double t0 = now_s();
    const size_t elem = 2 * sizeof(double);
    const void* dB = B;
    void* dX = X;
    int64_t lb = ldb, lx = ldx;
    if (mem == BFMF_HOST) {
      DevBuf& bb = h->g_B;
      DevBuf& xb = h->g_X;
      const size_t need = (size_t)h->n * nrhs * elem;
      if (bb.bytes < need) {
        bb.release();
        HIPCHK(dev_malloc((void**)&bb.p, need));
        bb.bytes = need;
      }
      if (xb.bytes < need) {
        xb.release();
        HIPCHK(dev_malloc((void**)&xb.p, need));
        xb.bytes = need;
      }
      HIPCHK(hipMemcpy2DAsync(bb.p, h->n * elem, B, ldb * elem, h->n * elem, nrhs, hipMemcpyHostToDevice,
                              h->stream));
      dB = bb.p;
      dX = xb.p;
      lb = lx = h->n;
    }
    int rc = 0;
    if (precond_only) {
      apply_preconditioner_dev(*h, dB, lb, dX, lx, nrhs);
      HIPCHK(hipStreamSynchronize(h->stream));
      h->timer.collect();
    } else {
      rc = gmres_dev(*h, dB, lb, dX, lx, nrhs, o);
    }
    if (mem == BFMF_HOST)
      HIPCHK(hipMemcpy2DAsync(X, ldx * elem, dX, lx * elem, h->n * elem, nrhs, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    o.seconds = now_s() - t0;
    if (io) *io = o;
    if (rc) throw Error(BFMF_E_NOCONV, "GMRES reached max_iter before convergence");
  });
}

bfmf_status bfmf_solve(bfmf_handle h, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                       int32_t mem, bfmf_solve_opts* io) {
  return solve_common(h, nrhs, B, ldb, X, ldx, mem, io, false);
}

bfmf_status bfmf_solve_async(bfmf_handle h, int64_t nrhs, const double* dB, int64_t ldb, double* dX, int64_t ldx,
                             void* hip_stream, bfmf_solve_opts* io) {
  return guarded(h, [&] {
    if (h->state != State::Factored) throw Error(BFMF_E_STATE, "solve_async before factor");
    if (nrhs <= 0 || !dB || !dX || ldb < h->n || ldx < h->n) throw Error(BFMF_E_INVAL, "solve_async: bad arguments");
    if (io && io->max_iter >= 0)
      throw Error(BFMF_E_INVAL, "solve_async: only the direct solve (max_iter < 0) is queued without host "
                                "synchronisation; GMRES needs the host at every iteration (use bfmf_solve)");
    const double t0 = now_s();
    hipStream_t own = h->stream, s = hip_stream ? (hipStream_t)hip_stream : h->stream;
    if (!h->async_ev) HIPCHK(hipEventCreateWithFlags(&h->async_ev, hipEventDisableTiming));
    if (s != own) {  // the handle's earlier work precedes this call's
      HIPCHK(hipEventRecord(h->async_ev, own));
      HIPCHK(hipStreamWaitEvent(s, h->async_ev, 0));
    }
    h->stream = s;  // every launch and staged copy of the application goes to the caller's stream
    try {
      apply_preconditioner_dev(*h, dB, ldb, dX, ldx, nrhs);
    } catch (...) {
      h->stream = own;
      throw;
    }
    h->stream = own;
    if (s != own) {  // and the handle's later work follows it
      HIPCHK(hipEventRecord(h->async_ev, s));
      HIPCHK(hipStreamWaitEvent(own, h->async_ev, 0));
    }
    if (io) {
      io->iters_max = 0;
      io->relres_max = -1;  // not computed: that would need the host to wait
      io->seconds = now_s() - t0;
    }
  });
}

bfmf_status bfmf_apply_preconditioner(bfmf_handle h, int64_t nrhs, const double* B, int64_t ldb, double* X,
                                      int64_t ldx, int32_t mem) {
  return solve_common(h, nrhs, B, ldb, X, ldx, mem, nullptr, true);
}

bfmf_status bfmf_get_symbolic(bfmf_handle h, bfmf_symbolic_view* out) {
  if (!h || !out) return BFMF_E_INVAL;
  if (h->state == State::Created) return BFMF_E_STATE;
  const Symbolic& s = h->sym;
  out->n = s.n;
  out->nfronts = s.nfronts();
  out->nlevels = s.nlevels;
  out->perm = s.perm.data();
  out->sbeg = s.sbeg.data();
  out->send = s.send.data();
  out->parent = s.parent.data();
  out->level = s.level.data();
  out->child_ptr = s.child_ptr.data();
  out->child_list = s.child_list.data();
  out->iu_ptr = s.iu_ptr.data();
  out->iu = s.iu.data();
  out->map = s.map.data();
  out->sep_ptr = s.sep_ptr.data();
  out->sep_nodes = (const int32_t*)s.sep_nodes.data();
  return BFMF_OK;
}

bfmf_status bfmf_get_stats(bfmf_handle h, bfmf_stats* out) {
  if (!h || !out) return BFMF_E_INVAL;
  *out = h->stats;
  out->device_bytes_peak = std::max<uint64_t>(h->stats.device_bytes_peak, h->device_bytes());
  return BFMF_OK;
}

bfmf_status bfmf_get_front(bfmf_handle h, int32_t front, int32_t what, void* out, int64_t ld) {
  return guarded(h, [&] {
    if (h->state != State::Factored) throw Error(BFMF_E_STATE, "get_front before factor");
    if (front < 0 || front >= h->sym.nfronts() || !out) throw Error(BFMF_E_INVAL, "get_front: bad front");
    const FrontPlan& p = h->fp[front];
    const size_t elem = 2 * sizeof(double);
    if (what == 2) {
      HIPCHK(hipMemcpy(out, h->d_piv.as<int32_t>() + p.piv_off, p.ns * sizeof(int32_t), hipMemcpyDeviceToHost));
      return;
    }
    if (ld < p.n) throw Error(BFMF_E_INVAL, "get_front: ld < n");
    if (h->compressed[front]) throw Error(BFMF_E_INVAL, "get_front: front is compressed");
    if (what == 0 && !h->fopts.keep_fronts) throw Error(BFMF_E_INVAL, "get_front: assembled fronts not kept");
    if (what != 0 && what != 1) throw Error(BFMF_E_INVAL, "get_front: bad 'what'");
    if (h->fopts.keep_fronts) {  // whole fronts, each in a slot of its own
      const DevBuf& src = what == 0 ? h->d_kept : h->d_work;
      HIPCHK(hipMemcpy2D(out, ld * elem, src.as<char>() + p.f_off * elem, p.n * elem, p.n * elem, p.n,
                         hipMemcpyDeviceToHost));
      return;
    }
    // the kept factor: [L U; F21'] then F12'; the contribution block has been reused
    char* o = (char*)out;
    for (int64_t j = 0; j < p.n; ++j) std::memset(o + j * ld * elem, 0, p.n * elem);
    const char* P = h->d_fac.as<char>() + p.p_off * elem;
    if (p.ns > 0)
      HIPCHK(hipMemcpy2D(o, ld * elem, P, p.n * elem, p.n * elem, p.ns, hipMemcpyDeviceToHost));
    if (p.ns > 0 && p.nu > 0)
      HIPCHK(hipMemcpy2D(o + p.ns * ld * elem, ld * elem, P + (int64_t)p.n * p.ns * elem, p.ns * elem, p.ns * elem,
                         p.nu, hipMemcpyDeviceToHost));
  });
}

bfmf_status bfmf_apply_front_block(bfmf_handle h, int32_t front, int32_t what, int32_t nrhs, const double* X,
                                   int64_t ldx, double* Y, int64_t ldy) {
  return guarded(h, [&] {
    if (h->state != State::Factored) throw Error(BFMF_E_STATE, "apply_front_block before factor");
    if (front < 0 || front >= h->sym.nfronts()) throw Error(BFMF_E_INVAL, "apply_front_block: bad front");
    if (!h->compressed[front] || !h->comp) throw Error(BFMF_E_INVAL, "apply_front_block: front is not compressed");
    comp_apply_block(h->comp, front, what, nrhs, X, ldx, Y, ldy);
  });
}

bfmf_status bfmf_extract_front(bfmf_handle h, int32_t front, int32_t nrows, const int32_t* rows, int32_t ncols,
                               const int32_t* cols, double* out, int64_t ldo) {
  return guarded(h, [&] {
    if (h->state != State::Factored) throw Error(BFMF_E_STATE, "extract_front before factor");
    if (front < 0 || front >= h->sym.nfronts()) throw Error(BFMF_E_INVAL, "extract_front: bad front");
    if (!h->fopts.keep_fronts)
      throw Error(BFMF_E_INVAL, "extract_front: the children's contribution blocks are kept only with keep_fronts");
    if (nrows <= 0 || ncols <= 0 || !rows || !cols || !out || ldo < nrows)
      throw Error(BFMF_E_INVAL, "extract_front: bad arguments");
    const int64_t n = h->fp[front].n;
    for (int32_t i = 0; i < nrows; ++i)
      if (rows[i] < 0 || rows[i] >= n) throw Error(BFMF_E_INVAL, "extract_front: row index out of the front");
    for (int32_t j = 0; j < ncols; ++j)
      if (cols[j] < 0 || cols[j] >= n) throw Error(BFMF_E_INVAL, "extract_front: column index out of the front");
    extract_front_entries(*h, front, std::vector<int32_t>(rows, rows + nrows), std::vector<int32_t>(cols, cols + ncols),
                          out, ldo);
  });
}

bfmf_status bfmf_get_kernel_stats(bfmf_handle h, int32_t kind, bfmf_kernel_stat* out) {
  static const char* names[K_COUNT] = {"assemble",      "panel_lu",       "schur_gemm",     "forward_sweep",
                                       "backward_sweep", "spmv",           "gmres_vector",   "butterfly_gemm",
                                       "interp_decomp",  "entry_extract",  "factor_store",   "preconditioner_graph"};
  if (!h || !out || kind < 0 || kind >= K_COUNT) return BFMF_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  std::strncpy(out->name, names[kind], sizeof(out->name) - 1);
  out->launches = h->timer.launches[kind];
  out->launches_all = std::max(h->timer.issued[kind], h->timer.launches[kind]);  // classes timed at every launch
  out->seconds = h->timer.seconds[kind];
  out->flops = h->timer.flops[kind];
  out->bytes = h->timer.bytes[kind];
  return BFMF_OK;
}

bfmf_status bfmf_reset_kernel_stats(bfmf_handle h) {
  if (!h) return BFMF_E_INVAL;
  h->timer.reset();
  for (int64_t& v : h->gemm_cfg_launches) v = 0;
  return BFMF_OK;
}

static_assert(GEMM_CFGS == BFMF_GEMM_TILES && GEMM_CFGS <= 16, "tile shapes of the C ABI");

bfmf_status bfmf_set_gemm_tile(int32_t cfg) {
  if (cfg < -1 || cfg >= GEMM_CFGS) return BFMF_E_INVAL;
  set_gemm_tile_override(cfg);
  return BFMF_OK;
}

bfmf_status bfmf_get_gemm_tile_launches(bfmf_handle h, int64_t* out, int32_t n) {
  if (!h || !out || n < GEMM_CFGS) return BFMF_E_INVAL;
  for (int i = 0; i < n; ++i) out[i] = i < GEMM_CFGS ? h->gemm_cfg_launches[i] : 0;
  return BFMF_OK;
}

int64_t bfmf_device_allocation_count(void) { return g_device_allocations.load(); }

const char* bfmf_status_str(bfmf_status s) {
  switch (s) {
    case BFMF_OK: return "ok";
    case BFMF_E_INVAL: return "invalid argument";
    case BFMF_E_NOMEM: return "out of device memory";
    case BFMF_E_STATE: return "call out of order";
    case BFMF_E_SINGULAR: return "exact zero pivot";
    case BFMF_E_NOCONV: return "GMRES did not converge";
    case BFMF_E_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

const char* bfmf_last_error(bfmf_handle h) { return h ? h->last_error.c_str() : bfmf::g_thread_error.c_str(); }

void bfmf_destroy(bfmf_handle h) {
  if (!h) return;
  if (h->device >= 0) (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  h->pgraph.release();
  if (h->async_ev) (void)hipEventDestroy(h->async_ev);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

}  // extern "C"
