// Numerical factorization of the dense fronts, the preconditioner sweeps and
// the FP64 GMRES driver.
//
// Factorization (Alg. 1): fronts are processed level by level from the
// deepest level to the root.  With opts.batched every kernel of a level is one
// launch over all fronts of the level; otherwise every front gets its own
// launches (the plain form).  The arena keeps every front in place: F11 holds
// L\U, F12 holds L^-1 P^T F12, F21 holds F21 U^-1 and F22 the contribution
// block C that the parent reads during its extend-add.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>

#include "context.hpp"
#include "kernels/kernels.hpp"

namespace bfmf {

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void alloc(DevBuf& b, size_t bytes) {
  b.release();
  if (bytes == 0) bytes = 16;
  hipError_t e = dev_malloc((void**)&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    throw Error(BFMF_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(BFMF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

hipEvent_t KernelTimer::take() {
  if (used == pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool[used++];
}

int KernelTimer::begin(hipStream_t s) {
  if (!enabled) return -1;
  Rec r;
  r.kind = -1;
  r.a = take();
  r.b = take();
  r.flops = r.bytes = 0;
  r.shape[0] = r.shape[1] = r.shape[2] = r.shape[3] = 0;
  HIPCHK(hipEventRecord(r.a, s));
  recs.push_back(r);
  return (int)recs.size() - 1;
}

int KernelTimer::begin_ext(hipEvent_t* start, hipEvent_t* stop) {
  if (!enabled) return -1;
  Rec r;
  r.kind = -1;
  r.a = take();
  r.b = take();
  r.flops = r.bytes = 0;
  r.shape[0] = r.shape[1] = r.shape[2] = r.shape[3] = 0;
  *start = r.a;
  *stop = r.b;
  recs.push_back(r);
  return (int)recs.size() - 1;
}

void KernelTimer::end_ext(int token, int kind, double fl, double by) {
  if (token < 0) return;
  Rec& r = recs[token];
  r.kind = kind;
  r.flops = fl;
  r.bytes = by;
}

void KernelTimer::end(int token, hipStream_t s, int kind, double fl, double by) {
  if (token < 0) return;
  Rec& r = recs[token];
  r.kind = kind;
  r.flops = fl;
  r.bytes = by;
  HIPCHK(hipEventRecord(r.b, s));
}

void KernelTimer::collect() {
  for (const Rec& r : recs) {
    if (r.kind < 0) continue;
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    launches[r.kind] += 1;
    seconds[r.kind] += ms * 1e-3;
    flops[r.kind] += r.flops;
    bytes[r.kind] += r.bytes;
    if (r.kind == K_BF_GEMM) {
      const int b = r.flops >= 1 ? std::min(63, (int)std::log2(r.flops)) : 0;
      hist_n[b] += 1;
      hist_s[b] += ms * 1e-3;
      hist_f[b] += r.flops;
      std::array<int, 4> key;
      for (int q = 0; q < 4; ++q) key[q] = r.shape[q] > 0 ? (int)std::log2((double)r.shape[q]) : -1;
      auto& v = shapes[key];
      v[0] += 1;
      v[1] += ms * 1e-3;
      v[2] += r.flops;
    }
  }
  recs.clear();
  used = 0;
}

void KernelTimer::reset() {
  recs.clear();
  used = 0;
  for (int k = 0; k < K_COUNT; ++k) {
    launches[k] = issued[k] = 0;
    seconds[k] = flops[k] = bytes[k] = 0;
  }
  for (int b = 0; b < 64; ++b) hist_n[b] = hist_s[b] = hist_f[b] = 0;
  for (double& x : pad) x = 0;
  for (int b = 0; b < 20; ++b) mhist[b] = nhist[b] = 0;
  shapes.clear();
}

KernelTimer::~KernelTimer() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

void factor_dense(Context& c) {
  const int32_t nf = c.sym.nfronts();
  const size_t elem = sizeof(double) * 2;
  // fronts compressed by Alg. 5: separator fronts with #I^s >= n_min
  c.compressed.assign(nf, 0);
  int ncomp = 0;
  for (int32_t f = 0; f < nf; ++f)
    if (c.fopts.n_min > 0 && !c.sym.leaf[f] && c.fp[f].ns >= c.fopts.n_min) {
      c.compressed[f] = 1;
      ++ncomp;
    }
  // contribution blocks kept in HOD-BF form: compressed fronts with a compressed parent
  c.cbcomp.assign(nf, 0);
  if (c.fopts.compress_cb)
    for (int32_t f = 0; f < nf; ++f) {
      const int32_t p = c.sym.parent[f];
      if (c.compressed[f] && p >= 0 && c.compressed[p] && c.fp[f].nu > 0) c.cbcomp[f] = 1;
    }
  // level order with the dense fronts of a level first
  const int nlev0 = (int)c.level_ptr.size() - 1;
  c.level_order.clear();
  c.level_ndense.assign(nlev0, 0);
  for (int L = 0; L < nlev0; ++L) {
    for (int k = c.level_ptr[L]; k < c.level_ptr[L + 1]; ++k)
      if (!c.compressed[c.level_fronts[k]]) c.level_order.push_back(c.level_fronts[k]);
    c.level_ndense[L] = (int)c.level_order.size() - c.level_ptr[L];
    for (int k = c.level_ptr[L]; k < c.level_ptr[L + 1]; ++k)
      if (c.compressed[c.level_fronts[k]]) c.level_order.push_back(c.level_fronts[k]);
  }
  // Memory.  A front lives in a level workspace from its assembly until the
  // level above has been assembled from its contribution block: dense fronts
  // take n^2 entries there, compressed fronts only their nu^2 block.  Children
  // are exactly one level below their parent, so two workspaces alternating
  // with the level's parity suffice.  The factor panels of a dense front
  // ([L U; F21'] and F12', n*ns + ns*nu entries) are copied to the kept
  // factor store after its Schur complement.  With keep_fronts every front
  // gets a workspace slot of its own (nothing reused), so its contribution
  // block stays readable.
  auto wsize = [&](int32_t f) {
    const FrontPlan& p = c.fp[f];
    if (c.cbcomp[f]) return (int64_t)0;  // its contribution block lives in HOD-BF form
    return c.compressed[f] ? (int64_t)p.nu * p.nu : (int64_t)p.n * p.n;
  };
  int64_t par_max[2] = {0, 0}, uniq = 0;
  for (int L = 0; L < nlev0; ++L) {
    int64_t lvl = 0;
    for (int k = c.level_ptr[L]; k < c.level_ptr[L + 1]; ++k) lvl += wsize(c.level_fronts[k]);
    par_max[L & 1] = std::max(par_max[L & 1], lvl);
    uniq += lvl;
  }
  int64_t fac = 0;
  for (int L = 0; L < nlev0; ++L) {
    int64_t off = c.fopts.keep_fronts ? 0 : ((L & 1) ? par_max[0] : 0);
    if (c.fopts.keep_fronts)
      for (int M = 0; M < L; ++M)
        for (int k = c.level_ptr[M]; k < c.level_ptr[M + 1]; ++k) off += wsize(c.level_fronts[k]);
    for (int k = c.level_ptr[L]; k < c.level_ptr[L + 1]; ++k) {
      const int32_t f = c.level_order[k];
      FrontPlan& p = c.fp[f];
      p.f_off = off;
      off += wsize(f);
      p.p_off = -1;
      if (!c.compressed[f]) {
        p.p_off = fac;
        fac += (int64_t)p.n * p.ns + (int64_t)p.ns * p.nu;
      }
    }
  }
  c.work_elems = c.fopts.keep_fronts ? uniq : par_max[0] + par_max[1];
  c.fac_elems = fac;
  const size_t need = (size_t)(c.work_elems + c.fac_elems + (c.fopts.keep_fronts ? uniq : 0)) * elem;
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  const size_t have = free_b + c.d_work.bytes + c.d_fac.bytes + c.d_kept.bytes;  // reused on a new factor
  const uint64_t budget = c.fopts.hbm_budget ? c.fopts.hbm_budget : (uint64_t)have;
  if (need > budget || need > have)
    throw Error(BFMF_E_NOMEM, "front workspaces and dense factors need " + std::to_string(need) + " bytes, budget " +
                                  std::to_string(std::min<uint64_t>(budget, have)));
  // the butterfly pool and scratch of the compressed fronts grow during the factorization: charged
  // against what the budget leaves (unbounded without a budget: growth then fails only in hipMalloc)
  c.fbudget.limit = c.fopts.hbm_budget ? budget - need : ~0ull;
  c.fbudget.held = 0;
  if (c.d_work.bytes < (size_t)c.work_elems * elem) alloc(c.d_work, (size_t)c.work_elems * elem);
  if (c.d_fac.bytes < (size_t)c.fac_elems * elem) alloc(c.d_fac, std::max<size_t>((size_t)c.fac_elems * elem, 16));
  if (c.fopts.keep_fronts) {
    if (c.d_kept.bytes < (size_t)uniq * elem) alloc(c.d_kept, (size_t)uniq * elem);
  } else {
    c.d_kept.release();
  }
  if (ncomp) {
    if (!c.comp) c.comp = comp_state_create(c);
    comp_state_reset(c.comp, c, nf);
    // grouped-GEMM tile tables of this device, measured once per process (before the factor clock starts)
    gemm_autotune<double>(c.device, c.stream);
    if (c.fopts.precision == BFMF_C64_MIXED) gemm_autotune<float>(c.device, c.stream);
  }
  // descriptors in level order
  char* arena = c.d_work.as<char>();
  char* facs = c.d_fac.as<char>();
  c.h_fds.assign(nf, FrontDesc());
  for (int32_t k = 0; k < nf; ++k) {
    const int32_t f = c.level_order[k];
    c.desc_index[f] = k;
    const FrontPlan& p = c.fp[f];
    FrontDesc& d = c.h_fds[k];
    std::memset(&d, 0, sizeof(d));
    d.F = arena + p.f_off * elem;
    if (p.p_off >= 0) {
      d.P = facs + p.p_off * elem;
      d.F12 = facs + (p.p_off + (int64_t)p.n * p.ns) * elem;
      d.ld12 = std::max(p.ns, 1);
    }
    d.n = p.n;
    d.ns = p.ns;
    d.nchild = p.nchild;
    d.front = f;
    d.sbeg = c.sym.sbeg[f];
    for (int q = 0; q < p.nchild; ++q) {
      const FrontPlan& cp = c.fp[p.child[q]];
      d.inv[q] = c.d_inv.as<int32_t>() + p.inv_off[q];
      if (c.cbcomp[p.child[q]]) {  // HOD-BF: its descriptor is set once the child is factored
        d.cb[q] = nullptr;
        d.cb_ld[q] = 1;
      } else if (c.compressed[p.child[q]]) {  // contribution block stored alone (ld nu)
        d.cb[q] = arena + cp.f_off * elem;
        d.cb_ld[q] = std::max(cp.nu, 1);
      } else {
        d.cb[q] = arena + (cp.f_off + cp.ns + (int64_t)cp.ns * cp.n) * elem;
        d.cb_ld[q] = cp.n;
      }
    }
    d.a_ptr = c.d_aptr.as<int64_t>() + p.aptr_off;
    d.a_row = c.d_arow.as<int32_t>();
    d.a_vidx = c.d_avidx.as<int64_t>();
    d.piv = c.d_piv.as<int32_t>() + p.piv_off;
    d.pperm = c.d_pperm.as<int32_t>() + p.piv_off;
    d.iu = c.d_iu32.as<int32_t>() + p.iu_off;
  }
  if (c.d_fds.bytes < nf * sizeof(FrontDesc)) alloc(c.d_fds, nf * sizeof(FrontDesc));
  HIPCHK(hipMemcpy(c.d_fds.p, c.h_fds.data(), nf * sizeof(FrontDesc), hipMemcpyHostToDevice));
  if (c.g_tmp_scatter.bytes < nf * sizeof(AxpbyTask)) alloc(c.g_tmp_scatter, nf * sizeof(AxpbyTask));
  c.fds_nrhs = -1;  // solve workspaces not set in these descriptors
  ++c.factor_gen;   // a captured preconditioner of the previous factorization is stale
  HIPCHK(hipMemsetAsync(c.d_status.p, 0, 16, c.stream));

  const double t0 = now();
  if (c.verbose) {
    c.hprof.reset();
    g_hprof = &c.hprof;
  }
  FrontDesc* dfds = c.d_fds.as<FrontDesc>();
  std::vector<int> hn, hns;
  const int nlev = (int)c.level_ptr.size() - 1;
  for (int L = 0; L < nlev; ++L) {
    const int b = c.level_ptr[L], e = b + c.level_ndense[L], e_all = c.level_ptr[L + 1];
    auto run = [&](int lo, int hi) {
      if (hi <= lo) return;
      hn.clear();
      hns.clear();
      int maxn = 0;
      double asm_bytes = 0, lu_flops = 0, sch_flops = 0, sch_bytes = 0, store_bytes = 0;
      int64_t maxstore = 0;
      for (int k = lo; k < hi; ++k) {
        const int32_t f = c.level_order[k];
        const FrontPlan& p = c.fp[f];
        hn.push_back(p.n);
        hns.push_back(p.ns);
        maxn = std::max(maxn, p.n);
        const double n = p.n, ns = p.ns, nu = p.nu;
        double cb = 0;
        for (int q = 0; q < p.nchild; ++q) cb += (double)c.fp[p.child[q]].nu * c.fp[p.child[q]].nu;
        const double na = (double)(c.h_aptr[p.aptr_off + p.n] - c.h_aptr[p.aptr_off]);
        asm_bytes += elem * (n * n + cb) + 28.0 * na + 4.0 * n * p.nchild + 8.0 * (n + 1);
        lu_flops += 8.0 / 3.0 * ns * ns * ns + 8.0 * ns * ns * nu;
        sch_flops += 8.0 * ns * nu * nu;
        sch_bytes += elem * (2.0 * ns * nu + 2.0 * nu * nu);
        store_bytes += 2.0 * elem * (n * ns + ns * nu);
        maxstore = std::max(maxstore, (int64_t)p.n * p.ns + (int64_t)p.ns * p.nu);
      }
      int tk = c.timer.begin(c.stream);
      check(launch_assemble<double>(dfds + lo, hi - lo, maxn, c.d_values.p, false, c.stream), "assemble");
      c.timer.end(tk, c.stream, K_ASSEMBLE, 0, asm_bytes);
      if (c.fopts.keep_fronts) {
        for (int k = lo; k < hi; ++k) {
          const FrontPlan& p = c.fp[c.level_order[k]];
          HIPCHK(hipMemcpyAsync(c.d_kept.as<char>() + p.f_off * elem, arena + p.f_off * elem,
                                (size_t)p.n * p.n * elem, hipMemcpyDeviceToDevice, c.stream));
        }
      }
      tk = c.timer.begin(c.stream);
      check(launch_partial_lu<double>(dfds + lo, hi - lo, hn.data(), hns.data(), c.d_status.as<int>(), c.stream),
            "partial LU");
      c.timer.end(tk, c.stream, K_LU, lu_flops, 0);
      tk = c.timer.begin(c.stream);
      if (c.fopts.precision == BFMF_C64_MIXED)  // complex64 form: the Schur product on FP32 MFMA
        check(launch_schur_mixed(dfds + lo, hi - lo, hn.data(), hns.data(), c.stream), "schur");
      else
        check(launch_schur<double>(dfds + lo, hi - lo, hn.data(), hns.data(), c.stream), "schur");
      c.timer.end(tk, c.stream, K_SCHUR, sch_flops, sch_bytes);
      tk = c.timer.begin(c.stream);
      check(launch_store_factor<double>(dfds + lo, hi - lo, maxstore, c.stream), "factor store");
      c.timer.end(tk, c.stream, K_STORE, 0, store_bytes);
    };
    if (c.fopts.batched) {
      run(b, e);
    } else {
      for (int k = b; k < e; ++k) run(k, k + 1);
    }
    // compressed fronts of this level (Alg. 5)
    if (e_all > e) {
      std::vector<int> cfr;
      std::vector<const FrontDesc*> cfd;
      std::vector<void*> ccb;
      for (int k = e; k < e_all; ++k) {
        const int32_t f = c.level_order[k];
        cfr.push_back(f);
        cfd.push_back(dfds + k);
        ccb.push_back(arena + c.fp[f].f_off * elem);
        const FrontDesc& d = c.h_fds[k];
        for (int q = 0; q < d.nchild; ++q)
          if (!d.cb[q] && !d.chb[q])
            throw Error(BFMF_E_INVAL, "internal: a child's contribution block is missing");
      }
      factor_compressed_level(c.comp, c, cfr, cfd, ccb);
      // the parents read the blocks built in HOD-BF form through these descriptors
      for (int32_t f : cfr) {
        if (!c.cbcomp[f]) continue;
        const int32_t p = c.sym.parent[f];
        const int kp = c.desc_index[p];
        const FrontPlan& pp = c.fp[p];
        const HodbfDev* dv = comp_cb_dev(c.comp, f);
        if (!dv) throw Error(BFMF_E_INVAL, "internal: contribution block in HOD-BF form without a descriptor");
        for (int q = 0; q < pp.nchild; ++q)
          if (pp.child[q] == f) c.h_fds[kp].chb[q] = dv;
        HIPCHK(hipMemcpyAsync(dfds + kp, &c.h_fds[kp], sizeof(FrontDesc), hipMemcpyHostToDevice, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
      }
    }
  }
  // the dense fronts' row interchanges as permutations, read by the blocked sweeps
  check(launch_pivot_perm(dfds, nf, c.stream), "pivot permutation");
  HIPCHK(hipStreamSynchronize(c.stream));
  c.stats.factor_seconds = now() - t0;
  if (c.verbose) {
    g_hprof = nullptr;
    const HostProf& h = c.hprof;
    fprintf(stderr,
            "[bfmf-host] factor %.3f s: blocked in syncs %.3f s (%lld), staging puts %.3f s (%lld), GEMM launch calls "
            "%.3f s (%lld), plan building %.3f s (%lld), run_plan total %.3f s (%lld); inclusive: entry "
            "constructions %.3f s, random constructions %.3f s, extraction %.3f s (%lld), proxy sampling %.3f s "
            "(%lld)\n",
            c.stats.factor_seconds, h.sec[HP_SYNC], (long long)h.n[HP_SYNC], h.sec[HP_PUT], (long long)h.n[HP_PUT],
            h.sec[HP_LAUNCH], (long long)h.n[HP_LAUNCH], h.sec[HP_PLAN], (long long)h.n[HP_PLAN], h.sec[HP_RUN],
            (long long)h.n[HP_RUN], h.sec[HP_ENTRY], h.sec[HP_RANDOM], h.sec[HP_EXTRACT], (long long)h.n[HP_EXTRACT],
            h.sec[HP_SAMPLE], (long long)h.n[HP_SAMPLE]);
  }
  c.timer.collect();
  if (c.verbose && c.timer.enabled) {
    fprintf(stderr, "[bfmf] butterfly GEMM launches (timed sample) by log2 flops: bucket count ms TFLOP/s\n");
    for (int b = 0; b < 64; ++b)
      if (c.timer.hist_n[b] > 0)
        fprintf(stderr, "[bfmf]   2^%-2d %8.0f %9.2f %7.2f\n", b, c.timer.hist_n[b], 1e3 * c.timer.hist_s[b],
                c.timer.hist_f[b] / std::max(c.timer.hist_s[b], 1e-30) / 1e12);
    std::vector<std::pair<double, std::array<int, 4>>> top;
    for (auto& kv : c.timer.shapes) top.push_back({kv.second[1], kv.first});
    std::sort(top.rbegin(), top.rend());
    const double* pd = c.timer.pad;
    if (pd[0] > 0) {
      fprintf(stderr,
              "[bfmf] butterfly GEMM padding to the tile (all launches): M %.3f N %.3f K %.3f all %.3f\n",
              pd[1] / pd[0], pd[2] / pd[0], pd[3] / pd[0], pd[4] / pd[0]);
      fprintf(stderr, "[bfmf] butterfly GEMM work by ceil(M/16), ceil(N/16) (share of multiply-adds):\n[bfmf]  ");
      for (int b = 1; b < 20; ++b) fprintf(stderr, " %d:%.3f/%.3f", b, c.timer.mhist[b] / pd[0], c.timer.nhist[b] / pd[0]);
      fprintf(stderr, "\n");
    }
    fprintf(stderr, "[bfmf] butterfly GEMM launch classes by time (log2 of tasks, max M, N, K): count ms TFLOP/s\n");
    for (size_t q = 0; q < std::min<size_t>(top.size(), 25); ++q) {
      const auto& v = c.timer.shapes[top[q].second];
      const auto& k = top[q].second;
      fprintf(stderr, "[bfmf]   %2d %2d %2d %2d %7.0f %8.2f %7.2f\n", k[0], k[1], k[2], k[3], v[0], 1e3 * v[1],
              v[2] / std::max(v[1], 1e-30) / 1e12);
    }
  }
  int st[3] = {0, 0, 0};
  HIPCHK(hipMemcpy(st, c.d_status.p, sizeof(st), hipMemcpyDeviceToHost));
  c.stats.singular_front = st[0] ? st[1] : -1;
  c.stats.singular_index = st[0] ? st[2] : -1;
  if (st[0]) throw Error(BFMF_E_SINGULAR, "exact zero pivot in front " + std::to_string(st[1]) + " at local index " +
                                              std::to_string(st[2]));
  double flops = 0, bytes = 0, dense_bytes = 0;
  for (int32_t f = 0; f < nf; ++f) {
    const double ns = c.fp[f].ns, nu = c.fp[f].nu;
    const double fb = (ns * ns + 2 * ns * nu) * elem;
    dense_bytes += fb;
    if (c.compressed[f]) continue;
    flops += 8.0 / 3.0 * ns * ns * ns + 8.0 * ns * ns * nu + 8.0 * ns * nu * nu;
    bytes += fb;
  }
  int maxrank = 0, chunked = 0;
  if (ncomp) {
    double cb = 0;
    compressed_stats(c.comp, cb, maxrank, chunked);
    bytes += cb;
  }
  c.stats.id_chunked = chunked;
  c.stats.cb_bytes = c.stats.cb_dense_bytes = 0;
  c.stats.cb_compressed = 0;
  if (ncomp) {
    uint64_t centre_peak = 0;
    compressed_cb_stats(c.comp, c.stats.cb_bytes, c.stats.cb_dense_bytes, c.stats.cb_compressed, centre_peak);
  }
  c.stats.workspace_bytes = (double)c.work_elems * 16.0;
  c.stats.factor_flops = flops;
  c.stats.factor_bytes = bytes;
  c.stats.dense_factor_bytes = dense_bytes;
  c.stats.max_rank = maxrank;
  c.stats.nfronts = nf;
  c.stats.compressed_fronts = ncomp;
  c.stats.dense_fronts = nf - ncomp;
  c.stats.nlevels = nlev;
  c.stats.solve_flops_per_rhs = 0;
  for (int32_t f = 0; f < nf; ++f) {
    const double ns = c.fp[f].ns, nu = c.fp[f].nu;
    c.stats.solve_flops_per_rhs += 8.0 * (ns * ns + 2 * ns * nu);
  }
}

void ensure_workspace(Context& c, int64_t nrhs) {
  const size_t elem = sizeof(double) * 2;
  if (c.ws_nrhs < nrhs) {
    alloc(c.d_W, (size_t)c.sum_n * nrhs * elem);
    alloc(c.d_y, (size_t)c.n * nrhs * elem);
    alloc(c.d_x, (size_t)c.n * nrhs * elem);
    c.ws_nrhs = nrhs;
    ++c.ws_gen;
    c.fds_nrhs = -1;
  }
  if (c.fds_nrhs == nrhs) return;  // the device descriptors already point into these workspaces
  // W pointers depend on nrhs: W_f at sum_{g<f} n_g * nrhs
  char* W = c.d_W.as<char>();
  const int32_t nf = c.sym.nfronts();
  for (int32_t k = 0; k < nf; ++k) {
    const int32_t f = c.level_order[k];
    const FrontPlan& p = c.fp[f];
    FrontDesc& d = c.h_fds[k];
    d.W = W + p.w_off * nrhs * elem;
    for (int q = 0; q < p.nchild; ++q) {
      const FrontPlan& cp = c.fp[p.child[q]];
      d.cw[q] = W + (cp.w_off * nrhs + cp.ns) * elem;
      d.cw_ld[q] = cp.n;
    }
  }
  HIPCHK(hipMemcpyAsync(c.d_fds.p, c.h_fds.data(), nf * sizeof(FrontDesc), hipMemcpyHostToDevice, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));  // the host copy of the descriptors is rewritten on the next change
  c.fds_nrhs = nrhs;
}

void apply_preconditioner_dev(Context& c, const void* dB, int64_t ldb, void* dX, int64_t ldx, int64_t nrhs) {
  ensure_workspace(c, nrhs);
  FrontDesc* dfds = c.d_fds.as<FrontDesc>();
  check(launch_permute_in<double>(dB, ldb, c.d_y.p, c.d_perm.as<int64_t>(), c.n, (int)nrhs, c.stream), "permute");
  const int nlev = (int)c.level_ptr.size() - 1;
  double lvl_bytes = 0, lvl_flops = 0;
  const double elem = 16.0;
  int maxns = 0;
  auto level_sizes = [&](int lo, int hi, int& maxn, int& maxnu) {
    maxn = 0;
    maxnu = 0;
    maxns = 0;
    lvl_bytes = lvl_flops = 0;
    for (int k = lo; k < hi; ++k) {
      const FrontPlan& p = c.fp[c.level_order[k]];
      maxn = std::max(maxn, p.n);
      maxnu = std::max(maxnu, p.nu);
      maxns = std::max(maxns, p.ns);
      const double ns = p.ns, nu = p.nu;
      // half of F11 (L or U) plus F21 or F12, read once; vectors in and out
      lvl_bytes += elem * (0.5 * ns * ns + ns * nu) + elem * 3.0 * (ns + nu) * nrhs;
      lvl_flops += 8.0 * (0.5 * ns * ns + ns * nu) * nrhs;
    }
  };
  for (int L = 0; L < nlev; ++L) {
    const int b = c.level_ptr[L], e = b + c.level_ndense[L], e_all = c.level_ptr[L + 1];
    if (e <= b) {
    } else if (c.fopts.batched) {
      int mn, mu;
      level_sizes(b, e, mn, mu);
      const int tk = c.timer.begin(c.stream);
      check(launch_forward_level<double>(dfds + b, e - b, mn, mu, maxns, c.d_y.p, c.n, (int)nrhs, c.stream), "fwd");
      c.timer.end(tk, c.stream, K_FWD, lvl_flops, lvl_bytes);
    } else {
      for (int k = b; k < e; ++k) {
        int mn, mu;
        level_sizes(k, k + 1, mn, mu);
        const int tk = c.timer.begin(c.stream);
        check(launch_forward_level<double>(dfds + k, 1, mn, mu, maxns, c.d_y.p, c.n, (int)nrhs, c.stream), "fwd");
        c.timer.end(tk, c.stream, K_FWD, lvl_flops, lvl_bytes);
      }
    }
    if (e_all > e && c.fopts.batched) {  // compressed fronts of the level together
      std::vector<int> fs, ns;
      std::vector<void*> Ws;
      int maxn = 0;
      for (int k = e; k < e_all; ++k) {
        fs.push_back(c.level_order[k]);
        ns.push_back(c.fp[c.level_order[k]].n);
        Ws.push_back(c.h_fds[k].W);
        maxn = std::max(maxn, c.fp[c.level_order[k]].n);
      }
      check(launch_fwd_gather<double>(dfds + e, e_all - e, maxn, c.d_y.p, c.n, (int)nrhs, c.stream), "fwd gather");
      forward_compressed_level(c.comp, c, fs, Ws, ns, (int)nrhs);
    } else {
      for (int k = e; k < e_all; ++k) {  // compressed fronts one after another
        const FrontPlan& p = c.fp[c.level_order[k]];
        check(launch_fwd_gather<double>(dfds + k, 1, p.n, c.d_y.p, c.n, (int)nrhs, c.stream), "fwd gather");
        forward_compressed(c.comp, c, c.level_order[k], c.h_fds[k].W, p.n, (int)nrhs);
      }
    }
  }
  for (int L = nlev - 1; L >= 0; --L) {
    const int b = c.level_ptr[L], e = b + c.level_ndense[L], e_all = c.level_ptr[L + 1];
    if (e_all > e && c.fopts.batched) {  // compressed fronts of the level together
      std::vector<int> fs, ns;
      std::vector<void*> Ws;
      std::vector<AxpbyTask> sc;
      int maxnu = 0;
      int64_t maxe = 0;
      for (int k = e; k < e_all; ++k) {
        const FrontPlan& p = c.fp[c.level_order[k]];
        fs.push_back(c.level_order[k]);
        ns.push_back(p.n);
        Ws.push_back(c.h_fds[k].W);
        maxnu = std::max(maxnu, p.nu);
        maxe = std::max<int64_t>(maxe, (int64_t)p.ns * nrhs);
        sc.push_back(AxpbyTask{(char*)c.d_x.p + c.sym.sbeg[c.level_order[k]] * 16, c.h_fds[k].W, c.n, p.n, p.ns,
                               (int32_t)nrhs, 0});  // x(I^s) = W(0:ns)
      }
      check(launch_bwd_gather<double>(dfds + e, e_all - e, maxnu, c.d_x.p, c.n, (int)nrhs, c.stream), "bwd gather");
      backward_compressed_level(c.comp, c, fs, Ws, ns, (int)nrhs);
      AxpbyTask* d_sc = (AxpbyTask*)c.g_tmp_scatter.p;
      if (c.g_tmp_scatter.bytes < sc.size() * sizeof(AxpbyTask))
        throw Error(BFMF_E_INVAL, "internal: scatter task buffer too small");
      c.stage.put(d_sc, sc.data(), sc.size() * sizeof(AxpbyTask), c.stream);
      check(launch_mix_batch<double, double>(d_sc, (int)sc.size(), maxe, 1.0, 0.0, 0.0, c.stream), "scatter");
    } else {
      for (int k = e; k < e_all; ++k) {  // compressed fronts one after another
        const FrontPlan& p = c.fp[c.level_order[k]];
        check(launch_bwd_gather<double>(dfds + k, 1, p.nu, c.d_x.p, c.n, (int)nrhs, c.stream), "bwd gather");
        backward_compressed(c.comp, c, c.level_order[k], c.h_fds[k].W, p.n, (int)nrhs);
        check(launch_axpby<double>((char*)c.d_x.p + c.sym.sbeg[c.level_order[k]] * 16, c.n, c.h_fds[k].W, p.n, p.ns,
                                   (int)nrhs, 1.0, 0.0, c.stream),
              "scatter");
      }
    }
    if (e <= b) {
    } else if (c.fopts.batched) {
      int mn, mu;
      level_sizes(b, e, mn, mu);
      const int tk = c.timer.begin(c.stream);
      check(launch_backward_level<double>(dfds + b, e - b, mn, mu, maxns, c.d_x.p, c.n, (int)nrhs, c.stream), "bwd");
      c.timer.end(tk, c.stream, K_BWD, lvl_flops, lvl_bytes);
    } else {
      for (int k = e - 1; k >= b; --k) {
        int mn, mu;
        level_sizes(k, k + 1, mn, mu);
        const int tk = c.timer.begin(c.stream);
        check(launch_backward_level<double>(dfds + k, 1, mn, mu, maxns, c.d_x.p, c.n, (int)nrhs, c.stream), "bwd");
        c.timer.end(tk, c.stream, K_BWD, lvl_flops, lvl_bytes);
      }
    }
  }
  check(launch_permute_out<double>(c.d_x.p, dX, ldx, c.d_perm.as<int64_t>(), c.n, (int)nrhs, c.stream), "permute");
}

// The preconditioner application in -> out replayed from a HIP graph.  The
// graph is captured from one application (after an eager one with the same
// sizes, so that no workspace grows while capturing), with the staged task
// lists copied from a pinned arena that the graph owns; it is rebuilt for
// other buffers, another column count, a new factorization or moved
// workspaces.  Returns false (and the caller applies eagerly) when capture is
// not possible; after a failed capture the factorization stays eager.
static bool apply_preconditioner_graph(Context& c, const void* in, void* out, int64_t nrhs, size_t stage_bytes) {
  PrecGraph& g = c.pgraph;
  if (!c.stream || g.failed_gen == c.factor_gen) return false;
  ensure_workspace(c, nrhs);
  const bool valid = g.exec && g.in == in && g.out == out && g.nrhs == nrhs && g.gen == c.factor_gen &&
                     g.ws_gen == c.ws_gen;
  if (!valid) {
    HIPCHK(hipStreamSynchronize(c.stream));  // no replay of the old graph in flight
    g.release();
    g.host_cap = stage_bytes + ((size_t)1 << 20);
    if (hipHostMalloc((void**)&g.host, g.host_cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      g.host = nullptr;
      g.failed_gen = c.factor_gen;
      return false;
    }
    c.stage.arena = g.host;
    c.stage.arena_cap = g.host_cap;
    c.stage.arena_head = 0;
    const bool timing = c.timer.enabled;
    c.timer.enabled = false;
    bool ok = hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      try {
        apply_preconditioner_dev(c, in, c.n, out, c.n, nrhs);
      } catch (const std::exception&) {
        ok = false;
      }
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(c.stream, &graph);
      ok = ok && ee == hipSuccess && graph;
      if (ok && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
      if (graph) g.graph = graph;
    }
    c.stage.arena = nullptr;
    c.timer.enabled = timing;
    if (!ok) {
      (void)hipGetLastError();
      g.release();
      g.failed_gen = c.factor_gen;
      return false;
    }
    g.in = in;
    g.out = out;
    g.nrhs = nrhs;
    g.gen = c.factor_gen;
    g.ws_gen = c.ws_gen;
  }
  const int tk = c.timer.begin(c.stream);
  HIPCHK(hipGraphLaunch(g.exec, c.stream));
  c.timer.end(tk, c.stream, K_PGRAPH, 0, 0);
  return true;
}

// ------------------------------------------------------------------ GMRES
void gmres_workspace(Context& c, int64_t nrhs, int m) {
  const size_t elem = 2 * sizeof(double);
  const size_t blk = (size_t)c.n * nrhs * elem;
  const size_t vbytes = blk * (m + 1);
  // The Krylov basis takes the level workspace of the factorization when that is large enough: the
  // workspace holds fronts only while bfmf_factor runs (128^3 with 32 columns: 33 GB of basis inside
  // 62 GB of workspace).  A later factorization invalidates the captured preconditioner graph anyway.
  if (!c.fopts.keep_fronts && c.d_work.bytes >= vbytes) {
    c.g_V.release();
    c.g_Vp = c.d_work.p;
  } else {
    if (c.g_V.bytes < vbytes) alloc(c.g_V, vbytes);
    c.g_Vp = c.g_V.p;
  }
  if (c.g_nrhs < nrhs || c.g_restart < m) {
    alloc(c.g_w, blk);
    alloc(c.g_r, blk);
    alloc(c.g_tmp, blk);
    alloc(c.g_scal, (size_t)(m + 2) * nrhs * elem * 2);
    alloc(c.g_part, (size_t)256 * nrhs * elem);
    c.g_nrhs = nrhs;
    c.g_restart = m;
  }
}

int gmres_dev(Context& c, const void* dB, int64_t ldb, void* dX, int64_t ldx, int64_t nrhs, bfmf_solve_opts& o) {
  typedef std::complex<double> cd;
  const int64_t N = c.n;
  const int m = std::max(1, o.restart);
  const size_t elem = sizeof(cd);
  gmres_workspace(c, nrhs, m);
  const bool use_graph = o.graphs != 0;  // replay the preconditioner of the iterations from a HIP graph
  size_t stage_bytes = 0;
  const int nblk = (int)std::min<int64_t>(256, (N + 255) / 256);
  cd* V = (cd*)c.g_Vp;
  cd* w = c.g_w.as<cd>();
  cd* r = c.g_r.as<cd>();
  cd* tmp = c.g_tmp.as<cd>();
  cd* hcol = c.g_scal.as<cd>();           // (m+2) x nrhs
  cd* ydev = hcol + (size_t)(m + 2) * nrhs;  // m x nrhs
  const int nr = (int)nrhs;
  const int64_t vstride = N * nrhs;
  auto Vi = [&](int i) { return V + (size_t)i * vstride; };
  const int64_t* rp = c.d_rowptr.as<int64_t>();
  const int32_t* ci = c.d_colind.as<int32_t>();
  const void* va = c.d_values.p;
  const double spmv_bytes = 20.0 * c.nnz + 8.0 * (N + 1) + 2.0 * elem * N * nrhs;
  const double spmv_flops = 8.0 * c.nnz * nrhs;
  auto spmv = [&](const void* X, int64_t ldx_, void* Y, int64_t ldy_, const void* B_, int64_t ldb_) {
    const int tk = c.timer.begin(c.stream);
    check(launch_spmv(rp, ci, va, X, ldx_, Y, ldy_, B_, ldb_, N, (int)nrhs, c.stream), "spmv");
    c.timer.end(tk, c.stream, K_SPMV, spmv_flops, spmv_bytes);
  };

  for (int q = 0; q < nr; ++q) HIPCHK(hipMemsetAsync((cd*)dX + q * ldx, 0, N * elem, c.stream));
  std::vector<cd> hb(nr);
  check(launch_dots(nullptr, 0, dB, ldb, N, nr, c.g_part.p, nblk, hcol, true, c.stream), "norm");
  HIPCHK(hipMemcpyAsync(hb.data(), hcol, nr * elem, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  std::vector<double> bnorm(nr), u0(nr, -1), tol_c(nr, o.rtol);
  for (int q = 0; q < nr; ++q) bnorm[q] = hb[q].real();
  std::vector<char> done(nr, 0);
  std::vector<int> iters(nr, 0);
  std::vector<cd> H((size_t)(m + 1) * m * nr), g((size_t)(m + 1) * nr), cs((size_t)m * nr), sn((size_t)m * nr);
  std::vector<cd> hh((size_t)(m + 2) * nr), yh((size_t)m * nr);
  std::vector<int> steps(nr);
  std::vector<double> relres(nr, 1.0);
  int total = 0;
  for (int q = 0; q < nr; ++q)
    if (bnorm[q] == 0) done[q] = 1;

  auto true_residual = [&]() {
    spmv(dX, ldx, r, N, dB, ldb);
    check(launch_dots(nullptr, 0, r, N, N, nr, c.g_part.p, nblk, hcol, true, c.stream), "norm");
    HIPCHK(hipMemcpyAsync(hh.data(), hcol, nr * elem, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    for (int q = 0; q < nr; ++q) relres[q] = bnorm[q] > 0 ? hh[q].real() / bnorm[q] : 0.0;
  };

  if (o.max_iter < 0) {  // direct solve: X = M^-1 B with the approximate factorization, no refinement
    apply_preconditioner_dev(c, dB, ldb, dX, ldx, nrhs);
    true_residual();
    c.timer.collect();
    o.iters_max = 0;
    o.relres_max = 0;
    bool ok = true;
    c.g_col_iters.assign(nr, 0);
    c.g_col_relres.assign(relres.begin(), relres.end());
    c.g_col_done.assign(nr, 1);
    for (int q = 0; q < nr; ++q) {
      o.relres_max = std::max(o.relres_max, relres[q]);
      c.g_col_done[q] = !(o.true_rtol > 0) || relres[q] <= o.true_rtol;
      ok &= (bool)c.g_col_done[q];
    }
    return ok ? 0 : 1;
  }

  while (total < o.max_iter) {
    bool any = false;
    for (int q = 0; q < nr; ++q) any |= !done[q];
    if (!any) break;
    // r = b - A x ; V0 = M^-1 r (eager: it also sizes the staged task lists of one application)
    spmv(dX, ldx, r, N, dB, ldb);
    const size_t put0 = c.stage.put_bytes;
    apply_preconditioner_dev(c, r, N, Vi(0), N, nr);
    stage_bytes = std::max(stage_bytes, c.stage.put_bytes - put0);
    check(launch_dots(nullptr, 0, Vi(0), N, N, nr, c.g_part.p, nblk, hcol, true, c.stream), "norm");
    HIPCHK(hipMemcpyAsync(hh.data(), hcol, nr * elem, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    std::vector<char> active(nr, 0);
    for (int q = 0; q < nr; ++q) {
      const double beta = hh[q].real();
      if (u0[q] < 0) u0[q] = beta;
      if (done[q]) continue;
      if (beta <= o.atol || (u0[q] > 0 && beta / u0[q] <= tol_c[q])) {
        done[q] = 1;
        continue;
      }
      active[q] = 1;
      std::fill(g.begin() + (size_t)q * (m + 1), g.begin() + (size_t)(q + 1) * (m + 1), cd(0));
      g[(size_t)q * (m + 1)] = beta;
      steps[q] = 0;
    }
    check(launch_scale_cols(hcol, Vi(0), N, Vi(0), N, N, nr, c.stream), "scale");
    bool cycle_active = false;
    for (int q = 0; q < nr; ++q) cycle_active |= active[q];
    if (!cycle_active) break;
    for (int j = 0; j < m && total < o.max_iter; ++j) {
      spmv(Vi(j), N, tmp, N, nullptr, 0);
      if (!(use_graph && apply_preconditioner_graph(c, tmp, w, nr, stage_bytes)))
        apply_preconditioner_dev(c, tmp, N, w, N, nr);
      for (int i = 0; i <= j; ++i) {  // modified Gram-Schmidt
        check(launch_dots(Vi(i), N, w, N, N, nr, c.g_part.p, nblk, hcol + (size_t)i * nr, false, c.stream), "dot");
        check(launch_axpy_cols(hcol + (size_t)i * nr, -1.0, Vi(i), N, w, N, N, nr, c.stream), "axpy");
      }
      check(launch_dots(nullptr, 0, w, N, N, nr, c.g_part.p, nblk, hcol + (size_t)(j + 1) * nr, true, c.stream),
            "norm");
      check(launch_scale_cols(hcol + (size_t)(j + 1) * nr, w, N, Vi(j + 1), N, N, nr, c.stream), "scale");
      HIPCHK(hipMemcpyAsync(hh.data(), hcol, (size_t)(j + 2) * nr * elem, hipMemcpyDeviceToHost, c.stream));
      HIPCHK(hipStreamSynchronize(c.stream));
      ++total;
      bool still = false;
      for (int q = 0; q < nr; ++q) {
        if (!active[q]) continue;
        cd* Hq = H.data() + (size_t)q * (m + 1) * m;
        cd* gq = g.data() + (size_t)q * (m + 1);
        cd* csq = cs.data() + (size_t)q * m;
        cd* snq = sn.data() + (size_t)q * m;
        for (int i = 0; i <= j + 1; ++i) Hq[i + (size_t)j * (m + 1)] = hh[(size_t)i * nr + q];
        for (int i = 0; i < j; ++i) {  // previous rotations
          cd a = Hq[i + (size_t)j * (m + 1)], b = Hq[i + 1 + (size_t)j * (m + 1)];
          Hq[i + (size_t)j * (m + 1)] = csq[i] * a + snq[i] * b;
          Hq[i + 1 + (size_t)j * (m + 1)] = -std::conj(snq[i]) * a + std::conj(csq[i]) * b;
        }
        cd a = Hq[j + (size_t)j * (m + 1)], b = Hq[j + 1 + (size_t)j * (m + 1)];
        const double den = std::sqrt(std::norm(a) + std::norm(b));
        if (den == 0) {
          csq[j] = 1;
          snq[j] = 0;
        } else if (std::abs(a) == 0) {
          csq[j] = 0;
          snq[j] = std::conj(b) / den;
        } else {
          csq[j] = std::abs(a) / den;
          snq[j] = (a / std::abs(a)) * std::conj(b) / den;
        }
        Hq[j + (size_t)j * (m + 1)] = csq[j] * a + snq[j] * b;
        Hq[j + 1 + (size_t)j * (m + 1)] = 0;
        gq[j + 1] = -std::conj(snq[j]) * gq[j];
        gq[j] = csq[j] * gq[j];
        steps[q] = j + 1;
        iters[q]++;
        const double res = std::abs(gq[j + 1]);
        if (res <= o.atol || res / u0[q] <= tol_c[q] || hh[(size_t)(j + 1) * nr + q].real() == 0) {
          active[q] = 0;
        } else {
          still = true;
        }
      }
      if (!still) break;
    }
    // x += V y per column
    int mmax = 0;
    std::fill(yh.begin(), yh.end(), cd(0));
    for (int q = 0; q < nr; ++q) {
      const int k = steps[q];
      if (k == 0) continue;
      mmax = std::max(mmax, k);
      cd* Hq = H.data() + (size_t)q * (m + 1) * m;
      cd* gq = g.data() + (size_t)q * (m + 1);
      for (int i = k - 1; i >= 0; --i) {
        cd s = gq[i];
        for (int l = i + 1; l < k; ++l) s -= Hq[i + (size_t)l * (m + 1)] * yh[l + (size_t)q * m];
        yh[i + (size_t)q * m] = s / Hq[i + (size_t)i * (m + 1)];
      }
      steps[q] = 0;
    }
    if (mmax > 0) {
      HIPCHK(hipMemcpyAsync(ydev, yh.data(), (size_t)m * nr * elem, hipMemcpyHostToDevice, c.stream));
      check(launch_basis_update(ydev, m, mmax, V, vstride, N, dX, ldx, N, nr, c.stream), "update");
    }
    // columns that met the preconditioned criterion: check the true residual
    bool need_true = o.true_rtol > 0;
    bool all_done = true;
    for (int q = 0; q < nr; ++q) all_done &= (bool)(done[q] || !active[q]);
    if (need_true) {
      true_residual();
      for (int q = 0; q < nr; ++q) {
        if (relres[q] > o.true_rtol) {
          // the preconditioned stop came too early for this column: tighten it
          if (done[q] || !active[q]) tol_c[q] *= 0.1;
          done[q] = 0;
        } else {
          done[q] = 1;
        }
      }
    } else {
      for (int q = 0; q < nr; ++q)
        if (!active[q]) done[q] = 1;
    }
    (void)all_done;
  }
  true_residual();
  c.timer.collect();
  o.iters_max = 0;
  o.relres_max = 0;
  for (int q = 0; q < nr; ++q) {
    o.iters_max = std::max(o.iters_max, iters[q]);
    o.relres_max = std::max(o.relres_max, relres[q]);
  }
  bool ok = true;
  for (int q = 0; q < nr; ++q) ok &= (bool)done[q];
  c.g_col_iters.assign(iters.begin(), iters.end());
  c.g_col_relres.assign(relres.begin(), relres.end());
  c.g_col_done.assign(done.begin(), done.end());
  return ok ? 0 : 1;
}

// ------------------------------------------------------------ slot GMRES
// Device arrays of a slot iteration (per slot, in dbuf): source pointers of the gathered columns,
// destination pointers of the new basis vectors, modes, MGS limits, basis-update counts, the norms of
// the preconditioned vectors and of the true residuals.
namespace {
struct SlotArrays {
  const void** src;
  void** dst;
  int32_t *mode, *lim, *mc;
  std::complex<double>*norm, *tn;
};
SlotArrays slot_arrays(DevBuf& b, int slots) {
  char* p = b.as<char>();
  SlotArrays a;
  a.src = (const void**)p;
  a.dst = (void**)(p + 8 * (size_t)slots);
  a.mode = (int32_t*)(p + 16 * (size_t)slots);
  a.lim = a.mode + slots;
  a.mc = a.lim + slots;
  a.norm = (std::complex<double>*)(p + ((28 * (size_t)slots + 15) & ~(size_t)15));
  a.tn = a.norm + slots;
  return a;
}
size_t slot_bytes(int slots) { return ((28 * (size_t)slots + 15) & ~(size_t)15) + 32 * (size_t)slots; }
}  // namespace

void SlotGmres::init(Context& ctx, int nslots, const bfmf_solve_opts& opts, void* dB, void* dX) {
  c = &ctx;
  slots = nslots;
  o = opts;
  if (o.restart <= 0) o.restart = 30;
  if (o.max_iter <= 0) o.max_iter = 300;
  m = o.restart;
  B = dB;
  X = dX;
  mode.assign(slots, IDLE);
  j.assign(slots, 0);
  iters.assign(slots, 0);
  u0.assign(slots, -1);
  tol_c.assign(slots, o.rtol);
  bnorm.assign(slots, -1);
  relres.assign(slots, 1);
  pc_met.assign(slots, 0);
  ok.assign(slots, 0);
  H.assign((size_t)(m + 1) * m * slots, 0);
  g.assign((size_t)(m + 1) * slots, 0);
  cs.assign((size_t)m * slots, 0);
  sn.assign((size_t)m * slots, 0);
  y.assign((size_t)m * slots, 0);
  gmres_workspace(ctx, slots, m);
  ensure_workspace(ctx, slots);
  if (dbuf.bytes < slot_bytes(slots)) {
    dbuf.release();
    HIPCHK(dev_malloc((void**)&dbuf.p, slot_bytes(slots)));
    dbuf.bytes = slot_bytes(slots);
  }
  last_width = -1;
}

void SlotGmres::admit(int q) {
  mode[q] = START;
  j[q] = 0;
  iters[q] = 0;
  u0[q] = -1;
  tol_c[q] = o.rtol;
  bnorm[q] = -1;
  relres[q] = 1;
  pc_met[q] = 0;
  ok[q] = 0;
}

bool SlotGmres::busy() const {
  for (int md : mode)
    if (md != IDLE) return true;
  return false;
}

void SlotGmres::step(std::vector<int>& finished) {
  typedef std::complex<double> cd;
  finished.clear();
  Context& cc = *c;
  const int64_t N = cc.n;
  int width = 0;
  for (int q = 0; q < slots; ++q)
    if (mode[q] != IDLE) width = q + 1;
  if (width == 0) return;
  int Wd = 1;  // the preconditioner runs on a power-of-two number of columns (one captured graph per width)
  while (Wd < width) Wd *= 2;
  Wd = std::min(Wd, slots);
  gmres_workspace(cc, slots, m);  // the basis may live in the level workspace: refresh its address
  const size_t elem = sizeof(cd);
  cd* V = (cd*)cc.g_Vp;
  cd* Vcur = cc.g_tmp.as<cd>();
  cd* T = cc.g_r.as<cd>();
  cd* w = cc.g_w.as<cd>();
  cd* hcol = cc.g_scal.as<cd>();
  cd* ydev = hcol + (size_t)(m + 2) * slots;
  const int64_t vstride = N * slots;
  const int nblk = (int)std::min<int64_t>(256, (N + 255) / 256);
  SlotArrays da = slot_arrays(dbuf, slots);
  // 1. the vector each column multiplies: x (restart: T = b - A x) or its current basis vector
  std::vector<const void*> src(Wd, nullptr);
  std::vector<int32_t> md(Wd, 0), lim(Wd, -1);
  int jmax = -1;
  for (int q = 0; q < Wd; ++q) {
    if (mode[q] == START) {
      src[q] = (cd*)X + (size_t)q * N;
      md[q] = 1;
    } else if (mode[q] == RUN) {
      src[q] = V + (size_t)j[q] * vstride + (size_t)q * N;
      md[q] = 2;
      lim[q] = j[q];
      jmax = std::max(jmax, j[q]);
    }
  }
  cc.stage.put(da.src, src.data(), Wd * sizeof(void*), cc.stream);
  cc.stage.put(da.mode, md.data(), Wd * sizeof(int32_t), cc.stream);
  cc.stage.put(da.lim, lim.data(), Wd * sizeof(int32_t), cc.stream);
  check(launch_slot_gather(da.src, Vcur, N, N, Wd, cc.stream), "slot gather");
  check(launch_spmv(cc.d_rowptr.as<int64_t>(), cc.d_colind.as<int32_t>(), cc.d_values.p, Vcur, N, T, N, nullptr, 0, N,
                    Wd, cc.stream),
        "spmv");
  check(launch_slot_fix(da.mode, B, N, T, N, N, Wd, cc.stream), "slot fix");
  check(launch_dots(nullptr, 0, T, N, N, Wd, cc.g_part.p, nblk, da.tn, true, cc.stream), "norm");
  // 2. w = M^-1 T: an eager application at a new width (it sizes the staged task lists), replays after
  if (Wd != last_width) {
    const size_t put0 = cc.stage.put_bytes;
    apply_preconditioner_dev(cc, T, N, w, N, Wd);
    stage_bytes = cc.stage.put_bytes - put0;
    last_width = Wd;
  } else if (!(o.graphs && apply_preconditioner_graph(cc, T, w, Wd, stage_bytes))) {
    apply_preconditioner_dev(cc, T, N, w, N, Wd);
  }
  // 3. modified Gram-Schmidt of the running columns against their own bases
  for (int i = 0; i <= jmax; ++i) {
    cd* Vi = V + (size_t)i * vstride;
    check(launch_dots(Vi, N, w, N, N, Wd, cc.g_part.p, nblk, hcol + (size_t)i * slots, false, cc.stream), "dot");
    check(launch_axpy_cols_masked(hcol + (size_t)i * slots, -1.0, Vi, N, w, N, N, Wd, da.lim, i, cc.stream), "axpy");
  }
  check(launch_dots(nullptr, 0, w, N, N, Wd, cc.g_part.p, nblk, da.norm, true, cc.stream), "norm");
  std::vector<cd> hh((size_t)(jmax + 1) * slots + 1), nrm(Wd), tn(Wd);
  if (jmax >= 0) HIPCHK(hipMemcpyAsync(hh.data(), hcol, (size_t)(jmax + 1) * slots * elem, hipMemcpyDeviceToHost, cc.stream));
  HIPCHK(hipMemcpyAsync(nrm.data(), da.norm, Wd * elem, hipMemcpyDeviceToHost, cc.stream));
  HIPCHK(hipMemcpyAsync(tn.data(), da.tn, Wd * elem, hipMemcpyDeviceToHost, cc.stream));
  HIPCHK(hipStreamSynchronize(cc.stream));
  // 4. per column: start a cycle, take a step, or end a cycle
  std::vector<void*> dst(Wd, nullptr);
  std::vector<int32_t> mc(Wd, 0);
  bool upd = false;
  for (int q = 0; q < Wd; ++q) {
    if (mode[q] == START) {
      const double t = tn[q].real();
      if (bnorm[q] < 0) bnorm[q] = t;  // x = 0 at admission: the first residual is b
      relres[q] = bnorm[q] > 0 ? t / bnorm[q] : 0.0;
      bool stop = false, good = false;
      if (bnorm[q] == 0) {
        stop = good = true;
      } else if (o.true_rtol > 0 && relres[q] <= o.true_rtol) {
        stop = good = true;
      } else if (!(o.true_rtol > 0) && pc_met[q]) {
        stop = good = true;
      } else if (iters[q] >= o.max_iter) {
        stop = true;
      }
      const double beta = nrm[q].real();
      if (!stop) {
        if (pc_met[q]) tol_c[q] *= 0.1;  // the preconditioned test was met too early for the true one
        pc_met[q] = 0;
        if (u0[q] < 0) u0[q] = beta;
        if (beta <= o.atol || !(beta > 0)) {
          stop = true;  // no further progress possible
          good = !(o.true_rtol > 0);
        } else {
          while (beta / u0[q] <= tol_c[q] && tol_c[q] > 1e-300) tol_c[q] *= 0.1;
        }
      }
      if (stop) {
        mode[q] = IDLE;
        ok[q] = good;
        finished.push_back(q);
        continue;
      }
      cd* gq = g.data() + (size_t)q * (m + 1);
      std::fill(gq, gq + m + 1, cd(0));
      gq[0] = beta;
      j[q] = 0;
      mode[q] = RUN;
      dst[q] = V + (size_t)q * N;  // V_0 = w / beta
    } else if (mode[q] == RUN) {
      const int jj = j[q];
      cd* Hq = H.data() + (size_t)q * (m + 1) * m;
      cd* gq = g.data() + (size_t)q * (m + 1);
      cd* csq = cs.data() + (size_t)q * m;
      cd* snq = sn.data() + (size_t)q * m;
      for (int i = 0; i <= jj; ++i) Hq[i + (size_t)jj * (m + 1)] = hh[(size_t)i * slots + q];
      Hq[jj + 1 + (size_t)jj * (m + 1)] = nrm[q];
      const double hnext = nrm[q].real();
      for (int i = 0; i < jj; ++i) {  // previous rotations
        cd a = Hq[i + (size_t)jj * (m + 1)], b = Hq[i + 1 + (size_t)jj * (m + 1)];
        Hq[i + (size_t)jj * (m + 1)] = csq[i] * a + snq[i] * b;
        Hq[i + 1 + (size_t)jj * (m + 1)] = -std::conj(snq[i]) * a + std::conj(csq[i]) * b;
      }
      cd a = Hq[jj + (size_t)jj * (m + 1)], b = Hq[jj + 1 + (size_t)jj * (m + 1)];
      const double den = std::sqrt(std::norm(a) + std::norm(b));
      if (den == 0) {
        csq[jj] = 1;
        snq[jj] = 0;
      } else if (std::abs(a) == 0) {
        csq[jj] = 0;
        snq[jj] = std::conj(b) / den;
      } else {
        csq[jj] = std::abs(a) / den;
        snq[jj] = (a / std::abs(a)) * std::conj(b) / den;
      }
      Hq[jj + (size_t)jj * (m + 1)] = csq[jj] * a + snq[jj] * b;
      Hq[jj + 1 + (size_t)jj * (m + 1)] = 0;
      gq[jj + 1] = -std::conj(snq[jj]) * gq[jj];
      gq[jj] = csq[jj] * gq[jj];
      iters[q]++;
      const double res = std::abs(gq[jj + 1]);
      const bool conv = res <= o.atol || res / u0[q] <= tol_c[q] || hnext == 0;
      if (conv || jj + 1 == m || iters[q] >= o.max_iter) {  // end of the cycle: x += V y
        const int k = jj + 1;
        cd* yq = y.data() + (size_t)q * m;
        std::fill(yq, yq + m, cd(0));
        for (int i = k - 1; i >= 0; --i) {
          cd sacc = gq[i];
          for (int l = i + 1; l < k; ++l) sacc -= Hq[i + (size_t)l * (m + 1)] * yq[l];
          yq[i] = sacc / Hq[i + (size_t)i * (m + 1)];
        }
        mc[q] = k;
        upd = true;
        pc_met[q] = conv;
        mode[q] = START;  // unless the check below finds it done, the next iteration restarts it
      } else {
        dst[q] = V + (size_t)(jj + 1) * vstride + (size_t)q * N;
        j[q] = jj + 1;
      }
    }
  }
  // 5. new basis vectors and solution updates
  bool any_dst = false;
  for (void* d : dst) any_dst |= d != nullptr;
  if (any_dst) {
    cc.stage.put(da.dst, dst.data(), Wd * sizeof(void*), cc.stream);
    check(launch_scale_cols_to(da.norm, w, N, da.dst, N, Wd, cc.stream), "scale");
  }
  if (upd) {
    cc.stage.put(da.mc, mc.data(), Wd * sizeof(int32_t), cc.stream);
    cc.stage.put(ydev, y.data(), (size_t)m * Wd * elem, cc.stream);
    check(launch_basis_update_masked(ydev, m, da.mc, V, vstride, N, X, N, N, Wd, cc.stream), "update");
    // the columns whose cycle ended: their true residual and the stopping test now (a residual, no
    // preconditioner application), so that a finished column leaves its slot at once
    check(launch_spmv(cc.d_rowptr.as<int64_t>(), cc.d_colind.as<int32_t>(), cc.d_values.p, X, N, T, N, B, N, N, Wd,
                      cc.stream),
          "spmv");
    check(launch_dots(nullptr, 0, T, N, N, Wd, cc.g_part.p, nblk, da.tn, true, cc.stream), "norm");
    HIPCHK(hipMemcpyAsync(tn.data(), da.tn, Wd * elem, hipMemcpyDeviceToHost, cc.stream));
    HIPCHK(hipStreamSynchronize(cc.stream));
    for (int q = 0; q < Wd; ++q) {
      if (mc[q] == 0) continue;
      relres[q] = bnorm[q] > 0 ? tn[q].real() / bnorm[q] : 0.0;
      const bool done = o.true_rtol > 0 ? relres[q] <= o.true_rtol : pc_met[q] != 0;
      if (done) {
        mode[q] = IDLE;
        ok[q] = 1;
        finished.push_back(q);
      }
    }
  }
}

}  // namespace bfmf
