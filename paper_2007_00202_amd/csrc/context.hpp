// The state behind a bfmf_handle: symbolic analysis, the device plan of the
// dense fronts, device buffers and counters.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>

#include <cstdint>
#include <array>
#include <chrono>
#include <map>
#include <memory>
#include <string>
#include <complex>
#include <vector>

#include "../../include/bfmf.h"
#include "analyze.hpp"
#include "devtypes.hpp"

namespace bfmf {

// RAII device allocation
// Every device allocation of the library goes through dev_malloc, which counts
// it (process-wide; bfmf_device_allocation_count reports the count).
inline std::atomic<int64_t> g_device_allocations{0};
inline hipError_t dev_malloc(void** p, size_t bytes) {
  g_device_allocations.fetch_add(1, std::memory_order_relaxed);
  return hipMalloc(p, bytes);
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

// Device bytes that growable buffers of a factorization may hold together (the
// hbm_budget left after the level workspaces and dense factors); growth beyond
// it raises E_NOMEM before anything is allocated.
struct Budget {
  uint64_t limit = ~0ull;
  uint64_t held = 0;
  bool fits(uint64_t add) const { return held + add <= limit; }
};

class Error : public std::exception {
 public:
  bfmf_status status;
  std::string msg;
  Error(bfmf_status s, std::string m) : status(s), msg(std::move(m)) {}
  const char* what() const noexcept override { return msg.c_str(); }
};

#define HIPCHK(expr)                                                                           \
  do {                                                                                         \
    hipError_t e__ = (expr);                                                                   \
    if (e__ != hipSuccess)                                                                     \
      throw ::bfmf::Error(BFMF_E_DEVICE, std::string(#expr " failed: ") + hipGetErrorString(e__)); \
  } while (0)

// Host-to-device uploads of task and index lists.  The host data is copied
// into a pinned ring and the device copy is enqueued on the stream, so the
// caller's vector may be freed at once and no synchronisation is needed.  The
// ring is reused after the stream has been synchronised (sync()), or, when it
// is full, after put() has synchronised the stream itself.
// Host-side time of a factorization by activity (BFMF_VERBOSE diagnostics).
enum HostSlot { HP_SYNC = 0, HP_PUT, HP_LAUNCH, HP_PLAN, HP_RUN, HP_ENTRY, HP_RANDOM, HP_EXTRACT, HP_SAMPLE, HP_COUNT };
struct HostProf {
  double sec[HP_COUNT] = {};
  int64_t n[HP_COUNT] = {};
  void reset() {
    for (int i = 0; i < HP_COUNT; ++i) sec[i] = 0, n[i] = 0;
  }
};
extern thread_local HostProf* g_hprof;  // the profile of the call in progress on this thread, or null
struct HostTimer {
  int slot;
  std::chrono::steady_clock::time_point t0;
  explicit HostTimer(int sl) : slot(sl) {
    if (g_hprof) t0 = std::chrono::steady_clock::now();
  }
  ~HostTimer() {
    if (!g_hprof) return;
    g_hprof->sec[slot] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    g_hprof->n[slot] += 1;
  }
};

struct Staging {
  char* host = nullptr;
  size_t cap = 0, head = 0;
  // while a graph is captured, puts go to this arena instead (never reused: the graph's copies read it
  // on every replay); put_bytes counts the ring's bytes since the last reset (sizes such an arena)
  char* arena = nullptr;
  size_t arena_cap = 0, arena_head = 0;
  size_t put_bytes = 0;
  void put(void* dst, const void* src, size_t bytes, hipStream_t s);
  void sync(hipStream_t s);
  Staging() = default;
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  ~Staging();
};

enum class State { Created, Analyzed, Factored };

enum KernelKind {
  K_ASSEMBLE = 0,
  K_LU = 1,
  K_SCHUR = 2,
  K_FWD = 3,
  K_BWD = 4,
  K_SPMV = 5,
  K_VEC = 6,
  K_BF_GEMM = 7,  // grouped GEMMs of butterfly products and constructions
  K_ID = 8,       // interpolative decompositions
  K_EXTRACT = 9,  // entry extraction from never-formed fronts and sketches
  K_STORE = 10,   // copy of the dense factors out of the level workspace
  K_PGRAPH = 11,  // one replay of the captured preconditioner (forward and backward sweeps)
  K_COUNT = 12
};

// HIP-event timing of kernel classes on the handle's stream.
struct KernelTimer {
  bool enabled = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double flops, bytes;
    int shape[4];  // butterfly GEMM launches: tasks, largest M, N, K
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  int64_t launches[K_COUNT] = {};  // timed launches
  int64_t issued[K_COUNT] = {};    // all launches while enabled
  int sample_every[K_COUNT] = {1, 1, 1, 1, 1, 1, 1, 8, 1, 1, 1, 1};  // time one launch in this many
  double seconds[K_COUNT] = {}, flops[K_COUNT] = {}, bytes[K_COUNT] = {};
  // timed butterfly GEMM launches by floor(log2(flops)): count, seconds, flops
  double hist_n[64] = {}, hist_s[64] = {}, hist_f[64] = {};
  // timed butterfly GEMM launches by log2 of (tasks, M, N, K): count, seconds, flops
  std::map<std::array<int, 4>, std::array<double, 3>> shapes;
  // every butterfly GEMM task (diagnostics, BFMF_VERBOSE): multiply-adds as given, and with M, N, K
  // padded to the launch's tile (one at a time, then all); multiply-adds by ceil(M/16) and ceil(N/16)
  double pad[5] = {};
  double mhist[20] = {}, nhist[20] = {};
  void set_shape(int token, int ntasks, int m, int n, int k) {
    if (token >= 0) recs[token].shape[0] = ntasks, recs[token].shape[1] = m, recs[token].shape[2] = n,
                    recs[token].shape[3] = k;
  }
  // whether to time the next launch of this class (counts it either way)
  // Launches to time: with sample_every = k > 1, a launch is taken when the
  // fractional part of i * (golden ratio) lies below 1/k (i = the class's
  // launch counter): about one in k, spread quasi-randomly, so the sample
  // does not alias with periodic launch sequences.
  bool want(int kind) {
    if (!enabled) return false;
    const uint64_t i = (uint64_t)issued[kind]++;
    if (sample_every[kind] <= 1) return true;
    const double frac = (double)((i * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
    return frac * sample_every[kind] < 1.0;
  }
  hipEvent_t take();
  int begin(hipStream_t s);
  void end(int token, hipStream_t s, int kind, double fl, double by);
  // a record whose two events the caller hands to a launch that timestamps them itself
  int begin_ext(hipEvent_t* start, hipEvent_t* stop);
  void end_ext(int token, int kind, double fl, double by);
  void collect();  // after the stream is synchronised
  void reset();
  ~KernelTimer();
};

// Host mirror of the per-front data that the kernels need.
struct FrontPlan {
  int32_t n = 0, ns = 0, nu = 0;
  int32_t nchild = 0;
  int32_t child[2] = {-1, -1};
  int64_t f_off = 0;      // element offset of F in the level workspace (dense: n^2, compressed: nu^2 block)
  int64_t p_off = -1;     // element offset of the kept factor (dense fronts: n*ns + ns*nu entries)
  int64_t inv_off[2] = {-1, -1};
  int64_t aptr_off = 0;   // into a_ptr (n+1 entries)
  int64_t piv_off = 0;    // into piv (ns entries)
  int64_t iu_off = 0;     // into iu32 (nu entries)
  int64_t w_off = 0;      // element offset of W per rhs column block (n entries per column)
  bool compressed = false;
};

// The preconditioner application in -> out (nrhs columns) captured as a HIP
// graph, replayed by the GMRES iterations; valid for one factorization and
// one set of solve workspaces.
struct PrecGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char* host = nullptr;  // pinned task lists that the graph's copies read
  size_t host_cap = 0;
  const void* in = nullptr;
  void* out = nullptr;
  int64_t nrhs = 0;
  uint64_t gen = 0, ws_gen = 0;
  uint64_t failed_gen = ~0ull;  // factorization for which capture failed (eager from then on)
  void release();
  ~PrecGraph() { release(); }
};

struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t async_ev = nullptr;  // orders bfmf_solve_async's stream with the handle's
  State state = State::Created;
  std::string last_error;

  // problem
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colind;
  std::vector<double> values;  // interleaved complex128, 2 nnz
  Symbolic sym;
  double analyze_seconds = 0;

  // plan
  std::vector<FrontPlan> fp;
  std::vector<int32_t> level_ptr, level_fronts;  // fronts grouped by level, deepest level first
  int64_t work_elems = 0;                        // level workspaces (both depth parities)
  int64_t fac_elems = 0;                         // kept factors of the dense fronts
  int64_t sum_n = 0;                             // sum of n_f
  std::vector<int64_t> h_aptr;
  std::vector<int32_t> h_arow;
  std::vector<int64_t> h_avidx;
  std::vector<int32_t> h_inv;

  // device: matrix and plan
  DevBuf d_rowptr, d_colind, d_values, d_perm;
  DevBuf d_aptr, d_arow, d_avidx, d_inv, d_iu32, d_piv, d_pperm, d_status;
  DevBuf d_fds;            // FrontDesc per front, in level order (level_fronts order)
  std::vector<FrontDesc> h_fds;
  std::vector<int32_t> desc_index;  // front id -> index in h_fds

  // device: numeric
  DevBuf d_work;           // fronts from assembly until the parent level is assembled
  DevBuf d_fac;            // factors of the dense fronts, kept for the sweeps
  DevBuf d_kept;           // debug copies of assembled fronts
  bfmf_factor_opts fopts{};
  int64_t gemm_cfg_launches[16] = {};  // grouped-GEMM launches per tile shape (since the last stats reset)
  bfmf_stats stats{};

  // device: solve workspaces
  DevBuf d_W, d_y, d_x;
  int64_t ws_nrhs = 0;
  int64_t fds_nrhs = -1;       // nrhs the device descriptors' workspace pointers are set for
  uint64_t factor_gen = 0;     // bumped by every factorization
  uint64_t ws_gen = 0;         // bumped when the solve workspaces move
  PrecGraph pgraph;
  DevBuf g_B, g_X, g_V, g_w, g_r, g_scal, g_part, g_tmp;
  DevBuf g_tmp_plan;  // device copy of the current grouped-GEMM task lists
  DevBuf g_tmp_scatter;  // task list of a level's batched scatter in the backward sweep (one per front)
  Staging stage;      // pinned ring of host-to-device uploads
  int64_t g_nrhs = 0, g_restart = 0;
  std::vector<int32_t> g_col_iters;   // per column of the last GMRES call: iterations,
  std::vector<double> g_col_relres;   // true relative residual,
  std::vector<uint8_t> g_col_done;    // and whether it met the stopping test
  void* g_Vp = nullptr;  // Krylov basis: g_V, or the idle level workspace d_work when it is large enough

  KernelTimer timer;

  // compressed fronts (Alg. 5): flag per front, dense fronts per level first
  std::vector<uint8_t> compressed;
  std::vector<uint8_t> cbcomp;        // compressed front whose contribution block is kept in HOD-BF form
  std::vector<int32_t> level_order;   // fronts in level order, dense first within a level
  std::vector<int32_t> level_ndense;  // dense fronts of each level
  void* comp = nullptr;               // CompState (compressed.cpp)
  Budget fbudget;                     // what the compressed fronts' pool and scratch may still take
  bool verbose = false;               // BFMF_VERBOSE: phase timings of compressed fronts on stderr
  HostProf hprof;                     // host time of the last factorization by activity (verbose only)

  uint64_t device_bytes() const;
  ~Context();
};

// message of the last failed call on this thread that had no handle to hold it
extern thread_local std::string g_thread_error;

// autotune.cpp: tile shape of a grouped-GEMM launch (measured table per device
// and precision, built on first use); a process-wide override (-1: autotuned)
template <class T>
void gemm_autotune(int device, hipStream_t s);
template <class T>
int choose_gemm_cfg(int device, hipStream_t s, const std::vector<GTask>& ph);
// one shape for the phase (returned), or -1 with each task's shape in task_cfg
template <class T>
int choose_gemm_cfg_split(int device, hipStream_t s, const std::vector<GTask>& ph, std::vector<int>& task_cfg);
template <class T>
void gemm_tune_table(int device, hipStream_t s, std::vector<double>& out);
void set_gemm_tile_override(int cfg);

// compressed.cpp
void* comp_state_create(Context& c);
void comp_state_destroy(void* p);
void comp_state_reset(void* p, Context& c, int nfronts);
void factor_compressed_level(void* state, Context& c, const std::vector<int>& fronts,
                             const std::vector<const FrontDesc*>& d_fds, const std::vector<void*>& cbs);
void forward_compressed(void* state, Context& c, int f, void* W, int n, int nrhs);
void backward_compressed(void* state, Context& c, int f, void* W, int n, int nrhs);
// all compressed fronts of a level at once (front ids, their workspaces W_f and sizes n_f)
void forward_compressed_level(void* state, Context& c, const std::vector<int>& fronts, const std::vector<void*>& Ws,
                              const std::vector<int>& ns, int nrhs);
void backward_compressed_level(void* state, Context& c, const std::vector<int>& fronts,
                               const std::vector<void*>& Ws, const std::vector<int>& ns, int nrhs);
void compressed_stats(void* state, double& bytes, int& maxrank, int& chunked);
// contribution blocks in HOD-BF form: their pool bytes, the bytes they take dense, their count,
// and the largest device memory their centre forms held at once
void compressed_cb_stats(void* state, double& bytes, double& dense_bytes, int& count, uint64_t& centre_peak);
// device bytes the centre forms of contribution blocks hold now
uint64_t comp_centre_held(void* state);
// device descriptor of front f's contribution block in HOD-BF form (null if it has none)
const HodbfDev* comp_cb_dev(void* state, int f);
uint64_t comp_state_bytes(void* state);  // device bytes held by the compressed fronts' pools
// out(i, j) = F(rows[i], cols[j]) of front f from A and the children's contribution blocks (host, ld ldo)
void extract_front_entries(Context& c, int f, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols,
                           double* out, int64_t ldo);
// Y = B X for a block of compressed front f (0 F11, 1 F11^-1, 2 F12, 3 F21, 4 S, 5 the contribution
// block in HOD-BF form); host complex128 arrays
void comp_apply_block(void* state, int f, int what, int nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy);

// Continuous-batching GMRES of the serving form: the columns ("slots") of B and X
// (device, n x slots, ld n) each run their own restarted GMRES(m) with the
// handle's preconditioner, at their own step; a column is admitted or retired
// between iterations, and its arithmetic does not depend on the other columns.
struct SlotGmres {
  enum { IDLE = 0, START = 1, RUN = 2 };
  Context* c = nullptr;
  int slots = 0, m = 30;
  bfmf_solve_opts o{};
  void* B = nullptr;
  void* X = nullptr;
  std::vector<int32_t> mode, j, iters;
  std::vector<double> u0, tol_c, bnorm, relres;
  std::vector<uint8_t> pc_met, ok;
  std::vector<std::complex<double>> H, g, cs, sn, y;  // per slot: (m+1) x m, m+1, m, m; y m x slots
  DevBuf dbuf;   // per-slot device arrays (pointers, modes, counts, norms)
  int last_width = -1;
  size_t stage_bytes = 0;
  void init(Context& ctx, int nslots, const bfmf_solve_opts& opts, void* dB, void* dX);
  void admit(int q);  // B(:, q) written and X(:, q) zeroed on the stream by the caller
  bool busy() const;
  // one iteration of every admitted column; `finished` gets the slots that completed (ok[q]: met the test)
  void step(std::vector<int>& finished);
};

// plan.cpp
void build_plan(Context& c);
void upload_plan(Context& c);
void upload_values(Context& c);
// numeric.cpp
void factor_dense(Context& c);
void ensure_workspace(Context& c, int64_t nrhs);
void apply_preconditioner_dev(Context& c, const void* dB, int64_t ldb, void* dX, int64_t ldx, int64_t nrhs);
int gmres_dev(Context& c, const void* dB, int64_t ldb, void* dX, int64_t ldx, int64_t nrhs, bfmf_solve_opts& o);
// device buffers of GMRES(m) for nrhs columns (grown, never shrunk)
void gmres_workspace(Context& c, int64_t nrhs, int m);

}  // namespace bfmf

// the opaque handle of the C ABI
struct bfmf_ctx : public bfmf::Context {};
