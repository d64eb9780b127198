// Tile-shape autotuner of the grouped GEMM that carries every butterfly
// product (the per-level block-diagonal products of an apply, Sec. 3, and the
// products of the constructions).
//
// On first use per device and precision, every tile shape is timed on
// synthetic grouped launches over a grid of task shapes: M (rows of a block),
// N (right-hand sides or probe columns) and K (inner dimension) in buckets.
// Each timing is the kernel's own duration (events attached to the dispatch)
// of a launch of P equal tasks, P chosen to fill the device, divided by P.  A
// launch then takes the shape whose predicted time, summed over its tasks from
// that table, is least.  All shapes add the products of an entry in the same
// order, so the choice changes the speed and never the result.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>

#include "context.hpp"
#include "kernels/kernels.hpp"

namespace bfmf {

namespace {

// rows in steps that separate the tile heights (16, 32, 48, 64, 96, 128, 256)
constexpr int NM = 9, NN = 6, NK = 4;
constexpr int MB[NM] = {16, 32, 48, 64, 80, 96, 128, 192, 256};
constexpr int NB[NN] = {16, 32, 64, 128, 256, 1024};
constexpr int KB[NK] = {16, 64, 256, 1024};

struct Table {
  bool ready = false;
  double us[GEMM_CFGS][NM][NN][NK];  // microseconds per task
  // fastest shape per bucket, without and with the skinny shape allowed (filled once ready)
  int8_t best[NM][NN][NK][2];
};

std::mutex g_mu;
std::map<std::pair<int, int>, Table> g_tables;  // (device, element size)
std::atomic<int> g_override{-1};

int bucket(const int* b, int n, int v) {
  for (int i = 0; i < n; ++i)
    if (v <= b[i]) return i;
  return n - 1;
}

// bucket of every value up to the largest bucket (1024), built once
struct BucketLut {
  int8_t m[1025], n[1025], k[1025];
  BucketLut() {
    for (int v = 0; v <= 1024; ++v) {
      m[v] = (int8_t)bucket(MB, NM, v);
      n[v] = (int8_t)bucket(NB, NN, v);
      k[v] = (int8_t)bucket(KB, NK, v);
    }
  }
};
const BucketLut& lut() {
  static const BucketLut l;
  return l;
}

void fill_best(Table& t) {
  for (int mi = 0; mi < NM; ++mi)
    for (int ni = 0; ni < NN; ++ni)
      for (int ki = 0; ki < NK; ++ki)
        for (int sk = 0; sk < 2; ++sk) {
          int b = 0;
          for (int cfg = 1; cfg < GEMM_CFGS; ++cfg) {
            if (cfg == GEMM_CFG_SKINNY && !sk) continue;
            if (t.us[cfg][mi][ni][ki] < t.us[b][mi][ni][ki]) b = cfg;
          }
          t.best[mi][ni][ki][sk] = (int8_t)b;
        }
}

void tchk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(BFMF_E_DEVICE, std::string("autotune: ") + what + ": " + hipGetErrorString(e));
}

// equal tasks of one shape: enough to fill the device with the 64 x 64 shape,
// at most 2^30 multiply-adds and 2^24 operand entries per launch
int tasks_for(int m, int n, int k) {
  const int64_t tiles = gemm_cfg_tiles(0, m, n);
  int64_t p = std::max<int64_t>(4, (2048 + tiles - 1) / tiles);
  p = std::min<int64_t>(p, std::max<int64_t>(4, ((int64_t)1 << 30) / ((int64_t)m * n * k)));
  p = std::min<int64_t>(p, std::max<int64_t>(1, ((int64_t)1 << 24) / ((int64_t)m * k + (int64_t)k * n + (int64_t)m * n)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(p, 4096));
}

template <class T>
void build_table(Table& t, hipStream_t s) {
  const size_t esz = 2 * sizeof(T);  // one complex entry
  // one buffer for the largest launch: P tasks with their own A, B and C
  int64_t max_elems = 0, max_tasks = 0, max_tiles = 0;
  for (int m : MB)
    for (int n : NB)
      for (int k : KB) {
        const int p = tasks_for(m, n, k);
        max_elems = std::max<int64_t>(max_elems, (int64_t)p * ((int64_t)m * k + (int64_t)k * n + (int64_t)m * n));
        max_tasks = std::max<int64_t>(max_tasks, p);
        for (int cfg = 0; cfg < GEMM_CFGS; ++cfg) max_tiles = std::max<int64_t>(max_tiles, p * gemm_cfg_tiles(cfg, m, n));
      }
  void* buf = nullptr;
  void* dtask = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tchk(dev_malloc((void**)&buf, (size_t)max_elems * esz), "operand buffer");
  tchk(dev_malloc((void**)&dtask, (size_t)max_tasks * (sizeof(GTask) + sizeof(int64_t)) + 64), "task buffer");
  tchk(hipMemsetAsync(buf, 0, (size_t)max_elems * esz, s), "clear");
  tchk(hipEventCreate(&e0), "event");
  tchk(hipEventCreate(&e1), "event");
  void* bases[4] = {buf, nullptr, nullptr, nullptr};
  std::vector<GTask> tasks;
  std::vector<int64_t> start;
  for (int mi = 0; mi < NM; ++mi)
    for (int ni = 0; ni < NN; ++ni)
      for (int ki = 0; ki < NK; ++ki) {
        const int m = MB[mi], n = NB[ni], k = KB[ki];
        const int p = tasks_for(m, n, k);
        tasks.assign(p, GTask());
        const int64_t stride = (int64_t)m * k + (int64_t)k * n + (int64_t)m * n;
        for (int i = 0; i < p; ++i) {
          GTask& g = tasks[i];
          std::memset(&g, 0, sizeof(g));
          g.a_off = i * stride;
          g.b_off = g.a_off + (int64_t)m * k;
          g.c_off = g.b_off + (int64_t)k * n;
          g.lda = m;
          g.ldb = k;
          g.ldc = m;
          g.M = m;
          g.N = n;
          g.K = k;
          g.opA = OP_N;
          g.opB = OP_N;
          g.abase = g.bbase = g.cbase = 0;
          g.beta = 1;
          g.alpha_re = 1.0;
        }
        tchk(hipMemcpyAsync(dtask, tasks.data(), p * sizeof(GTask), hipMemcpyHostToDevice, s), "tasks");
        int64_t* dstart = (int64_t*)((char*)dtask + p * sizeof(GTask));
        for (int cfg = 0; cfg < GEMM_CFGS; ++cfg) {
          double& out = t.us[cfg][mi][ni][ki];
          out = std::numeric_limits<double>::infinity();
          if (cfg == GEMM_CFG_SKINNY && n > GEMM_CFG_TN[GEMM_CFG_SKINNY]) continue;
          start.assign(p, 0);
          int64_t tiles = 0;
          for (int i = 0; i < p; ++i) {
            start[i] = tiles;
            tiles += gemm_cfg_tiles(cfg, m, n);
          }
          tchk(hipMemcpyAsync(dstart, start.data(), p * sizeof(int64_t), hipMemcpyHostToDevice, s), "tile starts");
          float best = std::numeric_limits<float>::infinity();
          for (int rep = 0; rep < 2; ++rep) {
            tchk(launch_grouped_gemm<T>((const GTask*)dtask, dstart, p, tiles, bases, cfg, s, e0, e1), "launch");
            tchk(hipEventSynchronize(e1), "sync");
            float ms = 0;
            tchk(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (rep > 0) best = std::min(best, ms);  // the first launch warms code and caches
          }
          out = 1e3 * best / p;
        }
        tchk(hipStreamSynchronize(s), "sync");  // the host vectors are reused
      }
  (void)max_tiles;
  tchk(hipStreamSynchronize(s), "sync");
  if (std::getenv("BFMF_VERBOSE")) {  // fastest shape and its time per task for every bucket
    for (int mi = 0; mi < NM; ++mi)
      for (int ni = 0; ni < NN; ++ni) {
        std::fprintf(stderr, "[bfmf-tune] %s M %3d N %4d:", sizeof(T) == 8 ? "c128" : "c64 ", MB[mi], NB[ni]);
        for (int ki = 0; ki < NK; ++ki) {
          int b = 0;
          for (int cfg = 1; cfg < GEMM_CFGS; ++cfg)
            if (t.us[cfg][mi][ni][ki] < t.us[b][mi][ni][ki]) b = cfg;
          std::fprintf(stderr, "  K %4d: %dx%d %7.2f us (64x64 %7.2f)", KB[ki], GEMM_CFG_TM[b], GEMM_CFG_TN[b],
                       t.us[b][mi][ni][ki], t.us[0][mi][ni][ki]);
        }
        std::fprintf(stderr, "\n");
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(dtask);
  (void)hipFree(buf);
  t.ready = true;
}

// BFMF_TILE_TABLE=path keeps the measured table in path.<bytes per complex entry>: a process finds the
// table there instead of measuring it (so that several processes, e.g. a benchmark and its profiled
// reruns, choose the same shapes); a missing or mismatched file is measured and written.
struct TableFile {
  char magic[8];
  int32_t cfgs, nm, nn, nk, esz, pad;
  double us[GEMM_CFGS][NM][NN][NK];
};

bool load_table(Table& t, const std::string& path, int esz) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  TableFile tf;
  const bool ok = std::fread(&tf, sizeof(tf), 1, f) == 1 && std::memcmp(tf.magic, "bfmftile", 8) == 0 &&
                  tf.cfgs == GEMM_CFGS && tf.nm == NM && tf.nn == NN && tf.nk == NK && tf.esz == esz;
  std::fclose(f);
  if (!ok) return false;
  std::memcpy(t.us, tf.us, sizeof(t.us));
  t.ready = true;
  return true;
}

void save_table(const Table& t, const std::string& path, int esz) {
  TableFile tf;
  std::memset(&tf, 0, sizeof(tf));
  std::memcpy(tf.magic, "bfmftile", 8);
  tf.cfgs = GEMM_CFGS;
  tf.nm = NM;
  tf.nn = NN;
  tf.nk = NK;
  tf.esz = esz;
  std::memcpy(tf.us, t.us, sizeof(t.us));
  if (FILE* f = std::fopen(path.c_str(), "wb")) {
    (void)std::fwrite(&tf, sizeof(tf), 1, f);
    std::fclose(f);
  }
}

template <class T>
const Table& table_for(int device, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  Table& t = g_tables[{device, (int)sizeof(T)}];
  if (!t.ready) {
    const char* env = std::getenv("BFMF_TILE_TABLE");
    const int esz = (int)(2 * sizeof(T));
    const std::string path = env ? std::string(env) + "." + std::to_string(esz) : std::string();
    if (path.empty() || !load_table(t, path, esz)) {
      build_table<T>(t, s);
      if (!path.empty()) save_table(t, path, esz);
    }
    fill_best(t);
  }
  return t;
}

struct Buckets {
  int mi, ni, ki;
  double scale;  // beyond the largest bucket: time in proportion
};
Buckets buckets_of(const GTask& g) {
  const BucketLut& l = lut();
  Buckets b;
  b.mi = g.M <= 1024 ? l.m[std::max(g.M, 0)] : NM - 1;
  b.ni = g.N <= 1024 ? l.n[std::max(g.N, 0)] : NN - 1;
  b.ki = g.K <= 1024 ? l.k[std::max(g.K, 0)] : NK - 1;
  b.scale = 1.0;
  if (g.M > MB[NM - 1]) b.scale *= (double)g.M / MB[NM - 1];
  if (g.N > NB[NN - 1]) b.scale *= (double)g.N / NB[NN - 1];
  if (g.K > KB[NK - 1]) b.scale *= (double)g.K / KB[NK - 1];
  return b;
}

double predict(const Table& t, int cfg, const GTask& g) {
  const Buckets b = buckets_of(g);
  return t.us[cfg][b.mi][b.ni][b.ki] * b.scale;
}

}  // namespace

void set_gemm_tile_override(int cfg) { g_override = cfg; }

template <class T>
void gemm_autotune(int device, hipStream_t s) {
  (void)table_for<T>(device, s);
}

template <class T>
int choose_gemm_cfg(int device, hipStream_t s, const std::vector<GTask>& ph) {
  bool skinny_ok = !ph.empty();
  for (const GTask& g : ph)
    skinny_ok = skinny_ok && g.N <= GEMM_CFG_TN[GEMM_CFG_SKINNY] && g.opA == OP_N && g.opB == OP_N;
  const int ov = g_override.load();
  if (ov >= 0 && ov < GEMM_CFGS) return (ov == GEMM_CFG_SKINNY && !skinny_ok) ? 0 : ov;
  const Table& t = table_for<T>(device, s);
  // at most 64 tasks, evenly spaced, enter the prediction
  const size_t stride = std::max<size_t>(1, ph.size() / 64);
  int arg = 0;
  double best = std::numeric_limits<double>::infinity();
  for (int cfg = 0; cfg < GEMM_CFGS; ++cfg) {
    if (cfg == GEMM_CFG_SKINNY && !skinny_ok) continue;
    double cost = 0;
    for (size_t i = 0; i < ph.size(); i += stride) cost += predict(t, cfg, ph[i]);
    if (cost < best) {
      best = cost;
      arg = cfg;
    }
  }
  return arg;
}

// Shapes for the tasks of one phase: either one shape for all (returned), or,
// when that pads tasks of very different heights, each task's own best shape
// (task_cfg filled, -1 returned; the caller launches one group per shape).
// Groups of fewer than kMinSplitTiles tiles stay with the phase's shape, and
// the split is taken only when the predicted time, with kLaunchUs for each
// extra launch, is at least 5% less.
template <class T>
int choose_gemm_cfg_split(int device, hipStream_t s, const std::vector<GTask>& ph, std::vector<int>& task_cfg) {
  constexpr double kLaunchUs = 6.0;
  constexpr int64_t kMinSplitTiles = 512;
  const int single = choose_gemm_cfg<T>(device, s, ph);
  if (g_override.load() >= 0 || ph.size() < 2) return single;
  const Table& t = table_for<T>(device, s);
  task_cfg.assign(ph.size(), single);
  double c_single = 0, c_split = 0;
  int64_t tiles[GEMM_CFGS] = {};
  std::vector<Buckets> bk(ph.size());
  for (size_t i = 0; i < ph.size(); ++i) {
    const GTask& g = ph[i];
    const bool sk = g.N <= GEMM_CFG_TN[GEMM_CFG_SKINNY] && g.opA == OP_N && g.opB == OP_N;
    const Buckets b = bk[i] = buckets_of(g);
    const int c = t.best[b.mi][b.ni][b.ki][sk ? 1 : 0];
    task_cfg[i] = c;
    tiles[c] += gemm_cfg_tiles(c, g.M, g.N);
    c_single += t.us[single][b.mi][b.ni][b.ki] * b.scale;
  }
  int groups = 0;
  for (size_t i = 0; i < ph.size(); ++i)
    if (tiles[task_cfg[i]] < kMinSplitTiles) task_cfg[i] = single;
  bool used[GEMM_CFGS] = {};
  for (size_t i = 0; i < ph.size(); ++i) {
    used[task_cfg[i]] = true;
    c_split += t.us[task_cfg[i]][bk[i].mi][bk[i].ni][bk[i].ki] * bk[i].scale;
  }
  for (bool u : used) groups += u ? 1 : 0;
  if (groups <= 1) return groups == 1 ? task_cfg[0] : single;
  if (c_split + kLaunchUs * (groups - 1) < 0.95 * c_single) return -1;
  return single;
}

template <class T>
void gemm_tune_table(int device, hipStream_t s, std::vector<double>& out) {
  const Table& t = table_for<T>(device, s);
  out.assign((const double*)t.us, (const double*)t.us + GEMM_CFGS * NM * NN * NK);
}

template void gemm_autotune<double>(int, hipStream_t);
template void gemm_autotune<float>(int, hipStream_t);
template int choose_gemm_cfg<double>(int, hipStream_t, const std::vector<GTask>&);
template int choose_gemm_cfg<float>(int, hipStream_t, const std::vector<GTask>&);
template int choose_gemm_cfg_split<double>(int, hipStream_t, const std::vector<GTask>&, std::vector<int>&);
template int choose_gemm_cfg_split<float>(int, hipStream_t, const std::vector<GTask>&, std::vector<int>&);
template void gemm_tune_table<double>(int, hipStream_t, std::vector<double>&);
template void gemm_tune_table<float>(int, hipStream_t, std::vector<double>&);

}  // namespace bfmf
