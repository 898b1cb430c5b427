// Host side of the C ABI: contexts, per-request device arenas, the ingest
// sequence, the iteration driver (one fused kernel launch per gradient-flow
// iteration for every active request) and the continuous-batching scheduler
// behind cvo_submit / cvo_poll.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <dlfcn.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/cvo.h"
#include "cvo_internal.h"
#include "cvo_step.h"

using namespace cvo;

namespace {

using Clock = std::chrono::steady_clock;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int round_up4(int v) { return (v + 3) / 4 * 4; }

// ---------------------------------------------------------------------------
// request description (host copy of everything the device needs)
// ---------------------------------------------------------------------------
struct Request {
  uint64_t ticket = 0;
  int mode = kModeRegister;
  int n = 0, m = 0, fd = 0, n_stages = 1, max_iters = 1, precision = 0, trace_on = 0;
  int step_rule = kStepFixed;
  int dof_mask = 0x3F;
  int chunk_min = kChunkMinDefault, chunks_max = kChunksMaxDefault;  // work-item sizing
  double xi0[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // direction of the coefficient evaluation
  double sigma = 0.1, sf = 0.2, a2 = -1.0, b2 = 1.0, eta = 1.0, kappa = 0.0, tol = 0.0, grad_tol = 0.0;
  double stage_tol = 0.0;
  int stage_iters[kMaxStages] = {0};
  double stage_ell[kMaxStages] = {0.0};
  double T0[16];
  // inputs: device pointers (borrowed or pointing into host_copy after upload)
  bool on_device = false;
  const float *sx = nullptr, *sfeat = nullptr, *tx = nullptr, *tfeat = nullptr;
  std::vector<float> hsx, hsf, htx, htf;  // host copies (submit with host inputs)
  int nclus = 0;   // target clusters (read back after ingest)
  size_t need_bytes = 0;  // exact device bytes once known (a request sent back to the queue)
  // device arenas: set-up data (A) and per-cluster iteration buffers (B)
  char* arena = nullptr;
  size_t arena_bytes = 0;
  char* arena_b = nullptr;
  size_t arena_b_bytes = 0;
  ReqStatic st{};
  ReqState* state = nullptr;
  double* trace_dev = nullptr;
  double* per_target_dev = nullptr;
  // completion
  int status = CVO_PENDING;
  cvo_result res{};
  double T_out[16];
  double coef[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // coefficient evaluation: F, A1..A4
  std::vector<double> trace;
  Clock::time_point t_submit;
};

struct Layout {
  size_t off_sx, off_sf, off_tx, off_tf;
  size_t off_xpart, off_zpart, off_xbox, off_zbox, off_T0, off_ell;
  size_t off_grid, off_ncell, off_skeys, off_tkeys, off_sperm, off_tperm;
  size_t off_count[kMaxStages + 1], off_radix[kMaxStages + 1], off_hist[kMaxStages + 1], off_sums[kMaxStages + 1];
  size_t off_segs, off_scans, off_clscan_args, off_zrec, off_zorig, off_xrec[kMaxStages], off_xrecptr;
  size_t off_clflag, off_clscan, off_clfirst, off_clsums, off_clstart, off_clcount;
  size_t cl_sums_stride;  // ints per stage in the clustering scan's tile sums
  size_t off_state;
  size_t total;
  int kcap, zs, xs, nblk_bbox;
};

// per-cluster iteration buffers, sized once the cluster count is known
struct LayoutB {
  size_t off_cinfo, off_cells, off_centry, off_tblk, off_sslots, off_csum, off_trace, off_pt;
  size_t total;
};

constexpr int kBboxBlocks = 256;
constexpr int kMaxPoints = 16000000;  // bounded by the single-level tile scan

int scan_tiles(long long len) { return (int)((len + kScanTile - 1) / kScanTile); }

Layout plan(const Request& q) {
  Layout L{};
  const int S = q.n_stages;
  L.kcap = std::min(std::max(1 << 16, 8 * q.n), (1 << 24) - 16);
  L.zs = round_up4(3 + q.fd);
  L.xs = round_up4(3 + q.fd);
  L.nblk_bbox = kBboxBlocks;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return r;
  };
  const size_t n = (size_t)q.n, m = (size_t)q.m, fd = (size_t)q.fd;
  if (!q.on_device) {
    L.off_sx = take(n * 3 * 4);
    L.off_sf = take(n * fd * 4);
    L.off_tx = take(m * 3 * 4);
    L.off_tf = take(m * fd * 4);
  }
  L.off_xpart = take(kBboxBlocks * 7 * 8);
  L.off_zpart = take(kBboxBlocks * 7 * 8);
  L.off_xbox = take(8 * 8);
  L.off_zbox = take(8 * 8);
  L.off_T0 = take(24 * 8);  // T0[16], then the direction xi0[6]
  L.off_ell = take(kMaxStages * 8);
  L.off_grid = take(sizeof(GridInfo) * kMaxStages);
  L.off_ncell = take(4 * (kMaxStages + 1));
  L.off_skeys = take(4 * n * S);
  L.off_tkeys = take(4 * m);
  L.off_sperm = take(4 * n * S);
  L.off_tperm = take(4 * m);
  for (int s = 0; s <= S; s++) {
    const size_t kc = (s < S) ? (size_t)L.kcap : (size_t)kZBuckets;
    const size_t nn = (s < S) ? n : m;
    const size_t hist = (size_t)kRadixBins * ((nn + kRadixTile - 1) / kRadixTile);
    L.off_count[s] = take(4 * (kc + 1));
    L.off_radix[s] = take(4 * 4 * nn);  // keys and indices, two of each
    L.off_hist[s] = take(4 * hist);
    L.off_sums[s] = take(4 * (size_t)(scan_tiles((long long)hist) + 1));
  }
  L.off_segs = take(sizeof(SortSeg) * (S + 1));
  L.off_scans = take(sizeof(ScanArgs) * (S + 1));
  L.off_clscan_args = take(sizeof(ScanArgs) * S);
  L.off_zrec = take(m * L.zs * 4);
  L.off_zorig = take(m * 4);
  const size_t xb = (q.precision == CVO_FP64) ? 8 : 4;
  for (int s = 0; s < S; s++) L.off_xrec[s] = take(n * L.xs * xb);
  L.off_xrecptr = take(sizeof(void*) * kMaxStages);
  L.cl_sums_stride = (size_t)(scan_tiles((long long)m) + 1);
  L.off_clflag = take(4 * m * S);
  L.off_clscan = take(4 * m * S);
  L.off_clfirst = take(4 * m * S);
  L.off_clsums = take(4 * L.cl_sums_stride * S);
  L.off_clstart = take(4 * m * S);
  L.off_clcount = take(4 * m * S);
  L.off_state = take(sizeof(ReqState));
  L.total = o;
  return L;
}

LayoutB plan_b(const Request& q, int nclus) {
  LayoutB L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return r;
  };
  const size_t nc = (size_t)nclus;
  L.off_cinfo = take(sizeof(ClusInfo) * nc);
  L.off_cells = take(sizeof(CellEntry) * nc * kCellCap);
  L.off_centry = take(sizeof(int) * nc * (size_t)q.chunks_max);
  L.off_tblk = take((q.precision == CVO_FP64 ? 8 : 4) * nc * (3 + (size_t)q.fd) * kWave);
  L.off_sslots = take(8 * nc * (size_t)q.chunks_max * kSlot);
  L.off_csum = take(8 * nc * kSlot);
  L.off_trace = q.trace_on ? take((size_t)q.max_iters * kTraceCols * 8) : 0;
  L.off_pt = (q.mode == kModeEvalTargets) ? take((size_t)q.m * 7 * 8) : 0;
  L.total = o;
  return L;
}

// Device memory of a request for admission.  Arena A is exact; arena B
// depends on the number of target clusters, known only after the ingest, and
// is estimated from ~2 clusters per 64 targets (spatially coherent clouds).
// Once the ingest has run, the scheduler charges the exact size (need_bytes)
// and sends a request whose exact size does not fit back to the queue.
size_t footprint(const Request& q) {
  if (q.need_bytes) return q.need_bytes;
  const Layout L = plan(q);
  const int nclus_est = (q.m + kWave - 1) / kWave * 2 + 64;
  return L.total + plan_b(q, std::min(nclus_est, q.m)).total;
}

}  // namespace

// ---------------------------------------------------------------------------
// work queue of the iteration launches on one stream
// ---------------------------------------------------------------------------
struct DevQueue {
  WorkQueue* q = nullptr;
  unsigned int* items = nullptr;
  unsigned int cap = 0;
  QueueRef ref() const { return QueueRef{q, items, cap}; }
  // capacity for a launch of max_items work items (the sum over its
  // requests of clusters x chunks_max); false if out of memory
  bool ensure(unsigned long long max_items) {
    if (!q && hipMalloc(&q, sizeof(WorkQueue)) != hipSuccess) {
      q = nullptr;
      return false;
    }
    const unsigned long long need = std::max(max_items, 1ull);
    if (need > 0xffffffffull) return false;
    if (need <= cap) return true;
    const unsigned long long want = std::min<unsigned long long>(std::max<unsigned long long>(need, 2ull * cap), 0xffffffffull);
    if (items) (void)hipFree(items);
    items = nullptr;
    cap = 0;
    if (hipMalloc(&items, want * sizeof(unsigned int)) != hipSuccess) {
      items = nullptr;
      return false;
    }
    cap = (unsigned int)want;
    return true;
  }
  // both counters to zero (before the first launch of a run on this stream)
  hipError_t reset(hipStream_t s) const { return hipMemsetAsync(q, 0, sizeof(WorkQueue), s); }
  void release() {
    if (q) (void)hipFree(q);
    if (items) (void)hipFree(items);
    q = nullptr;
    items = nullptr;
    cap = 0;
  }
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct cvo_ctx {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;  // eval/register stream (user-selectable)
  std::mutex call_mu;            // serialises eval/register
  std::string last_error;
  uint64_t budget = 0;
  int max_slots = 256;

  // pinned host staging
  void* pinned = nullptr;
  size_t pinned_bytes = 0;

  // cached arena for the synchronous path
  char* sync_arena = nullptr;
  size_t sync_arena_bytes = 0;
  char* sync_arena_b = nullptr;
  size_t sync_arena_b_bytes = 0;
  ReqStatic* d_reqs_sync = nullptr;
  int* d_clus_end_sync = nullptr;
  DevQueue queue_sync;
  char* fe_arena = nullptr;  // front-end buffers
  size_t fe_arena_bytes = 0;
  Request last_register;
  bool have_last = false;

  // iteration chunks replayed as HIP graphs (synchronous path and the
  // batched scheduler; read by the scheduler thread)
  std::atomic<bool> graphs{false};
  struct GraphKey {
    int nclus = -1, precision = -1, fd = -1, cut = -1, rule = -1, iters = -1;
    const void* items = nullptr;
    unsigned int cap = 0;
    hipStream_t stream = nullptr;
    bool operator==(const GraphKey& o) const {
      return nclus == o.nclus && precision == o.precision && fd == o.fd && cut == o.cut && rule == o.rule &&
             iters == o.iters && items == o.items && cap == o.cap && stream == o.stream;
    }
  };
  GraphKey graph_key;
  hipGraphExec_t graph_exec = nullptr;
  int64_t graph_captures = 0, graph_launches = 0;

  // profiling
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launches = 0;
  double prof_ms = 0.0;          // pair kernel
  double prof_prep_ms = 0.0;     // prepare kernel
  double prof_quart_ms = 0.0;    // pair kernel, quartic pass
  uint64_t prof_pairs = 0;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;

  // work-item sizing per size class (tuning table, loaded by cvo_create)
  struct TuneClass {
    int cutoff;      // 1: requests with a cutoff, 0: brute force
    int max_points;  // the class holds requests with max(n, m) <= max_points
    int chunk_min, chunks_max;
  };
  std::vector<TuneClass> tuning;
  std::string tuning_path;

  // serving
  std::mutex q_mu;
  std::condition_variable q_cv;     // scheduler wake-up
  std::condition_variable done_cv;  // pollers
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread sched;
  bool sched_started = false;
  hipStream_t serve_stream = nullptr;
  // stream-ordered device memory of served requests (a pool that keeps what
  // it has allocated, so admission and release do not synchronise the
  // device); null: plain hipMalloc / hipFree
  hipMemPool_t pool = nullptr;
  size_t max_pending = 65536;
  // serving counters (under q_mu)
  int64_t st_active = 0, st_completed = 0, st_failed = 0;
  int64_t st_graph_chunks = 0;  // scheduler chunks replayed from a captured graph
  uint64_t st_hbm_in_use = 0, st_hbm_peak = 0;
  // traces of polled batched tickets, newest last (cvo_trace after cvo_poll)
  std::unordered_map<uint64_t, std::vector<double>> kept_traces;
  std::deque<uint64_t> kept_order;
};

static int fail(cvo_ctx* c, hipError_t e, const char* what) {
  if (c) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    c->last_error = buf;
  }
  return CVO_EDEVICE;
}

#define HIPCHK(ctx, expr)                              \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return fail(ctx, e_, #expr); \
  } while (0)

// ---------------------------------------------------------------------------
// the allocation-free evaluation's device array: its address per device
// (looked up once, by cvo_create with that device current), and a lock per
// device that serialises the calls sharing it
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
constexpr int kStaticMaxPoints = 65536;  // points per cloud of cvo_eval_static
static std::mutex g_static_mu;
static void* g_static_ptr[kMaxDevices] = {};
static std::mutex g_static_call_mu[kMaxDevices];
static char g_static_host[kMaxDevices][64 * 1024];  // host staging of the set-up structures

static hipError_t init_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_static_mu);
  if (g_static_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = static_scratch_address(&p);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_static_ptr[device] = p;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// tuning table: {"classes": [{"cutoff": 0|1, "max_points": N, "work_item_min": N,
// "work_items_max": N}, ...], ...}.  Only the integer fields of the objects of
// the "classes" array are read; other fields are ignored.
// ---------------------------------------------------------------------------
static bool parse_tuning(const std::string& text, std::vector<cvo_ctx::TuneClass>& out) {
  const size_t arr = text.find("\"classes\"");
  if (arr == std::string::npos) return false;
  size_t p = text.find('[', arr);
  if (p == std::string::npos) return false;
  out.clear();
  // walk the array: each object at depth 1 is a class (nested objects and
  // quoted strings are skipped over)
  int depth = 0;
  size_t ob = std::string::npos;
  for (size_t k = p + 1; k < text.size(); k++) {
    const char ch = text[k];
    if (ch == '"') {
      for (k++; k < text.size() && text[k] != '"'; k++)
        if (text[k] == '\\') k++;
      continue;
    }
    if (ch == '{' && depth++ == 0) ob = k;
    if (ch == '}' && --depth == 0) {
      const std::string obj = text.substr(ob, k - ob + 1);
      auto field = [&](const char* key, long long* v) {
        const std::string kq = std::string("\"") + key + "\"";
        const size_t at = obj.find(kq);
        if (at == std::string::npos) return false;
        const size_t colon = obj.find(':', at + kq.size());
        if (colon == std::string::npos) return false;
        char* e = nullptr;
        const long long x = strtoll(obj.c_str() + colon + 1, &e, 10);
        if (e == obj.c_str() + colon + 1) return false;
        *v = x;
        return true;
      };
      long long cut, mp, cmin, cmax;
      if (!field("cutoff", &cut) || !field("max_points", &mp) || !field("work_item_min", &cmin) ||
          !field("work_items_max", &cmax))
        return false;
      if (cmin < kChunkMinLo || cmin > (1 << 20) || cmax < 1 || cmax > kChunksCap || mp < 1) return false;
      out.push_back(cvo_ctx::TuneClass{cut ? 1 : 0, (int)std::min<long long>(mp, INT32_MAX), (int)cmin, (int)cmax});
    }
    if (depth < 0 || (ch == ']' && depth == 0)) break;
  }
  return !out.empty() && depth == 0;
}

// The table next to the library (<package>/tuning.json, one level above
// lib/libcvo.so), or the file named by CVO_TUNING_FILE; none: the defaults.
static void load_tuning(cvo_ctx* c) {
  std::string path;
  if (const char* env = getenv("CVO_TUNING_FILE")) {
    path = env;
  } else {
    Dl_info info;
    if (dladdr((const void*)&load_tuning, &info) && info.dli_fname) {
      std::string lib = info.dli_fname;
      const size_t s1 = lib.rfind('/');
      const std::string dir = s1 == std::string::npos ? std::string(".") : lib.substr(0, s1);
      path = dir + "/../tuning.json";
    }
  }
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 20)) text.append(buf, got);
  fclose(f);
  std::vector<cvo_ctx::TuneClass> t;
  if (parse_tuning(text, t)) {
    c->tuning = t;
    c->tuning_path = path;
  }
}

// Work-item sizing of a request: the parameters' explicit values, else the
// first table class of the request's kind (cutoff or not) that holds
// max(n, m) points, else the defaults.  It depends only on the request
// itself, so a request runs the same work items alone and in a batch.
static void tune_request(const cvo_ctx* c, const cvo_params* p, Request& q) {
  int cmin = kChunkMinDefault, cmax = kChunksMaxDefault;
  const int pts = std::max(q.n, q.m);
  const int cut = q.kappa > 0.0 ? 1 : 0;
  for (const auto& t : c->tuning) {
    if (t.cutoff == cut && pts <= t.max_points) {
      cmin = t.chunk_min;
      cmax = t.chunks_max;
      break;
    }
  }
  if (p->work_item_min > 0) cmin = p->work_item_min;
  if (p->work_items_max > 0) cmax = p->work_items_max;
  q.chunk_min = cmin;
  q.chunks_max = cmax;
}

// ---------------------------------------------------------------------------
// validation and request construction
// ---------------------------------------------------------------------------
static bool finite_host(const float* p, size_t cnt) {
  for (size_t i = 0; i < cnt; i++)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static int build_request(const cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p,
                         const double* T0, int mode, Request& q) {
  if (!src || !tgt || !p || !T0) return CVO_EINVAL;
  if (src->n <= 0 || tgt->n <= 0) return CVO_EINVAL;
  if (src->n > kMaxPoints || tgt->n > kMaxPoints) return CVO_EINVAL;
  if (src->feat_dim < 1 || src->feat_dim > kMaxFeat || src->feat_dim != tgt->feat_dim) return CVO_EINVAL;
  if (!src->xyz || !src->feat || !tgt->xyz || !tgt->feat) return CVO_EINVAL;
  if (src->on_device != tgt->on_device) return CVO_EINVAL;
  if (!(p->sigma > 0.0) || !(p->feat_scale > 0.0) || !(p->b2 > 0.0) || !(p->eta > 0.0)) return CVO_EINVAL;
  if (!(p->cutoff_mult >= 0.0) || !std::isfinite(p->cutoff_mult) || !std::isfinite(p->a2)) return CVO_EINVAL;
  if (p->n_stages < 1 || p->n_stages > kMaxStages || !p->stage_ell) return CVO_EINVAL;
  if (p->n_stages > 1 && !p->stage_iters) return CVO_EINVAL;
  if (p->max_iters < 1 || !(p->tol >= 0.0)) return CVO_EINVAL;
  if (p->precision != CVO_FP32_KAHAN && p->precision != CVO_FP64) return CVO_EINVAL;
  if (p->step_rule != CVO_STEP_FIXED && p->step_rule != CVO_STEP_QUARTIC && p->step_rule != CVO_STEP_CONJUGATE)
    return CVO_EINVAL;
  if (!(p->grad_tol >= 0.0) || !(p->kernel_floor >= 0.0) || !std::isfinite(p->kernel_floor)) return CVO_EINVAL;
  if (p->dof_mask < 0 || p->dof_mask > 0x3F) return CVO_EINVAL;
  if (p->work_item_min < 0 || (p->work_item_min > 0 && (p->work_item_min < kChunkMinLo || p->work_item_min > (1 << 20))))
    return CVO_EINVAL;
  if (p->work_items_max < 0 || p->work_items_max > kChunksCap) return CVO_EINVAL;
  if (!(p->stage_tol >= 0.0) || !std::isfinite(p->stage_tol)) return CVO_EINVAL;
  // value sparsification (Table 1): sigma^2 exp(-r^2 / (2 ell^2)) >= floor
  // keeps exactly r <= ell sqrt(2 ln(sigma^2 / floor))
  if (p->kernel_floor > 0.0 && (p->cutoff_mult > 0.0 || !(p->sigma * p->sigma > p->kernel_floor)))
    return CVO_EINVAL;
  for (int s = 0; s < p->n_stages; s++) {
    if (!(p->stage_ell[s] > 0.0) || !std::isfinite(p->stage_ell[s])) return CVO_EINVAL;
    if (s < p->n_stages - 1 && p->stage_iters[s] < 1) return CVO_EINVAL;
  }
  for (int k = 0; k < 16; k++)
    if (!std::isfinite(T0[k])) return CVO_EINVAL;
  q.mode = mode;
  q.n = src->n;
  q.m = tgt->n;
  q.fd = src->feat_dim;
  q.n_stages = (mode == kModeRegister) ? p->n_stages : 1;
  q.max_iters = (mode == kModeRegister) ? p->max_iters : 1;
  q.precision = p->precision;
  q.trace_on = (mode == kModeRegister) ? (p->trace ? 1 : 0) : 0;
  q.step_rule = (mode == kModeRegister) ? p->step_rule : (mode == kModeQuartic ? kStepQuartic : kStepFixed);
  q.dof_mask = p->dof_mask == 0 ? 0x3F : p->dof_mask;
  q.sigma = p->sigma;
  q.sf = p->feat_scale;
  q.a2 = p->a2;
  q.b2 = p->b2;
  q.eta = p->eta;
  q.kappa = p->kernel_floor > 0.0 ? std::sqrt(2.0 * std::log(p->sigma * p->sigma / p->kernel_floor))
                                   : p->cutoff_mult;
  q.tol = p->tol;
  q.grad_tol = p->grad_tol;
  q.stage_tol = (mode == kModeRegister) ? p->stage_tol : 0.0;
  for (int s = 0; s < q.n_stages; s++) {
    q.stage_ell[s] = p->stage_ell[s];
    q.stage_iters[s] = (s < q.n_stages - 1) ? p->stage_iters[s] : INT_MAX;
  }
  memcpy(q.T0, T0, sizeof(q.T0));
  q.on_device = src->on_device != 0;
  if (!q.on_device) {
    if (!finite_host(src->xyz, 3ull * q.n) || !finite_host(src->feat, (size_t)q.fd * q.n) ||
        !finite_host(tgt->xyz, 3ull * q.m) || !finite_host(tgt->feat, (size_t)q.fd * q.m))
      return CVO_EINVAL;
  }
  q.sx = src->xyz;
  q.sfeat = src->feat;
  q.tx = tgt->xyz;
  q.tfeat = tgt->feat;
  tune_request(c, p, q);
  return CVO_OK;
}

// Enqueue the set-up sequence of one request into its arena A.  The host
// structures are staged through pinned memory (valid until the stream syncs).
static int enqueue_ingest(cvo_ctx* c, Request& q, const Layout& L, hipStream_t s, void* pinned_scratch) {
  char* A = q.arena;
  struct Staging {
    double T0[24];
    double ell[kMaxStages];
    SortSeg segs[kMaxStages + 1];
    ScanArgs scans[kMaxStages + 1];
    ScanArgs clscan[kMaxStages];
    void* xrecptr[kMaxStages];
  };
  static_assert(sizeof(Staging) < 16384, "staging area");
  Staging* h = (Staging*)pinned_scratch;
  memset(h->T0, 0, sizeof(h->T0));
  memcpy(h->T0, q.T0, sizeof(q.T0));
  memcpy(h->T0 + 16, q.xi0, sizeof(q.xi0));
  for (int k = 0; k < kMaxStages; k++) h->ell[k] = (k < q.n_stages) ? q.stage_ell[k] : 1.0;
  const int S = q.n_stages;
  int* ncell = (int*)(A + L.off_ncell);
  for (int sidx = 0; sidx <= S; sidx++) {
    SortSeg& g = h->segs[sidx];
    const bool tgt = sidx == S;
    g.keys = tgt ? (const int*)(A + L.off_tkeys) : (const int*)(A + L.off_skeys) + (size_t)sidx * q.n;
    g.nkeys = ncell + sidx;
    g.count = (int*)(A + L.off_count[sidx]);
    const size_t nn = (size_t)(tgt ? q.m : q.n);
    int* rx = (int*)(A + L.off_radix[sidx]);
    g.key_a = rx;
    g.idx_a = rx + nn;
    g.key_b = rx + 2 * nn;
    g.idx_b = rx + 3 * nn;
    g.hist = (int*)(A + L.off_hist[sidx]);
    g.perm = tgt ? (int*)(A + L.off_tperm) : (int*)(A + L.off_sperm) + (size_t)sidx * q.n;
    g.sums = (int*)(A + L.off_sums[sidx]);
    g.n = tgt ? q.m : q.n;
    g.kcap = tgt ? kZBuckets : L.kcap;
    g.nblocks = (int)((nn + kRadixTile - 1) / kRadixTile);
    ScanArgs& sa = h->scans[sidx];  // over the digit counts of a radix pass
    sa.data = g.hist;
    sa.lenp = nullptr;
    sa.len0 = kRadixBins * g.nblocks;
    sa.sums = g.sums;
  }
  for (int st = 0; st < S; st++) {
    h->clscan[st].data = (int*)(A + L.off_clscan) + (size_t)st * q.m;
    h->clscan[st].lenp = nullptr;
    h->clscan[st].len0 = q.m;
    h->clscan[st].sums = (int*)(A + L.off_clsums) + (size_t)st * L.cl_sums_stride;
  }
  for (int k = 0; k < kMaxStages; k++) h->xrecptr[k] = (k < S) ? (void*)(A + L.off_xrec[k]) : nullptr;

  HIPCHK(c, hipMemcpyAsync(A + L.off_T0, h->T0, sizeof(h->T0), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(A + L.off_ell, h->ell, sizeof(h->ell), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(A + L.off_segs, h->segs, sizeof(SortSeg) * (S + 1), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(A + L.off_scans, h->scans, sizeof(ScanArgs) * (S + 1), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(A + L.off_clscan_args, h->clscan, sizeof(ScanArgs) * S, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(A + L.off_xrecptr, h->xrecptr, sizeof(h->xrecptr), hipMemcpyHostToDevice, s));

  const float *sx = q.sx, *sf = q.sfeat, *tx = q.tx, *tf = q.tfeat;
  if (!q.on_device) {
    HIPCHK(c, hipMemcpyAsync(A + L.off_sx, q.sx, 12ull * q.n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(A + L.off_sf, q.sfeat, 4ull * q.fd * q.n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(A + L.off_tx, q.tx, 12ull * q.m, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(A + L.off_tf, q.tfeat, 4ull * q.fd * q.m, hipMemcpyHostToDevice, s));
    sx = (const float*)(A + L.off_sx);
    sf = (const float*)(A + L.off_sf);
    tx = (const float*)(A + L.off_tx);
    tf = (const float*)(A + L.off_tf);
  }
  IngestArgs a{};
  a.sx = sx;
  a.sfeat = sf;
  a.tx = tx;
  a.tfeat = tf;
  a.n = q.n;
  a.m = q.m;
  a.fd = q.fd;
  a.zs = L.zs;
  a.xs = L.xs;
  a.n_stages = S;
  a.precision = q.precision;
  a.kappa = q.kappa;
  a.cells_per_reach = 2;
  a.brute_div = 4;
  a.kcap = L.kcap;
  a.a2_param = q.a2;
  a.T0 = (const double*)(A + L.off_T0);
  a.xi0 = (q.mode == kModeQuartic) ? (const double*)(A + L.off_T0) + 16 : nullptr;
  a.stage_ell = (const double*)(A + L.off_ell);
  a.xpart = (double*)(A + L.off_xpart);
  a.zpart = (double*)(A + L.off_zpart);
  a.xbox = (double*)(A + L.off_xbox);
  a.zbox = (double*)(A + L.off_zbox);
  a.grid = (GridInfo*)(A + L.off_grid);
  a.ncell = ncell;
  a.src_keys = (int*)(A + L.off_skeys);
  a.tgt_keys = (int*)(A + L.off_tkeys);
  a.src_perm = (int*)(A + L.off_sperm);
  a.tgt_perm = (int*)(A + L.off_tperm);
  a.segs = (SortSeg*)(A + L.off_segs);
  a.sort_scans = (ScanArgs*)(A + L.off_scans);
  a.cl_scan_args = (ScanArgs*)(A + L.off_clscan_args);
  a.max_seg_n = std::max(q.n, q.m);
  a.max_kcap = std::max(L.kcap, kZBuckets);
  a.zrec = (float*)(A + L.off_zrec);
  a.zorig = (int*)(A + L.off_zorig);
  a.xrec_dev = (void* const*)(A + L.off_xrecptr);
  a.cl_flag = (int*)(A + L.off_clflag);
  a.cl_scan = (int*)(A + L.off_clscan);
  a.cl_first = (int*)(A + L.off_clfirst);
  a.cl_sums = (int*)(A + L.off_clsums);
  a.clus_start = (int*)(A + L.off_clstart);
  a.clus_count = (int*)(A + L.off_clcount);
  a.state = (ReqState*)(A + L.off_state);
  a.nblk_bbox = L.nblk_bbox;
  HIPCHK(c, launch_ingest(a, s));
  q.state = a.state;
  return CVO_OK;
}

// Fill q.st once the cluster count is known and arena B is allocated.
static int finish_setup(cvo_ctx* c, Request& q, const Layout& L, const LayoutB& LB, hipStream_t s) {
  (void)c;
  (void)s;
  char* A = q.arena;
  char* Bp = q.arena_b;
  ReqStatic& st = q.st;
  memset(&st, 0, sizeof(st));
  const int S = q.n_stages;
  st.state = (ReqState*)(A + L.off_state);
  st.zrec = (const float*)(A + L.off_zrec);
  st.zorig = (const int*)(A + L.off_zorig);
  for (int s = 0; s < kMaxStages; s++) {
    const int ss = s < q.n_stages ? s : 0;
    st.clus_start[s] = (const int*)(A + L.off_clstart) + (size_t)ss * q.m;
    st.clus_count[s] = (const int*)(A + L.off_clcount) + (size_t)ss * q.m;
  }
  for (int k = 0; k < S; k++) {
    st.xrec[k] = A + L.off_xrec[k];
    st.cstart[k] = (const int*)(A + L.off_count[k]);
  }
  st.grid = (const GridInfo*)(A + L.off_grid);
  st.cinfo = (ClusInfo*)(Bp + LB.off_cinfo);
  st.cells = (CellEntry*)(Bp + LB.off_cells);
  st.centry = (int*)(Bp + LB.off_centry);
  st.tblk = (void*)(Bp + LB.off_tblk);
  st.sslots = (double*)(Bp + LB.off_sslots);
  st.csum = (double*)(Bp + LB.off_csum);
  st.trace = q.trace_on ? (double*)(Bp + LB.off_trace) : nullptr;
  st.per_target = (q.mode == kModeEvalTargets) ? (double*)(Bp + LB.off_pt) : nullptr;
  st.m = q.m;
  st.n = q.n;
  st.fd = q.fd;
  st.zs = L.zs;
  st.xs = L.xs;
  st.nclus = q.nclus;
  st.n_stages = S;
  st.max_iters = q.max_iters;
  st.mode = q.mode;
  st.precision = q.precision;
  st.step_rule = q.step_rule;
  st.dof_mask = q.dof_mask;
  st.chunk_min = q.chunk_min;
  st.chunks_max = q.chunks_max;
  for (int k = 0; k < kMaxStages; k++) {
    st.stage_len[k] = (k < S - 1) ? q.stage_iters[k] : INT_MAX;
    st.stage_ell[k] = (k < S) ? q.stage_ell[k] : 1.0;
  }
  st.s2f = q.sigma * q.sigma * q.sf;
  st.b2 = q.b2;
  st.eta = q.eta;
  st.tol = q.tol;
  st.grad_tol = q.grad_tol;
  st.stage_tol = q.stage_tol;
  q.trace_dev = st.trace;
  q.per_target_dev = st.per_target;
  return CVO_OK;
}

static int ensure_pinned(cvo_ctx* c, size_t bytes) {
  if (c->pinned_bytes >= bytes) return CVO_OK;
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  size_t b = std::max(bytes, (size_t)1 << 20);
  HIPCHK(c, hipHostMalloc(&c->pinned, b, hipHostMallocDefault));
  c->pinned_bytes = b;
  return CVO_OK;
}

// Results of a finished request.  Does not publish the status: on the batched
// path a poller may delete the request as soon as it sees a terminal status,
// so only complete() sets it, under the queue lock, after every other field.
static void fill_result(Request& q, const ReqState& hs) {
  q.res.status = hs.status;
  q.res.iters = hs.iter;
  q.res.converged = hs.converged;
  q.res.F = hs.g[0];
  for (int a = 0; a < 3; a++) {
    q.res.omega[a] = hs.g[1 + a];
    q.res.v[a] = hs.g[4 + a];
  }
  for (int i = 0; i < 5; i++) q.coef[i] = hs.A[i];
  q.res.pairs_within = hs.pairs_within;
  q.res.pairs_examined = hs.pairs_examined;
  for (int k = 0; k < 12; k++) q.T_out[k] = hs.T[k];
  q.T_out[12] = q.T_out[13] = q.T_out[14] = 0.0;
  q.T_out[15] = 1.0;
}

static int grow(cvo_ctx* c, char** buf, size_t* have, size_t need, hipStream_t s) {
  if (*have >= need) return CVO_OK;
  HIPCHK(c, hipStreamSynchronize(s));
  if (*buf) HIPCHK(c, hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  const size_t want = align_up(need + (need >> 3), 1 << 20);
  if (hipMalloc(buf, want) != hipSuccess) {
    *buf = nullptr;
    return CVO_ENOMEM;
  }
  *have = want;
  return CVO_OK;
}

// The executable graph of `iters` consecutive iterations of the synchronous
// request (its launches captured from the stream once, replayed per chunk):
// the kernels read the request's state on the device, so one graph serves
// every chunk, and an exited request's kernels return at once.  Captured
// again when the launch layout changes.
static int chunk_graph(cvo_ctx* c, const Request& q, const QueueRef& QR, bool cut, int iters, hipStream_t s,
                       hipGraphExec_t* out) {
  cvo_ctx::GraphKey key;
  key.nclus = q.nclus;
  key.precision = q.precision;
  key.fd = q.fd;
  key.cut = cut ? 1 : 0;
  key.rule = q.step_rule;
  key.iters = iters;
  key.items = QR.items;
  key.cap = QR.cap;
  key.stream = s;
  if (c->graph_exec && c->graph_key == key) {
    *out = c->graph_exec;
    return CVO_OK;
  }
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  c->graph_exec = nullptr;
  HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters && e == hipSuccess; i++)
    e = launch_iteration_rule(q.step_rule, q.precision, q.fd, cut, c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR,
                              s);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, e != hipSuccess ? e : e2, "iteration graph capture");
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(c, e, "hipGraphInstantiate");
  c->graph_exec = ex;
  c->graph_key = key;
  c->graph_captures++;
  *out = ex;
  return CVO_OK;
}

// Synchronous single-request run (eval, eval-targets, register).
static int run_sync(cvo_ctx* c, Request& q, std::vector<double>* per_target_out) {
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const auto t0 = Clock::now();
  const Layout L = plan(q);
  if (c->budget && footprint(q) > c->budget) return CVO_ENOMEM;
  int rc = grow(c, &c->sync_arena, &c->sync_arena_bytes, L.total, s);
  if (rc) return rc;
  if (!c->d_reqs_sync) HIPCHK(c, hipMalloc(&c->d_reqs_sync, sizeof(ReqStatic)));
  if (!c->d_clus_end_sync) HIPCHK(c, hipMalloc(&c->d_clus_end_sync, sizeof(int)));
  q.arena = c->sync_arena;
  q.arena_bytes = L.total;
  rc = ensure_pinned(c, 64 * 1024);
  if (rc) return rc;
  char* pin = (char*)c->pinned;
  if (!c->ev_a) {
    HIPCHK(c, hipEventCreate(&c->ev_a));
    HIPCHK(c, hipEventCreate(&c->ev_b));
  }
  HIPCHK(c, hipEventRecord(c->ev_a, s));
  rc = enqueue_ingest(c, q, L, s, pin);
  if (rc) return rc;
  // the cluster count sizes the iteration buffers
  ReqState* hs = (ReqState*)(pin + 32768);
  HIPCHK(c, hipMemcpyAsync(hs, q.state, sizeof(ReqState), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  q.nclus = hs->nclus;
  if (hs->done) {  // invalid input detected on the device
    fill_result(q, *hs);
    q.status = hs->status;
    q.res.wall_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    return CVO_OK;
  }
  const LayoutB LB = plan_b(q, q.nclus);
  rc = grow(c, &c->sync_arena_b, &c->sync_arena_b_bytes, LB.total, s);
  if (rc) return rc;
  q.arena_b = c->sync_arena_b;
  q.arena_b_bytes = LB.total;
  rc = finish_setup(c, q, L, LB, s);
  if (rc) return rc;
  ReqStatic* hst = (ReqStatic*)(pin + 16384);
  int* hend = (int*)(pin + 16384 + sizeof(ReqStatic) + 64);
  *hst = q.st;
  *hend = q.nclus;
  HIPCHK(c, hipMemcpyAsync(c->d_reqs_sync, hst, sizeof(ReqStatic), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_clus_end_sync, hend, sizeof(int), hipMemcpyHostToDevice, s));

  if (!c->queue_sync.ensure((unsigned long long)q.nclus * q.chunks_max)) return CVO_ENOMEM;
  HIPCHK(c, c->queue_sync.reset(s));
  const QueueRef QR = c->queue_sync.ref();
  const bool cut = q.kappa > 0.0;
  const bool prof = c->profile && q.mode == kModeRegister;
  constexpr int kEv = 5;  // events per timed iteration
  if (prof && (int)c->ev_pool.size() < kEv * q.max_iters) {
    while ((int)c->ev_pool.size() < kEv * q.max_iters) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
  }
  int launched = 0;
  const int chunk = (q.tol > 0.0 || q.grad_tol > 0.0 || q.stage_tol > 0.0) ? 16 : q.max_iters;
  // roctx ranges (visible with rocprofv3 --marker-trace): the iteration
  // chunks of a synchronous call
  struct RangeGuard {
    ~RangeGuard() { roctxRangePop(); }
  };
  roctxRangePushA(q.mode == kModeRegister ? "cvo_register" : "cvo_eval");
  RangeGuard range_guard;
  // graph replay needs a capturable stream (not the legacy null stream)
  const bool use_graph = c->graphs && !prof && q.mode == kModeRegister && s != nullptr;
  for (int k = 0; k < q.max_iters;) {
    const int kend = std::min(q.max_iters, k + chunk);
    if (use_graph && kend - k == chunk) {
      hipGraphExec_t ex = nullptr;
      const int grc = chunk_graph(c, q, QR, cut, chunk, s, &ex);
      if (grc) return grc;
      HIPCHK(c, hipGraphLaunch(ex, s));
      c->graph_launches++;
      launched += chunk;
      k = kend;
    }
    for (; k < kend; k++) {
      if (prof) {
        hipEvent_t* ev = &c->ev_pool[kEv * k];
        HIPCHK(c, hipEventRecord(ev[0], s));
        HIPCHK(c, launch_prepare(c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR, s));
        HIPCHK(c, hipEventRecord(ev[1], s));
        HIPCHK(c, launch_pair_kernel(q.precision, q.fd, cut, c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR, s));
        HIPCHK(c, hipEventRecord(ev[2], s));
        if (q.step_rule != kStepFixed) {
          HIPCHK(c, launch_step(c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR, s, kPhaseGradient, false));
          HIPCHK(c, hipEventRecord(ev[3], s));
          HIPCHK(c, launch_quartic_pairs(q.precision, q.fd, cut, c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR,
                                         s));
          HIPCHK(c, hipEventRecord(ev[4], s));
          HIPCHK(c, launch_step(c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR, s, kPhaseQuartic, true));
        } else {
          HIPCHK(c, launch_step(c->d_reqs_sync, c->d_clus_end_sync, 1, q.nclus, QR, s));
        }
      } else {
        HIPCHK(c, launch_iteration_rule(q.step_rule, q.precision, q.fd, cut, c->d_reqs_sync, c->d_clus_end_sync, 1,
                                        q.nclus, QR, s));
      }
      launched++;
    }
    if (k < q.max_iters) {
      HIPCHK(c, hipMemcpyAsync(hs, q.state, sizeof(ReqState), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (hs->done) break;
    }
  }
  HIPCHK(c, hipEventRecord(c->ev_b, s));
  HIPCHK(c, hipMemcpyAsync(hs, q.state, sizeof(ReqState), hipMemcpyDeviceToHost, s));
  if (per_target_out) {
    per_target_out->resize((size_t)q.m * 7);
    HIPCHK(c, hipMemcpyAsync(per_target_out->data(), q.per_target_dev, (size_t)q.m * 7 * 8, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  fill_result(q, *hs);
  q.status = hs->status;
  q.res.device_bytes = L.total + LB.total;
  if (q.trace_on) {
    const int rows = std::min(hs->iter, q.max_iters);
    q.trace.resize((size_t)rows * kTraceCols);
    if (rows > 0)
      HIPCHK(c, hipMemcpy(q.trace.data(), q.trace_dev, q.trace.size() * 8, hipMemcpyDeviceToHost));
  }
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
  q.res.gpu_ms = ms;
  if (prof) {
    double tot = 0.0, prep = 0.0, quart = 0.0;
    for (int k = 0; k < launched; k++) {
      const hipEvent_t* ev = &c->ev_pool[kEv * k];
      float e1 = 0.f, e2 = 0.f, e3 = 0.f;
      HIPCHK(c, hipEventElapsedTime(&e1, ev[0], ev[1]));
      HIPCHK(c, hipEventElapsedTime(&e2, ev[1], ev[2]));
      if (q.step_rule != kStepFixed) HIPCHK(c, hipEventElapsedTime(&e3, ev[3], ev[4]));
      prep += e1;
      tot += e2;
      quart += e3;
    }
    c->prof_launches += launched;
    c->prof_ms += tot;
    c->prof_prep_ms += prep;
    c->prof_quart_ms += quart;
    c->prof_pairs += hs->pairs_within;
  }
  q.res.wall_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  return CVO_OK;
}

// ---------------------------------------------------------------------------
// continuous-batching scheduler (cvo_submit / cvo_poll)
// ---------------------------------------------------------------------------
namespace {

void complete(cvo_ctx* c, Request* q, int status) {
  std::lock_guard<std::mutex> g(c->q_mu);
  c->st_completed++;
  if (status != CVO_OK) c->st_failed++;
  q->status = status;
  q->res.status = status;
  q->res.wall_ms = std::chrono::duration<double, std::milli>(Clock::now() - q->t_submit).count();
  c->done_cv.notify_all();
}

// device memory of a served request, in the order of the serving stream
char* serve_alloc(cvo_ctx* c, size_t bytes, hipStream_t s) {
  void* p = nullptr;
  const hipError_t e = c->pool ? hipMallocFromPoolAsync(&p, bytes, c->pool, s) : hipMalloc(&p, bytes);
  return e == hipSuccess ? (char*)p : nullptr;
}
void serve_free(cvo_ctx* c, void* p, hipStream_t s) {
  if (!p) return;
  if (c->pool) (void)hipFreeAsync(p, s);
  else (void)hipFree(p);
}

// Both arenas go back after the work already enqueued on the serving stream.
void release(cvo_ctx* c, Request* q, uint64_t& in_use, hipStream_t s) {
  serve_free(c, q->arena, s);
  serve_free(c, q->arena_b, s);
  q->arena = nullptr;
  q->arena_b = nullptr;
  in_use -= q->arena_bytes;
  q->arena_bytes = 0;
}

// Pinned host memory per request of an admission batch: the ingest's
// staged structures, then (at kAdmitStateOff) the state read back.
constexpr int kAdmitBatch = 32;
constexpr size_t kPoolKeepBytes = size_t(4) << 30;  // kept in the pool while the scheduler is idle
constexpr size_t kAdmitStateOff = 32768;
constexpr size_t kAdmitSlot = 49152;
static_assert(kAdmitStateOff + sizeof(ReqState) <= kAdmitSlot, "admission slot");

// Admit one request, first half: allocate arena A, enqueue the ingest and
// the read-back of its state into the request's slot (the cluster count is
// read after the batch's synchronisation).  Returns CVO_OK or an error code.
int admit_enqueue(cvo_ctx* c, Request* q, hipStream_t s, char* slot) {
  const Layout L = plan(*q);
  q->arena = serve_alloc(c, L.total, s);
  if (!q->arena) return CVO_ENOMEM;
  int rc = enqueue_ingest(c, *q, L, s, slot);
  if (rc) return rc;
  if (hipMemcpyAsync(slot + kAdmitStateOff, q->state, sizeof(ReqState), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CVO_EDEVICE;
  return CVO_OK;
}

// After the synchronisation: the cluster count, and in *exact the request's
// exact device bytes (arenas A and B).
int admit_readback(Request* q, const char* slot, size_t* exact) {
  const ReqState* hs = (const ReqState*)(slot + kAdmitStateOff);
  if (hs->done) return hs->status ? hs->status : CVO_EINVAL;
  q->nclus = hs->nclus;
  *exact = plan(*q).total + plan_b(*q, q->nclus).total;
  return CVO_OK;
}

// Second half: allocate the iteration buffers (arena B) and fill the
// request's device constants.
int admit_finish(cvo_ctx* c, Request* q, hipStream_t s) {
  const Layout L = plan(*q);
  const LayoutB LB = plan_b(*q, q->nclus);
  q->arena_b = serve_alloc(c, LB.total, s);
  if (!q->arena_b) return CVO_ENOMEM;
  q->res.device_bytes = L.total + LB.total;
  return finish_setup(c, *q, L, LB, s);
}

void scheduler(cvo_ctx* c) {
  (void)hipSetDevice(c->device);
  hipStream_t s = c->serve_stream;
  std::vector<Request*> active;
  uint64_t in_use = 0;
  ReqStatic* d_reqs = nullptr;
  int* d_end = nullptr;
  int cap_reqs = 0;
  ReqStatic* h_reqs = nullptr;
  int* h_end = nullptr;
  ReqState* h_states = nullptr;
  ReqState* d_states = nullptr;  // the batch's states gathered for one read-back
  DevQueue queue;
  void* h_stage = nullptr;
  if (hipHostMalloc(&h_stage, kAdmitSlot * kAdmitBatch, hipHostMallocDefault) != hipSuccess) h_stage = nullptr;
  const int chunk = 8;
  // with cvo_set_graphs(1): a chunk's launches captured once per launch
  // layout (the groups of active requests, their cluster counts, the request
  // tables and the work list) and replayed while the layout stays the same
  hipGraphExec_t sg_exec = nullptr;
  std::vector<long long> sg_key;
  for (;;) {
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(c->q_mu);
      if (active.empty()) c->q_cv.wait(lk, [&] { return c->stop || !c->pending.empty(); });
      if (c->stop && c->pending.empty() && active.empty()) break;
      while (!c->pending.empty() && (int)(active.size() + admit.size()) < c->max_slots) {
        Request* q = c->pending.front();
        const size_t fp = footprint(*q);
        if (c->budget && fp > c->budget) {
          c->pending.pop_front();
          c->st_completed++;
          c->st_failed++;
          q->status = CVO_ENOMEM;
          q->res.status = CVO_ENOMEM;
          c->done_cv.notify_all();
          continue;
        }
        if (c->budget && in_use + fp > c->budget && !(active.empty() && admit.empty())) break;
        c->pending.pop_front();
        q->arena_bytes = fp;
        in_use += fp;
        admit.push_back(q);
      }
      c->st_active = (int64_t)(active.size() + admit.size());
      c->st_hbm_in_use = in_use;
      c->st_hbm_peak = std::max(c->st_hbm_peak, (uint64_t)in_use);
    }
    std::vector<Request*> requeue;
    // admissions in batches: the ingests of a batch are enqueued together and
    // the cluster counts read after one synchronisation
    std::vector<int> enq_rc(admit.size(), CVO_OK);
    bool synced = true;
    for (size_t k = 0; k < admit.size(); k++) {
      const size_t slot = k % kAdmitBatch;
      if (slot == 0) {
        const size_t end = std::min(admit.size(), k + kAdmitBatch);
        for (size_t j = k; j < end; j++)
          enq_rc[j] = h_stage ? admit_enqueue(c, admit[j], s, (char*)h_stage + (j - k) * kAdmitSlot) : CVO_ENOMEM;
        synced = hipStreamSynchronize(s) == hipSuccess;
      }
      Request* q = admit[k];
      size_t exact = 0;
      int rc = enq_rc[k];
      if (rc == CVO_OK)
        rc = synced ? admit_readback(q, (const char*)h_stage + slot * kAdmitSlot, &exact) : CVO_EDEVICE;
      if (rc == CVO_OK) {
        // charge the exact size; a request that no longer fits beside the
        // running ones waits in the queue with its exact size (its ingest is
        // redone on admission), one that cannot fit at all fails
        in_use = in_use - q->arena_bytes + exact;
        q->arena_bytes = exact;
        q->need_bytes = exact;
        if (c->budget && exact > c->budget) {
          rc = CVO_ENOMEM;
        } else if (c->budget && in_use > c->budget && !(active.empty() && q == admit.front())) {
          release(c, q, in_use, s);
          requeue.push_back(q);
          continue;
        } else {
          rc = admit_finish(c, q, s);
        }
      }
      if (rc != CVO_OK) {
        release(c, q, in_use, s);
        complete(c, q, rc);
        continue;
      }
      active.push_back(q);
    }
    {
      std::lock_guard<std::mutex> g(c->q_mu);
      for (auto it = requeue.rbegin(); it != requeue.rend(); ++it) c->pending.push_front(*it);
      c->st_active = (int64_t)active.size();
      c->st_hbm_in_use = in_use;
      c->st_hbm_peak = std::max(c->st_hbm_peak, (uint64_t)in_use);
    }
    if (active.empty()) continue;

    // one launch pair per iteration per kernel variant, for all active requests
    std::map<std::tuple<int, int, int, int>, std::vector<Request*>> groups;
    for (Request* q : active)
      groups[std::make_tuple(q->precision, q->fd, q->kappa > 0.0 ? 1 : 0, q->step_rule)].push_back(q);
    const int nreq = (int)active.size();
    if (nreq > cap_reqs) {
      if (d_reqs) (void)hipFree(d_reqs);
      if (d_end) (void)hipFree(d_end);
      if (d_states) (void)hipFree(d_states);
      if (h_reqs) (void)hipHostFree(h_reqs);
      if (h_end) (void)hipHostFree(h_end);
      if (h_states) (void)hipHostFree(h_states);
      d_reqs = nullptr;
      d_end = nullptr;
      d_states = nullptr;
      h_reqs = nullptr;
      h_end = nullptr;
      h_states = nullptr;
      cap_reqs = std::max(nreq, 2 * cap_reqs);
      if (hipMalloc(&d_reqs, sizeof(ReqStatic) * cap_reqs) != hipSuccess) d_reqs = nullptr;
      if (hipMalloc(&d_end, sizeof(int) * cap_reqs) != hipSuccess) d_end = nullptr;
      if (hipMalloc(&d_states, sizeof(ReqState) * cap_reqs) != hipSuccess) d_states = nullptr;
      if (hipHostMalloc(&h_reqs, sizeof(ReqStatic) * cap_reqs, hipHostMallocDefault) != hipSuccess) h_reqs = nullptr;
      if (hipHostMalloc(&h_end, sizeof(int) * cap_reqs, hipHostMallocDefault) != hipSuccess) h_end = nullptr;
      if (hipHostMalloc(&h_states, sizeof(ReqState) * cap_reqs, hipHostMallocDefault) != hipSuccess)
        h_states = nullptr;
    }
    struct G {
      int precision, fd, cut, rule, first, count, clusters;
      unsigned long long items;  // work items at most: sum of clusters x chunks_max
    };
    std::vector<G> gl;
    int pos = 0;
    std::vector<Request*> order;
    for (auto& kv : groups) {
      G g{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), pos,
          (int)kv.second.size(), 0, 0ull};
      int cl = 0;
      for (Request* q : kv.second) {
        h_reqs[pos] = q->st;
        cl += q->nclus;
        g.items += (unsigned long long)q->nclus * q->chunks_max;
        h_end[pos] = cl;
        order.push_back(q);
        pos++;
      }
      g.clusters = cl;
      gl.push_back(g);
    }
    unsigned long long most_items = 1;
    for (const G& g : gl) most_items = std::max(most_items, g.items);
    bool dev_ok = d_reqs && d_end && d_states && h_reqs && h_end && h_states && queue.ensure(most_items) &&
                  queue.reset(s) == hipSuccess &&
                  hipMemcpyAsync(d_reqs, h_reqs, sizeof(ReqStatic) * nreq, hipMemcpyHostToDevice, s) == hipSuccess &&
                  hipMemcpyAsync(d_end, h_end, sizeof(int) * nreq, hipMemcpyHostToDevice, s) == hipSuccess;
    roctxRangePushA("cvo_batch_iterations");
    auto launch_chunk = [&]() {
      hipError_t e = hipSuccess;
      for (int it = 0; it < chunk && e == hipSuccess; it++)
        for (const G& g : gl)
          if (e == hipSuccess)
            e = launch_iteration_rule(g.rule, g.precision, g.fd, g.cut != 0, d_reqs + g.first, d_end + g.first,
                                      g.count, g.clusters, queue.ref(), s);
      return e;
    };
    bool graphed = false;
    if (dev_ok && c->graphs.load()) {
      std::vector<long long> key = {(long long)(intptr_t)d_reqs, (long long)(intptr_t)d_end,
                                    (long long)(intptr_t)queue.q, (long long)(intptr_t)queue.items,
                                    (long long)queue.cap, chunk};
      for (const G& g : gl) key.insert(key.end(), {g.rule, g.precision, g.fd, g.cut, g.first, g.count, g.clusters});
      if (!sg_exec || key != sg_key) {
        if (sg_exec) (void)hipGraphExecDestroy(sg_exec);
        sg_exec = nullptr;
        // the capture records kernel launches only (the work list's reset
        // and the request tables' copies stay in front of it on the stream)
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
          const hipError_t e = launch_chunk();
          hipGraph_t gr = nullptr;
          const hipError_t e2 = hipStreamEndCapture(s, &gr);
          if (e == hipSuccess && e2 == hipSuccess && gr &&
              hipGraphInstantiate(&sg_exec, gr, nullptr, nullptr, 0) == hipSuccess)
            sg_key = key;
          else
            sg_exec = nullptr;
          if (gr) (void)hipGraphDestroy(gr);
        }
      }
      if (sg_exec) {
        graphed = true;
        if (hipGraphLaunch(sg_exec, s) != hipSuccess) dev_ok = false;
        else {
          std::lock_guard<std::mutex> g(c->q_mu);
          c->st_graph_chunks++;
        }
      }
    }
    if (dev_ok && !graphed && launch_chunk() != hipSuccess) dev_ok = false;
    if (dev_ok && (launch_gather_states(d_reqs, nreq, d_states, s) != hipSuccess ||
                   hipMemcpyAsync(h_states, d_states, sizeof(ReqState) * nreq, hipMemcpyDeviceToHost, s) !=
                       hipSuccess))
      dev_ok = false;
    if (dev_ok && hipStreamSynchronize(s) != hipSuccess) dev_ok = false;
    roctxRangePop();
    std::vector<Request*> still;
    for (int k = 0; k < nreq; k++) {
      Request* q = order[k];
      if (!dev_ok || h_states[k].done) {
        if (dev_ok) {
          fill_result(*q, h_states[k]);
          if (q->trace_on) {
            const int rows = std::min(h_states[k].iter, q->max_iters);
            q->trace.resize((size_t)rows * kTraceCols);
            if (rows > 0) (void)hipMemcpy(q->trace.data(), q->trace_dev, q->trace.size() * 8, hipMemcpyDeviceToHost);
          }
        }
        release(c, q, in_use, s);
        complete(c, q, dev_ok ? h_states[k].status : CVO_EDEVICE);
      } else {
        still.push_back(q);
      }
    }
    active.swap(still);
    bool idle = false;
    {
      std::lock_guard<std::mutex> g(c->q_mu);
      c->st_active = (int64_t)active.size();
      c->st_hbm_in_use = in_use;
      idle = active.empty() && c->pending.empty();
    }
    // with nothing left to run, the pool gives back what it holds beyond
    // kPoolKeepBytes (the frees enqueued above complete first)
    if (idle && c->pool && hipStreamSynchronize(s) == hipSuccess) (void)hipMemPoolTrimTo(c->pool, kPoolKeepBytes);
  }
  (void)hipStreamSynchronize(s);
  if (sg_exec) (void)hipGraphExecDestroy(sg_exec);
  if (d_reqs) (void)hipFree(d_reqs);
  if (d_end) (void)hipFree(d_end);
  if (d_states) (void)hipFree(d_states);
  if (h_reqs) (void)hipHostFree(h_reqs);
  if (h_end) (void)hipHostFree(h_end);
  if (h_states) (void)hipHostFree(h_states);
  if (h_stage) (void)hipHostFree(h_stage);
  queue.release();
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int cvo_create(int device, uint64_t hbm_budget_bytes, int max_slots, cvo_ctx** out) {
  if (!out) return CVO_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CVO_EDEVICE;
  if (max_slots < 0 || max_slots > 4096) return CVO_EINVAL;
  cvo_ctx* c = new (std::nothrow) cvo_ctx();
  if (!c) return CVO_ENOMEM;
  c->device = device;
  c->max_slots = max_slots > 0 ? max_slots : 256;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->serve_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return CVO_EDEVICE;
  }
  c->stream = c->own_stream;
  {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    uint64_t keep = UINT64_MAX;  // freed blocks stay in the pool for the next requests
    if (hipMemPoolCreate(&c->pool, &props) != hipSuccess) {
      c->pool = nullptr;
    } else if (hipMemPoolSetAttribute(c->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
      (void)hipMemPoolDestroy(c->pool);
      c->pool = nullptr;
    }
  }
  if (init_static_scratch(device) != hipSuccess) {
    (void)hipStreamDestroy(c->own_stream);
    (void)hipStreamDestroy(c->serve_stream);
    if (c->pool) (void)hipMemPoolDestroy(c->pool);
    delete c;
    return CVO_EDEVICE;
  }
  if (hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) hbm_budget_bytes = (uint64_t)(0.8 * (double)fr);
  }
  c->budget = hbm_budget_bytes;
  load_tuning(c);
  *out = c;
  return CVO_OK;
}

int cvo_destroy(cvo_ctx* c) {
  if (!c) return CVO_EINVAL;
  {
    std::lock_guard<std::mutex> g(c->q_mu);
    c->stop = true;
  }
  c->q_cv.notify_all();
  if (c->sched.joinable()) c->sched.join();
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->sync_arena) (void)hipFree(c->sync_arena);
  if (c->d_reqs_sync) (void)hipFree(c->d_reqs_sync);
  if (c->d_clus_end_sync) (void)hipFree(c->d_clus_end_sync);
  c->queue_sync.release();
  if (c->sync_arena_b) (void)hipFree(c->sync_arena_b);
  if (c->fe_arena) (void)hipFree(c->fe_arena);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ev_a) (void)hipEventDestroy(c->ev_a);
  if (c->ev_b) (void)hipEventDestroy(c->ev_b);
  for (auto& kv : c->tickets) delete kv.second;
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  if (c->serve_stream) (void)hipStreamDestroy(c->serve_stream);
  if (c->pool) (void)hipMemPoolDestroy(c->pool);
  delete c;
  return CVO_OK;
}

int cvo_set_stream(cvo_ctx* c, void* stream) {
  if (!c) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->call_mu);
  c->stream = stream ? (hipStream_t)stream : c->own_stream;
  return CVO_OK;
}

int cvo_set_graphs(cvo_ctx* c, int32_t enable) {
  if (!c) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->call_mu);
  c->graphs = enable != 0;
  return CVO_OK;
}

int cvo_set_profiling(cvo_ctx* c, int32_t enable) {
  if (!c) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->call_mu);
  c->profile = enable != 0;
  return CVO_OK;
}

int cvo_kernel_stats(cvo_ctx* c, int32_t reset, int64_t* launches, double* pair_ms, double* prepare_ms,
                     double* quartic_ms, uint64_t* pairs) {
  if (!c) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->call_mu);
  if (launches) *launches = c->prof_launches;
  if (pair_ms) *pair_ms = c->prof_ms;
  if (prepare_ms) *prepare_ms = c->prof_prep_ms;
  if (quartic_ms) *quartic_ms = c->prof_quart_ms;
  if (pairs) *pairs = c->prof_pairs;
  if (reset) {
    c->prof_launches = 0;
    c->prof_ms = 0.0;
    c->prof_prep_ms = 0.0;
    c->prof_quart_ms = 0.0;
    c->prof_pairs = 0;
  }
  return CVO_OK;
}

int cvo_eval(cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p, const double T[16],
             double* F, double omega[3], double v[3]) {
  if (!c) return CVO_EINVAL;
  Request q;
  int rc = build_request(c, src, tgt, p, T, kModeEval, q);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->call_mu);
  rc = run_sync(c, q, nullptr);
  if (rc) return rc;
  if (q.status) return q.status;
  if (F) *F = q.res.F;
  for (int a = 0; a < 3; a++) {
    if (omega) omega[a] = q.res.omega[a];
    if (v) v[a] = q.res.v[a];
  }
  return CVO_OK;
}

// cvo_eval without allocation: every device buffer of the evaluation (the
// request's set-up and iteration arenas, its constants, the work list) is
// carved out of the device's static array; host structures are staged through
// a static host buffer.  The same kernels as cvo_eval, on the context's stream.
static int run_eval_static(cvo_ctx* c, Request& q) {
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  char* base = (char*)g_static_ptr[c->device];
  if (!base) return CVO_EDEVICE;
  char* host = g_static_host[c->device];
  // layout: [ReqStatic | clus_end | WorkQueue] [arena A] [arena B] [work items]
  const size_t off_reqs = 0;
  const size_t off_end = align_up(sizeof(ReqStatic), 256);
  const size_t off_wq = off_end + 256;
  const size_t off_a = off_wq + align_up(sizeof(WorkQueue), 256);
  const Layout L = plan(q);
  const size_t off_b = align_up(off_a + L.total, 256);
  if (off_b > kStaticScratchBytes) {
    c->last_error = "cvo_eval_static: inputs exceed the static device array";
    return CVO_ENOMEM;
  }
  q.arena = base + off_a;
  q.arena_bytes = L.total;
  int rc = enqueue_ingest(c, q, L, s, host);
  if (rc) return rc;
  ReqState* hs = (ReqState*)(host + 32768);
  HIPCHK(c, hipMemcpyAsync(hs, q.state, sizeof(ReqState), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  q.nclus = hs->nclus;
  if (hs->done) {
    fill_result(q, *hs);
    q.status = hs->status;
    return CVO_OK;
  }
  const LayoutB LB = plan_b(q, q.nclus);
  const size_t off_items = align_up(off_b + LB.total, 256);
  const unsigned long long cap = (unsigned long long)std::max(q.nclus, 1) * q.chunks_max;
  if (off_items + cap * sizeof(unsigned int) > kStaticScratchBytes) {
    c->last_error = "cvo_eval_static: the target clusters' buffers exceed the static device array";
    return CVO_ENOMEM;
  }
  q.arena_b = base + off_b;
  q.arena_b_bytes = LB.total;
  rc = finish_setup(c, q, L, LB, s);
  if (rc) return rc;
  ReqStatic* hst = (ReqStatic*)(host + 16384);
  int* hend = (int*)(host + 16384 + sizeof(ReqStatic) + 64);
  *hst = q.st;
  *hend = q.nclus;
  ReqStatic* d_reqs = (ReqStatic*)(base + off_reqs);
  int* d_end = (int*)(base + off_end);
  const QueueRef QR{(WorkQueue*)(base + off_wq), (unsigned int*)(base + off_items), (unsigned int)cap};
  HIPCHK(c, hipMemcpyAsync(d_reqs, hst, sizeof(ReqStatic), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(d_end, hend, sizeof(int), hipMemcpyHostToDevice, s));
  // the work list starts empty (the array keeps the previous call's contents)
  HIPCHK(c, launch_zero(QR.q, sizeof(WorkQueue), s));
  HIPCHK(c, launch_iteration_rule(kStepFixed, q.precision, q.fd, q.kappa > 0.0, d_reqs, d_end, 1, q.nclus, QR, s));
  HIPCHK(c, hipMemcpyAsync(hs, q.state, sizeof(ReqState), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  fill_result(q, *hs);
  q.status = hs->status;
  q.res.device_bytes = off_items + cap * sizeof(unsigned int);
  return CVO_OK;
}

int cvo_quartic(cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p, const double T[16],
                const double omega[3], const double v[3], double coef[5]) {
  if (!c || !omega || !v || !coef) return CVO_EINVAL;
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(omega[a]) || !std::isfinite(v[a])) return CVO_EINVAL;
  Request q;
  int rc = build_request(c, src, tgt, p, T, kModeQuartic, q);
  if (rc) return rc;
  for (int a = 0; a < 3; a++) {
    q.xi0[a] = omega[a];
    q.xi0[3 + a] = v[a];
  }
  std::lock_guard<std::mutex> g(c->call_mu);
  rc = run_sync(c, q, nullptr);
  if (rc) return rc;
  if (q.status) return q.status;
  for (int i = 0; i < 5; i++) coef[i] = q.coef[i];
  return CVO_OK;
}

int cvo_eval_static(cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p, const double T[16],
                    double* F, double omega[3], double v[3]) {
  if (!c) return CVO_EINVAL;
  Request q;
  int rc = build_request(c, src, tgt, p, T, kModeEval, q);
  if (rc) return rc;
  if (q.n > kStaticMaxPoints || q.m > kStaticMaxPoints) {
    c->last_error = "cvo_eval_static: more than 65,536 points in a cloud";
    return CVO_ENOMEM;
  }
  if (c->device < 0 || c->device >= kMaxDevices) return CVO_EDEVICE;
  std::lock_guard<std::mutex> g(c->call_mu);
  std::lock_guard<std::mutex> gd(g_static_call_mu[c->device]);
  rc = run_eval_static(c, q);
  if (rc) return rc;
  if (q.status) return q.status;
  if (F) *F = q.res.F;
  for (int a = 0; a < 3; a++) {
    if (omega) omega[a] = q.res.omega[a];
    if (v) v[a] = q.res.v[a];
  }
  return CVO_OK;
}

int cvo_frontend(cvo_ctx* c, const cvo_rgbd_frame* f, int32_t k, float* xyz, float* feat, int32_t* n_out) {
  if (!c || !f || !xyz || !feat || !n_out || k < 1) return CVO_EINVAL;
  if (f->width < 1 || f->height < 1 || f->width > 16384 || f->height > 16384 || !f->depth || !f->rgb)
    return CVO_EINVAL;
  const long long P = (long long)f->width * f->height;
  if (P > (long long)kScanTile * kScanBlock) return CVO_EINVAL;
  if (!(f->fx > 0.0) || !(f->fy > 0.0) || !std::isfinite(f->fx) || !std::isfinite(f->fy) || !std::isfinite(f->cx) ||
      !std::isfinite(f->cy) || !std::isfinite(f->dmin) || !std::isfinite(f->dmax) || !(f->dmin <= f->dmax))
    return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->call_mu);
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  // arena: depth, rgb (host frames), I, key, tie, pos, two histograms,
  // control block, scan arguments and tile sums, outputs (host outputs)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const bool dev = f->on_device != 0;
  const size_t o_depth = dev ? 0 : take(4 * (size_t)P);
  const size_t o_rgb = dev ? 0 : take(12 * (size_t)P);
  const size_t o_I = take(4 * (size_t)P), o_key = take(4 * (size_t)P), o_tie = take(4 * (size_t)P),
               o_pos = take(4 * (size_t)P);
  const size_t o_hh = take(4 << 16), o_hl = take(4 << 16), o_ctl = take(sizeof(FeCtl)),
               o_scans = take(2 * sizeof(ScanArgs));
  const size_t ntiles = (size_t)((P + kScanTile - 1) / kScanTile) + 1;
  const size_t o_sums0 = take(4 * ntiles), o_sums1 = take(4 * ntiles);
  const size_t o_xyz = dev ? 0 : take(12 * (size_t)k);
  const size_t o_feat = dev ? 0 : take(20 * (size_t)k);
  int rc = grow(c, &c->fe_arena, &c->fe_arena_bytes, off, s);
  if (rc) return rc;
  rc = ensure_pinned(c, 64 * 1024);
  if (rc) return rc;
  char* A = c->fe_arena;
  FrontendArgs a{};
  a.W = f->width;
  a.H = f->height;
  a.k = k;
  a.dmin = (float)f->dmin;
  a.dmax = (float)f->dmax;
  a.fx = f->fx;
  a.fy = f->fy;
  a.cx = f->cx;
  a.cy = f->cy;
  if (dev) {
    a.depth = f->depth;
    a.rgb = f->rgb;
    a.xyz = xyz;
    a.feat = feat;
  } else {
    HIPCHK(c, hipMemcpyAsync(A + o_depth, f->depth, 4 * (size_t)P, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(A + o_rgb, f->rgb, 12 * (size_t)P, hipMemcpyHostToDevice, s));
    a.depth = (const float*)(A + o_depth);
    a.rgb = (const float*)(A + o_rgb);
    a.xyz = (float*)(A + o_xyz);
    a.feat = (float*)(A + o_feat);
  }
  a.I = (float*)(A + o_I);
  a.key = (unsigned*)(A + o_key);
  a.tie = (int*)(A + o_tie);
  a.pos = (int*)(A + o_pos);
  a.hist_hi = (unsigned*)(A + o_hh);
  a.hist_lo = (unsigned*)(A + o_hl);
  a.ctl = (FeCtl*)(A + o_ctl);
  a.scans = (ScanArgs*)(A + o_scans);
  ScanArgs* hs = (ScanArgs*)c->pinned;
  hs[0].data = a.tie;
  hs[0].lenp = nullptr;
  hs[0].len0 = (int)P;
  hs[0].sums = (int*)(A + o_sums0);
  hs[1].data = a.pos;
  hs[1].lenp = nullptr;
  hs[1].len0 = (int)P;
  hs[1].sums = (int*)(A + o_sums1);
  HIPCHK(c, hipMemcpyAsync(a.scans, hs, 2 * sizeof(ScanArgs), hipMemcpyHostToDevice, s));
  HIPCHK(c, launch_frontend(a, s));
  FeCtl* hc = (FeCtl*)((char*)c->pinned + 1024);
  HIPCHK(c, hipMemcpyAsync(hc, a.ctl, sizeof(FeCtl), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (hc->bad) return CVO_EINVAL;
  const int n = hc->n_out;
  if (!dev && n > 0) {
    HIPCHK(c, hipMemcpyAsync(xyz, a.xyz, 12 * (size_t)n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(feat, a.feat, 20 * (size_t)n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  *n_out = n;
  return CVO_OK;
}

int cvo_quartic_step(const double coef[5], double* t) {
  if (!coef || !t) return CVO_EINVAL;
  for (int i = 1; i < 5; i++)
    if (!std::isfinite(coef[i])) return CVO_EINVAL;
  return quartic_argmax(coef, t) ? 1 : 0;
}

int cvo_quartic_step_bounded(const double coef[5], double tmax, double* t) {
  if (!coef || !t || !(tmax > 0.0)) return CVO_EINVAL;
  for (int i = 1; i < 5; i++)
    if (!std::isfinite(coef[i])) return CVO_EINVAL;
  return quartic_argmax(coef, t, tmax) ? 1 : 0;
}

int cvo_eval_targets(cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p,
                     const double T[16], int32_t nsel, const int32_t* sel, double* out) {
  if (!c || !out || nsel < 0 || (nsel > 0 && !sel)) return CVO_EINVAL;
  Request q;
  int rc = build_request(c, src, tgt, p, T, kModeEvalTargets, q);
  if (rc) return rc;
  for (int k = 0; k < nsel; k++)
    if (sel[k] < 0 || sel[k] >= q.m) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->call_mu);
  std::vector<double> all;
  rc = run_sync(c, q, &all);
  if (rc) return rc;
  if (q.status) return q.status;
  if (nsel == 0) {
    memcpy(out, all.data(), all.size() * 8);
  } else {
    for (int k = 0; k < nsel; k++) memcpy(out + 7 * (size_t)k, all.data() + 7 * (size_t)sel[k], 7 * 8);
  }
  return CVO_OK;
}

int cvo_register(cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p, const double T0[16],
                 double T_out[16], cvo_result* res) {
  if (!c) return CVO_EINVAL;
  Request q;
  int rc = build_request(c, src, tgt, p, T0, kModeRegister, q);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->call_mu);
  rc = run_sync(c, q, nullptr);
  if (rc) return rc;
  if (T_out) memcpy(T_out, q.T_out, sizeof(q.T_out));
  if (res) *res = q.res;
  c->last_register = std::move(q);
  c->have_last = true;
  return c->last_register.status;
}

int cvo_submit(cvo_ctx* c, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* p, const double T0[16],
               uint64_t* ticket) {
  if (!c || !ticket) return CVO_EINVAL;
  Request* q = new (std::nothrow) Request();
  if (!q) return CVO_ENOMEM;
  int rc = build_request(c, src, tgt, p, T0, kModeRegister, *q);
  if (rc) {
    delete q;
    return rc;
  }
  if (!q->on_device) {
    q->hsx.assign(q->sx, q->sx + 3ull * q->n);
    q->hsf.assign(q->sfeat, q->sfeat + (size_t)q->fd * q->n);
    q->htx.assign(q->tx, q->tx + 3ull * q->m);
    q->htf.assign(q->tfeat, q->tfeat + (size_t)q->fd * q->m);
    q->sx = q->hsx.data();
    q->sfeat = q->hsf.data();
    q->tx = q->htx.data();
    q->tfeat = q->htf.data();
  }
  q->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(c->q_mu);
    if (c->pending.size() >= c->max_pending) {
      delete q;
      return CVO_EBUSY;
    }
    q->ticket = c->next_ticket++;
    c->tickets[q->ticket] = q;
    c->pending.push_back(q);
    if (!c->sched_started) {
      c->sched_started = true;
      c->sched = std::thread(scheduler, c);
    }
  }
  c->q_cv.notify_all();
  *ticket = q->ticket;
  return CVO_OK;
}

int cvo_serving_stats(cvo_ctx* c, cvo_serving_counters* out) {
  if (!c || !out) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->q_mu);
  out->pending = (int64_t)c->pending.size();
  out->active = c->st_active;
  out->completed = c->st_completed;
  out->failed = c->st_failed;
  out->hbm_in_use = c->st_hbm_in_use;
  out->hbm_budget = c->budget;
  out->hbm_peak = c->st_hbm_peak;
  out->graph_chunks = c->st_graph_chunks;
  return CVO_OK;
}

int cvo_set_queue_limit(cvo_ctx* c, int64_t max_pending) {
  if (!c || max_pending < 0) return CVO_EINVAL;
  std::lock_guard<std::mutex> g(c->q_mu);
  c->max_pending = (size_t)max_pending;
  return CVO_OK;
}

int cvo_poll(cvo_ctx* c, uint64_t ticket, int32_t wait_us, double T_out[16], cvo_result* res) {
  if (!c) return CVO_EINVAL;
  std::unique_lock<std::mutex> lk(c->q_mu);
  auto it = c->tickets.find(ticket);
  if (it == c->tickets.end()) return CVO_ENOTFOUND;
  Request* q = it->second;
  auto ready = [&] { return q->status != CVO_PENDING; };
  if (!ready()) {
    if (wait_us < 0)
      c->done_cv.wait(lk, ready);
    else if (wait_us > 0)
      c->done_cv.wait_for(lk, std::chrono::microseconds(wait_us), ready);
  }
  if (!ready()) return CVO_PENDING;
  if (T_out) memcpy(T_out, q->T_out, sizeof(q->T_out));
  if (res) *res = q->res;
  const int st = q->status;
  if (q->trace_on) {
    constexpr size_t kKeptTraces = 1024;
    c->kept_traces[ticket] = std::move(q->trace);
    c->kept_order.push_back(ticket);
    while (c->kept_order.size() > kKeptTraces) {
      c->kept_traces.erase(c->kept_order.front());
      c->kept_order.pop_front();
    }
  }
  c->tickets.erase(it);
  delete q;
  return st;
}

static int copy_trace(const std::vector<double>& tr, double* buf, int32_t cap) {
  const int rows = (int)(tr.size() / kTraceCols);
  const int w = std::min(rows, (int)cap);
  if (w > 0) memcpy(buf, tr.data(), (size_t)w * kTraceCols * 8);
  return w;
}

int cvo_trace(cvo_ctx* c, uint64_t ticket, double* buf, int32_t cap) {
  if (!c || cap < 0 || (cap > 0 && !buf)) return CVO_EINVAL;
  if (ticket == 0) {
    std::lock_guard<std::mutex> g(c->call_mu);
    if (!c->have_last) return CVO_ENOTFOUND;
    return copy_trace(c->last_register.trace, buf, cap);
  }
  // a batched ticket: the scheduler writes the trace before it publishes the
  // terminal status under q_mu
  std::lock_guard<std::mutex> g(c->q_mu);
  auto it = c->tickets.find(ticket);
  if (it != c->tickets.end()) {
    if (it->second->status == CVO_PENDING) return CVO_PENDING;
    return copy_trace(it->second->trace, buf, cap);
  }
  auto kt = c->kept_traces.find(ticket);
  if (kt == c->kept_traces.end()) return CVO_ENOTFOUND;
  return copy_trace(kt->second, buf, cap);
}

int cvo_tuning(cvo_ctx* c, int32_t n, int32_t m, int32_t cutoff, int32_t* work_item_min, int32_t* work_items_max,
               int32_t* table_classes) {
  if (!c || n < 1 || m < 1) return CVO_EINVAL;
  cvo_params p{};
  Request q;
  q.n = n;
  q.m = m;
  q.kappa = cutoff ? 1.0 : 0.0;
  tune_request(c, &p, q);
  if (work_item_min) *work_item_min = q.chunk_min;
  if (work_items_max) *work_items_max = q.chunks_max;
  if (table_classes) *table_classes = (int32_t)c->tuning.size();
  return CVO_OK;
}

const char* cvo_strerror(int code) {
  switch (code) {
    case CVO_OK: return "ok";
    case CVO_PENDING: return "pending";
    case CVO_EINVAL: return "invalid argument";
    case CVO_ENOMEM: return "request exceeds the device memory budget";
    case CVO_EBUSY: return "submission queue full";
    case CVO_ENOOVERLAP: return "no pair within reach (F <= 1e-300)";
    case CVO_EDEVICE: return "HIP device error";
    case CVO_ENOTFOUND: return "unknown ticket";
    default: return "unknown error";
  }
}

const char* cvo_last_error(cvo_ctx* c) { return c ? c->last_error.c_str() : ""; }

}  // extern "C"
