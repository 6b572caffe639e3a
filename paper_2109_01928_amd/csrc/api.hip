// C ABI of the Debye fitting library (declared in include/debyefit.h):
// argument validation on the host, launch planning and kernel dispatch.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/debyefit.h"
#include "common.hpp"
#include "fit_eval.hpp"

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(DEBYE_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define CHECK_HIP(expr, what)                   \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Lanes per wave that the schedule tries to keep busy: the GPU has 256 CUs x 4
// SIMDs; at two waves per SIMD a batch needs about 2048 waves to fill it.
constexpr int64_t TARGET_WAVES = 2048;
// LDS budget of one single-wave block: a CU has 160 KiB, and two waves per SIMD
// (eight per CU) need at most 20 KiB each
constexpr int LDS_PER_WAVE = 20 * 1024;
// concurrent streams over which the pole-count buckets of one evaluation are
// spread (one hardware queue each)
constexpr int MAX_SIDE_STREAMS = 4;

}  // namespace

namespace dfit {
// error text for debye_last_error() from the library's other host files
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace dfit

struct Bucket {
  int32_t N = 0, SP = 1, SF = 1, cpw = 64;
  int64_t n_cands = 0, n_tiles = 0, max_f = 0, work = 0;
  int64_t xcd_off[9] = {};   // tiles of XCD x: xcd_off[x] .. xcd_off[x+1]-1
  bool uni = false;          // split 1 and every tile holds one material: wave-uniform spectra loads
  double flops = 0;          // algorithmic FP64 work of one evaluation of the bucket
  std::vector<int32_t> mats;
  std::vector<float> tile_est;  // estimated duration of each tile (for the persistent launch's order)
  int32_t *d_lane_cand = nullptr, *d_lane_mat = nullptr, *d_mats = nullptr;
};

// a captured swarm iteration (step -> cost evaluation -> counter tick) and the
// arguments it was captured with
struct SwarmGraph {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int32_t *counter = nullptr;
  std::vector<unsigned char> key;
};

struct debye_plan {
  SwarmGraph graph, de_graph, da_graph;
  int32_t M = 0, max_poles = 0;
  int64_t n_freq = 0, n_cand = 0;
  std::vector<int64_t> f_off, cand_off;
  std::vector<int32_t> n_poles;
  std::vector<Bucket> buckets;
  std::map<int32_t, int32_t> sf_override;  // N (0 = all) -> frequency split
  std::map<int32_t, int32_t> sf_tuned;     // N -> split measured fastest by debye_plan_autotune
  uint64_t sched_gen = 0;                  // bumped by every tile rebuild; part of every graph key
  double *d_record = nullptr;
  int64_t rec_ld = 0;
  // fork/join of the buckets over side streams: bucket i runs on side[lane_of[i]]
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  std::vector<int> stream_of;
  // several buckets: how an evaluation is launched (DEBYE_LAUNCH_*), whether
  // the caller fixed it, and the persistent launch's tables
  int32_t launch = DEBYE_LAUNCH_BUCKETS;
  bool launch_fixed = false;
  dfit::RaggedBucket *d_rbuckets = nullptr;
  int64_t *d_items = nullptr;
  int32_t *d_counters = nullptr;
  int64_t item_off[9] = {};
  size_t ragged_lds = 0;
};

namespace {

void free_bucket(Bucket &b) {
  if (b.d_lane_cand) (void)hipFree(b.d_lane_cand);
  if (b.d_lane_mat) (void)hipFree(b.d_lane_mat);
  if (b.d_mats) (void)hipFree(b.d_mats);
  b.d_lane_cand = b.d_lane_mat = b.d_mats = nullptr;
}

int pick_split(const debye_plan &p, const Bucket &b) {
  auto it = p.sf_override.find(b.N);
  if (it == p.sf_override.end()) it = p.sf_override.find(0);
  const int max_sf = 64 / b.SP;
  if (it != p.sf_override.end() && it->second > 0) return std::min(it->second, max_sf);
  auto tuned = p.sf_tuned.find(b.N);
  if (tuned != p.sf_tuned.end()) return std::min(tuned->second, max_sf);
  // smallest power of two that gives TARGET_WAVES waves, without splitting
  // short spectra below 16 points per lane
  const int64_t avg_f = b.n_cands ? b.work / (b.n_cands * b.N) : 1;
  int sf = 1;
  while (sf < max_sf && (b.n_cands * b.SP * sf + 63) / 64 < TARGET_WAVES && avg_f / (2 * sf) >= 16) sf *= 2;
  // the SP > 1 path keeps each candidate's normal matrix in LDS: fewer
  // candidates per wave until two waves per SIMD fit
  const int lds = dfit::lds_bytes_per_candidate(b.N);
  while (lds > 0 && sf < max_sf && (64 / (b.SP * sf)) * lds > LDS_PER_WAVE) sf *= 2;
  return sf;
}

// Work tiles of a bucket and their split over the 8 XCDs (host only).  Work
// items are runs of one material's candidates (a material with more than
// 1/32 of the bucket's tiles is cut into pieces, so that a few big swarms
// still spread over the chip); the items, longest tiles first, go one by one
// to the XCD with the least estimated work (LPT), which keeps a material's
// spectra in one L2 and finishes the XCDs together.  Each XCD's candidates
// are packed into tiles in that order (a tile may span two materials of the
// same XCD).  uni: every tile's candidates of one material (and spectra of
// fewer than 2^29 points).
struct Schedule {
  std::vector<int32_t> lane_cand, lane_mat;
  int64_t xcd_off[9] = {};
  bool uni = false;
};

Schedule make_schedule(const int64_t *f_off, const int64_t *cand_off, const std::vector<int32_t> &mats, int N, int SP,
                       int SF) {
  const int cpw = 64 / (SP * SF);
  struct Item {
    int32_t m;
    int64_t c0, c1;   // candidates [c0, c1)
    double tile_t;    // estimated duration of one tile: points per lane plus the solve
  };
  int64_t total_tiles = 0, n_cands = 0;
  for (int32_t m : mats) {
    total_tiles += (cand_off[m + 1] - cand_off[m] + cpw - 1) / cpw;
    n_cands += cand_off[m + 1] - cand_off[m];
  }
  const int64_t max_item = std::max<int64_t>(1, total_tiles / 32) * cpw;  // candidates
  std::vector<Item> items;
  for (int32_t m : mats) {
    const int64_t F = f_off[m + 1] - f_off[m];
    const double t = (double)((F + SF - 1) / SF) + 0.05 * N * N;
    for (int64_t c = cand_off[m]; c < cand_off[m + 1]; c += max_item)
      items.push_back({m, c, std::min(c + max_item, cand_off[m + 1]), t});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.tile_t > y.tile_t; });
  std::vector<std::vector<int32_t>> xc(8), xm(8);
  double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (const Item &it : items) {
    const int x = (int)(std::min_element(load, load + 8) - load);
    load[x] += it.tile_t * (double)(it.c1 - it.c0) / cpw;
    for (int64_t c = it.c0; c < it.c1; ++c) {
      xc[x].push_back((int32_t)c);
      xm[x].push_back(it.m);
    }
  }
  Schedule sc;
  std::vector<int32_t> &lc = sc.lane_cand, &lm = sc.lane_mat;
  lc.reserve(n_cands + 8 * cpw);
  lm.reserve(n_cands + 8 * cpw);
  for (int x = 0; x < 8; ++x) {
    lc.insert(lc.end(), xc[x].begin(), xc[x].end());
    lm.insert(lm.end(), xm[x].begin(), xm[x].end());
    while (lc.size() % cpw) {
      lc.push_back(-1);
      lm.push_back(0);
    }
    sc.xcd_off[x + 1] = (int64_t)lc.size() / cpw;
  }
  const int64_t n_tiles = (int64_t)lc.size() / cpw;
  sc.uni = true;
  for (int32_t m : mats)
    if (f_off[m + 1] - f_off[m] >= ((int64_t)1 << 29)) sc.uni = false;  // 32-bit byte offsets
  for (int64_t t = 0; sc.uni && t < n_tiles; ++t)
    for (int64_t l = t * cpw; l < (t + 1) * cpw; ++l)
      if (lc[l] >= 0 && lm[l] != lm[t * cpw]) {
        sc.uni = false;
        break;
      }
  return sc;
}

int build_tiles(debye_plan &p, Bucket &b) {
  // captured graphs hold the old tile buffers: the new generation keys them out
  ++p.sched_gen;
  free_bucket(b);
  b.SF = pick_split(p, b);
  b.cpw = 64 / (b.SP * b.SF);
  const Schedule sc = make_schedule(p.f_off.data(), p.cand_off.data(), b.mats, b.N, b.SP, b.SF);
  for (int x = 0; x < 9; ++x) b.xcd_off[x] = sc.xcd_off[x];
  b.uni = sc.uni;
  const std::vector<int32_t> &lc = sc.lane_cand, &lm = sc.lane_mat;
  b.n_tiles = (int64_t)lc.size() / b.cpw;
  if (b.n_tiles == 0) return DEBYE_OK;
  // estimated tile duration: the longest spectrum of its candidates, per
  // frequency lane, times a per-point cost that follows the kernel's
  // executed instructions (Gram accumulators, basis values, ring moves,
  // the other passes), plus the dense solve
  {
    const int SP = b.SP, NB = (b.N + SP - 1) / SP, D = SP == 1 ? 0 : NB * SP / 2;
    const int NG = SP == 1 ? b.N * (b.N + 1) / 2 : NB * (D + 1);
    const double per_point = NG + 12.0 * NB + 60.0 + (SP > 1 ? 2.0 * D + 24.0 : 0.0);
    b.tile_est.assign(b.n_tiles, 0.0f);
    for (int64_t t = 0; t < b.n_tiles; ++t) {
      int64_t fmax = 0;
      for (int64_t l = t * b.cpw; l < (t + 1) * b.cpw; ++l)
        if (lc[l] >= 0) fmax = std::max(fmax, p.f_off[lm[l] + 1] - p.f_off[lm[l]]);
      b.tile_est[t] = (float)((double)((fmax + b.SF - 1) / b.SF) * per_point + 0.5 * (double)b.N * b.N * b.N);
    }
  }
  if (hipMalloc(&b.d_lane_cand, lc.size() * 4) != hipSuccess || hipMalloc(&b.d_lane_mat, lm.size() * 4) != hipSuccess ||
      hipMalloc(&b.d_mats, b.mats.size() * 4) != hipSuccess)
    return fail(DEBYE_ENOMEM, "plan: device allocation failed");
  CHECK_HIP(hipMemcpy(b.d_lane_cand, lc.data(), lc.size() * 4, hipMemcpyHostToDevice), "plan upload");
  CHECK_HIP(hipMemcpy(b.d_lane_mat, lm.data(), lm.size() * 4, hipMemcpyHostToDevice), "plan upload");
  CHECK_HIP(hipMemcpy(b.d_mats, b.mats.data(), b.mats.size() * 4, hipMemcpyHostToDevice), "plan upload");
  return DEBYE_OK;
}

// Tables of the persistent launch (plans with several pole-count buckets):
// one descriptor per bucket, and per XCD the union of the buckets' tiles of
// that XCD (each bucket's lists are already balanced over the XCDs by work),
// longest estimated duration first.  Rebuilt after every re-tiling.
int build_ragged(debye_plan &p) {
  if (p.d_rbuckets) (void)hipFree(p.d_rbuckets);
  if (p.d_items) (void)hipFree(p.d_items);
  p.d_rbuckets = nullptr;
  p.d_items = nullptr;
  for (int x = 0; x < 9; ++x) p.item_off[x] = 0;
  p.ragged_lds = 0;
  if (p.buckets.size() < 2) return DEBYE_OK;
  ++p.sched_gen;   // captured graphs hold the old tables
  std::vector<dfit::RaggedBucket> rb(p.buckets.size());
  std::vector<std::vector<std::pair<float, int64_t>>> per_xcd(8);
  for (size_t i = 0; i < p.buckets.size(); ++i) {
    const Bucket &bk = p.buckets[i];
    rb[i] = dfit::RaggedBucket{bk.N, bk.SF, bk.cpw, bk.uni ? 1 : 0, bk.d_lane_cand, bk.d_lane_mat};
    p.ragged_lds = std::max(p.ragged_lds, (size_t)dfit::lds_bytes_per_candidate(bk.N) * bk.cpw);
    for (int x = 0; x < 8; ++x)
      for (int64_t t = bk.xcd_off[x]; t < bk.xcd_off[x + 1]; ++t)
        per_xcd[x].push_back({bk.tile_est[t], ((int64_t)i << 40) | t});
  }
  std::vector<int64_t> items;
  for (int x = 0; x < 8; ++x) {
    std::stable_sort(per_xcd[x].begin(), per_xcd[x].end(),
                     [](const std::pair<float, int64_t> &u, const std::pair<float, int64_t> &v) { return u.first > v.first; });
    for (const auto &it : per_xcd[x]) items.push_back(it.second);
    p.item_off[x + 1] = (int64_t)items.size();
  }
  if (!p.d_counters && hipMalloc(&p.d_counters, 8 * sizeof(int32_t)) != hipSuccess) {
    p.d_counters = nullptr;
    return fail(DEBYE_ENOMEM, "plan: persistent-launch counters allocation failed");
  }
  if (hipMalloc(&p.d_rbuckets, rb.size() * sizeof(dfit::RaggedBucket)) != hipSuccess ||
      hipMalloc(&p.d_items, std::max<size_t>(items.size(), 1) * 8) != hipSuccess)
    return fail(DEBYE_ENOMEM, "plan: persistent-launch tables allocation failed");
  CHECK_HIP(hipMemcpy(p.d_rbuckets, rb.data(), rb.size() * sizeof(dfit::RaggedBucket), hipMemcpyHostToDevice),
            "plan upload");
  if (!items.empty())
    CHECK_HIP(hipMemcpy(p.d_items, items.data(), items.size() * 8, hipMemcpyHostToDevice), "plan upload");
  return DEBYE_OK;
}

// blocks of the persistent launch: eight one-wave blocks per CU (two waves
// per SIMD), each looping over its XCD's items
constexpr int32_t RAGGED_BLOCKS = 256 * 8;

int check_batch(const debye_batch *b) {
  if (!b) return fail(DEBYE_EINVAL, "batch is NULL");
  if (b->n_mat < 1) return fail(DEBYE_ERANGE, "n_mat must be >= 1 (got %d)", b->n_mat);
  if (b->max_poles < 1 || b->max_poles > DEBYE_MAX_POLES)
    return fail(DEBYE_ERANGE, "max_poles must be in 1..%d (got %d)", DEBYE_MAX_POLES, b->max_poles);
  if (b->n_freq < 1) return fail(DEBYE_ERANGE, "n_freq must be >= 1");
  if (b->n_cand < 0) return fail(DEBYE_ERANGE, "n_cand must be >= 0");
  if (!b->f_off || !b->cand_off || !b->n_poles || !b->omega || !b->eps_re || !b->eps_im)
    return fail(DEBYE_EINVAL, "batch has a NULL device pointer");
  return DEBYE_OK;
}

int check_plan_batch(const debye_plan *p, const debye_batch *b, int64_t ld) {
  if (!p) return fail(DEBYE_EINVAL, "plan is NULL");
  int rc = check_batch(b);
  if (rc) return rc;
  if (b->n_mat != p->M || b->n_cand != p->n_cand || b->n_freq != p->n_freq || b->max_poles != p->max_poles)
    return fail(DEBYE_EINVAL, "batch shape does not match the plan (M %d/%d, candidates %lld/%lld, points %lld/%lld)",
                b->n_mat, p->M, (long long)b->n_cand, (long long)p->n_cand, (long long)b->n_freq, (long long)p->n_freq);
  if (ld < p->max_poles) return fail(DEBYE_ERANGE, "ld (%lld) < max_poles (%d)", (long long)ld, p->max_poles);
  return DEBYE_OK;
}

static_assert((unsigned)DEBYE_FLAG_NO_SIGN_FLIP == (unsigned)dfit::FLAG_NO_SIGN_FLIP &&
                  (unsigned)DEBYE_FLAG_NO_REFINE == (unsigned)dfit::FLAG_NO_REFINE &&
                  (unsigned)DEBYE_FLAG_DD_REFINE == (unsigned)dfit::FLAG_DD_REFINE,
              "the kernels read the ABI's flag bits");

int check_damping(double damping, uint32_t flags) {
  if (!(damping >= 0.0) || !std::isfinite(damping)) return fail(DEBYE_ERANGE, "damping must be finite and >= 0");
  if (flags & ~(uint32_t)(DEBYE_FLAG_NO_SIGN_FLIP | DEBYE_FLAG_NO_REFINE | DEBYE_FLAG_DD_REFINE))
    return fail(DEBYE_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & DEBYE_FLAG_NO_REFINE) && (flags & DEBYE_FLAG_DD_REFINE))
    return fail(DEBYE_EINVAL, "DEBYE_FLAG_NO_REFINE and DEBYE_FLAG_DD_REFINE exclude each other");
  return DEBYE_OK;
}

// the adjoint kernels and the polish have no double-double refinement
int check_grad_flags(uint32_t flags) {
  if (flags & DEBYE_FLAG_DD_REFINE)
    return fail(DEBYE_EINVAL, "DEBYE_FLAG_DD_REFINE is for forward evaluations only");
  return DEBYE_OK;
}

dfit::FitArgs fit_args(const debye_plan *p, const Bucket &bk, const debye_batch *b, const double *theta, int64_t ld,
                       double damping, uint32_t flags) {
  dfit::FitArgs a{};
  a.f_off = b->f_off;
  a.omega = b->omega;
  a.eps_re = b->eps_re;
  a.eps_im = b->eps_im;
  a.theta = theta;
  a.ld = ld;
  a.damping = damping;
  a.flags = flags;
  a.freq_split = bk.SF;
  a.cand_per_wave = bk.cpw;
  a.lane_cand = bk.d_lane_cand;
  a.lane_mat = bk.d_lane_mat;
  for (int x = 0; x < 9; ++x) a.xcd_off[x] = bk.xcd_off[x];
  (void)p;
  return a;
}

// ---- captured optimiser iterations ----
void graph_destroy(SwarmGraph &g) {
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.ev_in) (void)hipEventDestroy(g.ev_in);
  if (g.ev_out) (void)hipEventDestroy(g.ev_out);
  if (g.stream) (void)hipStreamDestroy(g.stream);
  if (g.counter) (void)hipFree(g.counter);
  g = SwarmGraph();
}

// move the work onto the graph's own stream (ordered after the caller's)
int graph_enter(SwarmGraph &g, hipStream_t caller) {
  if (!g.stream) {
    CHECK_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking), "graph stream");
    CHECK_HIP(hipEventCreateWithFlags(&g.ev_in, hipEventDisableTiming), "graph event");
    CHECK_HIP(hipEventCreateWithFlags(&g.ev_out, hipEventDisableTiming), "graph event");
    if (hipMalloc(&g.counter, sizeof(int32_t)) != hipSuccess) return fail(DEBYE_ENOMEM, "graph counter");
  }
  CHECK_HIP(hipEventRecord(g.ev_in, caller), "event");
  CHECK_HIP(hipStreamWaitEvent(g.stream, g.ev_in, 0), "event wait");
  return DEBYE_OK;
}

int graph_leave(SwarmGraph &g, hipStream_t caller) {
  CHECK_HIP(hipEventRecord(g.ev_out, g.stream), "event");
  CHECK_HIP(hipStreamWaitEvent(caller, g.ev_out, 0), "event wait");
  return DEBYE_OK;
}

// Replay `iters` iterations of body(stream, counter) from one captured graph;
// the device counter holds the iteration number, t0 for the first replay, and
// the body ends with its increment.  The capture is reused while `key` (every
// argument the captured nodes depend on) is unchanged.
template <class BODY>
int graph_replay(SwarmGraph &g, const std::vector<unsigned char> &key, int32_t t0, int32_t iters, BODY &&body) {
  if (iters <= 0) return DEBYE_OK;
  hipStream_t s = g.stream;
  if (!g.exec || g.key != key) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    const int rc = body(s, g.counter);
    const hipError_t e2 = rc ? hipSuccess : dfit::launch_tick(g.counter, s);
    const hipError_t e3 = hipStreamEndCapture(s, &graph);
    if (rc || e2 != hipSuccess || e3 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc ? rc : hip_fail(e2 != hipSuccess ? e2 : e3, "graph capture");
    }
    const hipError_t e4 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e4 != hipSuccess) {
      g.exec = nullptr;
      return hip_fail(e4, "graph instantiate");
    }
    g.key = key;
  }
  CHECK_HIP(dfit::launch_set_counter(g.counter, t0, s), "counter");
  for (int32_t t = 0; t < iters; ++t) CHECK_HIP(hipGraphLaunch(g.exec, s), "graph launch");
  return DEBYE_OK;
}

struct KeyBytes {
  std::vector<unsigned char> v;
  template <class T> void put(const T &x) {
    const unsigned char *c = (const unsigned char *)&x;
    v.insert(v.end(), c, c + sizeof(T));
  }
};

// Enqueue launch(bucket, stream) for every non-empty bucket.  With several
// buckets they fork from `stream` onto the plan's side streams and join back,
// so different pole counts overlap on the GPU; under stream capture the fork
// and join become parallel branches of the graph.
template <class LAUNCH> int for_buckets(const debye_plan *p, hipStream_t stream, LAUNCH &&launch) {
  if (p->side.empty()) {
    for (const Bucket &bk : p->buckets)
      if (bk.n_tiles) {
        int rc = launch(bk, stream);
        if (rc) return rc;
      }
    return DEBYE_OK;
  }
  const int n_side = (int)p->side.size();
  CHECK_HIP(hipEventRecord(p->ev_fork, stream), "fork event");
  for (int j = 0; j < n_side; ++j) CHECK_HIP(hipStreamWaitEvent(p->side[j], p->ev_fork, 0), "fork wait");
  int rc = DEBYE_OK;
  for (size_t i = 0; i < p->buckets.size() && rc == DEBYE_OK; ++i)
    if (p->buckets[i].n_tiles) rc = launch(p->buckets[i], p->side[p->stream_of[i]]);
  // join every side stream, also after a failed launch, so no capture is left open
  for (int j = 0; j < n_side; ++j) {
    CHECK_HIP(hipEventRecord(p->ev_join[j], p->side[j]), "join event");
    CHECK_HIP(hipStreamWaitEvent(stream, p->ev_join[j], 0), "join wait");
  }
  return rc;
}

}  // namespace

namespace {
int fit_eval_impl(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld, double damping,
                  uint32_t flags, double *cost, double *weights, double *eps_inf, int8_t *status,
                  const int32_t *skip_mat, hipStream_t stream);
}  // namespace

extern "C" {

const char *debye_last_error(void) { return g_error.c_str(); }
const char *debye_version(void) { return "debyefit 0.1 (gfx950, FP64)"; }

int debye_plan_create(const debye_batch *shape, const int64_t *f_off_host, const int64_t *cand_off_host,
                      const int32_t *n_poles_host, uint32_t flags, debye_plan **out) {
  if (!out) return fail(DEBYE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_batch(shape);
  if (rc) return rc;
  if (!f_off_host || !cand_off_host || !n_poles_host) return fail(DEBYE_EINVAL, "host shape arrays are NULL");
  if (flags & ~(uint32_t)DEBYE_PLAN_TARGET_GRAD) return fail(DEBYE_EINVAL, "unknown plan flag bits 0x%x", flags);
  const int32_t M = shape->n_mat;
  if (f_off_host[0] != 0 || cand_off_host[0] != 0) return fail(DEBYE_EINVAL, "offsets must start at 0");
  int32_t maxN = 0;
  for (int32_t m = 0; m < M; ++m) {
    if (f_off_host[m + 1] - f_off_host[m] < 1)
      return fail(DEBYE_ERANGE, "material %d has %lld frequency points (need >= 1)", m,
                  (long long)(f_off_host[m + 1] - f_off_host[m]));
    if (cand_off_host[m + 1] < cand_off_host[m]) return fail(DEBYE_EINVAL, "cand_off is decreasing at %d", m);
    if (n_poles_host[m] < 1 || n_poles_host[m] > DEBYE_MAX_POLES)
      return fail(DEBYE_ERANGE, "material %d: n_poles %d outside 1..%d", m, n_poles_host[m], DEBYE_MAX_POLES);
    maxN = std::max(maxN, n_poles_host[m]);
  }
  if (f_off_host[M] != shape->n_freq || cand_off_host[M] != shape->n_cand)
    return fail(DEBYE_EINVAL, "n_freq / n_cand do not match the offsets");
  if (maxN != shape->max_poles) return fail(DEBYE_EINVAL, "max_poles (%d) != max of n_poles (%d)", shape->max_poles, maxN);
  if (cand_off_host[M] > INT32_MAX) return fail(DEBYE_ERANGE, "more than 2^31-1 candidates");

  debye_plan *p = new debye_plan();
  p->M = M;
  p->max_poles = maxN;
  p->n_freq = shape->n_freq;
  p->n_cand = shape->n_cand;
  p->f_off.assign(f_off_host, f_off_host + M + 1);
  p->cand_off.assign(cand_off_host, cand_off_host + M + 1);
  p->n_poles.assign(n_poles_host, n_poles_host + M);
  std::map<int32_t, Bucket> by_n;
  for (int32_t m = 0; m < M; ++m) {
    const int64_t P = cand_off_host[m + 1] - cand_off_host[m];
    if (P == 0) continue;
    Bucket &b = by_n[n_poles_host[m]];
    b.N = n_poles_host[m];
    b.SP = dfit::pole_split(b.N);
    b.mats.push_back(m);
    b.n_cands += P;
    const int64_t F = f_off_host[m + 1] - f_off_host[m];
    b.max_f = std::max(b.max_f, F);
    b.work += P * F * b.N;
    b.flops += (double)P * ((double)F * (b.N * b.N + 13.0 * b.N + 5.0) + b.N * b.N * (b.N / 3.0 + 2.0));
  }
  for (auto &kv : by_n) p->buckets.push_back(std::move(kv.second));
  // per-candidate adjoint records for the target gradient (set-up, so that
  // debye_fit_eval_grad itself never allocates)
  if (flags & DEBYE_PLAN_TARGET_GRAD) {
    p->rec_ld = 4 * p->max_poles + 2;   // [w | z | mu | tau | eps_inf, gc]
    if (hipMalloc(&p->d_record, (size_t)std::max<int64_t>(p->n_cand, 1) * p->rec_ld * 8) != hipSuccess) {
      p->d_record = nullptr;
      debye_plan_destroy(p);
      return fail(DEBYE_ENOMEM, "plan: adjoint record allocation failed");
    }
  }
  // largest work first
  std::stable_sort(p->buckets.begin(), p->buckets.end(), [](const Bucket &x, const Bucket &y) { return x.flops > y.flops; });
  for (auto &b : p->buckets) {
    rc = build_tiles(*p, b);
    if (rc) {
      debye_plan_destroy(p);
      return rc;
    }
  }
  if ((rc = build_ragged(*p))) {
    debye_plan_destroy(p);
    return rc;
  }
  // several pole counts: the buckets run concurrently on side streams, each
  // bucket (largest first) on the stream with the least work so far
  const int n_side = std::min<int>(MAX_SIDE_STREAMS, (int)p->buckets.size());
  if (n_side > 1) {
    p->side.assign(n_side, nullptr);
    p->ev_join.assign(n_side, nullptr);
    bool ok = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int j = 0; j < n_side && ok; ++j)
      ok = hipStreamCreateWithFlags(&p->side[j], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&p->ev_join[j], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      debye_plan_destroy(p);
      return fail(DEBYE_EHIP, "plan: stream or event creation failed");
    }
    std::vector<double> load(n_side, 0.0);
    for (const Bucket &b : p->buckets) {
      const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      p->stream_of.push_back(j);
      load[j] += b.flops;
    }
  }
  *out = p;
  return DEBYE_OK;
}

int debye_plan_destroy(debye_plan *p) {
  if (!p) return DEBYE_OK;
  graph_destroy(p->graph);
  graph_destroy(p->de_graph);
  graph_destroy(p->da_graph);
  for (hipStream_t st : p->side)
    if (st) (void)hipStreamSynchronize(st);
  for (auto &b : p->buckets) free_bucket(b);
  if (p->d_record) (void)hipFree(p->d_record);
  if (p->d_rbuckets) (void)hipFree(p->d_rbuckets);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counters) (void)hipFree(p->d_counters);
  for (hipStream_t st : p->side)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : p->ev_join)
    if (ev) (void)hipEventDestroy(ev);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  delete p;
  return DEBYE_OK;
}

int debye_plan_set_freq_split(debye_plan *p, int32_t n_poles, int32_t split) {
  if (!p) return fail(DEBYE_EINVAL, "plan is NULL");
  if (split < 0 || split > 64 || (split & (split - 1))) return fail(DEBYE_ERANGE, "split must be 0 or a power of two <= 64");
  if (split == 0) p->sf_override.erase(n_poles);
  else p->sf_override[n_poles] = split;
  for (auto &b : p->buckets) {
    int rc = build_tiles(*p, b);
    if (rc) return rc;
  }
  return build_ragged(*p);
}

int debye_plan_set_launch(debye_plan *p, int32_t mode) {
  if (!p) return fail(DEBYE_EINVAL, "plan is NULL");
  if (mode != DEBYE_LAUNCH_AUTO && mode != DEBYE_LAUNCH_BUCKETS && mode != DEBYE_LAUNCH_PERSISTENT)
    return fail(DEBYE_EINVAL, "unknown launch mode %d", mode);
  p->launch_fixed = mode != DEBYE_LAUNCH_AUTO;
  const int32_t m = mode == DEBYE_LAUNCH_AUTO ? DEBYE_LAUNCH_BUCKETS : mode;
  if (m != p->launch) ++p->sched_gen;
  p->launch = m;
  return DEBYE_OK;
}

int debye_plan_get_launch(const debye_plan *p) {
  if (!p) return fail(DEBYE_EINVAL, "plan is NULL");
  return p->buckets.size() > 1 ? p->launch : DEBYE_LAUNCH_BUCKETS;
}

int debye_plan_autotune(debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld, double damping,
                        uint32_t flags, int32_t reps, hipStream_t stream) {
  int rc = check_plan_batch(p, b, ld);
  if (rc) return rc;
  if ((rc = check_damping(damping, flags))) return rc;
  if (!log10_tau) return fail(DEBYE_EINVAL, "log10_tau is NULL");
  if (reps < 1 || reps > 100) return fail(DEBYE_ERANGE, "reps must be in 1..100");
  double *cost = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&](int r) {
    (void)hipStreamSynchronize(stream);
    if (cost) (void)hipFree(cost);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return r;
  };
  if (hipMalloc(&cost, (size_t)std::max<int64_t>(p->n_cand, 1) * 8) != hipSuccess)
    return cleanup(fail(DEBYE_ENOMEM, "autotune: cost buffer allocation failed"));
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return cleanup(fail(DEBYE_EHIP, "autotune: event creation failed"));
  // time `reps` launches of a bucket at its current schedule
  auto time_bucket = [&](Bucket &bk, int n, float *ms) -> int {
    dfit::FitArgs a = fit_args(p, bk, b, log10_tau, ld, damping, flags);
    a.cost = cost;
    hipError_t e = hipEventRecord(e0, stream);
    for (int r = 0; r < n && e == hipSuccess; ++r) e = dfit::launch_fit(bk.N, a, bk.n_tiles, false, bk.uni, stream);
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    return e == hipSuccess ? DEBYE_OK : hip_fail(e, "autotune launch");
  };
  for (Bucket &bk : p->buckets) {
    if (!bk.n_cands || p->sf_override.count(bk.N) || p->sf_override.count(0)) continue;
    const int64_t avg_f = bk.work / (bk.n_cands * bk.N);
    std::vector<int> splits;
    for (int sf = 1; sf <= 64 / bk.SP; sf *= 2) {
      if (sf > 1 && avg_f / sf < 8) break;
      splits.push_back(sf);
    }
    // bring the clocks up first (about 30 ms of this bucket's work), so that
    // the first split timed is not penalised
    float ms = 0;
    p->sf_tuned[bk.N] = splits[0];
    if ((rc = build_tiles(*p, bk)) || (rc = time_bucket(bk, 1, &ms))) return cleanup(rc);
    const int warm = std::min(200, std::max(1, (int)(30.0f / std::max(ms, 0.01f))));
    if ((rc = time_bucket(bk, warm, &ms))) return cleanup(rc);
    // three rounds over the splits, the best time of each (box-to-box and
    // run-to-run spread is a few percent, about the margin between splits)
    std::vector<float> best(splits.size(), INFINITY);
    for (int round = 0; round < 3; ++round)
      for (size_t i = 0; i < splits.size(); ++i) {
        p->sf_tuned[bk.N] = splits[i];
        if ((rc = build_tiles(*p, bk)) || (rc = time_bucket(bk, reps, &ms))) return cleanup(rc);
        best[i] = std::min(best[i], ms);
      }
    // a wider split must win clearly (3 %): it costs reductions, and timing
    // noise should not flip the schedule between runs
    size_t pick = 0;
    for (size_t i = 1; i < splits.size(); ++i)
      if (best[i] < 0.97f * best[pick]) pick = i;
    p->sf_tuned[bk.N] = splits[pick];
    if ((rc = build_tiles(*p, bk))) return cleanup(rc);
  }
  if ((rc = build_ragged(*p))) return cleanup(rc);
  // several buckets: the forked per-bucket launches against the one
  // persistent launch, whole evaluations on the tuned tiles (three rounds,
  // the best of each; the persistent launch must win by 3 %)
  if (p->buckets.size() > 1 && !p->launch_fixed) {
    auto time_eval = [&](int32_t mode, int n, float *ms) -> int {
      p->launch = mode;
      hipError_t e = hipEventRecord(e0, stream);
      int r = DEBYE_OK;
      for (int k = 0; k < n && r == DEBYE_OK && e == hipSuccess; ++k)
        r = debye_fit_eval(p, b, log10_tau, ld, damping, flags, cost, nullptr, nullptr, nullptr, stream);
      if (r) return r;
      if (e == hipSuccess) e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
      return e == hipSuccess ? DEBYE_OK : hip_fail(e, "autotune launch");
    };
    float best[2] = {INFINITY, INFINITY}, ms = 0;
    const int32_t modes[2] = {DEBYE_LAUNCH_BUCKETS, DEBYE_LAUNCH_PERSISTENT};
    for (int m = 0; m < 2; ++m)
      if ((rc = time_eval(modes[m], 1, &ms))) return cleanup(rc);
    for (int round = 0; round < 3; ++round)
      for (int m = 0; m < 2; ++m) {
        if ((rc = time_eval(modes[m], reps, &ms))) return cleanup(rc);
        best[m] = std::min(best[m], ms);
      }
    p->launch = best[1] < 0.97f * best[0] ? DEBYE_LAUNCH_PERSISTENT : DEBYE_LAUNCH_BUCKETS;
    ++p->sched_gen;
  }
  return cleanup(DEBYE_OK);
}

int debye_schedule_preview(const int64_t *f_off, const int64_t *cand_off, const int32_t *mats, int32_t n_mats,
                           int32_t n_poles, int32_t pole_split, int32_t freq_split, int32_t *lane_cand,
                           int32_t *lane_mat, int64_t capacity, int64_t *xcd_off, int32_t *uniform) {
  if (!f_off || !cand_off || (n_mats > 0 && !mats) || !xcd_off || !uniform)
    return fail(DEBYE_EINVAL, "NULL pointer");
  if (n_mats < 0 || n_poles < 1 || n_poles > DEBYE_MAX_POLES || (pole_split != 1 && pole_split != 2 && pole_split != 4) ||
      freq_split < 1 || freq_split * pole_split > 64 || (freq_split & (freq_split - 1)))
    return fail(DEBYE_ERANGE, "schedule preview: bad sizes");
  const std::vector<int32_t> ms(mats, mats + n_mats);
  const Schedule sc = make_schedule(f_off, cand_off, ms, n_poles, pole_split, freq_split);
  for (int x = 0; x < 9; ++x) xcd_off[x] = sc.xcd_off[x];
  *uniform = sc.uni ? 1 : 0;
  const int64_t n = (int64_t)sc.lane_cand.size();
  if (lane_cand && lane_mat) {
    if (capacity < n) return fail(DEBYE_ERANGE, "schedule preview: capacity %lld < %lld slots", (long long)capacity,
                                  (long long)n);
    std::copy(sc.lane_cand.begin(), sc.lane_cand.end(), lane_cand);
    std::copy(sc.lane_mat.begin(), sc.lane_mat.end(), lane_mat);
  }
  return (int)std::min<int64_t>(n, INT32_MAX);
}

int debye_plan_info(const debye_plan *p, int32_t i, int32_t *n_poles, int32_t *pole_split, int32_t *freq_split,
                    int64_t *n_tiles, int32_t *uniform) {
  if (!p) return fail(DEBYE_EINVAL, "plan is NULL");
  if (i < 0) return (int)p->buckets.size();
  if (i >= (int)p->buckets.size()) return fail(DEBYE_ERANGE, "bucket index out of range");
  const Bucket &b = p->buckets[i];
  if (n_poles) *n_poles = b.N;
  if (pole_split) *pole_split = b.SP;
  if (freq_split) *freq_split = b.SF;
  if (n_tiles) *n_tiles = b.n_tiles;
  if (uniform) *uniform = b.uni ? 1 : 0;
  return DEBYE_OK;
}

int debye_afe(const debye_batch *b, const double *log10_tau, int64_t ld, const double *weights, const double *eps_inf,
              double *afe, hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (ld < b->max_poles) return fail(DEBYE_ERANGE, "ld < max_poles");
  if (!log10_tau || !weights || !eps_inf || !afe) return fail(DEBYE_EINVAL, "NULL pointer");
  if (b->n_cand > INT32_MAX) return fail(DEBYE_ERANGE, "more than 2^31-1 candidates");
  dfit::AfeArgs a{b->n_mat, b->f_off, b->cand_off, b->n_poles, b->omega, b->eps_re, b->eps_im,
                  log10_tau, weights, eps_inf, ld, afe};
  CHECK_HIP(dfit::launch_afe(a, b->n_cand, stream), "debye_afe launch");
  return DEBYE_OK;
}

int debye_basis(const double *omega, int64_t F, const double *log10_tau, int64_t ld, int64_t n_cand, int32_t N,
                double *re, double *im, hipStream_t stream) {
  if (!omega || !log10_tau || !re || !im) return fail(DEBYE_EINVAL, "NULL pointer");
  if (F < 1 || N < 1 || N > DEBYE_MAX_POLES || n_cand < 0) return fail(DEBYE_ERANGE, "bad size (F %lld, N %d)", (long long)F, N);
  if (ld < N) return fail(DEBYE_ERANGE, "ld < N");
  if (n_cand == 0) return DEBYE_OK;
  CHECK_HIP(dfit::launch_basis(omega, F, log10_tau, ld, n_cand, N, re, im, stream), "debye_basis launch");
  return DEBYE_OK;
}

int debye_fit_eval(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld, double damping,
                   uint32_t flags, double *cost, double *weights, double *eps_inf, int8_t *status, hipStream_t stream) {
  return fit_eval_impl(p, b, log10_tau, ld, damping, flags, cost, weights, eps_inf, status, nullptr, stream);
}

}  // extern "C"

namespace {
// debye_fit_eval with an optional mask of materials to leave out ([M],
// nonzero = skip: waves holding only such candidates exit at once and their
// outputs are left as they were)
int fit_eval_impl(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld, double damping,
                  uint32_t flags, double *cost, double *weights, double *eps_inf, int8_t *status,
                  const int32_t *skip_mat, hipStream_t stream) {
  int rc = check_plan_batch(p, b, ld);
  if (rc) return rc;
  if ((rc = check_damping(damping, flags))) return rc;
  if (!log10_tau || !cost) return fail(DEBYE_EINVAL, "log10_tau and cost must not be NULL");
  if (p->launch == DEBYE_LAUNCH_PERSISTENT && p->buckets.size() > 1 && !(flags & DEBYE_FLAG_DD_REFINE)) {
    // one launch over every bucket, on the caller's stream
    dfit::RaggedArgs r{};
    r.common = fit_args(p, p->buckets[0], b, log10_tau, ld, damping, flags);
    r.common.cost = cost;
    r.common.weights = weights;
    r.common.eps_inf = eps_inf;
    r.common.status = status;
    r.common.skip_mat = skip_mat;
    r.buckets = p->d_rbuckets;
    r.items = p->d_items;
    for (int x = 0; x < 9; ++x) r.item_off[x] = p->item_off[x];
    r.counters = p->d_counters;
    CHECK_HIP(dfit::launch_fit_ragged(r, RAGGED_BLOCKS, p->ragged_lds, stream), "debye_fit_eval persistent launch");
    return DEBYE_OK;
  }
  return for_buckets(p, stream, [&](const Bucket &bk, hipStream_t s) -> int {
    dfit::FitArgs a = fit_args(p, bk, b, log10_tau, ld, damping, flags);
    a.cost = cost;
    a.weights = weights;
    a.eps_inf = eps_inf;
    a.status = status;
    a.skip_mat = skip_mat;
    CHECK_HIP(dfit::launch_fit(bk.N, a, bk.n_tiles, false, bk.uni, s), "debye_fit_eval launch");
    return DEBYE_OK;
  });
}
}  // namespace

namespace {
// cost + adjoint launches of every bucket; `record` ([n_cand][rec_ld]
// doubles) holds the per-candidate adjoint records the target-gradient
// kernel reads back (NULL without target gradients)
int fit_eval_grad_launch(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld,
                         double damping, uint32_t flags, const double *grad_cost, double *cost,
                         double *grad_log10_tau, double *grad_eps_re, double *grad_eps_im, int8_t *status,
                         double *record, int64_t rec_ld, hipStream_t stream, const int32_t *skip_mat = nullptr) {
  const bool targets = grad_eps_re != nullptr;
  if (targets) {
    // materials without candidates get zero target gradients (a fill kernel,
    // not a memset, so that the call can be captured into a graph)
    CHECK_HIP(dfit::launch_fill(grad_eps_re, p->n_freq, 0.0, stream), "fill");
    CHECK_HIP(dfit::launch_fill(grad_eps_im, p->n_freq, 0.0, stream), "fill");
  }
  return for_buckets(p, stream, [&](const Bucket &bk, hipStream_t s) -> int {
    dfit::FitArgs a = fit_args(p, bk, b, log10_tau, ld, damping, flags);
    a.cost = cost;
    a.status = status;
    a.grad_cost = grad_cost;
    a.grad_theta = grad_log10_tau;
    a.record = targets ? record : nullptr;
    a.rec_ld = rec_ld;
    a.skip_mat = targets ? nullptr : skip_mat;
    CHECK_HIP(dfit::launch_fit(bk.N, a, bk.n_tiles, true, bk.uni, s), "debye_fit_eval_grad launch");
    if (!targets) return DEBYE_OK;
    dfit::TargetGradArgs t{};
    t.f_off = b->f_off;
    t.cand_off = b->cand_off;
    t.omega = b->omega;
    t.eps_re = b->eps_re;
    t.eps_im = b->eps_im;
    t.theta = log10_tau;
    t.ld = ld;
    t.record = record;
    t.rec_ld = rec_ld;
    t.mat_list = bk.d_mats;
    t.grad_re = grad_eps_re;
    t.grad_im = grad_eps_im;
    // the bucket's materials only: disjoint from the other buckets' points
    CHECK_HIP(dfit::launch_target_grad(bk.N, t, bk.max_f, (int32_t)bk.mats.size(), s), "target gradient launch");
    return DEBYE_OK;
  });
}

int fit_eval_grad_check(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld,
                        double damping, uint32_t flags, const double *cost, const double *grad_eps_re,
                        const double *grad_eps_im) {
  int rc = check_plan_batch(p, b, ld);
  if (rc) return rc;
  if ((rc = check_damping(damping, flags))) return rc;
  if ((rc = check_grad_flags(flags))) return rc;
  if (!log10_tau || !cost) return fail(DEBYE_EINVAL, "log10_tau and cost must not be NULL");
  if ((grad_eps_re == nullptr) != (grad_eps_im == nullptr))
    return fail(DEBYE_EINVAL, "grad_eps_re and grad_eps_im must both be set or both be NULL");
  return DEBYE_OK;
}

}  // namespace

namespace dfit {
// debye_fit_eval_grad with the target-gradient records in a buffer the caller
// provides: after the argument checks, and only when target gradients are
// requested, `record_buffer` is asked for a device buffer of at least the
// bytes the batch needs ([n_cand][4 max_poles + 2] doubles); it returns
// DEBYE_OK and the address, or an error code (e.g. DEBYE_ERANGE when it is
// too small).  Nothing is allocated here.
int fit_eval_grad_external(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld,
                           double damping, uint32_t flags, const double *grad_cost, double *cost,
                           double *grad_log10_tau, double *grad_eps_re, double *grad_eps_im, int8_t *status,
                           int (*record_buffer)(size_t bytes, double **out), hipStream_t stream) {
  int rc = fit_eval_grad_check(p, b, log10_tau, ld, damping, flags, cost, grad_eps_re, grad_eps_im);
  if (rc) return rc;
  if (!grad_eps_re)
    return fit_eval_grad_launch(p, b, log10_tau, ld, damping, flags, grad_cost, cost, grad_log10_tau, nullptr,
                                nullptr, status, nullptr, 0, stream);
  const int64_t rec_ld = 4 * (int64_t)p->max_poles + 2;
  double *rec = nullptr;
  if ((rc = record_buffer((size_t)std::max<int64_t>(p->n_cand, 1) * (size_t)rec_ld * 8, &rec))) return rc;
  return fit_eval_grad_launch(p, b, log10_tau, ld, damping, flags, grad_cost, cost, grad_log10_tau, grad_eps_re,
                              grad_eps_im, status, rec, rec_ld, stream);
}
}  // namespace dfit

extern "C" {

int debye_fit_eval_grad(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld,
                        double damping, uint32_t flags, const double *grad_cost, double *cost,
                        double *grad_log10_tau, double *grad_eps_re, double *grad_eps_im, int8_t *status,
                        hipStream_t stream) {
  int rc = fit_eval_grad_check(p, b, log10_tau, ld, damping, flags, cost, grad_eps_re, grad_eps_im);
  if (rc) return rc;
  if (grad_eps_re && !p->d_record)
    return fail(DEBYE_EINVAL, "target gradients need a plan created with DEBYE_PLAN_TARGET_GRAD");
  return fit_eval_grad_launch(p, b, log10_tau, ld, damping, flags, grad_cost, cost, grad_log10_tau, grad_eps_re,
                              grad_eps_im, status, p->d_record, p->rec_ld, stream);
}

int debye_material_eval(int32_t M, const int8_t *kind, const double *params, const int64_t *f_off, int64_t n_freq,
                        const double *omega, uint64_t noise_seed, double *eps_re, double *eps_im, double *jac,
                        hipStream_t stream) {
  if (M < 1) return fail(DEBYE_ERANGE, "M must be >= 1");
  if (n_freq < 1) return fail(DEBYE_ERANGE, "n_freq must be >= 1");
  if (!kind || !params || !f_off || !omega || !eps_re || !eps_im) return fail(DEBYE_EINVAL, "NULL pointer");
  dfit::MaterialArgs a{M, kind, params, f_off, n_freq, omega, noise_seed, eps_re, eps_im, jac};
  CHECK_HIP(dfit::launch_material(a, stream), "debye_material_eval launch");
  return DEBYE_OK;
}

int debye_material_vjp(int32_t M, const int64_t *f_off, int64_t n_freq, const double *jac, const double *grad_re,
                       const double *grad_im, double *grad_params, hipStream_t stream) {
  if (M < 1) return fail(DEBYE_ERANGE, "M must be >= 1");
  if (n_freq < 1) return fail(DEBYE_ERANGE, "n_freq must be >= 1");
  if (!f_off || !jac || !grad_re || !grad_im || !grad_params) return fail(DEBYE_EINVAL, "NULL pointer");
  CHECK_HIP(dfit::launch_material_vjp(M, f_off, jac, grad_re, grad_im, grad_params, stream), "debye_material_vjp launch");
  return DEBYE_OK;
}

static int pso_check(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_pso_params p) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (ld < b->max_poles) return fail(DEBYE_ERANGE, "ld < max_poles");
  if (!lb || !ub) return fail(DEBYE_EINVAL, "lb/ub are NULL");
  if (!std::isfinite(p.inertia) || !std::isfinite(p.c1) || !std::isfinite(p.c2))
    return fail(DEBYE_ERANGE, "PSO coefficients must be finite");
  return DEBYE_OK;
}

int debye_pso_init(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_pso_params p, double *x,
                   double *v, double *pbest_x, double *pbest_cost, double *gbest_cost, int64_t *gbest_idx,
                   hipStream_t stream) {
  int rc = pso_check(b, ld, lb, ub, p);
  if (rc) return rc;
  if (!x || !v || !pbest_x || !pbest_cost || !gbest_cost || !gbest_idx) return fail(DEBYE_EINVAL, "NULL state pointer");
  dfit::PsoArgs a{};
  a.M = b->n_mat;
  a.cand_off = b->cand_off;
  a.n_poles = b->n_poles;
  a.ld = ld;
  a.lb = lb;
  a.ub = ub;
  a.seed = p.seed;
  a.x = x;
  a.v = v;
  a.pbest_x = pbest_x;
  a.pbest_cost = pbest_cost;
  a.gbest_cost = gbest_cost;
  a.gbest_idx = gbest_idx;
  CHECK_HIP(dfit::launch_pso_init(a, b->n_cand, stream), "debye_pso_init launch");
  return DEBYE_OK;
}

int debye_pso_step(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_pso_params p, int32_t t,
                   int32_t move, const double *cost, double *x, double *v, double *pbest_x, double *pbest_cost,
                   double *gbest_x, double *gbest_cost, int64_t *gbest_idx, double *history, int64_t hist_ld,
                   hipStream_t stream) {
  int rc = pso_check(b, ld, lb, ub, p);
  if (rc) return rc;
  if (t < 1) return fail(DEBYE_ERANGE, "iteration t must be >= 1");
  if (history && hist_ld < t) return fail(DEBYE_ERANGE, "hist_ld (%lld) < t (%d)", (long long)hist_ld, t);
  if (!cost || !x || !v || !pbest_x || !pbest_cost || !gbest_x || !gbest_cost || !gbest_idx)
    return fail(DEBYE_EINVAL, "NULL state pointer");
  dfit::PsoArgs a{};
  a.M = b->n_mat;
  a.cand_off = b->cand_off;
  a.n_poles = b->n_poles;
  a.ld = ld;
  a.lb = lb;
  a.ub = ub;
  a.inertia = p.inertia;
  a.c1 = p.c1;
  a.c2 = p.c2;
  a.seed = p.seed;
  a.t = t;
  a.move = move ? 1 : 0;
  a.cost = cost;
  a.x = x;
  a.v = v;
  a.pbest_x = pbest_x;
  a.pbest_cost = pbest_cost;
  a.gbest_x = gbest_x;
  a.gbest_cost = gbest_cost;
  a.gbest_idx = gbest_idx;
  a.history = history;
  a.hist_ld = hist_ld;
  CHECK_HIP(dfit::launch_pso_step(a, stream), "debye_pso_step launch");
  return DEBYE_OK;
}

static dfit::PsoArgs pso_args(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_pso_params p,
                               int32_t t, int32_t move, const debye_swarm *sw) {
  dfit::PsoArgs a{};
  a.M = b->n_mat;
  a.cand_off = b->cand_off;
  a.n_poles = b->n_poles;
  a.ld = ld;
  a.lb = lb;
  a.ub = ub;
  a.inertia = p.inertia;
  a.c1 = p.c1;
  a.c2 = p.c2;
  a.seed = p.seed;
  a.t = t;
  a.move = move;
  a.cost = sw->cost;
  a.x = sw->x;
  a.v = sw->v;
  a.pbest_x = sw->pbest_x;
  a.pbest_cost = sw->pbest_cost;
  a.gbest_x = sw->gbest_x;
  a.gbest_cost = sw->gbest_cost;
  a.gbest_idx = sw->gbest_idx;
  a.history = sw->history;
  a.hist_ld = sw->hist_ld;
  return a;
}

int debye_pso_run(const debye_plan *pc, const debye_batch *b, int64_t ld, const double *lb, const double *ub,
                  debye_pso_params p, int32_t iters, double damping, uint32_t flags, const debye_swarm *sw,
                  int32_t use_graph, hipStream_t stream) {
  int rc = check_plan_batch(pc, b, ld);
  if (rc) return rc;
  if ((rc = check_damping(damping, flags))) return rc;
  if ((rc = pso_check(b, ld, lb, ub, p))) return rc;
  if (!sw || !sw->x || !sw->v || !sw->pbest_x || !sw->pbest_cost || !sw->gbest_x || !sw->gbest_cost ||
      !sw->gbest_idx || !sw->cost)
    return fail(DEBYE_EINVAL, "NULL swarm pointer");
  if (iters < 0) return fail(DEBYE_ERANGE, "iters must be >= 0");
  if (sw->history && sw->hist_ld < (int64_t)iters + 1) return fail(DEBYE_ERANGE, "hist_ld must be >= iters + 1");
  debye_plan *plan = const_cast<debye_plan *>(pc);
  SwarmGraph &g = plan->graph;
  hipStream_t s = stream;
  if (use_graph) {
    if ((rc = graph_enter(g, stream))) return rc;
    s = g.stream;
  }
  dfit::PsoArgs a0 = pso_args(b, ld, lb, ub, p, 0, 0, sw);
  CHECK_HIP(dfit::launch_pso_init(a0, b->n_cand, s), "swarm init");
  if ((rc = debye_fit_eval(plan, b, sw->x, ld, damping, flags, sw->cost, nullptr, nullptr, sw->status, s))) return rc;
  if (!use_graph) {
    for (int32_t t = 1; t <= iters; ++t) {
      CHECK_HIP(dfit::launch_pso_step(pso_args(b, ld, lb, ub, p, t, 1, sw), s), "swarm step");
      if ((rc = debye_fit_eval(plan, b, sw->x, ld, damping, flags, sw->cost, nullptr, nullptr, sw->status, s)))
        return rc;
    }
  } else {
    KeyBytes key;
    key.put(*b);
    key.put(ld);
    key.put(lb);
    key.put(ub);
    key.put(p);
    key.put(damping);
    key.put(flags);
    key.put(*sw);
    key.put(plan->sched_gen);
    rc = graph_replay(g, key.v, 1, iters, [&](hipStream_t gs, int32_t *counter) -> int {
      dfit::PsoArgs a = pso_args(b, ld, lb, ub, p, 0, 1, sw);
      a.t_dev = counter;
      CHECK_HIP(dfit::launch_pso_step(a, gs), "swarm step");
      return debye_fit_eval(plan, b, sw->x, ld, damping, flags, sw->cost, nullptr, nullptr, sw->status, gs);
    });
    if (rc) return rc;
  }
  CHECK_HIP(dfit::launch_pso_step(pso_args(b, ld, lb, ub, p, iters + 1, 0, sw), s), "final bests");
  if (use_graph) return graph_leave(g, stream);
  return DEBYE_OK;
}

// ---- differential evolution ----
static int de_check(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_de_params p) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (ld < b->max_poles) return fail(DEBYE_ERANGE, "ld < max_poles");
  if (!lb || !ub) return fail(DEBYE_EINVAL, "lb/ub are NULL");
  if (!(p.f_lo >= 0.0 && p.f_lo <= p.f_hi && p.f_hi <= 2.0) || !(p.cr >= 0.0 && p.cr <= 1.0))
    return fail(DEBYE_ERANGE, "DE parameters out of range (0 <= f_lo <= f_hi <= 2, 0 <= cr <= 1)");
  return DEBYE_OK;
}

static dfit::DeArgs de_args(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_de_params p,
                            int32_t t) {
  dfit::DeArgs a{};
  a.M = b->n_mat;
  a.cand_off = b->cand_off;
  a.n_poles = b->n_poles;
  a.ld = ld;
  a.lb = lb;
  a.ub = ub;
  a.f_lo = p.f_lo;
  a.f_hi = p.f_hi;
  a.cr = p.cr;
  a.seed = p.seed;
  a.t = t;
  return a;
}

int debye_de_init(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_de_params p, double *x,
                  double *fit, double *best_cost, int64_t *best_idx, hipStream_t stream) {
  int rc = de_check(b, ld, lb, ub, p);
  if (rc) return rc;
  if (!x || !fit || !best_cost || !best_idx) return fail(DEBYE_EINVAL, "NULL population pointer");
  dfit::DeArgs a = de_args(b, ld, lb, ub, p, 0);
  a.x = x;
  a.fit = fit;
  a.best_cost = best_cost;
  a.best_idx = best_idx;
  CHECK_HIP(dfit::launch_de_init(a, b->n_cand, stream), "DE init");
  return DEBYE_OK;
}

int debye_de_trial(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_de_params p, int32_t t,
                   const double *x, double *u, hipStream_t stream) {
  int rc = de_check(b, ld, lb, ub, p);
  if (rc) return rc;
  if (!x || !u) return fail(DEBYE_EINVAL, "NULL population pointer");
  if (t < 1) return fail(DEBYE_ERANGE, "generation must be >= 1");
  dfit::DeArgs a = de_args(b, ld, lb, ub, p, t);
  a.x = const_cast<double *>(x);
  a.u = u;
  CHECK_HIP(dfit::launch_de_trial(a, b->n_cand, stream), "DE trial");
  return DEBYE_OK;
}

int debye_de_select(const debye_batch *b, int64_t ld, int32_t t, const double *u, const double *cost_u, double *x,
                    double *fit, double *best_x, double *best_cost, int64_t *best_idx, double *history,
                    int64_t hist_ld, hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (ld < b->max_poles) return fail(DEBYE_ERANGE, "ld < max_poles");
  if (!u || !cost_u || !x || !fit || !best_x || !best_cost || !best_idx) return fail(DEBYE_EINVAL, "NULL pointer");
  if (t < 0 || (history && hist_ld <= t)) return fail(DEBYE_ERANGE, "generation must be >= 0 and < hist_ld");
  dfit::DeArgs a = de_args(b, ld, nullptr, nullptr, debye_de_params{0, 0, 0, 0}, t);
  a.u = const_cast<double *>(u);
  a.cost_u = cost_u;
  a.x = x;
  a.fit = fit;
  a.best_x = best_x;
  a.best_cost = best_cost;
  a.best_idx = best_idx;
  a.history = history;
  a.hist_ld = hist_ld;
  CHECK_HIP(dfit::launch_de_select(a, stream), "DE select");
  return DEBYE_OK;
}

int debye_de_run(const debye_plan *pc, const debye_batch *b, int64_t ld, const double *lb, const double *ub,
                 debye_de_params p, int32_t iters, double damping, uint32_t flags, const debye_population *pop,
                 int32_t use_graph, hipStream_t stream) {
  int rc = check_plan_batch(pc, b, ld);
  if (rc) return rc;
  if ((rc = check_damping(damping, flags))) return rc;
  if ((rc = de_check(b, ld, lb, ub, p))) return rc;
  if (!pop || !pop->x || !pop->u || !pop->fit || !pop->cost || !pop->best_x || !pop->best_cost || !pop->best_idx)
    return fail(DEBYE_EINVAL, "NULL population pointer");
  if (iters < 0) return fail(DEBYE_ERANGE, "iters must be >= 0");
  if (pop->history && pop->hist_ld < (int64_t)iters + 1) return fail(DEBYE_ERANGE, "hist_ld must be >= iters + 1");
  debye_plan *plan = const_cast<debye_plan *>(pc);
  SwarmGraph &g = plan->de_graph;
  hipStream_t s = stream;
  if (use_graph) {
    if ((rc = graph_enter(g, stream))) return rc;
    s = g.stream;
  }
  auto sel = [&](int32_t t) {
    dfit::DeArgs a = de_args(b, ld, lb, ub, p, t);
    a.u = pop->u;
    a.cost_u = pop->cost;
    a.x = pop->x;
    a.fit = pop->fit;
    a.best_x = pop->best_x;
    a.best_cost = pop->best_cost;
    a.best_idx = pop->best_idx;
    a.history = pop->history;
    a.hist_ld = pop->hist_ld;
    return a;
  };
  dfit::DeArgs a0 = sel(0);
  CHECK_HIP(dfit::launch_de_init(a0, b->n_cand, s), "DE init");
  // generation 0: the initial population is its own trial set
  if ((rc = debye_fit_eval(plan, b, pop->x, ld, damping, flags, pop->cost, nullptr, nullptr, pop->status, s)))
    return rc;
  CHECK_HIP(hipMemcpyAsync(pop->u, pop->x, (size_t)b->n_cand * ld * 8, hipMemcpyDeviceToDevice, s), "copy");
  CHECK_HIP(dfit::launch_de_select(a0, s), "DE select");
  auto generation = [&](hipStream_t gs, int32_t t, const int32_t *t_dev) -> int {
    dfit::DeArgs a = sel(t);
    a.t_dev = t_dev;
    CHECK_HIP(dfit::launch_de_trial(a, b->n_cand, gs), "DE trial");
    int r = debye_fit_eval(plan, b, pop->u, ld, damping, flags, pop->cost, nullptr, nullptr, pop->status, gs);
    if (r) return r;
    CHECK_HIP(dfit::launch_de_select(a, gs), "DE select");
    return DEBYE_OK;
  };
  if (!use_graph) {
    for (int32_t t = 1; t <= iters; ++t)
      if ((rc = generation(s, t, nullptr))) return rc;
    return DEBYE_OK;
  }
  KeyBytes key;
  key.put(*b);
  key.put(ld);
  key.put(lb);
  key.put(ub);
  key.put(p);
  key.put(damping);
  key.put(flags);
  key.put(*pop);
  key.put(pc->sched_gen);
  rc = graph_replay(g, key.v, 1, iters, [&](hipStream_t gs, int32_t *counter) { return generation(gs, 0, counter); });
  if (rc) return rc;
  return graph_leave(g, stream);
}

// ---- annealing ----
static int da_check(const debye_batch *b, int64_t ld, debye_da_params p) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (ld < b->max_poles) return fail(DEBYE_ERANGE, "ld < max_poles");
  if (!(p.qv > 1.0 && p.qv < 3.0) || !(p.qa < 1.0) || !(p.t0 > 0.0) || !std::isfinite(p.t0) || !std::isfinite(p.qa))
    return fail(DEBYE_ERANGE, "annealing parameters out of range (1 < qv < 3, qa < 1, t0 > 0)");
  return DEBYE_OK;
}

static dfit::DaArgs da_args(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_da_params p,
                            int32_t t) {
  dfit::DaArgs a{};
  a.M = b->n_mat;
  a.cand_off = b->cand_off;
  a.n_poles = b->n_poles;
  a.ld = ld;
  a.lb = lb;
  a.ub = ub;
  a.qv = p.qv;
  a.qa = p.qa;
  a.t0 = p.t0;
  a.seed = p.seed;
  a.t = t;
  return a;
}

int debye_da_init(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_da_params p, double *x,
                  double *fit, double *best_cost, int64_t *best_idx, hipStream_t stream) {
  int rc = da_check(b, ld, p);
  if (rc) return rc;
  if (!lb || !ub || !x || !fit || !best_cost || !best_idx) return fail(DEBYE_EINVAL, "NULL pointer");
  dfit::DaArgs a = da_args(b, ld, lb, ub, p, 0);
  a.x = x;
  a.fit = fit;
  a.best_cost = best_cost;
  a.best_idx = best_idx;
  CHECK_HIP(dfit::launch_da_init(a, b->n_cand, stream), "annealing init");
  return DEBYE_OK;
}

int debye_da_visit(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_da_params p, int32_t t,
                   const double *x, double *y, hipStream_t stream) {
  int rc = da_check(b, ld, p);
  if (rc) return rc;
  if (!lb || !ub || !x || !y) return fail(DEBYE_EINVAL, "NULL pointer");
  if (t < 1) return fail(DEBYE_ERANGE, "generation must be >= 1");
  dfit::DaArgs a = da_args(b, ld, lb, ub, p, t);
  a.x = const_cast<double *>(x);
  a.u = y;
  CHECK_HIP(dfit::launch_da_visit(a, b->n_cand, stream), "annealing visit");
  return DEBYE_OK;
}

int debye_da_accept(const debye_batch *b, int64_t ld, debye_da_params p, int32_t t, const double *y,
                    const double *cost_y, double *x, double *fit, double *best_x, double *best_cost, int64_t *best_idx,
                    double *history, int64_t hist_ld, hipStream_t stream) {
  int rc = da_check(b, ld, p);
  if (rc) return rc;
  if (!y || !cost_y || !x || !fit || !best_x || !best_cost || !best_idx) return fail(DEBYE_EINVAL, "NULL pointer");
  if (t < 0 || (history && hist_ld <= t)) return fail(DEBYE_ERANGE, "generation must be >= 0 and < hist_ld");
  dfit::DaArgs a = da_args(b, ld, nullptr, nullptr, p, t);
  a.u = const_cast<double *>(y);
  a.cost_u = cost_y;
  a.x = x;
  a.fit = fit;
  a.best_x = best_x;
  a.best_cost = best_cost;
  a.best_idx = best_idx;
  a.history = history;
  a.hist_ld = hist_ld;
  CHECK_HIP(dfit::launch_da_accept(a, stream), "annealing accept");
  return DEBYE_OK;
}

int debye_da_run(const debye_plan *pc, const debye_batch *b, int64_t ld, const double *lb, const double *ub,
                 debye_da_params p, int32_t iters, double damping, uint32_t flags, const debye_population *pop,
                 int32_t use_graph, hipStream_t stream) {
  int rc = check_plan_batch(pc, b, ld);
  if (rc) return rc;
  if ((rc = check_damping(damping, flags))) return rc;
  if ((rc = da_check(b, ld, p))) return rc;
  if (!lb || !ub) return fail(DEBYE_EINVAL, "lb/ub are NULL");
  if (!pop || !pop->x || !pop->u || !pop->fit || !pop->cost || !pop->best_x || !pop->best_cost || !pop->best_idx)
    return fail(DEBYE_EINVAL, "NULL population pointer");
  if (iters < 0) return fail(DEBYE_ERANGE, "iters must be >= 0");
  if (pop->history && pop->hist_ld < (int64_t)iters + 1) return fail(DEBYE_ERANGE, "hist_ld must be >= iters + 1");
  debye_plan *plan = const_cast<debye_plan *>(pc);
  SwarmGraph &g = plan->da_graph;
  hipStream_t s = stream;
  if (use_graph) {
    if ((rc = graph_enter(g, stream))) return rc;
    s = g.stream;
  }
  auto args = [&](int32_t t) {
    dfit::DaArgs a = da_args(b, ld, lb, ub, p, t);
    a.u = pop->u;
    a.cost_u = pop->cost;
    a.x = pop->x;
    a.fit = pop->fit;
    a.best_x = pop->best_x;
    a.best_cost = pop->best_cost;
    a.best_idx = pop->best_idx;
    a.history = pop->history;
    a.hist_ld = pop->hist_ld;
    return a;
  };
  dfit::DaArgs a0 = args(0);
  CHECK_HIP(dfit::launch_da_init(a0, b->n_cand, s), "annealing init");
  if ((rc = debye_fit_eval(plan, b, pop->x, ld, damping, flags, pop->cost, nullptr, nullptr, pop->status, s)))
    return rc;
  CHECK_HIP(hipMemcpyAsync(pop->u, pop->x, (size_t)b->n_cand * ld * 8, hipMemcpyDeviceToDevice, s), "copy");
  CHECK_HIP(dfit::launch_da_accept(a0, s), "annealing accept");
  auto generation = [&](hipStream_t gs, int32_t t, const int32_t *t_dev) -> int {
    dfit::DaArgs a = args(t);
    a.t_dev = t_dev;
    CHECK_HIP(dfit::launch_da_visit(a, b->n_cand, gs), "annealing visit");
    int r = debye_fit_eval(plan, b, pop->u, ld, damping, flags, pop->cost, nullptr, nullptr, pop->status, gs);
    if (r) return r;
    CHECK_HIP(dfit::launch_da_accept(a, gs), "annealing accept");
    return DEBYE_OK;
  };
  if (!use_graph) {
    for (int32_t t = 1; t <= iters; ++t)
      if ((rc = generation(s, t, nullptr))) return rc;
    return DEBYE_OK;
  }
  KeyBytes key;
  key.put(*b);
  key.put(ld);
  key.put(lb);
  key.put(ub);
  key.put(p);
  key.put(damping);
  key.put(flags);
  key.put(*pop);
  key.put(pc->sched_gen);
  rc = graph_replay(g, key.v, 1, iters, [&](hipStream_t gs, int32_t *counter) { return generation(gs, 0, counter); });
  if (rc) return rc;
  return graph_leave(g, stream);
}

// ---- L-BFGS polish: a context that owns the workspace and the plans (one
// candidate per material, for the gradient and the full steps; ta and tb
// trials per material, for the two later stages of the line search), so that
// the calls below only enqueue work
constexpr int32_t POLISH_STAGE_A = 4;   // halvings tried right after a failed full step

struct debye_polish {
  int32_t M = 0, max_poles = 0, mem = 0, max_trials = 0, steps = 0, ta = 0, tb = 0;
  int64_t ld = 0, n_freq = 0;
  double c1 = 0;
  debye_plan *p1 = nullptr, *pA = nullptr, *pB = nullptr;
  void *ws = nullptr;         // one allocation for every buffer below
  int64_t *off_a = nullptr, *off_b = nullptr;   // [M+1] candidate offsets of the two later stages
  double *grad, *S, *Y, *rho, *dir, *gd, *trial_theta, *trial_cost, *new_theta, *new_cost, *new_grad, *cost, *acc_cost;
  int32_t *hist_n, *hist_head, *accepted, *done, *stalled;
  int8_t *trial_status, *new_status;
};

namespace {
int polish_check(const debye_polish *pp, const debye_batch *b, double damping, uint32_t flags) {
  if (!pp) return fail(DEBYE_EINVAL, "polish context is NULL");
  int rc = check_batch(b);
  if (rc) return rc;
  if (b->n_mat != pp->M || b->n_cand != pp->M || b->n_freq != pp->n_freq || b->max_poles != pp->max_poles)
    return fail(DEBYE_EINVAL, "batch does not match the polish context (one candidate per material)");
  if ((rc = check_damping(damping, flags))) return rc;
  return check_grad_flags(flags);
}

dfit::LbfgsArgs polish_args(const debye_polish *pp, const debye_batch *b, double *theta, const double *lb,
                            const double *ub, double *cost_hist) {
  dfit::LbfgsArgs la{};
  la.M = pp->M;
  la.n_poles = b->n_poles;
  la.ld = pp->ld;
  la.mem = pp->mem;
  la.max_trials = pp->max_trials;
  la.ta = pp->ta;
  la.tb = pp->tb;
  la.c1 = pp->c1;
  la.lb = lb;
  la.ub = ub;
  la.theta = theta;
  la.cost = pp->cost;
  la.acc_cost = pp->acc_cost;
  la.grad = pp->grad;
  la.S = pp->S;
  la.Y = pp->Y;
  la.rho = pp->rho;
  la.hist_n = pp->hist_n;
  la.hist_head = pp->hist_head;
  la.dir = pp->dir;
  la.gd = pp->gd;
  la.trial_theta = pp->trial_theta;
  la.trial_cost = pp->trial_cost;
  la.trial_status = pp->trial_status;
  la.done = pp->done;
  la.stalled = pp->stalled;
  la.new_theta = pp->new_theta;
  la.accepted = pp->accepted;
  la.new_cost = pp->new_cost;
  la.new_grad = pp->new_grad;
  la.new_status = pp->new_status;
  la.cost_hist = cost_hist;
  la.steps = pp->steps;
  return la;
}
}  // namespace

int debye_polish_create(const debye_batch *shape, const int64_t *f_off_host, const int32_t *n_poles_host, int64_t ld,
                        debye_lbfgs_params lp, debye_polish **out) {
  if (!out) return fail(DEBYE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_batch(shape);
  if (rc) return rc;
  if (!f_off_host || !n_poles_host) return fail(DEBYE_EINVAL, "host shape arrays are NULL");
  if (ld < shape->max_poles) return fail(DEBYE_ERANGE, "ld < max_poles");
  if (shape->n_cand != shape->n_mat) return fail(DEBYE_EINVAL, "polish needs exactly one candidate per material");
  if (lp.steps < 0 || lp.mem < 1 || lp.mem > DFIT_MAX_MEM || lp.max_trials < 1 || lp.max_trials > 64 ||
      !(lp.c1 > 0.0 && lp.c1 < 1.0))
    return fail(DEBYE_ERANGE, "L-BFGS parameters out of range (steps >= 0, mem 1..%d, trials 1..64, 0 < c1 < 1)",
                DFIT_MAX_MEM);
  const int32_t M = shape->n_mat;
  const int T = lp.max_trials;
  const int32_t ta = std::min(POLISH_STAGE_A, T - 1), tb = T - 1 - ta;
  std::vector<int64_t> one(M + 1), offs_a(M + 1), offs_b(M + 1);
  for (int32_t m = 0; m <= M; ++m) {
    one[m] = m;
    offs_a[m] = (int64_t)m * ta;
    offs_b[m] = (int64_t)m * tb;
  }
  debye_polish *pp = new debye_polish();
  pp->M = M;
  pp->max_poles = shape->max_poles;
  pp->mem = lp.mem;
  pp->max_trials = T;
  pp->ta = ta;
  pp->tb = tb;
  pp->steps = lp.steps;
  pp->c1 = lp.c1;
  pp->ld = ld;
  pp->n_freq = shape->n_freq;
  auto bail = [&](int r) {
    debye_polish_destroy(pp);
    return r;
  };
  const int64_t n1 = (int64_t)M * ld, nT = (int64_t)M * T;
  const size_t doubles = (size_t)(n1 /*grad*/ + 2 * (int64_t)M * lp.mem * ld /*S,Y*/ + (int64_t)M * lp.mem /*rho*/ +
                                  n1 /*dir*/ + M /*gd*/ + nT * ld /*trial theta*/ + nT /*trial cost*/ + n1 /*new theta*/ +
                                  M /*new cost*/ + n1 /*new grad*/ + M /*cost*/ + M /*accepted cost*/);
  const size_t bytes = (size_t)2 * (M + 1) * 8 + doubles * 8 + (size_t)5 * M * 4 + (size_t)nT + (size_t)M + 64;
  if (hipMalloc(&pp->ws, bytes) != hipSuccess) {
    pp->ws = nullptr;
    return bail(fail(DEBYE_ENOMEM, "polish workspace allocation failed"));
  }
  pp->off_a = (int64_t *)pp->ws;
  pp->off_b = pp->off_a + M + 1;
  double *dp = (double *)(pp->off_b + M + 1);
  auto take = [&](int64_t n) {
    double *r = dp;
    dp += n;
    return r;
  };
  pp->grad = take(n1);
  pp->S = take((int64_t)M * lp.mem * ld);
  pp->Y = take((int64_t)M * lp.mem * ld);
  pp->rho = take((int64_t)M * lp.mem);
  pp->dir = take(n1);
  pp->gd = take(M);
  pp->trial_theta = take(nT * ld);
  pp->trial_cost = take(nT);
  pp->new_theta = take(n1);
  pp->new_cost = take(M);
  pp->new_grad = take(n1);
  pp->cost = take(M);
  pp->acc_cost = take(M);
  int32_t *ip = (int32_t *)dp;
  pp->hist_n = ip;
  pp->hist_head = ip + M;
  pp->accepted = ip + 2 * M;
  pp->done = ip + 3 * M;
  pp->stalled = ip + 4 * M;
  pp->trial_status = (int8_t *)(ip + 5 * M);
  pp->new_status = pp->trial_status + nT;
  if (hipMemcpy(pp->off_a, offs_a.data(), (M + 1) * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pp->off_b, offs_b.data(), (M + 1) * 8, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(DEBYE_EHIP, "polish: upload of the trial offsets failed"));
  std::vector<int64_t> f_h(f_off_host, f_off_host + M + 1);
  if ((rc = debye_plan_create(shape, f_h.data(), one.data(), n_poles_host, 0, &pp->p1))) return bail(rc);
  debye_batch bt = *shape;
  if (ta > 0) {
    bt.cand_off = pp->off_a;
    bt.n_cand = (int64_t)M * ta;
    if ((rc = debye_plan_create(&bt, f_h.data(), offs_a.data(), n_poles_host, 0, &pp->pA))) return bail(rc);
  }
  if (tb > 0) {
    bt.cand_off = pp->off_b;
    bt.n_cand = (int64_t)M * tb;
    if ((rc = debye_plan_create(&bt, f_h.data(), offs_b.data(), n_poles_host, 0, &pp->pB))) return bail(rc);
  }
  *out = pp;
  return DEBYE_OK;
}

int debye_polish_destroy(debye_polish *pp) {
  if (!pp) return DEBYE_OK;
  debye_plan_destroy(pp->p1);
  debye_plan_destroy(pp->pA);
  debye_plan_destroy(pp->pB);
  if (pp->ws) {
    (void)hipDeviceSynchronize();   // no work of the context may still read the workspace
    (void)hipFree(pp->ws);
  }
  delete pp;
  return DEBYE_OK;
}

int debye_polish_begin(debye_polish *pp, const debye_batch *b, const double *theta, double damping, uint32_t flags,
                       hipStream_t stream) {
  int rc = polish_check(pp, b, damping, flags);
  if (rc) return rc;
  if (!theta) return fail(DEBYE_EINVAL, "theta is NULL");
  // empty history (a fill kernel, not a memset, so that the call can be captured)
  CHECK_HIP(dfit::launch_fill_i32(pp->hist_n, 2 * (int64_t)pp->M, 0, stream), "fill");
  CHECK_HIP(dfit::launch_fill_i32(pp->stalled, (int64_t)pp->M, 0, stream), "fill");
  return debye_fit_eval_grad(pp->p1, b, theta, pp->ld, damping, flags, nullptr, pp->cost, pp->grad, nullptr, nullptr,
                             pp->new_status, stream);
}

int debye_polish_step(debye_polish *pp, const debye_batch *b, double *theta, const double *lb, const double *ub,
                      double damping, uint32_t flags, int32_t step, double *cost_hist, hipStream_t stream) {
  int rc = polish_check(pp, b, damping, flags);
  if (rc) return rc;
  if (!theta || !lb || !ub) return fail(DEBYE_EINVAL, "NULL pointer");
  if (step < 0 || (cost_hist && step >= pp->steps))
    return fail(DEBYE_ERANGE, "step %d outside 0..%d", step, pp->steps - 1);
  dfit::LbfgsArgs la = polish_args(pp, b, theta, lb, ub, cost_hist);
  la.step = step;
  const int32_t M = pp->M;
  const int64_t ld = pp->ld;
  hipError_t e = dfit::launch_lbfgs_direction(la, stream);
  if (e != hipSuccess) return hip_fail(e, "lbfgs direction");
  // stage 0: the full step of every material still moving (rows 0 .. M-1 of
  // the trial arrays).  A material whose step found no acceptable trial is
  // stalled for good: its point, gradient and history stay as they were, so
  // every later step would rebuild the same trials and reject them again.
  if ((rc = fit_eval_impl(pp->p1, b, pp->trial_theta, ld, damping, flags, pp->trial_cost, nullptr, nullptr,
                          pp->trial_status, pp->stalled, stream)))
    return rc;
  if ((e = dfit::launch_lbfgs_first(la, stream)) != hipSuccess) return hip_fail(e, "lbfgs first trial");
  // stages A and B: the next ta halvings, then the rest, each only for the
  // materials the earlier stages left undecided
  debye_batch bt = *b;
  int64_t row = M;
  int32_t t_lo = 1;
  for (int stage = 0; stage < 2; ++stage) {
    const int32_t n = stage == 0 ? pp->ta : pp->tb;
    if (n == 0) continue;
    bt.cand_off = stage == 0 ? pp->off_a : pp->off_b;
    bt.n_cand = (int64_t)M * n;
    if ((rc = fit_eval_impl(stage == 0 ? pp->pA : pp->pB, &bt, pp->trial_theta + row * ld, ld, damping, flags,
                            pp->trial_cost + row, nullptr, nullptr, pp->trial_status + row, pp->done, stream)))
      return rc;
    if ((e = dfit::launch_lbfgs_select(la, t_lo, t_lo + n - 1, stream)) != hipSuccess)
      return hip_fail(e, "lbfgs select");
    row += (int64_t)M * n;
    t_lo += n;
  }
  // cost and gradient at the accepted points (the stalled materials, which
  // accepted none, are left out)
  if ((rc = fit_eval_grad_launch(pp->p1, b, pp->new_theta, pp->ld, damping, flags, nullptr, pp->new_cost, pp->new_grad,
                                 nullptr, nullptr, pp->new_status, nullptr, 0, stream, pp->stalled)))
    return rc;
  if ((e = dfit::launch_lbfgs_update(la, stream)) != hipSuccess) return hip_fail(e, "lbfgs update");
  return DEBYE_OK;
}

int debye_lbfgs_polish(debye_polish *pp, const debye_batch *b, double *theta, const double *lb, const double *ub,
                       double damping, uint32_t flags, double *cost_hist, hipStream_t stream) {
  int rc = polish_check(pp, b, damping, flags);
  if (rc) return rc;
  if (!theta || !lb || !ub) return fail(DEBYE_EINVAL, "NULL pointer");
  if (pp->steps == 0) return DEBYE_OK;
  if ((rc = debye_polish_begin(pp, b, theta, damping, flags, stream))) return rc;
  for (int32_t s = 0; s < pp->steps; ++s)
    if ((rc = debye_polish_step(pp, b, theta, lb, ub, damping, flags, s, cost_hist, stream))) return rc;
  return DEBYE_OK;
}

}  // extern "C"
