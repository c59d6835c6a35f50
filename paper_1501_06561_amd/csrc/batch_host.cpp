// Host side of the many-sketch batch (see include/fdsketch.h and
// fdsk_batch.hpp): per-sketch workspace, the round schedule of an append or
// finalize call, and the C ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fdsk_batch.hpp"
#include "fdsk_tune.hpp"
#include "fdsketch.h"

using namespace fdsk;

struct fdsk_batch {
  int S = 0;
  hipStream_t stream = nullptr;
  std::vector<fdsk_config> cfg;
  std::vector<GroupSketch> sk;     // host copy of the device descriptors
  std::vector<int> occ, cur, new0; // schedule state per sketch
  std::vector<int64_t> rows_in;
  std::vector<int32_t> rows_out;
  void* arena = nullptr;
  GroupSketch* d_sk = nullptr;
  DevStats* d_stats = nullptr;
  void* d_tasks = nullptr;         // task lists of the current call
  size_t tasks_cap = 0;
  // Appends run each size class of buffer rows as its own lock-step schedule
  // on its own stream, ordered after the caller's stream by events.
  static constexpr int kClasses = 4;
  hipStream_t lane[kClasses] = {};
  hipEvent_t ev_in = nullptr, ev_out[kClasses] = {};
  void* d_tasks_c[kClasses] = {};
  size_t tasks_cap_c[kClasses] = {};
  // The rebuild's tuned rows per workgroup per size class and precision (0
  // FP64, 1 BF16x3); a launch takes its first task's class (the rows per
  // workgroup change no result).  The Gram's tuned K slice length is each
  // sketch's own (GroupSketch::kchunk).
  int rebuild_rt[kClasses][2] = {{32, 32}, {32, 32}, {32, 32}, {32, 32}};
  bool finalized = false;
  int err = 0;
  std::string msg;
  // Stage profiling (FDSK_FLAG_PROFILE): event pairs with the launch's
  // algorithmic work, recorded on the class streams.
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  struct Mark { int stage; hipEvent_t a, b; double work; };
  std::vector<Mark> marks;
  // The captured graph of the last append call and the task lists it reads
  // (owned by the cache, so other calls cannot overwrite them).
  bool use_graph = false;
  struct GraphCache {
    bool valid = false;
    int dt = 0, cap = 0;
    std::vector<GroupIngest> hi[kClasses];
    std::vector<GroupRR> hr[kClasses];
    std::vector<size_t> oi[kClasses], orr[kClasses];
    void* d_tasks[kClasses] = {};
    size_t tasks_cap[kClasses] = {};
    hipGraph_t graph[kClasses] = {};
    hipGraphExec_t exec[kClasses] = {};
  } gc;
};

namespace {

thread_local std::string g_batch_err;

int berr(fdsk_batch* b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) {
    b->err = code;
    b->msg = buf;
  } else {
    g_batch_err = buf;
  }
  return code;
}

int rup(int x, int a) { return (x + a - 1) / a * a; }

size_t dtype_bytes(fdsk_dtype t) {
  switch (t) {
    case FDSK_F64: return 8;
    case FDSK_F32: return 4;
    case FDSK_BF16: return 2;
  }
  return 0;
}

RuleParams rule_for(const fdsk_config& c) {
  RuleParams rp{};
  rp.variant = static_cast<int>(c.variant);
  rp.l = c.l;
  int s = static_cast<int>(std::ceil(c.alpha * c.l * (1.0 - 1e-12)));
  s = std::min(std::max(s, 1), c.l);
  int r = c.l - s;
  switch (c.variant) {
    case FDSK_FD: rp.t = c.l; rp.r = 0; break;
    case FDSK_ISVD: rp.t = c.l; rp.r = c.l - 1; break;
    case FDSK_ALPHA: rp.t = c.l; rp.r = r; break;
    case FDSK_FAST_ALPHA: rp.t = r + (s + 1) / 2; rp.r = r; break;
    default: rp.t = c.l; rp.r = 0; break;   // SSD / CFD: refused by sketch_batch_create
  }
  rp.keep = rp.t - 1;
  return rp;
}

// The tasks of one call, grouped by round.
struct Plan {
  std::vector<std::vector<GroupIngest>> ing;
  std::vector<std::vector<GroupRR>> rr;
};

// Size class of a buffer (the register reduction's classes; above 208
// rows the packed-triangle head runs first).
int size_class(int m) { return m <= 64 ? 0 : (m <= 128 ? 1 : (m <= 208 ? 2 : 3)); }

// A plan's task lists flattened for upload, with each round's offsets.  The
// host vectors stay alive until the stream that copies them is synchronised.
struct Staged {
  std::vector<GroupIngest> hi;
  std::vector<GroupRR> hr;
  std::vector<size_t> oi, orr;
  GroupIngest* d_ing = nullptr;
  GroupRR* d_rr = nullptr;
};

// Sort each round's ReduceRanks in descending order of buffer rows, so that
// the longest workgroups are dispatched first (the order changes no result:
// every task works on its own sketch), and flatten the rounds into one task
// list per kind with each round's offsets.
void flatten_plan(const fdsk_batch* b, Plan& p, Staged& sg) {
  for (auto& v : p.rr)
    std::stable_sort(v.begin(), v.end(), [b](const GroupRR& x, const GroupRR& y) {
      return b->sk[x.sk].m > b->sk[y.sk].m;
    });
  size_t ni = 0, nr = 0;
  for (auto& v : p.ing) ni += v.size();
  for (auto& v : p.rr) nr += v.size();
  sg.hi.reserve(ni);
  sg.hr.reserve(nr);
  const size_t rounds = std::max(p.ing.size(), p.rr.size());
  sg.oi.assign(rounds + 1, 0);
  sg.orr.assign(rounds + 1, 0);
  for (size_t r = 0; r < rounds; ++r) {
    sg.oi[r] = sg.hi.size();
    sg.orr[r] = sg.hr.size();
    if (r < p.ing.size()) sg.hi.insert(sg.hi.end(), p.ing[r].begin(), p.ing[r].end());
    if (r < p.rr.size()) sg.hr.insert(sg.hr.end(), p.rr[r].begin(), p.rr[r].end());
  }
  sg.oi[rounds] = sg.hi.size();
  sg.orr[rounds] = sg.hr.size();
}

// Upload a flattened plan on stream st into the task buffer (grown if
// needed; callers synchronise before reusing it).
int upload_plan(fdsk_batch* b, Staged& sg, hipStream_t st, void*& d_tasks, size_t& tasks_cap) {
  const size_t ni = sg.hi.size(), nr = sg.hr.size();
  const size_t ing_bytes = (ni * sizeof(GroupIngest) + 255) / 256 * 256;
  const size_t bytes = ing_bytes + nr * sizeof(GroupRR) + 256;
  if (bytes > tasks_cap) {
    if (d_tasks) {
      hipError_t e = hipStreamSynchronize(st);
      if (e == hipSuccess) e = hipFree(d_tasks);
      d_tasks = nullptr;
      tasks_cap = 0;
      if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch tasks: %s", hipGetErrorString(e));
    }
    if (hipMalloc(&d_tasks, bytes) != hipSuccess)
      return berr(b, FDSK_ENOMEM, "batch task lists of %zu bytes", bytes);
    tasks_cap = bytes;
  }
  sg.d_ing = static_cast<GroupIngest*>(d_tasks);
  sg.d_rr = reinterpret_cast<GroupRR*>(static_cast<char*>(d_tasks) + ing_bytes);
  hipError_t e = hipSuccess;
  if (ni) e = hipMemcpyAsync(sg.d_ing, sg.hi.data(), ni * sizeof(GroupIngest), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && nr)
    e = hipMemcpyAsync(sg.d_rr, sg.hr.data(), nr * sizeof(GroupRR), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch task upload: %s", hipGetErrorString(e));
  return 0;
}

int stage_plan(fdsk_batch* b, Plan& p, hipStream_t st, void*& d_tasks, size_t& tasks_cap, Staged& sg) {
  flatten_plan(b, p, sg);
  return upload_plan(b, sg, st, d_tasks, tasks_cap);
}

hipEvent_t take_event(fdsk_batch* b) {
  hipEvent_t e = nullptr;
  if (!b->ev_pool.empty()) {
    e = b->ev_pool.back();
    b->ev_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Profiling: an event on the stream before a stage's launches (or nullptr).
hipEvent_t mark(fdsk_batch* b, hipStream_t st) {
  if (!b->profile) return nullptr;
  hipEvent_t e = take_event(b);
  if (e && hipEventRecord(e, st) != hipSuccess) return nullptr;
  return e;
}

void add_mark(fdsk_batch* b, int stage, hipEvent_t a, hipStream_t st, double work) {
  if (!a) return;
  hipEvent_t e = mark(b, st);
  if (e) b->marks.push_back({stage, a, e, work});
}

// Launch round r of a staged plan on stream st, at most `cap` sketches per
// launch.  With profiling, each stage's launches are bracketed by events and
// credited with the algorithmic work of their tasks.
hipError_t launch_round(fdsk_batch* b, const Plan& p, const Staged& sg, size_t r, int dt, int cap,
                        hipStream_t st) {
  hipError_t e = hipSuccess;
  static const std::vector<GroupIngest> empty_i;
  static const std::vector<GroupRR> empty_r;
  const auto& vi = r < p.ing.size() ? p.ing[r] : empty_i;
  const auto& vr = r < p.rr.size() ? p.rr[r] : empty_r;
  const double es = static_cast<double>(dtype_bytes(static_cast<fdsk_dtype>(dt)));
  for (size_t c0 = 0; c0 < vi.size() && e == hipSuccess; c0 += cap) {
    const int nt = static_cast<int>(std::min<size_t>(cap, vi.size() - c0));
    int max_f = 0;
    double bytes = 0.0;
    for (int t = 0; t < nt; ++t) {
      max_f = std::max(max_f, vi[c0 + t].f);
      bytes += static_cast<double>(vi[c0 + t].f) * b->sk[vi[c0 + t].sk].d * (es + 8.0);
    }
    hipEvent_t a = mark(b, st);
    e = launch_group_ingest(b->d_sk, sg.d_ing + sg.oi[r] + c0, nt, max_f, dt, st);
    add_mark(b, FDSK_STAGE_INGEST, a, st, bytes);
  }
  for (size_t c0 = 0; c0 < vr.size() && e == hipSuccess; c0 += cap) {
    const int nt = static_cast<int>(std::min<size_t>(cap, vr.size() - c0));
    int max_mp = 0, max_m = 0, max_ldc = 0, max_keep = 0, ks = 1, max_c = 0;
    bool p0 = false, p1 = false, p3 = false;   // precisions present in this launch
    double w_gram = 0, w_head = 0, w_trid = 0, w_dc = 0, w_bt = 0, w_reb = 0;
    for (int t = 0; t < nt; ++t) {
      const GroupSketch& s = b->sk[vr[c0 + t].sk];
      max_mp = std::max(max_mp, s.mp);
      max_m = std::max(max_m, s.m);
      max_ldc = std::max(max_ldc, s.ldc);
      max_keep = std::max(max_keep, s.rp.keep);
      max_c = std::max(max_c, std::min(s.m, s.l));
      p0 |= s.npass == 0;
      p1 |= s.npass == 1;
      p3 |= s.npass == 3;
      const int kc = task_kchunk(s.kchunk, s.ldc);
      ks = std::max(ks, (s.ldc + kc - 1) / kc);
      const double m = s.m, d = s.d, np = std::max(s.npass, 1);
      w_gram += np * m * (m + 1.0) * d;
      // Householder reduction: 4/3 n^3 over n columns, split between the
      // packed-triangle head (the first m - 208 columns) and the registers.
      const double hcols = std::max(0.0, m - 208.0), tail = m - hcols;
      w_head += 4.0 / 3.0 * (m * m * m - tail * tail * tail);
      w_trid += 4.0 / 3.0 * tail * tail * tail;
      w_dc += 4.0 / 3.0 * m * m * m;
      w_bt += 2.0 * m * m * std::min(s.m, s.l);
      w_reb += np * 2.0 * s.rp.keep * m * d;
    }
    const GroupRR* tt = sg.d_rr + sg.orr[r] + c0;
    const int g = size_class(b->sk[vr[c0].sk].m);
    hipEvent_t a = mark(b, st);
    if (p1 || p3) e = launch_group_gram_lowp(b->d_sk, tt, nt, max_mp, max_ldc, p1, p3, ks, -1, st);
    if (e == hipSuccess) e = launch_group_gram(b->d_sk, tt, nt, max_mp, p0, ks, -1, st);
    add_mark(b, FDSK_STAGE_GRAM, a, st, w_gram);
    hipEvent_t eig0 = mark(b, st);
    if (e == hipSuccess && max_m > 208) {
      a = mark(b, st);
      e = launch_group_tridiag_head(b->d_sk, tt, nt, max_m, st);
      add_mark(b, FDSK_STAGE_TRIDIAG_HEAD, a, st, w_head);
    }
    a = mark(b, st);
    if (e == hipSuccess) e = launch_group_tridiag(b->d_sk, tt, nt, max_m, st);
    add_mark(b, FDSK_STAGE_TRIDIAG, a, st, w_trid);
    a = mark(b, st);
    if (e == hipSuccess) e = launch_group_dc(b->d_sk, tt, nt, max_m, st);
    add_mark(b, FDSK_STAGE_DC, a, st, w_dc);
    a = mark(b, st);
    if (e == hipSuccess) e = launch_group_backtr(b->d_sk, tt, nt, max_m, max_c, st);
    add_mark(b, FDSK_STAGE_BACKTR, a, st, w_bt);
    add_mark(b, FDSK_STAGE_EIG, eig0, st, w_head + w_trid + w_dc + w_bt);
    a = mark(b, st);
    if (e == hipSuccess) e = launch_group_shrink(b->d_sk, tt, nt, st);
    add_mark(b, FDSK_STAGE_SHRINK, a, st, 0.0);
    a = mark(b, st);
    if (e == hipSuccess && p0)
      e = launch_group_rebuild(b->d_sk, tt, nt, max_ldc, max_keep, b->rebuild_rt[g][0], st);
    if (e == hipSuccess && (p1 || p3))
      e = launch_group_rebuild_lowp(b->d_sk, tt, nt, max_ldc, max_keep, p1, p3, b->rebuild_rt[g][1], st);
    add_mark(b, FDSK_STAGE_REBUILD, a, st, w_reb);
  }
  return e;
}

// Upload a plan and launch it round by round on the batch's stream, then
// synchronise it (the task buffer is reused by the next call).
int run_plan(fdsk_batch* b, Plan& p, int dt, int cap) {
  Staged sg;
  int rc = stage_plan(b, p, b->stream, b->d_tasks, b->tasks_cap, sg);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  const size_t rounds = std::max(p.ing.size(), p.rr.size());
  for (size_t r = 0; r < rounds && e == hipSuccess; ++r) e = launch_round(b, p, sg, r, dt, cap, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return 0;
}

// The class streams.  HIP maps ordinary streams onto a small per-process
// pool of hardware queues (four by default) and shares a queue between
// streams once the pool is used up; two classes on one queue run one after
// the other.  Which streams end up sharing depends on every stream the
// process created before, so the class streams are created with a CU mask
// holding every CU: such a stream gets a hardware queue of its own and
// still runs on the whole GPU.  Where that is refused, an ordinary
// non-blocking stream is used.
hipError_t create_lane(hipStream_t* st) {
  int dev = 0;
  hipDeviceProp_t p{};
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&p, dev);
  if (e == hipSuccess && p.multiProcessorCount > 0) {
    const int ncu = p.multiProcessorCount;
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (int c = 0; c < ncu; ++c) mask[c / 32] |= 1u << (c % 32);
    if (hipExtStreamCreateWithCUMask(st, static_cast<uint32_t>(mask.size()), mask.data()) == hipSuccess)
      return hipSuccess;
    (void)hipGetLastError();
  }
  return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
}

int ensure_lanes(fdsk_batch* b) {
  constexpr int K = fdsk_batch::kClasses;
  if (b->ev_in) return 0;
  hipError_t e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  for (int g = 0; g < K && e == hipSuccess; ++g) {
    e = create_lane(&b->lane[g]);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out[g], hipEventDisableTiming);
  }
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch streams: %s", hipGetErrorString(e));
  return 0;
}

template <class T>
bool same_list(const std::vector<T>& a, const std::vector<T>& b) {
  return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) == 0);
}

// Whether the cached graph launches exactly the flattened plans sg.
bool cache_matches(const fdsk_batch* b, const Staged* sg, int dt, int cap) {
  const auto& c = b->gc;
  if (!c.valid || c.dt != dt || c.cap != cap) return false;
  for (int g = 0; g < fdsk_batch::kClasses; ++g)
    if (!same_list(c.hi[g], sg[g].hi) || !same_list(c.hr[g], sg[g].hr) || !same_list(c.oi[g], sg[g].oi) ||
        !same_list(c.orr[g], sg[g].orr))
      return false;
  return true;
}

void drop_graph(fdsk_batch* b) {
  auto& c = b->gc;
  for (int g = 0; g < fdsk_batch::kClasses; ++g) {
    if (c.exec[g]) (void)hipGraphExecDestroy(c.exec[g]);
    if (c.graph[g]) (void)hipGraphDestroy(c.graph[g]);
    c.exec[g] = nullptr;
    c.graph[g] = nullptr;
  }
  c.valid = false;
}

// The cached per-class graphs launched on the class streams, after the
// caller's stream, which then waits for all of them.
hipError_t launch_graphs(fdsk_batch* b) {
  constexpr int K = fdsk_batch::kClasses;
  hipError_t e = hipEventRecord(b->ev_in, b->stream);
  for (int g = 0; g < K && e == hipSuccess; ++g)
    if (b->gc.exec[g]) {
      e = hipStreamWaitEvent(b->lane[g], b->ev_in, 0);
      if (e == hipSuccess) e = hipGraphLaunch(b->gc.exec[g], b->lane[g]);
      if (e == hipSuccess) e = hipEventRecord(b->ev_out[g], b->lane[g]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_out[g], 0);
    }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e;
}

// Enqueue every round of the class plans: each class on its own stream,
// after `origin` (event ev_in), rounds interleaved across the classes as
// they are enqueued; `origin` then waits for all of them.
hipError_t enqueue_classes(fdsk_batch* b, Plan* plans, const Staged* sg, const bool* used, size_t rounds,
                           int dt, int cap, hipStream_t origin) {
  constexpr int K = fdsk_batch::kClasses;
  hipError_t e = hipEventRecord(b->ev_in, origin);
  for (int g = 0; g < K && e == hipSuccess; ++g)
    if (used[g]) e = hipStreamWaitEvent(b->lane[g], b->ev_in, 0);
  for (size_t r = 0; r < rounds && e == hipSuccess; ++r)
    for (int g = 0; g < K && e == hipSuccess; ++g)
      if (used[g]) e = launch_round(b, plans[g], sg[g], r, dt, cap, b->lane[g]);
  for (int g = 0; g < K && e == hipSuccess; ++g)
    if (used[g]) {
      e = hipEventRecord(b->ev_out[g], b->lane[g]);
      if (e == hipSuccess) e = hipStreamWaitEvent(origin, b->ev_out[g], 0);
    }
  return e;
}

// Run one plan per size class, each on its own stream ordered after the
// caller's stream, which then waits for all of them.  Direct launches enqueue
// the rounds as they are planned.  Graph: each class's rounds are captured
// from its own stream into a graph of their own (the classes stay
// concurrent), instantiated and launched there; a call with the same
// schedule as the cached graphs replays them.  Everything is synchronised
// before returning (the host task lists and the task buffers are reused by
// the next call).
int run_class_plans(fdsk_batch* b, Plan* plans, int dt, int cap) {
  constexpr int K = fdsk_batch::kClasses;
  int rc = ensure_lanes(b);
  if (rc) return rc;
  Staged sg[K];
  size_t rounds = 0;
  bool used[K] = {};
  for (int g = 0; g < K; ++g) {
    used[g] = !plans[g].ing.empty() || !plans[g].rr.empty();
    if (!used[g]) continue;
    flatten_plan(b, plans[g], sg[g]);
    rounds = std::max(rounds, std::max(plans[g].ing.size(), plans[g].rr.size()));
  }
  hipError_t e = hipSuccess;
  const bool graph = b->use_graph && !b->profile;
  if (graph && cache_matches(b, sg, dt, cap)) {
    e = launch_graphs(b);
    if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch graph launch: %s", hipGetErrorString(e));
    return 0;
  }
  if (graph) {
    drop_graph(b);
    auto& c = b->gc;
    for (int g = 0; g < K; ++g)
      if (used[g]) {
        rc = upload_plan(b, sg[g], b->stream, c.d_tasks[g], c.tasks_cap[g]);
        if (rc) return rc;
      }
    e = hipStreamSynchronize(b->stream);     // task lists in place before any replay
    for (int g = 0; g < K && e == hipSuccess; ++g) {
      if (!used[g]) continue;
      e = hipStreamBeginCapture(b->lane[g], hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) break;
      for (size_t r = 0; r < rounds && e == hipSuccess; ++r)
        e = launch_round(b, plans[g], sg[g], r, dt, cap, b->lane[g]);
      hipGraph_t gr = nullptr;
      const hipError_t ee = hipStreamEndCapture(b->lane[g], &gr);
      if (e == hipSuccess) e = ee;
      c.graph[g] = gr;
      if (e == hipSuccess) e = hipGraphInstantiate(&c.exec[g], gr, nullptr, nullptr, 0);
    }
    if (e == hipSuccess) e = launch_graphs(b);
    if (e != hipSuccess) {
      drop_graph(b);
      return berr(b, FDSK_EDEVICE, "batch graph: %s", hipGetErrorString(e));
    }
    c.valid = true;
    c.dt = dt;
    c.cap = cap;
    for (int g = 0; g < K; ++g) {
      c.hi[g] = std::move(sg[g].hi);
      c.hr[g] = std::move(sg[g].hr);
      c.oi[g] = std::move(sg[g].oi);
      c.orr[g] = std::move(sg[g].orr);
    }
    return 0;
  }
  for (int g = 0; g < K; ++g)
    if (used[g]) {
      rc = upload_plan(b, sg[g], b->lane[g], b->d_tasks_c[g], b->tasks_cap_c[g]);
      if (rc) return rc;
    }
  e = enqueue_classes(b, plans, sg, used, rounds, dt, cap, b->stream);
  // Synchronise every class stream (the host copies above and the task
  // buffers are reused), then the caller's.
  for (int g = 0; g < K; ++g)
    if (used[g]) {
      const hipError_t es = hipStreamSynchronize(b->lane[g]);
      if (e == hipSuccess) e = es;
    }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return 0;
}

// Pick every size class's Gram K slice length and rebuild rows per
// workgroup (see fdsk_tune.hpp), per precision, on the new batch's zeroed
// workspaces: one task per sketch of the class and precision, timed over
// launches of all of them, a quarter, a sixteenth and one (the rounds of a
// call hold fewer and fewer sketches as the short streams finish).  The
// candidates write zeros into Gp, G and the second buffers.  The chosen
// slice length goes into the sketches' descriptors (uploaded by the
// caller).
hipError_t tune_batch(fdsk_batch* b) {
  constexpr int K = fdsk_batch::kClasses;
  if (tune_mode() == TUNE_OFF) return hipSuccess;
  const std::string dev = tune_device_tag();
  std::vector<GroupRR> tasks[K][2];
  for (int i = 0; i < b->S; ++i) {
    const GroupSketch& D = b->sk[i];
    tasks[size_class(D.m)][D.npass ? 1 : 0].push_back({i, 0, 0, 0, 1});
  }
  size_t total = 0;
  for (int g = 0; g < K; ++g)
    for (int q = 0; q < 2; ++q) {
      std::stable_sort(tasks[g][q].begin(), tasks[g][q].end(),
                       [b](const GroupRR& x, const GroupRR& y) { return b->sk[x.sk].m > b->sk[y.sk].m; });
      total += tasks[g][q].size();
    }
  GroupRR* d_t = nullptr;
  hipError_t e = hipMalloc(&d_t, total * sizeof(GroupRR));
  if (e != hipSuccess) return e;
  size_t off = 0;
  for (int g = 0; g < K && e == hipSuccess; ++g)
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
      const auto& v = tasks[g][q];
      if (v.empty()) continue;
      const GroupRR* tt = d_t + off;
      e = hipMemcpy(d_t + off, v.data(), v.size() * sizeof(GroupRR), hipMemcpyHostToDevice);
      off += v.size();
      if (e != hipSuccess) break;
      const int N = static_cast<int>(v.size());
      int max_mp = 0, max_ldc = 0, max_keep = 0;
      for (const auto& t : v) {
        max_mp = std::max(max_mp, b->sk[t.sk].mp);
        max_ldc = std::max(max_ldc, b->sk[t.sk].ldc);
        max_keep = std::max(max_keep, b->sk[t.sk].rp.keep);
      }
      std::vector<int> counts{N};
      for (int c : {(N + 3) / 4, (N + 15) / 16, 1})
        if (c != counts.back()) counts.push_back(c);
      const std::string key = "|p" + std::to_string(q ? 3 : 0) + "|m" + std::to_string(max_mp) + "|d" +
                              std::to_string(tune_bucket(max_ldc)) + "|n" + std::to_string(tune_bucket(N));
      hipStream_t st = b->stream;
      const int kc = tune_pick(dev + "|bgram" + key, {0, 256, 512, 1024}, 0, st, [&](int cand) {
        hipError_t ee = hipSuccess;
        for (int nt : counts) {
          int ks = 1;
          for (int j = 0; j < nt; ++j) {
            const int ldc = b->sk[v[j].sk].ldc, c = task_kchunk(cand, ldc);
            ks = std::max(ks, (ldc + c - 1) / c);
          }
          if (q && ee == hipSuccess)
            ee = launch_group_gram_lowp(b->d_sk, tt, nt, max_mp, max_ldc, false, true, ks, cand, st);
          if (ee == hipSuccess) ee = launch_group_gram(b->d_sk, tt, nt, max_mp, !q, ks, cand, st);
        }
        return ee;
      });
      for (const auto& t : v) b->sk[t.sk].kchunk = kc;
      if (max_keep > 32)
        b->rebuild_rt[g][q] = tune_pick(dev + "|brebuild" + key, {32, 64}, 32, st, [&](int rt) {
          hipError_t ee = hipSuccess;
          for (int nt : counts) {
            if (ee != hipSuccess) break;
            ee = q ? launch_group_rebuild_lowp(b->d_sk, tt, nt, max_ldc, max_keep, false, true, rt, st)
                   : launch_group_rebuild(b->d_sk, tt, nt, max_ldc, max_keep, rt, st);
          }
          return ee;
        });
    }
  const hipError_t es = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = es;
  (void)hipFree(d_t);
  return e;
}

}  // namespace

extern "C" {

const char* sketch_batch_last_error(const fdsk_batch* b) {
  return b ? b->msg.c_str() : g_batch_err.c_str();
}

int sketch_batch_create(int32_t S, const fdsk_config* cfgs, void* hip_stream, fdsk_batch** out) {
  if (!out || !cfgs || S < 1) return berr(nullptr, FDSK_EINVAL, "bad arguments");
  *out = nullptr;
  for (int i = 0; i < S; ++i) {
    const fdsk_config& c = cfgs[i];
    const int m = c.buffer_rows == 0 ? 2 * c.l : c.buffer_rows;
    if (c.d < 1 || c.d > 65536 || c.l < 1 || m < c.l)
      return berr(nullptr, FDSK_EINVAL, "sketch %d: bad sizes", i);
    if (m > kBatchMax)
      return berr(nullptr, FDSK_EUNSUPPORTED, "sketch %d: buffer rows %d > %d", i, m, kBatchMax);
    if (c.variant == FDSK_SSD || c.variant == FDSK_CFD)
      return berr(nullptr, FDSK_EUNSUPPORTED, "SSD and CFD run on single sketches only");
    if (c.variant < FDSK_FD || c.variant > FDSK_FAST_ALPHA) return berr(nullptr, FDSK_EINVAL, "bad variant");
    if ((c.variant == FDSK_ALPHA || c.variant == FDSK_FAST_ALPHA) && !(c.alpha > 0.0 && c.alpha <= 1.0))
      return berr(nullptr, FDSK_EINVAL, "sketch %d: alpha must lie in (0, 1]", i);
    if (c.precision == FDSK_P_FP8X3)
      return berr(nullptr, FDSK_EUNSUPPORTED, "sketch %d: the FP8 Gram is single-sketch only", i);
    if (c.precision == FDSK_P_BF16)
      return berr(nullptr, FDSK_EUNSUPPORTED,
                  "sketch %d: single-pass BF16 is not a sketching precision (use FDSK_P_BF16X3)", i);
    if (c.precision != FDSK_P_FP64 && c.precision != FDSK_P_BF16X3)
      return berr(nullptr, FDSK_EINVAL, "sketch %d: unknown precision", i);
    if (c.flags & ~(FDSK_FLAG_PROFILE | FDSK_FLAG_GRAPH))
      return berr(nullptr, FDSK_EUNSUPPORTED, "sketch %d: batched sketches take only the PROFILE and GRAPH flags",
                  i);
    if (c.flags != cfgs[0].flags)
      return berr(nullptr, FDSK_EINVAL, "sketch %d: every sketch of a batch takes the same flags", i);
  }
  fdsk_batch* b = new fdsk_batch;
  b->S = S;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->profile = (cfgs[0].flags & FDSK_FLAG_PROFILE) != 0;
  b->use_graph = (cfgs[0].flags & FDSK_FLAG_GRAPH) != 0;
  b->cfg.assign(cfgs, cfgs + S);
  b->sk.resize(S);
  b->occ.assign(S, 0);
  b->cur.assign(S, 0);
  b->new0.assign(S, 0);
  b->rows_in.assign(S, 0);
  b->rows_out.assign(S, 0);
  // One arena: every sketch's buffers, then the descriptors and statistics.
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  constexpr int NB = 12;   // C0 C1 Gp G W V Ut S1 S2 lam rownorm bf16 halves (of C0, C1, then Ut)
  std::vector<size_t> o(static_cast<size_t>(S) * NB);
  for (int i = 0; i < S; ++i) {
    const fdsk_config& c = cfgs[i];
    GroupSketch& D = b->sk[i];
    std::memset(&D, 0, sizeof D);
    D.d = static_cast<int>(c.d);
    D.l = c.l;
    D.m = c.buffer_rows == 0 ? 2 * c.l : c.buffer_rows;
    D.mp = rup(D.m, 32);
    D.ldc = rup(D.d, 64);
    D.rp = rule_for(c);
    D.npass = c.precision == FDSK_P_BF16 ? 1 : (c.precision == FDSK_P_BF16X3 ? 3 : 0);
    const size_t cb = static_cast<size_t>(D.mp) * D.ldc * 8, g = static_cast<size_t>(D.mp) * D.mp * 8;
    size_t* q = &o[static_cast<size_t>(i) * NB];
    q[0] = take(cb);
    q[1] = take(cb);
    q[2] = take(g * gp_parts(D.ldc));
    for (int k = 3; k < 9; ++k) q[k] = take(g);
    q[9] = take(static_cast<size_t>(D.mp) * 8);
    q[10] = take(static_cast<size_t>(D.mp) * 8);
    q[11] = take(D.npass > 0 ? 2 * bf16_workspace_bytes(D.mp, D.ldc) +
                                   4 * static_cast<size_t>(D.mp) * D.mp : 0);
  }
  const size_t oDesc = take(sizeof(GroupSketch) * S), oStats = take(sizeof(DevStats) * S);
  hipError_t e = hipMalloc(&b->arena, off);
  if (e != hipSuccess) {
    delete b;
    return berr(nullptr, FDSK_ENOMEM, "batch workspace of %zu bytes: %s", off, hipGetErrorString(e));
  }
  char* a = static_cast<char*>(b->arena);
  b->d_sk = reinterpret_cast<GroupSketch*>(a + oDesc);
  b->d_stats = reinterpret_cast<DevStats*>(a + oStats);
  for (int i = 0; i < S; ++i) {
    GroupSketch& D = b->sk[i];
    const size_t* q = &o[static_cast<size_t>(i) * NB];
    double** f[9] = {&D.C0, &D.C1, &D.Gp, &D.G, &D.W, &D.V, &D.Ut, &D.S1, &D.S2};
    for (int k = 0; k < 9; ++k) *f[k] = reinterpret_cast<double*>(a + q[k]);
    D.lam = reinterpret_cast<double*>(a + q[9]);
    D.rownorm = reinterpret_cast<double*>(a + q[10]);
    D.bh0 = D.npass > 0 ? reinterpret_cast<uint16_t*>(a + q[11]) : nullptr;
    D.bh1 = D.npass > 0 ? D.bh0 + bf16_workspace_bytes(D.mp, D.ldc) / sizeof(uint16_t) : nullptr;
    D.uh = D.npass > 0 ? D.bh1 + bf16_workspace_bytes(D.mp, D.ldc) / sizeof(uint16_t) : nullptr;
    D.st = b->d_stats + i;
  }
  e = hipMemsetAsync(b->arena, 0, off, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_sk, b->sk.data(), sizeof(GroupSketch) * S, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = tune_batch(b);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_sk, b->sk.data(), sizeof(GroupSketch) * S, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    (void)hipFree(b->arena);
    delete b;
    return berr(nullptr, FDSK_EDEVICE, "batch init: %s", hipGetErrorString(e));
  }
  *out = b;
  return 0;
}

int sketch_batch_append(fdsk_batch* b, const void* const* rows, const int64_t* n_rows,
                        const int64_t* strides, fdsk_dtype dtype, fdsk_mem mem, int32_t grid_size) {
  if (!b) return berr(nullptr, FDSK_EINVAL, "null batch");
  if (b->err) return b->err;
  if (b->finalized) return berr(b, FDSK_ESTATE, "append after finalize");
  if (!rows || !n_rows || !strides) return berr(b, FDSK_EINVAL, "null argument");
  if (mem != FDSK_MEM_DEVICE && mem != FDSK_MEM_HOST) return berr(b, FDSK_EINVAL, "bad mem kind");
  const size_t es = dtype_bytes(dtype);
  if (es == 0) return berr(b, FDSK_EINVAL, "bad dtype");
  if (grid_size < 0) return berr(b, FDSK_EINVAL, "grid_size < 0");
  for (int i = 0; i < b->S; ++i) {
    if (n_rows[i] < 0) return berr(b, FDSK_EINVAL, "sketch %d: n_rows < 0", i);
    if (n_rows[i] > 0 && (!rows[i] || strides[i] < b->sk[i].d))
      return berr(b, FDSK_EINVAL, "sketch %d: bad rows or stride", i);
  }
  // Host rows: every sketch's rows of the call packed into one device
  // buffer (leading dimension d_i), then the device path.
  std::vector<const void*> drows(rows, rows + b->S);
  std::vector<int64_t> dstrides(strides, strides + b->S);
  void* stage = nullptr;
  if (mem == FDSK_MEM_HOST) {
    size_t total = 0;
    for (int i = 0; i < b->S; ++i) total += static_cast<size_t>(n_rows[i]) * b->sk[i].d * es;
    if (total > 0) {
      if (hipMalloc(&stage, total) != hipSuccess)
        return berr(b, FDSK_ENOMEM, "staging %zu bytes of host rows", total);
      size_t off = 0;
      hipError_t e = hipSuccess;
      for (int i = 0; i < b->S && e == hipSuccess; ++i) {
        if (n_rows[i] == 0) continue;
        const size_t rb = static_cast<size_t>(b->sk[i].d) * es;
        char* dst = static_cast<char*>(stage) + off;
        e = hipMemcpy2DAsync(dst, rb, rows[i], strides[i] * es, rb, n_rows[i], hipMemcpyHostToDevice, b->stream);
        drows[i] = dst;
        dstrides[i] = b->sk[i].d;
        off += rb * n_rows[i];
      }
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
      if (e != hipSuccess) {
        (void)hipFree(stage);
        return berr(b, FDSK_EDEVICE, "staging host rows: %s", hipGetErrorString(e));
      }
    }
  }
  // Lay out every sketch's ingests and ReduceRanks of this call by round,
  // one plan per size class.
  Plan plans[fdsk_batch::kClasses];
  for (int i = 0; i < b->S; ++i) {
    const GroupSketch& D = b->sk[i];
    Plan& p = plans[size_class(D.m)];
    int64_t pos = 0;
    size_t r = 0;
    long last_rr = -1;               // round of this call's last ReduceRank of sketch i
    while (pos < n_rows[i]) {
      const int f = static_cast<int>(std::min<int64_t>(D.m - b->occ[i], n_rows[i] - pos));
      GroupIngest t;
      t.src = static_cast<const char*>(drows[i]) + pos * dstrides[i] * static_cast<int64_t>(es);
      t.stride = dstrides[i];
      t.sk = i;
      t.f = f;
      t.row0 = b->occ[i];
      t.cur = b->cur[i];
      // Rows that fill the buffer are consumed by the ReduceRank that
      // follows in this call.
      t.w64 = (D.npass == 0 || b->occ[i] + f < D.m) ? 1 : 0;
      t.pad = 0;
      if (p.ing.size() <= r) p.ing.resize(r + 1);
      p.ing[r].push_back(t);
      b->occ[i] += f;
      pos += f;
      if (b->occ[i] < D.m) break;
      if (p.rr.size() <= r) p.rr.resize(r + 1);
      p.rr[r].push_back(GroupRR{i, b->cur[i], b->new0[i], D.m, D.npass == 0 ? 1 : 0});
      last_rr = static_cast<long>(r);
      b->cur[i] ^= 1;
      b->occ[i] = D.rp.keep;
      b->new0[i] = D.rp.keep;
      ++r;
    }
    // The last ReduceRank's rows may be copied out by finalize.
    if (last_rr >= 0) p.rr[last_rr].back().w64 = 1;
    b->rows_in[i] += n_rows[i];
  }
  const int rc = run_class_plans(b, plans, static_cast<int>(dtype), grid_size > 0 ? grid_size : b->S);
  if (stage) (void)hipFree(stage);   // run_class_plans synchronised every stream
  return rc;
}

int sketch_batch_finalize(fdsk_batch* b, void* const* B_out, const int64_t* ldb, fdsk_dtype out_dtype,
                          fdsk_mem mem, int32_t grid_size, int32_t* rows_out) {
  if (!b) return berr(nullptr, FDSK_EINVAL, "null batch");
  if (b->err) return b->err;
  if (b->finalized) return berr(b, FDSK_ESTATE, "finalize called twice");
  if (!B_out || !ldb) return berr(b, FDSK_EINVAL, "null argument");
  if (mem != FDSK_MEM_DEVICE) return berr(b, FDSK_EUNSUPPORTED, "batched outputs must be on the device");
  if (out_dtype != FDSK_F64 && out_dtype != FDSK_F32) return berr(b, FDSK_EINVAL, "output dtype");
  if (grid_size < 0) return berr(b, FDSK_EINVAL, "grid_size < 0");
  for (int i = 0; i < b->S; ++i)
    if (!B_out[i] || ldb[i] < b->sk[i].d) return berr(b, FDSK_EINVAL, "sketch %d: bad output", i);
  // Sketches holding more than l rows: zero the free rows and reduce once
  // more; the others: account for the rows appended since their last
  // ReduceRank.
  std::vector<GroupSpan> spans;
  int nzero = 0;
  Plan p;
  p.rr.resize(1);
  for (int i = 0; i < b->S; ++i) {
    const GroupSketch& D = b->sk[i];
    if (b->occ[i] > D.l && b->occ[i] < D.m) {
      spans.push_back(GroupSpan{i, b->cur[i], b->occ[i], D.m});
      ++nzero;
    }
  }
  for (int i = 0; i < b->S; ++i) {
    const GroupSketch& D = b->sk[i];
    if (b->occ[i] > D.l) {
      p.rr[0].push_back(GroupRR{i, b->cur[i], b->new0[i], b->occ[i], 1});
      b->cur[i] ^= 1;
      b->occ[i] = D.rp.keep;
      b->new0[i] = D.rp.keep;
    } else if (b->occ[i] > b->new0[i]) {
      spans.push_back(GroupSpan{i, b->cur[i], b->new0[i], b->occ[i]});
      b->new0[i] = b->occ[i];
    }
  }
  void* d_span = nullptr;
  hipError_t e = hipSuccess;
  if (!spans.empty()) {
    e = hipMalloc(&d_span, spans.size() * sizeof(GroupSpan));
    if (e != hipSuccess) return berr(b, FDSK_ENOMEM, "batch finalize spans");
    e = hipMemcpyAsync(d_span, spans.data(), spans.size() * sizeof(GroupSpan), hipMemcpyHostToDevice,
                       b->stream);
    GroupSpan* ds = static_cast<GroupSpan*>(d_span);
    if (e == hipSuccess) e = launch_group_zero(b->d_sk, ds, nzero, b->stream);
    if (e == hipSuccess)
      e = launch_group_pending(b->d_sk, ds + nzero, static_cast<int>(spans.size()) - nzero, b->stream);
  }
  int rc = 0;
  if (e == hipSuccess) rc = run_plan(b, p, FDSK_F64, grid_size > 0 ? grid_size : b->S);
  if (d_span) (void)hipFree(d_span);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch finalize: %s", hipGetErrorString(e));
  if (rc) return rc;
  for (int i = 0; i < b->S && e == hipSuccess; ++i) {
    const GroupSketch& D = b->sk[i];
    b->rows_out[i] = std::min(b->occ[i], D.l);
    e = launch_copy_out(b->cur[i] ? D.C1 : D.C0, D.ldc, b->rows_out[i], D.l, D.d, B_out[i], ldb[i],
                        static_cast<int>(out_dtype), b->stream);
  }
  std::vector<DevStats> ds(b->S);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ds.data(), b->d_stats, sizeof(DevStats) * b->S, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch finalize: %s", hipGetErrorString(e));
  b->finalized = true;
  int bad = -1;
  for (int i = 0; i < b->S; ++i) {
    if (rows_out) rows_out[i] = b->rows_out[i];
    if (ds[i].nonfinite && bad < 0) bad = i;
  }
  if (bad >= 0) return berr(b, FDSK_ENONFINITE, "sketch %d: a NaN or Inf reached the sketch", bad);
  return 0;
}

int sketch_batch_stats(const fdsk_batch* cb, int32_t index, fdsk_report* out) {
  fdsk_batch* b = const_cast<fdsk_batch*>(cb);
  if (!b || !out || index < 0 || index >= b->S) return berr(b, FDSK_EINVAL, "bad arguments");
  DevStats h{};
  hipError_t e = hipMemcpyAsync(&h, b->d_stats + index, sizeof h, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch stats: %s", hipGetErrorString(e));
  std::memset(out, 0, sizeof *out);
  out->fro2_A = h.fro2A;
  out->delta_sum = h.Delta;
  out->shrink_total = h.Stot;
  out->n_rows = b->rows_in[index];
  out->n_reduce = h.n_rr;
  out->rows_out = b->rows_out[index];
  out->eig_unconverged = h.eig_unconv;
  out->eig_sweeps = static_cast<int64_t>(h.eig_sweeps);
  out->cov_err = out->proj_err_k = out->proj_full_over_fro2 = std::nan("");
  out->fro2_B = out->lambda_max = out->lambda_min = std::nan("");
  return 0;
}

int sketch_batch_reset(fdsk_batch* b) {
  if (!b) return berr(nullptr, FDSK_EINVAL, "null batch");
  // Rows beyond a sketch's occupancy are never read before they are written
  // again (a reduction runs on a full buffer; finalize zeroes the free rows
  // first), so only the accumulators and the host schedule start over.
  hipError_t e = hipMemsetAsync(b->d_stats, 0, sizeof(DevStats) * b->S, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch reset: %s", hipGetErrorString(e));
  std::fill(b->occ.begin(), b->occ.end(), 0);
  std::fill(b->cur.begin(), b->cur.end(), 0);
  std::fill(b->new0.begin(), b->new0.end(), 0);
  std::fill(b->rows_in.begin(), b->rows_in.end(), 0);
  std::fill(b->rows_out.begin(), b->rows_out.end(), 0);
  b->finalized = false;
  b->err = 0;
  b->msg.clear();
  for (auto& mk : b->marks) {
    b->ev_pool.push_back(mk.a);
    b->ev_pool.push_back(mk.b);
  }
  b->marks.clear();
  std::sort(b->ev_pool.begin(), b->ev_pool.end());
  b->ev_pool.erase(std::unique(b->ev_pool.begin(), b->ev_pool.end()), b->ev_pool.end());
  return 0;
}

int sketch_batch_profile(fdsk_batch* b, fdsk_profile* out) {
  if (!b || !out) return berr(b, FDSK_EINVAL, "null argument");
  hipError_t e = hipStreamSynchronize(b->stream);
  for (int g = 0; g < fdsk_batch::kClasses && e == hipSuccess; ++g)
    if (b->lane[g]) e = hipStreamSynchronize(b->lane[g]);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch profile: %s", hipGetErrorString(e));
  std::memset(out, 0, sizeof *out);
  for (auto& mk : b->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, mk.a, mk.b) == hipSuccess) {
      out->ms[mk.stage] += ms;
      out->launches[mk.stage] += 1;
      out->work[mk.stage] += mk.work;
    }
  }
  return 0;
}

void sketch_batch_destroy(fdsk_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (int g = 0; g < fdsk_batch::kClasses; ++g) {
    if (b->lane[g]) {
      (void)hipStreamSynchronize(b->lane[g]);
      (void)hipStreamDestroy(b->lane[g]);
    }
    if (b->ev_out[g]) (void)hipEventDestroy(b->ev_out[g]);
    if (b->d_tasks_c[g]) (void)hipFree(b->d_tasks_c[g]);
    if (b->gc.d_tasks[g]) (void)hipFree(b->gc.d_tasks[g]);
  }
  for (auto& mk : b->marks) {
    b->ev_pool.push_back(mk.a);
    b->ev_pool.push_back(mk.b);
  }
  std::sort(b->ev_pool.begin(), b->ev_pool.end());
  b->ev_pool.erase(std::unique(b->ev_pool.begin(), b->ev_pool.end()), b->ev_pool.end());
  for (auto e : b->ev_pool) (void)hipEventDestroy(e);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->d_tasks) (void)hipFree(b->d_tasks);
  if (b->arena) (void)hipFree(b->arena);
  delete b;
}

}  // extern "C"
