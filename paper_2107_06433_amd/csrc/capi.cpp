// Host runtime of the C ABI declared in include/wmd.h: argument validation,
// workspace layout, corpus preparation and the launch sequence of a query.
#include "wmd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <list>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "wmd_internal.h"

using namespace wmd;

namespace {

thread_local std::string g_err;

wmd_status fail(wmd_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define WMD_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(WMD_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

template <class T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

bool mul_ok(size_t a, size_t b, size_t* out) {
  if (a && b > SIZE_MAX / a) return false;
  *out = a * b;
  return true;
}

}  // namespace

// Query workspace of wmd_query_static (see wmd.h): a device array of fixed
// size.  Every GPU the library runs on holds its own copy until the process
// ends.  Host code never uses this name as an address: scratch_address()
// resolves the copy of the current device with hipGetSymbolAddress, and that
// pointer is what the kernels receive.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the scratch array on device `dev`, which must be current;
// resolved once per device.
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

// One Sinkhorn launch of a query's plan: the length buckets that one-wave
// items hold merged into one launch, or one bucket with a shape of its own.
// Plans depend on the padded query width S only through the kernel shape, so
// queries whose units have equal keys share one launch (SinkQuerySet).
struct SinkUnit {
  bool merged = false;
  MergePlan plan;                 // merged: shape, member buckets (longest first), row bodies
  int nb = 0;                     // buckets in the unit
  int bk[kMergeMax] = {};         // their indices, in launch order
  SinkConfig cfg{};               // one bucket: its shape
  double nzb = 0.0, ndd = 0.0;    // entries and documents the unit covers
  std::string name;
  std::vector<int64_t> key;
};

struct wmd_corpus {
  int device = 0;
  void* scratch = nullptr;  // this device's copy of the static query scratch
  int64_t V = 0, N = 0, nnz = 0, U = 0;
  int d = 0, dp = 0;
  const float* emb = nullptr;
  const int64_t* doc_ptr = nullptr;
  CorpusLayout L{};
  void* ws = nullptr;
  // documents grouped by length bucket, then the NaN-scoring (empty) ones
  int64_t bucket_off[kNumBuckets + 1] = {};
  int64_t empty_off = 0, empty_count = 0;
  int64_t bucket_nnz[kNumBuckets] = {};  // entries of the documents in each bucket
  int* docs() const { return at<int>(ws, L.docs); }

  // per-launch timing (wmd_set_timing); timing_mu serialises timed calls
  struct Rec { std::string name; size_t ev; double flops, bytes; int query, S, cap, ndocs; };
  std::atomic<bool> timing{false};
  std::vector<hipEvent_t> events;  // pool, reused; pairs (start, end)
  std::vector<Rec> recs;
  std::mutex timing_mu;

  // Side streams (default priority) that run the independent Sinkhorn
  // launches of a call concurrently, forked from and joined back into the
  // caller's stream with events.  Each caller stream gets a set of its own,
  // so calls on different streams never queue behind each other here; a call
  // holds its set's lock while it enqueues (through the end of a capture).
  static constexpr int kSide = 4;
  struct SideSet {
    hipStream_t side[kSide] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kSide] = {};
    std::mutex mu;
    ~SideSet() {
      for (int i = 0; i < kSide; ++i) {
        if (side[i]) (void)hipStreamDestroy(side[i]);
        if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
      }
      if (fork_ev) (void)hipEventDestroy(fork_ev);
    }
  };
  static constexpr size_t kMaxSideSets = 16;  // further caller streams run without forking
  std::map<hipStream_t, std::unique_ptr<SideSet>> sides;
  std::mutex sides_mu;

  // captured launch sequences (WMD_QUERY_GRAPH), most recent first
  struct GraphEntry { std::vector<uint64_t> key; hipGraph_t graph; hipGraphExec_t exec; };
  std::list<GraphEntry> graphs;
  std::mutex graph_mu;
  static constexpr size_t kMaxGraphs = 128;

  // launch planning: merge mode, Sinkhorn shapes pinned per (padded query
  // width, bucket capacity), and the per-width plans derived from them
  std::mutex cfg_mu;
  int merge = WMD_MERGE_ALL;
  std::map<std::pair<int, int>, SinkConfig> pinned;
  std::map<int, std::shared_ptr<const std::vector<SinkUnit>>> plans;

  ~wmd_corpus() {
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr size_t kMaxTimedLaunches = 1000000;

// Launch tag of a timing record: query (the first one of a multi-query
// launch), padded width S, bucket capacity (0: several buckets) and documents.
struct Tag { int query = -1, S = 0, cap = 0, ndocs = 0; };

// Launches `fn` on stream s; in a timed call (the caller holds timing_mu),
// brackets it with two events and records its algorithmic work.
template <class F>
hipError_t timed_launch(wmd_corpus* c, bool timed, hipStream_t s, const std::string& name, double flops,
                        double bytes, const Tag& tag, F&& fn) {
  if (!timed || c->recs.size() >= kMaxTimedLaunches) return fn();
  const size_t ev = 2 * c->recs.size();
  while (c->events.size() < ev + 2) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    c->events.push_back(e);
  }
  hipError_t err = hipEventRecord(c->events[ev], s);
  if (err != hipSuccess) return err;
  err = fn();
  if (err != hipSuccess) return err;
  err = hipEventRecord(c->events[ev + 1], s);
  if (err != hipSuccess) return err;
  c->recs.push_back({name, ev, flops, bytes, tag.query, tag.S, tag.cap, tag.ndocs});
  return hipSuccess;
}

// The side-stream set of caller stream s (created on first use), or null
// when the corpus already serves its maximum number of caller streams.
wmd_status side_set(wmd_corpus* c, hipStream_t s, wmd_corpus::SideSet** out) {
  *out = nullptr;
  std::lock_guard<std::mutex> lock(c->sides_mu);
  auto it = c->sides.find(s);
  if (it != c->sides.end()) {
    *out = it->second.get();
    return WMD_OK;
  }
  if (c->sides.size() >= wmd_corpus::kMaxSideSets) return WMD_OK;
  std::unique_ptr<wmd_corpus::SideSet> set(new (std::nothrow) wmd_corpus::SideSet());
  if (!set) return fail(WMD_ERR_INVALID_ARGUMENT, "out of host memory");
  for (int i = 0; i < wmd_corpus::kSide; ++i) {
    WMD_HIP(hipStreamCreateWithFlags(&set->side[i], hipStreamNonBlocking));
    WMD_HIP(hipEventCreateWithFlags(&set->join_ev[i], hipEventDisableTiming));
  }
  WMD_HIP(hipEventCreateWithFlags(&set->fork_ev, hipEventDisableTiming));
  *out = set.get();
  c->sides.emplace(s, std::move(set));
  return WMD_OK;
}

}  // namespace

extern "C" {

const char* wmd_last_error(void) { return g_err.c_str(); }

size_t wmd_corpus_workspace_bytes(int64_t V, int32_t d, int64_t N, int64_t nnz) {
  if (V < 1 || d < 1 || d > 4096 || N < 1 || nnz < 0) return 0;
  size_t t;
  if (!mul_ok((size_t)V, (size_t)padded_dim(d) * 6, &t)) return 0;
  return CorpusLayout::make(V, d, N, nnz).total;
}

wmd_status wmd_create_corpus(const wmd_corpus_desc* desc, void* stream, wmd_corpus** out) {
  g_err.clear();
  if (!out) return fail(WMD_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(WMD_ERR_INVALID_ARGUMENT, "desc is NULL");
  const wmd_corpus_desc& D = *desc;
  if (D.V < 1 || D.V > INT32_MAX - 1) return fail(WMD_ERR_INVALID_ARGUMENT, "V must be in [1, 2^31-2]");
  if (D.d < 1 || D.d > 4096) return fail(WMD_ERR_INVALID_ARGUMENT, "d must be in [1, 4096]");
  if (D.N < 1 || D.N > INT32_MAX) return fail(WMD_ERR_INVALID_ARGUMENT, "N must be in [1, 2^31-1]");
  if (D.nnz < 0) return fail(WMD_ERR_INVALID_ARGUMENT, "nnz must be >= 0");
  if (!D.emb || !D.doc_ptr || (D.nnz > 0 && (!D.word_ids || !D.weights)) || !D.workspace)
    return fail(WMD_ERR_INVALID_ARGUMENT, "NULL device pointer in corpus descriptor");
  const size_t need = wmd_corpus_workspace_bytes(D.V, D.d, D.N, D.nnz);
  if (need == 0) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus sizes overflow");
  if (D.workspace_bytes < need)
    return fail(WMD_ERR_WORKSPACE_TOO_SMALL, "corpus workspace needs " + std::to_string(need) + " bytes");
  if ((uintptr_t)D.workspace % 256 != 0) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus workspace must be 256-byte aligned");

  hipStream_t s = static_cast<hipStream_t>(stream);
  // doc_ptr is needed on the host for validation and the length buckets
  std::vector<int64_t> ptr((size_t)D.N + 1);
  WMD_HIP(hipMemcpyAsync(ptr.data(), D.doc_ptr, sizeof(int64_t) * ptr.size(), hipMemcpyDeviceToHost, s));
  WMD_HIP(hipStreamSynchronize(s));
  if (ptr[0] != 0 || ptr[(size_t)D.N] != D.nnz)
    return fail(WMD_ERR_INVALID_ARGUMENT, "doc_ptr must start at 0 and end at nnz");
  for (int64_t k = 0; k < D.N; ++k) {
    const int64_t len = ptr[(size_t)k + 1] - ptr[(size_t)k];
    if (len < 0) return fail(WMD_ERR_INVALID_ARGUMENT, "doc_ptr must be non-decreasing");
    if (len > kMaxDocLen)
      return fail(WMD_ERR_NOT_SUPPORTED, "document " + std::to_string(k) + " has more than 4096 entries");
  }

  std::unique_ptr<wmd_corpus> c(new (std::nothrow) wmd_corpus());
  if (!c) return fail(WMD_ERR_INVALID_ARGUMENT, "out of host memory");
  WMD_HIP(hipGetDevice(&c->device));
  WMD_HIP(scratch_address(c->device, &c->scratch));
  c->V = D.V; c->N = D.N; c->nnz = D.nnz; c->d = D.d; c->dp = padded_dim(D.d);
  c->emb = D.emb; c->doc_ptr = D.doc_ptr;
  c->L = CorpusLayout::make(D.V, D.d, D.N, D.nnz);
  c->ws = D.workspace;
  const CorpusLayout& L = c->L;
  void* ws = D.workspace;

  int* err = at<int>(ws, L.err);
  int* map = at<int>(ws, L.map);
  WMD_HIP(launch_fill_i32(err, 64, 0, s));
  WMD_HIP(launch_fill_i32(map, D.V + 1, D.compact_vocab ? 0 : 1, s));
  if (D.nnz > 0) WMD_HIP(launch_prep_entries(D.word_ids, D.weights, D.nnz, D.V, D.compact_vocab ? map : at<int>(ws, L.used), err, s));
  int herr = 0;
  WMD_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  WMD_HIP(hipStreamSynchronize(s));
  if (herr & 1) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus word id outside [0, V)");
  if (herr & 2) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus weight negative or not finite");

  WMD_HIP(launch_prep_docs(D.doc_ptr, D.weights, D.N, at<float>(ws, L.wn), at<int>(ws, L.dpos), s));
  WMD_HIP(launch_prep_scan(map, D.V, s));
  WMD_HIP(launch_prep_compact(map, D.V, at<int>(ws, L.used), D.word_ids, D.nnz, at<int>(ws, L.wl), s));
  int U = 0;
  WMD_HIP(hipMemcpyAsync(&U, map + D.V, sizeof(int), hipMemcpyDeviceToHost, s));
  WMD_HIP(hipStreamSynchronize(s));
  c->U = U;
  if (U > 0)
    WMD_HIP(launch_prep_emb(D.emb, D.d, c->dp, at<int>(ws, L.used), U, at<float>(ws, L.e32),
                            at<uint16_t>(ws, L.e16), at<float>(ws, L.en), s));

  // length buckets; documents with no positive weight go last and score NaN
  std::vector<int> dpos((size_t)D.N);
  WMD_HIP(hipMemcpyAsync(dpos.data(), at<int>(ws, L.dpos), sizeof(int) * dpos.size(), hipMemcpyDeviceToHost, s));
  WMD_HIP(hipStreamSynchronize(s));
  std::vector<std::vector<int>> lists(kNumBuckets + 1);
  for (int64_t k = 0; k < D.N; ++k) {
    const int64_t len = ptr[(size_t)k + 1] - ptr[(size_t)k];
    if (len == 0 || !dpos[(size_t)k]) { lists[kNumBuckets].push_back((int)k); continue; }
    int b = 0;
    while (kBucketCap[b] < len) ++b;
    lists[b].push_back((int)k);
    c->bucket_nnz[b] += len;
  }
  // longest documents first inside a bucket (ties by id): the items that take
  // longest start first, and the two documents of a half-wave item have
  // similar lengths, so a smaller row body fits both more often
  for (int b = 0; b < kNumBuckets; ++b)
    std::stable_sort(lists[b].begin(), lists[b].end(), [&](int x, int y) {
      return ptr[(size_t)x + 1] - ptr[(size_t)x] > ptr[(size_t)y + 1] - ptr[(size_t)y];
    });
  std::vector<int> flat;
  flat.reserve((size_t)D.N);
  for (int b = 0; b <= kNumBuckets; ++b) {
    if (b < kNumBuckets) c->bucket_off[b] = (int64_t)flat.size();
    else c->empty_off = (int64_t)flat.size();
    flat.insert(flat.end(), lists[b].begin(), lists[b].end());
  }
  c->bucket_off[kNumBuckets] = c->empty_off;
  c->empty_count = (int64_t)lists[kNumBuckets].size();
  // per-document records in the same order: first entry (lo, hi), length, id
  std::vector<int4> rec(flat.size());
  for (size_t i = 0; i < flat.size(); ++i) {
    const int k = flat[i];
    const int64_t b0 = ptr[(size_t)k];
    rec[i] = make_int4((int)(uint32_t)(b0 & 0xffffffff), (int)(b0 >> 32), (int)(ptr[(size_t)k + 1] - b0), k);
  }
  WMD_HIP(hipMemcpyAsync(c->docs(), flat.data(), sizeof(int) * flat.size(), hipMemcpyHostToDevice, s));
  WMD_HIP(hipMemcpyAsync(at<int4>(ws, L.drec), rec.data(), sizeof(int4) * rec.size(), hipMemcpyHostToDevice, s));
  WMD_HIP(hipStreamSynchronize(s));
  *out = c.release();
  return WMD_OK;
}

wmd_status wmd_get_corpus_info(const wmd_corpus* c, wmd_corpus_info* info) {
  g_err.clear();
  if (!c || !info) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->V = c->V; info->N = c->N; info->nnz = c->nnz; info->d = c->d; info->d_padded = c->dp;
  info->U = c->U; info->empty_docs = c->empty_count; info->n_buckets = kNumBuckets;
  for (int b = 0; b < kNumBuckets; ++b) {
    info->bucket_docs[b] = c->bucket_off[b + 1] - c->bucket_off[b];
    info->bucket_cap[b] = kBucketCap[b];
  }
  return WMD_OK;
}

wmd_status wmd_destroy(wmd_corpus* c) {
  g_err.clear();
  delete c;
  return WMD_OK;
}

}  // extern "C"

namespace {

struct QueryPlan {
  int B = 0;
  int64_t C = 0;
  std::vector<int64_t> col0, S;
};

wmd_status plan_query(const wmd_corpus* c, int32_t B, const int64_t* qp, QueryPlan* plan) {
  if (!c) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus is NULL");
  if (B < 1) return fail(WMD_ERR_INVALID_ARGUMENT, "B must be >= 1");
  if (!qp) return fail(WMD_ERR_INVALID_ARGUMENT, "q_ptr_host is NULL");
  if (qp[0] != 0) return fail(WMD_ERR_INVALID_ARGUMENT, "q_ptr must start at 0");
  plan->B = B;
  plan->col0.resize((size_t)B);
  plan->S.resize((size_t)B);
  int64_t C = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = qp[b + 1] - qp[b];
    if (n < 1) return fail(WMD_ERR_INVALID_ARGUMENT, "query " + std::to_string(b) + " has no entries");
    if (n > kMaxQueryLen)
      return fail(WMD_ERR_NOT_SUPPORTED, "query " + std::to_string(b) + " has more than 2048 entries");
    plan->col0[(size_t)b] = C;
    plan->S[(size_t)b] = round4(n);
    C += round4(n);
  }
  if (C > INT32_MAX / 2) return fail(WMD_ERR_NOT_SUPPORTED, "too many query words in one call");
  plan->C = C;
  return WMD_OK;
}

QueryLayout layout_for(const wmd_corpus* c, const QueryPlan& p, int schedule) {
  const bool need_u = schedule == WMD_SCHEDULE_PER_ITERATION || schedule == WMD_SCHEDULE_UNFUSED;
  const bool need_w = schedule == WMD_SCHEDULE_UNFUSED;
  return QueryLayout::make(p.B, p.C, c->U, c->dp, c->N, c->nnz, need_u, need_w);
}

}  // namespace

extern "C" {

size_t wmd_query_workspace_bytes(const wmd_corpus* c, int32_t B, const int64_t* q_ptr_host, int32_t schedule) {
  g_err.clear();
  QueryPlan plan;
  if (plan_query(c, B, q_ptr_host, &plan) != WMD_OK) return 0;
  if (schedule < WMD_SCHEDULE_AUTO || schedule > WMD_SCHEDULE_UNFUSED) return 0;
  return layout_for(c, plan, schedule).total;
}

// The Sinkhorn launch units of a query of padded width S, built once per
// width and kept until the merge mode or a pinned shape changes.  Per query,
// the length buckets that one-wave items hold share one launch; the others
// (and any bucket with a pinned shape) get launches of their own.
static wmd_status units_for(wmd_corpus* c, int S, std::shared_ptr<const std::vector<SinkUnit>>* out) {
  std::lock_guard<std::mutex> lock(c->cfg_mu);
  auto hit = c->plans.find(S);
  if (hit != c->plans.end()) {
    *out = hit->second;
    return WMD_OK;
  }
  auto units = std::make_shared<std::vector<SinkUnit>>();
  int caps[kNumBuckets], nds[kNumBuckets], bks[kNumBuckets], nm = 0;
  for (int bk = 0; bk < kNumBuckets; ++bk) {
    const int64_t nd = c->bucket_off[bk + 1] - c->bucket_off[bk];
    if (nd == 0) continue;
    caps[nm] = kBucketCap[bk]; nds[nm] = (int)nd; bks[nm] = bk; ++nm;
  }
  bool in_merge[kNumBuckets] = {};
  MergePlan mp;
  if (c->merge == WMD_MERGE_ALL && nm > 1 && plan_merge(S, caps, nds, nm, &mp) && mp.n > 1) {
    SinkUnit u;
    u.merged = true;
    u.plan = mp;
    u.nb = mp.n;
    u.key = {1, mp.tc, mp.trmax, mp.lg_cg, mp.n};
    for (int g = 0; g < mp.n; ++g) {
      const int bk = bks[mp.member[g]];
      in_merge[bk] = true;
      u.bk[g] = bk;
      u.nzb += (double)c->bucket_nnz[bk];
      u.ndd += (double)nds[mp.member[g]];
      u.key.push_back(bk);
      u.key.push_back(mp.body[g]);
    }
    u.name = "sink_merge_kernel<" + std::to_string(mp.tc) + "," + std::to_string(mp.trmax) + "," +
             std::to_string(mp.lg_cg) + ">x" + std::to_string(mp.n);
    units->push_back(std::move(u));
  }
  for (int bk = 0; bk < kNumBuckets; ++bk) {
    const int64_t nd = c->bucket_off[bk + 1] - c->bucket_off[bk];
    if (nd == 0 || in_merge[bk]) continue;
    SinkUnit u;
    u.nb = 1;
    u.bk[0] = bk;
    auto pin = c->pinned.find({S, kBucketCap[bk]});
    if (pin != c->pinned.end()) {
      u.cfg = pin->second;
    } else if (!choose_sink_config(S, kBucketCap[bk], (int)nd, &u.cfg)) {
      return fail(WMD_ERR_NOT_SUPPORTED, "no kernel shape for query width " + std::to_string(S) +
                                             " and documents of up to " + std::to_string(kBucketCap[bk]) + " words");
    }
    u.nzb = (double)c->bucket_nnz[bk];
    u.ndd = (double)nd;
    const SinkConfig& cfg = u.cfg;
    u.key = {0, bk, cfg.tc, cfg.tr, cfg.lg_cg, cfg.nwaves, cfg.maxw, cfg.stream ? 1 : 0};
    u.name = cfg.stream ? std::string("sink_stream_kernel")
                        : cfg.multiwave ? "sink_kernel<" + std::to_string(cfg.tc) + "," + std::to_string(cfg.tr) +
                                              "," + std::to_string(cfg.lg_cg) + "," + std::to_string(cfg.maxw) +
                                              ">x" + std::to_string(cfg.nwaves)
                                        : "sink_merge_kernel<" + std::to_string(cfg.tc) + "," +
                                              std::to_string(cfg.tr) + "," + std::to_string(cfg.lg_cg) + ">x1";
    units->push_back(std::move(u));
  }
  c->plans.emplace(S, units);
  *out = units;
  return WMD_OK;
}

// Descriptor checks that need nothing from the corpus object (which is not
// dereferenced before they pass).
static wmd_status check_query_desc(const wmd_corpus* c, const wmd_query_desc* q, const float* out,
                                   const void* workspace) {
  if (!c || !q) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL corpus or query descriptor");
  if (!out || !workspace) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL output or workspace");
  if (!q->q_ptr || !q->q_ids || !q->q_weights) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL device query pointer");
  if (!(q->lambda > 0.f) || !std::isfinite(q->lambda)) return fail(WMD_ERR_INVALID_ARGUMENT, "lambda must be finite and > 0");
  if (q->max_iter < 0 || q->max_iter > 100000) return fail(WMD_ERR_INVALID_ARGUMENT, "max_iter must be in [0, 100000]");
  if (q->cdist != WMD_CDIST_FP32 && q->cdist != WMD_CDIST_BF16) return fail(WMD_ERR_INVALID_ARGUMENT, "unknown cdist precision");
  if (q->schedule < WMD_SCHEDULE_AUTO || q->schedule > WMD_SCHEDULE_UNFUSED) return fail(WMD_ERR_INVALID_ARGUMENT, "unknown schedule");
  if (!(q->tol >= 0.f) || !std::isfinite(q->tol)) return fail(WMD_ERR_INVALID_ARGUMENT, "tol must be finite and >= 0");
  if (q->tol > 0.f && q->schedule != WMD_SCHEDULE_AUTO && q->schedule != WMD_SCHEDULE_RESIDENT)
    return fail(WMD_ERR_NOT_SUPPORTED, "a tolerance stop needs the resident schedule");
  return WMD_OK;
}

// Enqueues the whole path of one call.  `side`: the caller stream's side set,
// locked by the caller, or null to keep every launch on the caller's stream.
// `timed`: record per-launch events (the caller holds timing_mu).
static wmd_status enqueue_query(wmd_corpus* c, const wmd_query_desc* q, float* out, void* workspace,
                                size_t workspace_bytes, void* stream, bool in_graph, wmd_corpus::SideSet* side,
                                bool timed) {
  wmd_status st = check_query_desc(c, q, out, workspace);
  if (st != WMD_OK) return st;
  QueryPlan plan;
  st = plan_query(c, q->B, q->q_ptr_host, &plan);
  if (st != WMD_OK) return st;
  const int schedule = q->schedule == WMD_SCHEDULE_AUTO ? WMD_SCHEDULE_RESIDENT : q->schedule;
  const QueryLayout L = layout_for(c, plan, schedule);
  if (workspace_bytes < L.total)
    return fail(WMD_ERR_WORKSPACE_TOO_SMALL, "query workspace needs " + std::to_string(L.total) + " bytes");
  if ((uintptr_t)workspace % 256 != 0) return fail(WMD_ERR_INVALID_ARGUMENT, "query workspace must be 256-byte aligned");
  int dev = 0;
  WMD_HIP(hipGetDevice(&dev));
  if (dev != c->device) return fail(WMD_ERR_INVALID_ARGUMENT, "current device differs from the corpus device");
  // launch units of every query (by padded width)
  std::vector<std::shared_ptr<const std::vector<SinkUnit>>> qunits((size_t)q->B);
  for (int b = 0; b < q->B; ++b) {
    st = units_for(c, (int)plan.S[(size_t)b], &qunits[(size_t)b]);
    if (st != WMD_OK) return st;
  }

  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = workspace;
  const CorpusLayout& CL = c->L;
  const Tag none{};

  // a1: query selection and slot layout
  SelectParams sp{};
  sp.q_ptr = q->q_ptr; sp.q_ids = q->q_ids; sp.q_w = q->q_weights;
  sp.B = q->B; sp.V = c->V; sp.d = c->d; sp.dp = c->dp; sp.emb = c->emb;
  sp.err = at<int>(ws, L.err); sp.vr = at<int>(ws, L.vr); sp.qid = at<int>(ws, L.qid);
  sp.r = at<float>(ws, L.r); sp.cinfo = at<int2>(ws, L.cinfo); sp.qinfo = at<int2>(ws, L.qinfo);
  sp.qn = at<float>(ws, L.qn);
  sp.q32 = at<float>(ws, L.q32); sp.q16 = at<uint16_t>(ws, L.q16);
  sp.want_bf16 = q->cdist == WMD_CDIST_BF16;
  const double T = (double)q->q_ptr_host[q->B];  // raw query entries = sum of v_r
  const double esz = q->cdist == WMD_CDIST_BF16 ? 2.0 : 4.0;
  const double sel_bytes = T * 8.0 + T * c->d * 4.0 + (double)plan.C * c->dp * (4.0 + esz);

  // a2 + a3: cost matrix and K for every query word in one GEMM
  float* kt = at<float>(ws, L.kt);
  CdistParams cp{};
  cp.e32 = at<float>(c->ws, CL.e32); cp.e16 = at<uint16_t>(c->ws, CL.e16); cp.en = at<float>(c->ws, CL.en);
  cp.used = at<int>(c->ws, CL.used); cp.U = c->U;
  cp.q32 = sp.q32; cp.q16 = sp.q16; cp.qn = sp.qn; cp.qid = sp.qid; cp.cinfo = sp.cinfo;
  cp.C = plan.C; cp.dp = c->dp; cp.lam = q->lambda; cp.kt = kt;
  float* km = at<float>(ws, L.km);
  cp.km = km;
  cp.one_query = q->B == 1;
  // one short query whose cost matrix takes the skinny kernel: that kernel
  // selects the query itself (no separate launch, the selection's latency
  // hidden behind the vocabulary stream)
  const bool bf16 = q->cdist == WMD_CDIST_BF16;
  const bool fuse = q->B == 1 && q->q_ptr_host[1] <= 64 && cdist_fuses_select(cp, bf16);
  if (fuse) {
    cp.sel_n = (int)q->q_ptr_host[1];
    cp.q_ids = q->q_ids; cp.q_w = q->q_weights; cp.V = c->V; cp.d = c->d; cp.emb = c->emb;
    cp.err = sp.err; cp.vr = sp.vr; cp.r = sp.r; cp.qid_out = sp.qid; cp.cinfo_out = sp.cinfo;
  } else {
    WMD_HIP(timed_launch(c, timed, s, "select_kernel", 0.0, sel_bytes, none, [&] { return launch_select(sp, s); }));
  }
  if (c->U > 0) {
    // algorithmic work: 2 U d flops per query word; read the U x d vocabulary
    // rows and the query rows once, write K^T
    const double U = (double)c->U;
    const double flops = 2.0 * U * T * c->d;
    const double bytes = U * c->d * esz + T * c->d * esz + U * 4.0 + U * (double)plan.C * 4.0 +
                         (fuse ? sel_bytes : 0.0);
    // the tile shape is picked inside the launch; its name is filled in afterwards
    const char* name = "cdist_kernel";
    const size_t nrec = timed ? c->recs.size() : 0;
    bool shifted = false;
    WMD_HIP(timed_launch(c, timed, s, "", flops, bytes, none, [&] { return launch_cdist(cp, bf16, s, &name, &shifted); }));
    if (timed && c->recs.size() > nrec) c->recs.back().name = std::string(name) + (fuse ? "+select" : "");
    if (!shifted) {
      // row shifts of K^T: read the distances, write K and one shift per row
      const double cells = U * (double)plan.C;
      const int max_S = (int)*std::max_element(plan.S.begin(), plan.S.end());
      WMD_HIP(timed_launch(c, timed, s, "gibbs_rows_kernel", 2.0 * cells, 8.0 * cells + 4.0 * U * q->B, none, [&] {
        return launch_gibbs_rows(kt, km, sp.qinfo, c->U, q->B, max_S, q->lambda, s);
      }));
    }
  }

  // iterations per document: 0 for documents that are never iterated (no
  // positive weight); the Sinkhorn launches overwrite the others
  if (q->iters) {
    const int64_t n = (int64_t)q->B * c->N;
    WMD_HIP(launch_fill_i32(q->iters, n, schedule == WMD_SCHEDULE_RESIDENT ? 0 : q->max_iter, s));
  }

  // a4-a6: Sinkhorn iterations and the final pass.  Resident schedule: the
  // units of all queries with equal keys share one launch (at most
  // kMaxLaunchQueries queries each), in order of first appearance; the other
  // schedules (comparison baselines) and the streaming fallback launch per
  // query.  Launches are independent of each other; with several they are
  // spread over the caller stream's side streams.
  struct Launch { const SinkUnit* u; std::vector<int> qs; };
  std::vector<Launch> launches;
  {
    std::map<std::vector<int64_t>, size_t> open;  // key -> launch still taking queries
    for (int b = 0; b < q->B; ++b)
      for (const SinkUnit& u : *qunits[(size_t)b]) {
        const bool share =
            schedule == WMD_SCHEDULE_RESIDENT && !u.cfg.stream && !(q->flags & WMD_QUERY_PER_QUERY_LAUNCHES);
        if (share) {
          auto it = open.find(u.key);
          if (it != open.end() && launches[it->second].qs.size() < (size_t)kMaxLaunchQueries) {
            launches[it->second].qs.push_back(b);
            continue;
          }
          open[u.key] = launches.size();
        }
        launches.push_back({&u, {b}});
      }
  }
  const int groups = (int)launches.size();
  // inside a graph, branches cost nothing on the host; eagerly, the event
  // traffic only pays off with more groups
  const bool fork = side && (in_graph ? groups > 1 : groups > 3);
  // side streams in use: every one that waits on the fork must be joined
  // again (a stream left out of the join would end a capture unjoined)
  const int nside = fork ? std::min(groups, wmd_corpus::kSide) : 0;
  if (fork) {
    WMD_HIP(hipEventRecord(side->fork_ev, s));
    for (int i = 0; i < nside; ++i) WMD_HIP(hipStreamWaitEvent(side->side[i], side->fork_ev, 0));
  }
  float* ubuf = at<float>(ws, L.u);
  float* wbuf = at<float>(ws, L.w);
  const int4* drec = at<int4>(c->ws, CL.drec);
  // parameters of query b (base + b for a query set's base: b = 0)
  auto params_of = [&](int b) {
    const int64_t col0 = plan.col0[(size_t)b];
    SinkParams p{};
    p.kt = kt + (size_t)col0 * (size_t)c->U;
    p.km = km + (size_t)b * (size_t)c->U;
    p.r = sp.r + col0;
    p.vr = sp.vr + b;
    p.wl = at<int>(c->ws, CL.wl); p.wn = at<float>(c->ws, CL.wn);
    p.S = (int)plan.S[(size_t)b];
    p.inv_lam = 1.0f / q->lambda;
    p.tol = q->tol;
    p.iters_out = (q->iters && schedule == WMD_SCHEDULE_RESIDENT) ? q->iters + (size_t)b * (size_t)c->N : nullptr;
    p.out = out + (size_t)b * (size_t)c->N;
    p.u = ubuf + (size_t)col0 * (size_t)c->N;
    p.w = wbuf + (size_t)b * (size_t)c->nnz;
    return p;
  };
  int group = 0;
  for (const Launch& ln : launches) {
    const SinkUnit& u = *ln.u;
    hipStream_t gs = fork ? side->side[group % nside] : s;
    ++group;
    const int b0 = ln.qs[0];
    const bool multi = ln.qs.size() > 1;
    SinkQuerySet qset{};
    if (multi) {
      qset.nq = (int)ln.qs.size();
      qset.U = c->U;
      qset.N = c->N;
      for (size_t i = 0; i < ln.qs.size(); ++i) {
        const int b = ln.qs[i];
        qset.q[i] = make_int4(b, (int)plan.col0[(size_t)b], (int)plan.S[(size_t)b], 0);
      }
    }
    const SinkParams p = multi ? params_of(0) : params_of(b0);
    Tag tag{b0, (int)plan.S[(size_t)b0], u.merged ? 0 : kBucketCap[u.bk[0]], (int)u.ndd};
    auto launch = [&](const SinkParams& a) -> hipError_t {
      if (u.merged) {
        SinkParams m = a;
        m.drec = drec;
        int off[kMergeMax], nd[kMergeMax];
        for (int g = 0; g < u.nb; ++g) {
          off[g] = (int)c->bucket_off[u.bk[g]];
          nd[g] = (int)(c->bucket_off[u.bk[g] + 1] - c->bucket_off[u.bk[g]]);
        }
        int grid = 0;
        return launch_sink_merged(m, u.plan, off, nd, gs, &grid, multi ? &qset : nullptr);
      }
      SinkParams one = a;
      one.drec = drec + c->bucket_off[u.bk[0]];
      one.ndocs = (int)u.ndd;
      return launch_sink(one, u.cfg, sink_grid(u.cfg, one.ndocs), gs, multi ? &qset : nullptr);
    };
    // algorithmic work per document and iteration (n_k entries, v_r query words):
    // 4 v_r n_k + n_k + 2 v_r flops; 8 n_k + 4 v_r n_k + 8 v_r bytes when u and the
    // K^T rows travel through memory every pass.  The final pass does
    // 4 v_r n_k + 2 n_k flops.  Summed over the launch's queries.
    const double nzb = u.nzb, ndd = u.ndd;
    double vsum = 0.0;
    for (int b : ln.qs) vsum += (double)(q->q_ptr_host[b + 1] - q->q_ptr_host[b]);
    const double nq = (double)ln.qs.size();
    const double it_flops = 4.0 * vsum * nzb + nq * nzb + 2.0 * vsum * ndd;
    const double it_bytes = 8.0 * nq * nzb + 4.0 * vsum * nzb + 8.0 * vsum * ndd;
    const double fin_flops = 4.0 * vsum * nzb + 2.0 * nq * nzb;
    auto go = [&](const SinkParams& a, double fl, double by) {
      return timed_launch(c, timed, gs, u.name, fl, by, tag, [&] { return launch(a); });
    };
    if (schedule == WMD_SCHEDULE_RESIDENT) {
      SinkParams a = p;
      a.iters = q->max_iter; a.do_final = 1;
      // resident: the entries, the document records and the K^T rows are read once
      WMD_HIP(go(a, q->max_iter * it_flops + fin_flops, 8.0 * nq * nzb + 4.0 * vsum * nzb + 20.0 * nq * ndd));
    } else {
      for (int it = 0; it < q->max_iter; ++it) {
        if (schedule == WMD_SCHEDULE_PER_ITERATION) {
          SinkParams a = p;
          a.iters = 1; a.load_u = it > 0; a.store_u = 1;
          WMD_HIP(go(a, it_flops, it_bytes));
        } else {
          SinkParams a = p;  // SDDMM: w_j = c_j / (K_j . u)
          a.iters = 1; a.load_u = it > 0; a.store_w = 1;
          WMD_HIP(go(a, 2.0 * vsum * nzb + nq * nzb, 12.0 * nq * nzb + 4.0 * vsum * nzb + 4.0 * vsum * ndd));
          SinkParams m = p;  // SpMM: acc = K w, u = r / acc
          m.iters = 1; m.load_w = 1; m.store_u = 1;
          WMD_HIP(go(m, 2.0 * vsum * nzb + 2.0 * vsum * ndd, 8.0 * nq * nzb + 4.0 * vsum * nzb + 4.0 * vsum * ndd));
        }
      }
      SinkParams f = p;
      f.iters = 0; f.load_u = q->max_iter > 0; f.do_final = 1;
      WMD_HIP(go(f, fin_flops, 8.0 * nq * nzb + 4.0 * vsum * nzb + 4.0 * vsum * ndd + 20.0 * nq * ndd));
    }
  }
  if (c->empty_count > 0)
    for (int b = 0; b < q->B; ++b) {
      const Tag tag{b, 0, 0, (int)c->empty_count};
      WMD_HIP(timed_launch(c, timed, s, "nan_docs_kernel", 0.0, 8.0 * c->empty_count, tag, [&] {
        return launch_nan_docs(c->docs() + c->empty_off, c->empty_count, out + (size_t)b * (size_t)c->N, s);
      }));
    }
  if (fork)
    for (int i = 0; i < nside; ++i) {
      WMD_HIP(hipEventRecord(side->join_ev[i], side->side[i]));
      WMD_HIP(hipStreamWaitEvent(s, side->join_ev[i], 0));
    }
  return WMD_OK;
}

wmd_status wmd_set_merge(wmd_corpus* c, int32_t mode) {
  g_err.clear();
  if (!c) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus is NULL");
  if (mode != WMD_MERGE_ALL && mode != WMD_MERGE_NONE) return fail(WMD_ERR_INVALID_ARGUMENT, "unknown merge mode");
  std::lock_guard<std::mutex> lock(c->cfg_mu);
  c->merge = mode;
  c->plans.clear();
  return WMD_OK;
}

wmd_status wmd_set_timing(wmd_corpus* c, int32_t enable) {
  g_err.clear();
  if (!c) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus is NULL");
  std::lock_guard<std::mutex> lock(c->timing_mu);
  c->timing = enable != 0;
  c->recs.clear();
  return WMD_OK;
}

wmd_status wmd_get_timing(wmd_corpus* c, wmd_kernel_stat* stats, int32_t capacity, int32_t* count) {
  g_err.clear();
  if (!c || !count || (capacity > 0 && !stats)) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL argument");
  std::lock_guard<std::mutex> lock(c->timing_mu);
  std::vector<std::string> names;
  std::vector<wmd_kernel_stat> acc;
  for (const auto& r : c->recs) {
    WMD_HIP(hipEventSynchronize(c->events[r.ev + 1]));
    float ms = 0.f;
    WMD_HIP(hipEventElapsedTime(&ms, c->events[r.ev], c->events[r.ev + 1]));
    size_t i = 0;
    while (i < names.size() && names[i] != r.name) ++i;
    if (i == names.size()) {
      names.push_back(r.name);
      wmd_kernel_stat z{};
      std::snprintf(z.name, sizeof(z.name), "%s", r.name.c_str());
      acc.push_back(z);
    }
    acc[i].launches += 1;
    acc[i].total_ms += ms;
    acc[i].flops += r.flops;
    acc[i].bytes += r.bytes;
  }
  const int32_t n = (int32_t)acc.size();
  for (int32_t i = 0; i < n && i < capacity; ++i) stats[i] = acc[(size_t)i];
  *count = n;
  return WMD_OK;
}

static uint64_t bits_of(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

wmd_status wmd_query(wmd_corpus* c, const wmd_query_desc* q, float* out, void* workspace, size_t workspace_bytes,
                     void* stream) {
  g_err.clear();
  wmd_status st = check_query_desc(c, q, out, workspace);
  if (st != WMD_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // a timed call holds timing_mu throughout (its records and event pool are shared)
  std::unique_lock<std::mutex> timing_lock(c->timing_mu, std::defer_lock);
  bool timed = c->timing.load();
  if (timed) {
    timing_lock.lock();
    timed = c->timing.load();
    if (!timed) timing_lock.unlock();
  }
  wmd_corpus::SideSet* side = nullptr;
  st = side_set(c, s, &side);
  if (st != WMD_OK) return st;
  // the side set stays locked until the call's launches (or its capture) are complete
  std::unique_lock<std::mutex> side_lock;
  if (side) side_lock = std::unique_lock<std::mutex>(side->mu);
  const bool graph = (q->flags & WMD_QUERY_GRAPH) && stream != nullptr && !timed;
  if (!graph) return enqueue_query(c, q, out, workspace, workspace_bytes, stream, false, side, timed);
  if (q->B < 1 || !q->q_ptr_host) return fail(WMD_ERR_INVALID_ARGUMENT, "B must be >= 1 with host offsets");
  // every argument the captured launches depend on
  std::vector<uint64_t> key = {(uint64_t)(uintptr_t)out, (uint64_t)(uintptr_t)workspace, (uint64_t)workspace_bytes,
                               (uint64_t)(uintptr_t)q->q_ptr, (uint64_t)(uintptr_t)q->q_ids,
                               (uint64_t)(uintptr_t)q->q_weights, (uint64_t)(uintptr_t)q->iters,
                               (uint64_t)q->B, bits_of(q->lambda), (uint64_t)q->max_iter, (uint64_t)q->cdist,
                               (uint64_t)q->schedule, bits_of(q->tol), (uint64_t)(uintptr_t)stream,
                               (uint64_t)q->flags};
  for (int b = 0; b <= q->B; ++b) key.push_back((uint64_t)q->q_ptr_host[b]);
  {
    std::lock_guard<std::mutex> lock(c->cfg_mu);
    key.push_back((uint64_t)c->merge);
    for (const auto& p : c->pinned) {
      key.push_back(((uint64_t)p.first.first << 32) | (uint32_t)p.first.second);
      key.push_back(((uint64_t)p.second.tc << 48) | ((uint64_t)p.second.tr << 32) |
                    ((uint64_t)p.second.lg_cg << 16) | ((uint64_t)p.second.nwaves << 8) | (uint64_t)p.second.maxw);
    }
  }
  int dev = 0;
  WMD_HIP(hipGetDevice(&dev));
  if (dev != c->device) return fail(WMD_ERR_INVALID_ARGUMENT, "current device differs from the corpus device");
  std::lock_guard<std::mutex> graph_lock(c->graph_mu);
  for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
    if (it->key != key) continue;
    c->graphs.splice(c->graphs.begin(), c->graphs, it);  // most recent first
    WMD_HIP(hipGraphLaunch(c->graphs.front().exec, s));
    return WMD_OK;
  }
  WMD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  st = enqueue_query(c, q, out, workspace, workspace_bytes, stream, true, side, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (st != WMD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(WMD_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(WMD_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  c->graphs.push_front({std::move(key), g, x});
  if (c->graphs.size() > wmd_corpus::kMaxGraphs) {
    (void)hipGraphExecDestroy(c->graphs.back().exec);
    (void)hipGraphDestroy(c->graphs.back().graph);
    c->graphs.pop_back();
  }
  WMD_HIP(hipGraphLaunch(x, s));
  return WMD_OK;
}

wmd_status wmd_get_launches(wmd_corpus* c, wmd_launch_rec* recs, int32_t capacity, int32_t* count) {
  g_err.clear();
  if (!c || !count || (capacity > 0 && !recs)) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL argument");
  std::lock_guard<std::mutex> lock(c->timing_mu);
  int32_t n = 0;
  for (const auto& r : c->recs) {
    if (n < capacity) {
      WMD_HIP(hipEventSynchronize(c->events[r.ev + 1]));
      float ms = 0.f;
      WMD_HIP(hipEventElapsedTime(&ms, c->events[r.ev], c->events[r.ev + 1]));
      wmd_launch_rec& o = recs[n];
      std::memset(&o, 0, sizeof(o));
      std::snprintf(o.name, sizeof(o.name), "%s", r.name.c_str());
      o.query = r.query; o.S = r.S; o.cap = r.cap; o.ndocs = r.ndocs; o.ms = ms;
    }
    ++n;
  }
  *count = n;
  return WMD_OK;
}

static wmd_sink_shape to_shape(const SinkConfig& c) {
  wmd_sink_shape s{};
  s.tc = c.tc; s.tr = c.tr; s.lg_cg = c.lg_cg; s.maxw = c.maxw; s.nwaves = c.nwaves; s.stream = c.stream ? 1 : 0;
  return s;
}

wmd_status wmd_sink_candidates(const wmd_corpus* c, int32_t S, int32_t cap, wmd_sink_shape* out, int32_t capacity,
                               int32_t* count) {
  g_err.clear();
  if (!c || !count || (capacity > 0 && !out)) return fail(WMD_ERR_INVALID_ARGUMENT, "NULL argument");
  if (S < 4 || S % 4 || cap < 1) return fail(WMD_ERR_INVALID_ARGUMENT, "S must be a positive multiple of 4, cap >= 1");
  int bk = 0;
  while (bk < kNumBuckets - 1 && kBucketCap[bk] < cap) ++bk;
  const int nd = (int)(c->bucket_off[bk + 1] - c->bucket_off[bk]);
  std::vector<SinkConfig> v(512);
  const int n = sink_candidates(S, cap, nd > 0 ? nd : 1, v.data(), (int)v.size());
  for (int i = 0; i < n && i < capacity && i < (int)v.size(); ++i) out[i] = to_shape(v[(size_t)i]);
  *count = n;
  return WMD_OK;
}

wmd_status wmd_set_sink_shape(wmd_corpus* c, int32_t S, int32_t cap, const wmd_sink_shape* shape) {
  g_err.clear();
  if (!c) return fail(WMD_ERR_INVALID_ARGUMENT, "corpus is NULL");
  if (!shape) {
    std::lock_guard<std::mutex> lock(c->cfg_mu);
    c->pinned.erase({S, cap});
    c->plans.clear();
    return WMD_OK;
  }
  SinkConfig cfg{shape->tc, shape->tr, shape->lg_cg, shape->nwaves, shape->maxw > 1, shape->stream != 0, shape->maxw};
  if (cfg.stream) cfg = SinkConfig{0, 0, 6, 4, false, true, 4};
  if (!sink_config_fits(cfg, S, cap)) return fail(WMD_ERR_INVALID_ARGUMENT, "shape cannot run this (S, cap)");
  std::lock_guard<std::mutex> lock(c->cfg_mu);
  c->pinned[{S, cap}] = cfg;
  c->plans.clear();
  return WMD_OK;
}

size_t wmd_query_static_capacity(void) { return kScratchBytes; }

wmd_status wmd_query_static(wmd_corpus* c, const wmd_query_desc* q, float* out, void* stream) {
  g_err.clear();
  wmd_status st = check_query_desc(c, q, out, c ? c->scratch : nullptr);
  if (st != WMD_OK) return st;
  if (q->flags & WMD_QUERY_GRAPH)
    return fail(WMD_ERR_NOT_SUPPORTED, "wmd_query_static does not capture graphs (instantiating one allocates)");
  if (c->timing)
    return fail(WMD_ERR_NOT_SUPPORTED, "wmd_query_static does not run while per-kernel timing is enabled");
  QueryPlan plan;
  st = plan_query(c, q->B, q->q_ptr_host, &plan);
  if (st != WMD_OK) return st;
  const int schedule = q->schedule == WMD_SCHEDULE_AUTO ? WMD_SCHEDULE_RESIDENT : q->schedule;
  const size_t need = layout_for(c, plan, schedule).total;
  if (need > kScratchBytes)
    return fail(WMD_ERR_NOT_SUPPORTED, "this call needs " + std::to_string(need) +
                                           " bytes of query workspace; the static scratch holds " +
                                           std::to_string(kScratchBytes) + " (use wmd_query with a workspace)");
  // no side streams: creating a caller stream's set would create streams
  return enqueue_query(c, q, out, c->scratch, kScratchBytes, stream, false, nullptr, false);
}

wmd_status wmd_query_errors(const void* workspace, int32_t B, int32_t* codes, void* stream) {
  g_err.clear();
  if (!workspace || !codes || B < 1) return fail(WMD_ERR_INVALID_ARGUMENT, "bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  WMD_HIP(hipMemcpyAsync(codes, workspace, sizeof(int32_t) * (size_t)B, hipMemcpyDeviceToHost, s));
  WMD_HIP(hipStreamSynchronize(s));
  return WMD_OK;
}

}  // extern "C"
