// Private declarations shared by the host runtime (capi.cpp) and the kernel
// translation units.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wmd {

constexpr int kMaxDocLen = 4096;     // longest document the fused kernels hold
constexpr int kMaxQueryLen = 2048;   // raw entries per query
constexpr int kNumBuckets = 9;       // document-length capacities 16 .. 4096
constexpr int kBucketCap[kNumBuckets] = {16, 32, 64, 128, 256, 512, 1024, 2048, 4096};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t round4(int64_t x) { return (x + 3) & ~int64_t(3); }
// Row length of the internal embedding copies: a multiple of both GEMM k-steps.
inline int padded_dim(int d) { return (d + 63) / 64 * 64; }

// ---------------------------------------------------------------- layouts

// Corpus workspace: derived arrays built once by wmd_create_corpus.
struct CorpusLayout {
  size_t err, wn, wl, map, used, dpos, docs, drec, en, e32, e16, total;
  static CorpusLayout make(int64_t V, int d, int64_t N, int64_t nnz) {
    CorpusLayout L{};
    const int dp = padded_dim(d);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.err = take(64 * sizeof(int));
    L.wn = take(sizeof(float) * (size_t)nnz);           // normalised weights
    L.wl = take(sizeof(int) * (size_t)nnz);             // compacted word ids
    L.map = take(sizeof(int) * (size_t)(V + 1));        // vocab id -> compacted row
    L.used = take(sizeof(int) * (size_t)V);             // compacted row -> vocab id
    L.dpos = take(sizeof(int) * (size_t)N);             // doc has positive mass
    L.docs = take(sizeof(int) * (size_t)N);             // docs grouped by length bucket
    L.drec = take(sizeof(int4) * (size_t)N);            // (first entry lo/hi, length, id) per doc, same order
    L.en = take(sizeof(float) * (size_t)V);             // |e|^2 of compacted rows
    L.e32 = take(sizeof(float) * (size_t)V * dp);       // compacted embeddings, f32
    L.e16 = take(sizeof(uint16_t) * (size_t)V * dp);    // same, bf16
    L.total = o;
    return L;
  }
};

// Query workspace: everything one wmd_query call writes.  The per-query error
// codes sit at offset 0 so that wmd_query_errors() can find them from the
// workspace pointer alone.
struct QueryLayout {
  size_t err, vr, qid, r, cinfo, qinfo, qn, q32, q16, kt, km, u, w, total;
  static QueryLayout make(int B, int64_t C, int64_t U, int dp, int64_t N, int64_t nnz,
                          bool need_u, bool need_w) {
    QueryLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.err = take(sizeof(int) * (size_t)B);
    L.vr = take(sizeof(int) * (size_t)B);
    L.qid = take(sizeof(int) * (size_t)C);
    L.r = take(sizeof(float) * (size_t)C);
    L.cinfo = take(sizeof(int2) * (size_t)C);
    L.qinfo = take(sizeof(int2) * (size_t)B);           // per query: first column, width S
    L.qn = take(sizeof(float) * (size_t)C);
    L.q32 = take(sizeof(float) * (size_t)C * dp);
    L.q16 = take(sizeof(uint16_t) * (size_t)C * dp);
    L.kt = take(sizeof(float) * (size_t)C * (size_t)U);
    L.km = take(sizeof(float) * (size_t)B * (size_t)U);  // per query and row: the row's shift m_j
    L.u = need_u ? take(sizeof(float) * (size_t)C * (size_t)N) : o;
    L.w = need_w ? take(sizeof(float) * (size_t)nnz * (size_t)B) : o;
    L.total = o;
    return L;
  }
};

// ------------------------------------------------------- kernel parameters

struct SelectParams {
  const int64_t* q_ptr; const int32_t* q_ids; const float* q_w;
  int B; int64_t V; int d; int dp;
  const float* emb;
  int* err; int* vr; int* qid; float* r; int2* cinfo; int2* qinfo; float* qn; float* q32; uint16_t* q16;
  int want_bf16;
};

// The Gibbs kernel is stored row-scaled: row j of query b's block holds
// exp(-lambda (M_ij - m_j)) with m_j = min_i M_ij over the query's words, and
// km[b U + j] = m_j.  Scaling a column of K by any positive factor leaves
// Algorithm 1's u iterates and its distance unchanged (v absorbs the factor),
// so this is the same computation; every stored row then has maximum 1 and
// cannot underflow as a whole.  With one query in the call (one_query) the
// cost-matrix kernel applies the shift itself; otherwise it stores the plain
// distances (+inf in unused slots) and gibbs_rows_kernel applies it.
struct CdistParams {
  const float* e32; const uint16_t* e16; const float* en; const int* used; int64_t U;
  const float* q32; const uint16_t* q16; const float* qn; const int* qid; const int2* cinfo;
  int64_t C; int dp; float lam;
  float* kt;
  float* km;               // B x U row shifts (written here when one_query)
  int one_query;
  // Fused selection (sel_n > 0): one query of sel_n <= 64 entries and C = its
  // padded width.  Every block selects it and reads the embedding rows of its
  // words itself; block 0 also writes err, vr, r, qid and cinfo (the _out
  // pointers to the same buffers as qid and cinfo), the outputs
  // of the selection kernel that the later kernels read.  q32, q16 and qn are
  // then neither read nor written.
  int sel_n;
  const int32_t* q_ids; const float* q_w; int64_t V; int d; const float* emb;
  int* err; int* vr; float* r; int* qid_out; int2* cinfo_out;
};

// One fused SDDMM-SpMM launch over the documents of one length bucket for one
// query.  The same kernel runs every schedule; flags pick the variant.
struct SinkParams {
  const float* kt;        // K^T block of the query: U rows x S floats (1 in unused slots),
                          // row j scaled by exp(lambda m_j) (see CdistParams)
  const float* km;        // U row shifts m_j of the query
  const float* r;         // S slots of the normalised query histogram (0 = unused slot)
  const int* vr;          // device: number of used slots (0 = invalid query)
  const int4* drec;       // documents of the bucket: (first entry lo, hi, length, id)
  const int* wl; const float* wn;
  int ndocs;
  int S;
  float inv_lam;          // 1 / lambda: the final pass recovers M = m_j - ln(K) / lambda
  float* out;             // row of this query, indexed by document id
  float* u;               // N x S scalings (per-iteration schedules), doc-major
  float* w;               // nnz sparse intermediate (unfused schedule)
  int iters;              // iterations run by this launch (the cap when tol > 0)
  int load_u, store_u, do_final, store_w, load_w;
  float tol;              // > 0: stop a document once max_i |dx_i| / x_i <= tol
  int* iters_out;         // per document of this query (indexed by id), or null
};

// Several queries of one call in one Sinkhorn launch.  Every query of a call
// sees the same documents, so queries whose launch plans are identical (same
// kernel shape, same length buckets and row bodies) share one launch: its
// blocks run the plan once per query of the set, each with that query's K^T
// block, row shifts, r, v_r and output row.  The SinkParams of such a launch
// hold the call's base pointers (column 0 / query 0).
constexpr int kMaxLaunchQueries = 64;
struct SinkQuerySet {
  int nq;                       // 0: the launch runs the one query its SinkParams describe
  int64_t U, N;                 // K^T rows per query, documents per output row
  int4 q[kMaxLaunchQueries];    // per query: (index b in the call, first column, padded width S, 0)
};

// The parameters of query i of the set.
__host__ __device__ inline SinkParams for_query(const SinkParams& base, const SinkQuerySet& qs, int i) {
  SinkParams p = base;
  const int4 q = qs.q[i];
  p.kt = base.kt + (size_t)q.y * (size_t)qs.U;
  p.km = base.km + (size_t)q.x * (size_t)qs.U;
  p.r = base.r + q.y;
  p.vr = base.vr + q.x;
  p.out = base.out + (size_t)q.x * (size_t)qs.N;
  if (base.iters_out) p.iters_out = base.iters_out + (size_t)q.x * (size_t)qs.N;
  p.S = q.z;
  return p;
}

// Several length buckets of one query (or of each query of a set) in one
// launch of one-wave items (groups longest documents first; see
// sink_merge_kernel).
constexpr int kMergeMax = 8;
struct SinkMerge {
  SinkParams p;           // drec and ndocs are replaced per group
  SinkQuerySet qs;        // several queries: group g's blocks are nq runs of its per-query blocks
  int ngroups;
  int end[kMergeMax];     // one past the group's last block
  int off[kMergeMax];     // the group's first document record
  int ndocs[kMergeMax];
  int body[kMergeMax];    // rows per lane TRMAX >> (body & 3); body & 4: half-wave items
};

// Register-resident shape: tc x tr cells per lane, 2^lg_cg column lanes, an item
// spans `nwaves` waves of one block when multiwave (maxw = 4 or 16: the block
// size the kernel was compiled for), else one wave with four items per block.
// With `stream`: the one-block-per-item fallback that re-reads K^T rows on
// every pass.
struct SinkConfig { int tc, tr, lg_cg, nwaves; bool multiwave; bool stream; int maxw; };

// --------------------------------------------------------- launch wrappers
// Each returns the hipError_t of its launch.

hipError_t launch_fill_i32(int* p, int64_t n, int value, hipStream_t s);
hipError_t launch_prep_entries(const int32_t* ids, const float* w, int64_t nnz, int64_t V,
                               int* flags, int* err, hipStream_t s);
hipError_t launch_prep_docs(const int64_t* doc_ptr, const float* w, int64_t N, float* wn,
                            int* dpos, hipStream_t s);
hipError_t launch_prep_scan(int* map, int64_t V, hipStream_t s);
hipError_t launch_prep_compact(const int* map, int64_t V, int* used, const int32_t* ids,
                               int64_t nnz, int* wl, hipStream_t s);
hipError_t launch_prep_emb(const float* emb, int d, int dp, const int* used, int64_t U,
                           float* e32, uint16_t* e16, float* en, hipStream_t s);

hipError_t launch_select(const SelectParams& p, hipStream_t s);
// `name` receives the kernel and tile shape that was launched; `shifted` is set
// when that kernel stored the row-scaled K itself (one query, skinny kernel),
// otherwise it stored distances and launch_gibbs_rows must follow.
hipError_t launch_cdist(const CdistParams& p, bool bf16, hipStream_t s, const char** name, bool* shifted);
// Row shift of the stored distances of B queries (after a launch_cdist with
// one_query = 0): m_j = min over each query's used columns, K = exp(-lambda
// (M - m_j)), unused columns (+inf) become 1.
// max_S: the widest query's padded width (sizes the grid).
hipError_t launch_gibbs_rows(float* kt, float* km, const int2* qinfo, int64_t U, int B, int max_S, float lam,
                             hipStream_t s);
// whether launch_cdist can run with the selection fused in (sel_n > 0)
bool cdist_fuses_select(const CdistParams& p, bool bf16);
// grid: blocks for one query; with qs.nq > 0 the launch has nq times as many.
hipError_t launch_sink(const SinkParams& p, const SinkConfig& cfg, int grid, hipStream_t s,
                       const SinkQuerySet* qs = nullptr);
hipError_t launch_nan_docs(const int* docs, int64_t ndocs, float* out, hipStream_t s);

// Host-side shape choice for one (padded query width, bucket capacity, documents)
// triple: feasible shapes by increasing model cost (the streaming fallback last).
int sink_candidates(int S, int cap, int ndocs, SinkConfig* out, int max);
bool choose_sink_config(int S, int cap, int ndocs, SinkConfig* cfg);
bool sink_config_supported(const SinkConfig& cfg);
// Whether `cfg` can run documents of up to `cap` words at padded query width S.
bool sink_config_fits(const SinkConfig& cfg, int S, int cap);
int sink_grid(const SinkConfig& cfg, int ndocs);
int sink_block(const SinkConfig& cfg);

// One launch over several length buckets of one query (one-wave items).
// member[g] indexes the caller's bucket list, longest documents first; group g
// runs with trmax >> (body[g] & 3) rows per lane, as half-wave items (two per
// wave) when body[g] & 4.
struct MergePlan {
  int tc = 0, trmax = 0, lg_cg = 0;
  int n = 0;
  int member[kMergeMax] = {};
  int body[kMergeMax] = {};
};
bool plan_merge(int S, const int* cap, const int* ndocs, int nb, MergePlan* out);
// off / ndocs: per group, in plan order; p.drec is the start of all records.
hipError_t launch_sink_merged(const SinkParams& p, const MergePlan& plan, const int* off, const int* ndocs,
                              hipStream_t s, int* grid_out, const SinkQuerySet* qs = nullptr);

}  // namespace wmd
