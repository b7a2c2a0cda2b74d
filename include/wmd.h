/*
 * wmd.h -- C ABI of the gfx950 Sinkhorn Word Mover's Distance library.
 *
 * The library scores query documents against a resident corpus of target
 * documents with the entropic (Sinkhorn) word mover's distance of
 * arXiv 2107.06433, Algorithm 1:
 *
 *   select the query's nonzero words (r), M = Euclidean cost between the
 *   query words and the vocabulary, K = exp(-lambda M), x = 1/v_r, then
 *   max_iter times  x = diag(1/r) K (c .* 1/(K^T (1/x))),  and finally
 *   u = 1/x, v = c .* 1/(K^T u), d_k = sum(u .* ((K .* M) v))_k.
 *
 * The sparse steps run as the fused SDDMM-SpMM of Section III-C: for every
 * nonzero c_jk the dot product s = K_j . u_k and the update x_k += K_j c_jk / s
 * happen together, so the sparse intermediate v is never stored.
 *
 * Conventions for every function below
 *  - All device pointers refer to memory on the device that is current when
 *    the call is made; the library never allocates device memory.  Device
 *    buffers are supplied by the caller (typically torch tensors) and are
 *    BORROWED: they must stay valid for as long as the library may use them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - Functions return a wmd_status and never throw.  On failure
 *    wmd_last_error() returns a message for the calling thread.
 *  - Distances are float32.  Arithmetic is float32 throughout the iteration;
 *    only the cost-matrix GEMM may use bf16 inputs (WMD_CDIST_BF16).
 */
#ifndef WMD_H
#define WMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WMD_OK = 0,
  WMD_ERR_INVALID_ARGUMENT = 1,    /* bad pointer, size, id, weight or option      */
  WMD_ERR_WORKSPACE_TOO_SMALL = 2, /* workspace_bytes below the *_workspace_bytes() */
  WMD_ERR_DEVICE = 3,              /* a HIP call failed; message holds its string   */
  WMD_ERR_NOT_SUPPORTED = 4        /* a shape beyond the library's limits           */
} wmd_status;

/* Precision of the cost-matrix GEMM  q_i . e_j  (Section III-B-1, cdist).
 * FP32: float32 inputs and accumulation.  BF16: bf16-rounded inputs, float32
 * accumulation; the norms |q|^2, |e|^2, the square root, exp and every
 * Sinkhorn step stay float32 either way. */
typedef enum { WMD_CDIST_FP32 = 0, WMD_CDIST_BF16 = 1 } wmd_cdist;

/* How the max_iter fused SDDMM-SpMM passes are scheduled.
 *  RESIDENT      one launch per query (per document-length bucket where a
 *                bucket needs several waves per document, see wmd_set_merge)
 *                runs every iteration and the final pass; each document's
 *                rows of K^T are gathered once and kept in registers.
 *  PER_ITERATION one launch per iteration (u round-trips through device
 *                memory, rows of K^T re-gathered each pass), as Section III-C
 *                runs one SDDMM_SpMM call per loop trip, then a final launch.
 *  UNFUSED       SDDMM and SpMM as two launches per iteration with the sparse
 *                intermediate w stored in device memory (the unfused baseline
 *                of the fusion experiment, Section V).
 *  AUTO          RESIDENT. */
typedef enum {
  WMD_SCHEDULE_AUTO = 0,
  WMD_SCHEDULE_RESIDENT = 1,
  WMD_SCHEDULE_PER_ITERATION = 2,
  WMD_SCHEDULE_UNFUSED = 3
} wmd_schedule;

typedef struct wmd_corpus wmd_corpus; /* opaque host object */

/* ------------------------------------------------------------------ corpus */

/* The target documents: the paper's V x N histogram matrix c (Section III-B-2),
 * stored column by column (CSC, i.e. document-major), and the V x d word
 * embedding table `vecs`. */
typedef struct {
  int64_t V;                /* vocabulary size, >= 1                                  */
  int32_t d;                /* embedding width, 1..4096                               */
  const float* emb;         /* device, V*d float32, row-major (word j = row j)        */
  int64_t N;                /* number of target documents, >= 1                       */
  int64_t nnz;              /* total (word, weight) entries, >= 0                     */
  const int64_t* doc_ptr;   /* device, N+1 int64: doc k owns entries doc_ptr[k]..[k+1]*/
  const int32_t* word_ids;  /* device, nnz int32 in [0, V); repeats are summed         */
  const float* weights;     /* device, nnz float32, finite, >= 0; raw counts are fine:
                               each document is normalised to sum 1 (Section III-B-1).
                               A document whose weights sum to 0 scores NaN.            */
  int32_t compact_vocab;    /* nonzero: evaluate the cost matrix only for the words
                               that occur in the corpus (results are identical)        */
  void* workspace;          /* device, >= wmd_corpus_workspace_bytes(), 256-byte
                               aligned (hipMalloc and torch allocations are); holds the
                               normalised weights, compacted embeddings (f32 + bf16),
                               squared norms and document-length buckets.  Borrowed.   */
  size_t workspace_bytes;
} wmd_corpus_desc;

/* Bytes of corpus workspace needed for these sizes (0 on overflow). */
size_t wmd_corpus_workspace_bytes(int64_t V, int32_t d, int64_t N, int64_t nnz);

/* Validates the corpus on the device (ids in range, weights finite and >= 0,
 * doc_ptr non-decreasing from 0 to nnz, at most 4096 entries per document),
 * normalises every document, builds the compacted vocabulary and the
 * document-length buckets.  Synchronises `stream` before returning.
 * Invalid data -> WMD_ERR_INVALID_ARGUMENT and *out = NULL. */
wmd_status wmd_create_corpus(const wmd_corpus_desc* desc, void* stream, wmd_corpus** out);

typedef struct {
  int64_t V, N, nnz;
  int32_t d, d_padded;      /* d_padded: row length of the internal embedding copies */
  int64_t U;                /* vocabulary rows the cost matrix is evaluated on        */
  int64_t empty_docs;       /* documents that score NaN (no positive weight)          */
  int32_t n_buckets;        /* document-length buckets (capacity 16, 32, ... 4096)    */
  int64_t bucket_docs[16];  /* documents per bucket                                   */
  int32_t bucket_cap[16];   /* longest document a bucket holds                        */
} wmd_corpus_info;

wmd_status wmd_get_corpus_info(const wmd_corpus* c, wmd_corpus_info* info);

/* Frees the host object and its cached launch plans.  NULL is a no-op.
 * Borrowed device buffers are left to the caller. */
wmd_status wmd_destroy(wmd_corpus* c);

/* ----------------------------------------------------------------- queries */

/* B query documents in one call.  Query b owns entries q_ptr[b]..q_ptr[b+1]
 * of q_ids / q_weights; repeated ids are summed, zero weights dropped and
 * the histogram normalised to 1 on the device (Algorithm 1, first step).
 * The offsets are needed twice: on the host to plan the launches and on the
 * device for the kernels; both copies must hold the same values. */
typedef struct {
  int32_t B;                  /* number of queries, >= 1                               */
  const int64_t* q_ptr_host;  /* host, B+1, non-decreasing from 0; every query >= 1
                                 entry and at most 2048 entries                        */
  const int64_t* q_ptr;       /* device copy of q_ptr_host                             */
  const int32_t* q_ids;       /* device, q_ptr[B] word ids                             */
  const float* q_weights;     /* device, q_ptr[B] weights                              */
  float lambda;               /* entropic weight, finite, > 0: K = exp(-lambda M).
                                 Range: K is float32.  Each row of K (one vocabulary
                                 word against the query's words) is stored scaled by
                                 exp(lambda m_j), m_j the row's smallest cost: exact for
                                 the iteration (the document-side scaling absorbs the
                                 factor) and taken out again in the final pass, so no
                                 row underflows.  A query word
                                 whose lambda (M_ij - m_j) exceeds about 87 (exp below
                                 the smallest normal float) for every word of a
                                 document still breaks the float32 iteration there:
                                 that document scores +Inf (below).  With N(0, 1/d)
                                 embeddings at d = 300, results keep float32 accuracy
                                 for lambda from 1 to 300 (tested); in few dimensions
                                 distances spread further and the limit comes sooner
                                 (d = 8: some documents flagged at lambda 50).         */
  int32_t max_iter;           /* Sinkhorn-Knopp iterations, 0..100000                  */
  int32_t cdist;              /* wmd_cdist                                             */
  int32_t schedule;           /* wmd_schedule                                          */
  float tol;                  /* 0: exactly max_iter iterations (the paper's cut-off).
                                 > 0: a document stops as soon as an iteration changes
                                 its x by at most tol, max_i |x_new_i - x_i| / x_new_i
                                 <= tol (Algorithm 1 loops until x stops changing), and at
                                 max_iter at the latest.  Resident schedule only.       */
  int32_t* iters;             /* device, B*N int32 or NULL: iterations each document ran */
  int32_t flags;              /* WMD_QUERY_* bits                                       */
} wmd_query_desc;

/* flags: capture the call's launch sequence into a HIP graph on first use and
 * replay it when a later call on the same corpus has identical arguments
 * (pointers, sizes, offsets, lambda, iterations, options).  Independent
 * launch groups become parallel graph branches.  Needs a non-NULL stream;
 * ignored while per-kernel timing is enabled.  A corpus keeps its 128 most
 * recently used graphs. */
#define WMD_QUERY_GRAPH 1
/* flags: give every query its own Sinkhorn launches.  By default (resident
 * schedule) the queries of a call whose launch plans are identical -- the
 * same kernel shape, length buckets and row bodies, which depend on the query
 * width only through the shape -- share one launch of up to 64 queries.  The
 * results are the same bit for bit either way. */
#define WMD_QUERY_PER_QUERY_LAUNCHES 2

/* Bytes of query workspace for B queries with these offsets and schedule
 * (0 on invalid input).  Dominated by K^T: 4 * U * sum_b S_b bytes, S_b =
 * entries of query b rounded up to a multiple of 4 (the final pass recovers
 * M from K, so no cost matrix is stored). */
size_t wmd_query_workspace_bytes(const wmd_corpus* c, int32_t B, const int64_t* q_ptr_host,
                                 int32_t schedule);

/* Enqueues the whole hot path for B queries on `stream` and returns without
 * waiting (Algorithm 1 for every query against every document): query selection, cost matrix + K (one GEMM over all queries;
 * a call with one query of at most 64 entries, at most 32 padded columns and
 * an embedding width of at most 384 (f32) or 768 (bf16) selects it inside
 * the GEMM's launch), the Sinkhorn iterations and the final pass.  `out` (device, B*N float32,
 * row b = query b) is written when the stream reaches the end of the call.
 * Host-side argument errors are reported synchronously.  Errors found on the
 * device (a query id outside [0, V), a negative or non-finite weight, no
 * positive weight) make that query's row NaN and are read back with
 * wmd_query_errors().  Per document: a finite distance; NaN for a document
 * without positive weight or a row of an invalid query; +Inf where the float32
 * scaling broke down for a document with words (K underflow, see lambda).
 * The workspace must be 256-byte aligned.  Calls that
 * share a workspace must be ordered on one stream; calls with separate
 * workspaces may run concurrently. */
wmd_status wmd_query(wmd_corpus* c, const wmd_query_desc* q, float* out, void* workspace,
                     size_t workspace_bytes, void* stream);

/* wmd_query without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The query workspace is a static device array of
 * wmd_query_static_capacity() bytes (64 MiB), one copy per GPU, held until the
 * process ends; this call allocates nothing and calls no allocating routine.
 * Inputs and `out` are the caller's, as for wmd_query; the distances are the
 * same bit for bit.  A call whose workspace would exceed the array
 * (wmd_query_workspace_bytes) returns WMD_ERR_NOT_SUPPORTED, as do the graph
 * flag and per-kernel timing (both would allocate).  Every call on one GPU
 * uses the same array: calls that may overlap on the device (other streams,
 * other threads, other corpora) race and must be ordered by the caller.
 * Nothing in the array needs to start at zero (every launch writes what it
 * reads first).  Device error codes stay in the array; a row of an invalid
 * query is NaN as with wmd_query. */
size_t wmd_query_static_capacity(void);
wmd_status wmd_query_static(wmd_corpus* c, const wmd_query_desc* q, float* out, void* stream);

/* Per-query device error codes of the last wmd_query on `workspace`
 * (0 = ok, 1 = id out of range, 2 = bad weight, 3 = no positive weight).
 * Copies B int32 into host `codes` and synchronises `stream`. */
wmd_status wmd_query_errors(const void* workspace, int32_t B, int32_t* codes, void* stream);

/* ------------------------------------------------------- instrumentation */

/* Per-kernel timing for measurement tools.  While enabled on a corpus, every
 * wmd_query on it brackets each kernel launch with a pair of HIP events on the
 * caller's stream and records the launch's algorithmic work (flops and bytes
 * the method must move, not what the hardware counted).  Enabling clears
 * earlier records; at most 1,000,000 launches are kept. */
typedef struct {
  char name[96];      /* kernel and template shape, e.g. "sink_kernel<5,16,0>" */
  int64_t launches;
  double total_ms;    /* summed event-to-event duration of those launches      */
  double flops;       /* summed algorithmic floating-point operations          */
  double bytes;       /* summed algorithmic bytes read or written              */
} wmd_kernel_stat;

wmd_status wmd_set_timing(wmd_corpus* c, int32_t enable);

/* Waits for every recorded event, then writes one entry per kernel name
 * (at most `capacity`) and their number to *count. */
wmd_status wmd_get_timing(wmd_corpus* c, wmd_kernel_stat* stats, int32_t capacity, int32_t* count);

/* One record per timed launch, in launch order: the kernel name, the padded
 * query width S and length-bucket capacity of a Sinkhorn launch (0 for other
 * kernels), its document count and the event-to-event duration. */
typedef struct {
  char name[96];
  int32_t query, S, cap, ndocs;
  double ms;
} wmd_launch_rec;

wmd_status wmd_get_launches(wmd_corpus* c, wmd_launch_rec* recs, int32_t capacity, int32_t* count);

/* ------------------------------------------------------- kernel shapes */

/* A shape of the fused Sinkhorn kernel: each lane keeps tc query words x tr
 * document words of K^T in registers; 2^lg_cg lanes span the query words; a
 * document occupies one wave (maxw = 1, four documents per block) or nwaves
 * waves of a block compiled for at most maxw (4, 8 or 16) waves.  stream = 1 is
 * the fallback that re-reads K^T rows on every pass (other fields ignored). */
typedef struct {
  int32_t tc, tr, lg_cg, maxw, nwaves, stream;
} wmd_sink_shape;

/* The shapes that can run documents of up to `cap` words against a query of
 * padded width S (a multiple of 4) on this corpus's device, best estimate of
 * the built-in cost model first.  Writes at most `capacity`. */
wmd_status wmd_sink_candidates(const wmd_corpus* c, int32_t S, int32_t cap, wmd_sink_shape* out, int32_t capacity,
                               int32_t* count);

/* Pins the shape this corpus uses for (S, cap) when that bucket launches on
 * its own (see wmd_set_merge), e.g. from a measured tuning table; NULL removes
 * the pin.  A shape that cannot run (S, cap) is rejected with
 * WMD_ERR_INVALID_ARGUMENT. */
wmd_status wmd_set_sink_shape(wmd_corpus* c, int32_t S, int32_t cap, const wmd_sink_shape* shape);

/* How a query's length buckets are grouped into Sinkhorn launches.  Work
 * items (query, document) are independent (Section III-C), so the grouping
 * changes the time, and at most the float32 rounding of a bucket that runs
 * with a different lane layout; each result stays deterministic.
 *   WMD_MERGE_ALL:  every bucket whose documents one wave per item can hold
 *                   (up to 16 rows per lane) joins one launch per query, the
 *                   longest documents first (default)
 *   WMD_MERGE_NONE: one launch per bucket
 * Pinned shapes (wmd_set_sink_shape) apply to the buckets that launch on
 * their own. */
#define WMD_MERGE_ALL 0
#define WMD_MERGE_NONE 1
wmd_status wmd_set_merge(wmd_corpus* c, int32_t mode);

/* Message of the last failed call on this thread ("" if none). */
const char* wmd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WMD_H */
