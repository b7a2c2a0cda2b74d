// Corpus preparation (run once by wmd_create_corpus) and query selection
// (the first step of every wmd_query).
#include "lanes.h"
#include "query_rows.h"
#include "wmd_internal.h"

namespace wmd {

namespace {

__global__ void fill_i32_kernel(int* p, int64_t n, int value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Validate every (word, weight) entry and mark the words that occur.
__global__ void prep_entries_kernel(const int32_t* ids, const float* w, int64_t nnz, int64_t V,
                                    int* flags, int* err) {
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t id = ids[e];
    const float x = w[e];
    if (id < 0 || id >= V) bad |= 1;
    else flags[id] = 1;
    if (!(x >= 0.f) || isinf(x)) bad |= 2;
  }
  if (bad) atomicOr(err, bad);
}

// Normalise each document to sum 1 (Section III-B-1).  The sum is taken in
// double and each weight is divided in double before rounding to float.
__global__ void prep_docs_kernel(const int64_t* doc_ptr, const float* w, int64_t N, float* wn, int* dpos) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = doc_ptr[k], e = doc_ptr[k + 1];
    double s = 0.0;
    for (int64_t j = b; j < e; ++j) s += (double)w[j];
    dpos[k] = s > 0.0;
    for (int64_t j = b; j < e; ++j) wn[j] = s > 0.0 ? (float)((double)w[j] / s) : 0.f;
  }
}

// Exclusive prefix sum of flags[0..V) in place; map[V] = total.  One block.
__global__ void __launch_bounds__(1024) prep_scan_kernel(int* map, int64_t V) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (V + 1023) / 1024;
  const int64_t b = t * chunk, e = b + chunk < V ? b + chunk : V;
  int s = 0;
  for (int64_t i = b; i < e; ++i) s += map[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;  // exclusive
  for (int64_t i = b; i < e; ++i) {
    int f = map[i];
    map[i] = run;
    run += f;
  }
  if (t == 1023) map[V] = part[1023];
}

__global__ void prep_compact_kernel(const int* map, int64_t V, int* used, const int32_t* ids, int64_t nnz, int* wl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += stride)
    if (map[v + 1] > map[v]) used[map[v]] = (int)v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) wl[e] = map[ids[e]];
}

// One wave per compacted row: zero-padded f32 and bf16 copies and |e|^2.
__global__ void prep_emb_kernel(const float* emb, int d, int dp, const int* used, int64_t U,
                                float* e32, uint16_t* e16, float* en) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t row = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); row < U; row += waves) {
    const float* src = emb + (size_t)used[row] * d;
    double s = 0.0;
    for (int t = lane; t < dp; t += 64) {
      const float x = t < d ? src[t] : 0.f;
      e32[(size_t)row * dp + t] = x;
      e16[(size_t)row * dp + t] = f32_to_bf16(x);
      s += (double)x * (double)x;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) en[row] = (float)s;
  }
}

// Algorithm 1, first step, for one query per block: validate the entries,
// sum repeated ids, drop zero weights, normalise r in double, and lay out the
// query's S slots (S = entries rounded up to 4) of the GEMM's column space:
// word id, r, the query's column base and width, the f32/bf16 embedding row
// and its squared norm.  Slots past the selected words get id -1, r = 0.
__global__ void __launch_bounds__(256) select_kernel(SelectParams p) {
  __shared__ int s_id[kMaxQueryLen];
  __shared__ float s_w[kMaxQueryLen];
  __shared__ double s_m[kMaxQueryLen];
  __shared__ int s_slot[kMaxQueryLen];
  __shared__ int s_wflag[4];
  __shared__ long long s_col0;
  __shared__ int s_vr, s_err;
  __shared__ double s_tot;
  const int b = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t beg = p.q_ptr[b];
  const int n = (int)(p.q_ptr[b + 1] - beg);
  const int S = (n + 3) & ~3;
  const int nn = n < kMaxQueryLen ? n : kMaxQueryLen;
  // column base of this query: the padded widths of the queries before it,
  // summed by the last wave (lane partials, then a fixed butterfly)
  if (wave == 3) {
    long long part = 0;
    for (int bb = lane; bb < b; bb += 64) part += (p.q_ptr[bb + 1] - p.q_ptr[bb] + 3) & ~3LL;
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) s_col0 = part;
  }
  if (n <= 64) {
    if (wave == 0) select_small(p.q_ids, p.q_w, p.V, beg, n, S, lane, s_id, s_m, s_slot, &s_err, &s_vr, &s_tot);
    __syncthreads();
  } else {
  // entries into LDS, with their error flags ORed per wave
  int lf = 0;
  for (int i = t; i < nn; i += 256) {
    const int id = p.q_ids[beg + i];
    const float x = p.q_w[beg + i];
    s_id[i] = id;
    s_w[i] = x;
    if (id < 0 || id >= p.V) lf |= 1;
    if (!(x >= 0.f) || isinf(x)) lf |= 2;
  }
  const bool f1 = __ballot(lf & 1) != 0, f2 = __ballot(lf & 2) != 0;
  if (lane == 0) s_wflag[wave] = (f1 ? 1 : 0) | (f2 ? 2 : 0);
  __syncthreads();
  // merge repeats into their first occurrence, summing in entry order
  for (int i = t; i < nn; i += 256) {
    const int id = s_id[i];
    bool first = true;
    for (int j = 0; j < i; ++j)
      if (s_id[j] == id) { first = false; break; }
    double m = 0.0;
    if (first)
      for (int j = i; j < nn; ++j)
        if (s_id[j] == id) m += (double)s_w[j];
    s_m[i] = first ? m : 0.0;
  }
  __syncthreads();
  // slots in entry order and the total weight, by the first wave: per chunk
  // of 64 entries a ballot prefix and a fixed butterfly sum, chunks in order
  if (wave == 0) {
    int c = 0;
    double tot = 0.0;
    for (int i0 = 0; i0 < nn; i0 += 64) {
      const int i = i0 + lane;
      const double m = i < nn ? s_m[i] : 0.0;
      const bool sel = m > 0.0;
      const unsigned long long mask = __ballot(sel);
      if (sel) s_slot[c + __popcll(mask & ((1ull << lane) - 1))] = i;
      c += __popcll(mask);
      double part = sel ? m : 0.0;
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
      tot += part;
    }
    for (int k = c + lane; k < S && k < kMaxQueryLen; k += 64) s_slot[k] = -1;
    if (lane == 0) {
      int e = s_wflag[0] | s_wflag[1] | s_wflag[2] | s_wflag[3];
      if (n > kMaxQueryLen) e |= 4;
      if (e == 0 && c == 0) e = 8;
      s_err = e;
      s_vr = e ? 0 : c;
      s_tot = tot;
    }
  }
  __syncthreads();
  }
  const int err = s_err;
  const int vr = s_vr;
  const double tot = s_tot;
  const int64_t col0 = s_col0;
  if (t == 0) {
    p.err[b] = err & 1 ? 1 : err & 2 ? 2 : err & 4 ? 4 : err & 8 ? 3 : 0;
    p.vr[b] = vr;
    p.qinfo[b] = make_int2((int)col0, S);
  }
  for (int s = t; s < S; s += 256) {
    const int i = s < vr && s < kMaxQueryLen ? s_slot[s] : -1;
    p.qid[col0 + s] = i >= 0 ? s_id[i] : -1;
    p.r[col0 + s] = i >= 0 ? (float)(s_m[i] / tot) : 0.f;
    p.cinfo[col0 + s] = make_int2((int)col0, S);
  }
  // embedding rows of the slots and their squared norms: 8 lanes per slot,
  // 32 slots per pass (query_row)
  const int g = t >> 3, lane8 = t & 7;
  for (int s0 = 0; s0 < S; s0 += 32) {
    const int s = s0 + g;
    const int i = s < vr && s < kMaxQueryLen ? s_slot[s] : -1;
    const int q = i >= 0 ? s_id[i] : -1;
    double nrm = 0.0;
    if (s < S) {
      float* d32 = p.q32 + (size_t)(col0 + s) * p.dp;
      uint16_t* d16 = p.q16 + (size_t)(col0 + s) * p.dp;
      const bool bf = p.want_bf16;
      nrm = query_row(p.emb, p.d, p.dp, q, lane8, [&](int k, float4 v) {
        *(float4*)(d32 + k) = v;
        if (bf) *(uint2*)(d16 + k) = pack_bf16x4(v);
      });
    }
    nrm = sum_row_lanes(nrm);
    if (s < S && lane8 == 0) p.qn[col0 + s] = (float)nrm;
  }
}

__global__ void nan_docs_kernel(const int* docs, int64_t ndocs, float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ndocs; i += (int64_t)gridDim.x * blockDim.x)
    out[docs[i]] = __int_as_float(0x7FC00000);
}

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

hipError_t launch_fill_i32(int* p, int64_t n, int value, hipStream_t s) {
  fill_i32_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, n, value);
  return hipGetLastError();
}

hipError_t launch_prep_entries(const int32_t* ids, const float* w, int64_t nnz, int64_t V, int* flags,
                               int* err, hipStream_t s) {
  prep_entries_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(ids, w, nnz, V, flags, err);
  return hipGetLastError();
}

hipError_t launch_prep_docs(const int64_t* doc_ptr, const float* w, int64_t N, float* wn, int* dpos,
                            hipStream_t s) {
  prep_docs_kernel<<<grid_for(N, 256), 256, 0, s>>>(doc_ptr, w, N, wn, dpos);
  return hipGetLastError();
}

hipError_t launch_prep_scan(int* map, int64_t V, hipStream_t s) {
  prep_scan_kernel<<<1, 1024, 0, s>>>(map, V);
  return hipGetLastError();
}

hipError_t launch_prep_compact(const int* map, int64_t V, int* used, const int32_t* ids, int64_t nnz, int* wl,
                               hipStream_t s) {
  prep_compact_kernel<<<grid_for(V > nnz ? V : nnz, 256), 256, 0, s>>>(map, V, used, ids, nnz, wl);
  return hipGetLastError();
}

hipError_t launch_prep_emb(const float* emb, int d, int dp, const int* used, int64_t U, float* e32,
                           uint16_t* e16, float* en, hipStream_t s) {
  prep_emb_kernel<<<grid_for(U, 4), 256, 0, s>>>(emb, d, dp, used, U, e32, e16, en);
  return hipGetLastError();
}

hipError_t launch_select(const SelectParams& p, hipStream_t s) {
  select_kernel<<<p.B, 256, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_nan_docs(const int* docs, int64_t ndocs, float* out, hipStream_t s) {
  if (ndocs <= 0) return hipSuccess;
  nan_docs_kernel<<<grid_for(ndocs, 256), 256, 0, s>>>(docs, ndocs, out);
  return hipGetLastError();
}

}  // namespace wmd
