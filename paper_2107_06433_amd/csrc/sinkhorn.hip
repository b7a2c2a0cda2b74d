// Launch side of the fused Sinkhorn kernels: the streaming fallback, the
// table of instantiated register-resident shapes and the choice among them.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "sink_kernel.h"

namespace wmd {

namespace {

// Fallback for items whose K^T block does not fit in registers (very wide
// queries against very long documents): one 256-thread block per item, u and
// w in LDS, the K^T rows re-read from memory on every pass.  Phase 1: each
// wave takes rows j = wave, wave+4, ...; its lanes split the row's columns,
// and a wave sum gives s_j, then w_j.  Phase 2: the same rows, lanes own
// columns, partial sums per wave go through LDS and are added in wave order.
constexpr int kStreamMaxS = 2048;

__device__ __forceinline__ float sum_wave(float x) {
  float v[1] = {x};
  sum_low<6>(v);
  return v[0];
}

__global__ void __launch_bounds__(256) sink_stream_kernel(SinkParams p) {
  __shared__ float su[kStreamMaxS];
  __shared__ float sw[kMaxDocLen];
  __shared__ float sacc[4][kStreamMaxS / 2];
  __shared__ float sred[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = p.S;
  const int vr = *p.vr;
  for (int item = blockIdx.x; item < p.ndocs; item += gridDim.x) {
    const int4 rec = p.drec[item];
    const int64_t beg = rec_begin(rec);
    const int n = rec.z, k = rec.w;
    for (int c = threadIdx.x; c < S; c += 256)
      su[c] = p.load_u ? p.u[(size_t)k * S + c] : (p.r[c] > 0.f ? (float)vr : 0.f);
    if (p.load_w)
      for (int j = threadIdx.x; j < n; j += 256) sw[j] = p.w[beg + j];
    __syncthreads();
    for (int it = 0; it < p.iters; ++it) {
      if (!p.load_w) {
        for (int j = wave; j < n; j += 4) {
          const float* row = p.kt + (size_t)p.wl[beg + j] * S;
          float a = 0.f;
          for (int c = lane; c < S; c += 64) a = fmaf(row[c], su[c], a);
          a = sum_wave(a);
          const float cj = p.wn[beg + j];
          if (lane == 0) {
            const float wj = cj > 0.f ? fast_div(cj, a) : 0.f;
            sw[j] = wj;
            if (p.store_w) p.w[beg + j] = wj;
          }
        }
        __syncthreads();
        if (p.store_w) continue;
      }
      // columns in halves of kStreamMaxS/2 so the partial sums fit in LDS
      for (int c0 = 0; c0 < S; c0 += kStreamMaxS / 2) {
        float acc[kStreamMaxS / 2 / 64];
#pragma unroll
        for (int i = 0; i < kStreamMaxS / 2 / 64; ++i) acc[i] = 0.f;
        for (int j = wave; j < n; j += 4) {
          const float* row = p.kt + (size_t)p.wl[beg + j] * S;
          const float wj = sw[j];
#pragma unroll
          for (int i = 0; i < kStreamMaxS / 2 / 64; ++i) {
            const int c = c0 + lane + 64 * i;
            if (c < S) acc[i] = fmaf(row[c], wj, acc[i]);
          }
        }
#pragma unroll
        for (int i = 0; i < kStreamMaxS / 2 / 64; ++i) sacc[wave][lane + 64 * i] = acc[i];
        __syncthreads();
        for (int c = c0 + threadIdx.x; c < S && c < c0 + kStreamMaxS / 2; c += 256) {
          const float a = ((sacc[0][c - c0] + sacc[1][c - c0]) + sacc[2][c - c0]) + sacc[3][c - c0];
          const float rc = p.r[c];
          su[c] = rc > 0.f ? fast_div(rc, a) : 0.f;
        }
        __syncthreads();
      }
    }
    if (p.store_u)
      for (int c = threadIdx.x; c < S; c += 256) p.u[(size_t)k * S + c] = su[c];
    if (p.do_final) {
      // d_k = sum_j c_j (m_j - (ln 2 / lambda) (K_j . (u log2 K_j)) / (K_j . u))
      // for the row-scaled K (M_ij = m_j - ln(K_ij) / lambda)
      const float scale = kNegLn2 * p.inv_lam;
      float part = 0.f;
      for (int j = wave; j < n; j += 4) {
        const int wj = p.wl[beg + j];
        const float* row = p.kt + (size_t)wj * S;
        float a = 0.f, b = 0.f;
        for (int c = lane; c < S; c += 64) {
          const float ku = row[c] * su[c];
          a += ku;
          b = fmaf(ku, log2_gibbs(row[c]), b);
        }
        a = sum_wave(a);
        b = sum_wave(b);
        const float cj = p.wn[beg + j];
        if (cj > 0.f) part += cj * fmaf(scale, fast_div(b, a), p.km[wj]);
      }
      if (lane == 0) sred[wave] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        const float tot = ((sred[0] + sred[1]) + sred[2]) + sred[3];
        p.out[k] = vr > 0 ? flag_range(tot) : __int_as_float(0x7FC00000);
        if (p.iters_out) p.iters_out[k] = p.iters;  // no tolerance stop on this path
      }
    }
    __syncthreads();
  }
}

// regs and spills are those of the resident-only variant: shapes are chosen
// for the resident schedule, and the other schedules (comparison baselines)
// run the general variant of the same shape.
struct Shape {
  SinkEntry e;
  int regs;      // VGPRs per lane of the compiled kernel
  bool spills;   // uses private (scratch) memory
};

const std::vector<Shape>& shapes() {
  static std::vector<Shape> all;
  static std::once_flag once;
  std::call_once(once, [] {
    const SinkEntry* (*tabs[])(int*) = {sink_table_cg0, sink_table_cg1, sink_table_cg2, sink_table_cg3,
                                         sink_table_cg4, sink_table_cg5, sink_table_cg6};
    for (auto tab : tabs) {
      int n = 0;
      const SinkEntry* t = tab(&n);
      for (int i = 0; i < n; ++i) {
        if (!t[i].fn) continue;
        hipFuncAttributes a{};
        int regs = 128;
        bool spills = false;
        if (hipFuncGetAttributes(&a, t[i].fn) == hipSuccess) {
          if (a.numRegs > 0) regs = a.numRegs;
          spills = a.localSizeBytes > 0;
        }
        all.push_back(Shape{t[i], regs, spills});
      }
    }
  });
  return all;
}

// The compiled variant for a launch: the resident-only one when the launch
// neither loads nor stores u or w.
const void* kernel_for(const Shape& sh, const SinkParams& p) {
  const bool resident = !p.load_u && !p.store_u && !p.load_w && !p.store_w;
  return resident ? sh.e.fn : sh.e.fn_sched;
}

const Shape* find_shape(const SinkConfig& c) {
  for (const Shape& s : shapes())
    if (s.e.tc == c.tc && s.e.tr == c.tr && s.e.lg_cg == c.lg_cg && s.e.maxw == c.maxw) return &s;
  return nullptr;
}

// Multi-wave items: per-wave column partials and column results, both
// doubled for the alternation by iteration parity, and r per column.
size_t lds_bytes(const SinkConfig& c) {
  const size_t cols = (size_t)(1 << c.lg_cg) * c.tc;
  // two parity buffers of per-wave column partials, two of column results, r
  return c.multiwave ? sizeof(float) * (2 * c.nwaves * cols + 3 * cols) : 0;
}

}  // namespace

bool sink_config_supported(const SinkConfig& c) {
  return c.stream ? true : find_shape(c) != nullptr;
}

int sink_block(const SinkConfig& c) { return c.stream ? 256 : c.multiwave ? 64 * c.nwaves : 256; }

int sink_grid(const SinkConfig& c, int ndocs) {
  const int items = (c.stream || c.multiwave) ? 1 : 4;
  int g = (ndocs + items - 1) / items;
  return g < 1 ? 1 : g;
}

// Cost model over the compiled shapes.  Per wave and iteration a shape
// issues about I = 2 tr tc FMAs, tr lg_cg + tc (6 - lg_cg) DPP/permlane sums,
// 2 instructions per row and per column for the reciprocals, and for
// multi-wave items the two-phase LDS sum (about 2 tc + nwaves, plus two
// barriers counted as 40).  With W = items x nwaves waves
// on 1024 SIMDs the time is the larger of the issue-bound estimate
// W I 4 / 1024 cycles and the latency-bound one: rounds of `occupancy`
// resident waves per SIMD, each taking ~8 cycles per dependent instruction.
namespace {

double model_cost(const Shape& sh, int nw, int ndocs) {
  const SinkEntry& e = sh.e;
  const bool mw = e.maxw > 1;
  const int regs = (sh.regs + 7) & ~7;
  int occ = 512 / regs;
  occ = occ > 8 ? 8 : occ;
  const double I = 2.0 * e.tr * e.tc + e.tr * e.lg_cg + e.tc * (6 - e.lg_cg) + 2.0 * e.tr + 2.0 * e.tc +
                   (mw ? 2.0 * e.tc + nw + 20.0 * nw : 0.0);
  const double waves = (double)ndocs * nw;
  const double t_issue = waves * I * 4.0 / 1024.0;
  const double rounds = std::ceil(waves / (1024.0 * occ));
  const double t_lat = rounds * I * 8.0;
  return t_issue > t_lat ? t_issue : t_lat;
}

// The waves per document a shape needs for `cap` rows, or 0 if it cannot hold them.
int waves_for(const SinkEntry& e, int S, int cap) {
  const int CG = 1 << e.lg_cg, RSW = 64 >> e.lg_cg;
  if (e.tc * CG < S || (e.tc - 1) * CG >= S) return 0;  // the smallest tc that covers S
  if (e.maxw == 1) {
    if (RSW * e.tr < cap || (e.tr > 1 && RSW * (e.tr / 2) >= cap)) return 0;
    return 1;
  }
  const int nw = (cap + RSW * e.tr - 1) / (RSW * e.tr);
  return (nw < 2 || nw > e.maxw) ? 0 : nw;
}

}  // namespace

bool sink_config_fits(const SinkConfig& c, int S, int cap) {
  if (c.stream) return S <= kStreamMaxS && cap <= kMaxDocLen;
  const Shape* sh = find_shape(c);
  if (!sh || sh->spills) return false;
  const int nw = waves_for(sh->e, S, cap);
  return nw > 0 && nw == c.nwaves && lds_bytes(c) <= 65536;
}

// Cost model over the compiled shapes.  Per wave and iteration a shape
// issues about I = 2 tr tc FMAs, tr lg_cg + tc (6 - lg_cg) DPP/permlane sums,
// 2 instructions per row and per column for the reciprocals, and for
// multi-wave items the two-phase LDS sum (about 2 tc + nwaves, plus barriers).
// With W = items x nwaves waves on 1024 SIMDs the time is the larger of the
// issue-bound estimate W I 4 / 1024 cycles and the latency-bound one: rounds
// of `occupancy` resident waves per SIMD, ~8 cycles per dependent instruction.
// Measured tuning tables override this choice per (S, cap).
int sink_candidates(int S, int cap, int ndocs, SinkConfig* out, int max) {
  std::vector<std::pair<double, SinkConfig>> all;
  for (const Shape& sh : shapes()) {
    if (sh.spills) continue;
    const int nw = waves_for(sh.e, S, cap);
    if (!nw) continue;
    const bool mw = sh.e.maxw > 1;
    SinkConfig c{sh.e.tc, sh.e.tr, sh.e.lg_cg, nw, mw, false, sh.e.maxw};
    if (lds_bytes(c) > 65536) continue;
    const int regs = (sh.regs + 7) & ~7;
    const int occ = 512 / regs > 8 ? 8 : 512 / regs;
    if (mw && (4 * occ) / nw < 1) continue;
    all.push_back({model_cost(sh, nw, ndocs), c});
  }
  std::stable_sort(all.begin(), all.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  int n = 0;
  for (const auto& a : all) {
    if (n < max) out[n] = a.second;
    ++n;
  }
  if (S <= kStreamMaxS && cap <= kMaxDocLen) {
    if (n < max) out[n] = SinkConfig{0, 0, 6, 4, false, true, 4};
    ++n;
  }
  return n;
}

bool choose_sink_config(int S, int cap, int ndocs, SinkConfig* out) {
  SinkConfig c[1];
  if (sink_candidates(S, cap, ndocs, c, 1) < 1) return false;
  *out = c[0];
  return true;
}

hipError_t launch_sink(const SinkParams& p, const SinkConfig& c, int grid, hipStream_t s, const SinkQuerySet* qs) {
  const int nq = qs ? qs->nq : 0;
  if (nq < 0 || nq > kMaxLaunchQueries) return hipErrorInvalidValue;
  if (c.stream) {
    if (nq > 0) return hipErrorInvalidValue;  // the fallback runs one query per launch
    if (p.S > kStreamMaxS) return hipErrorInvalidValue;
    sink_stream_kernel<<<grid, 256, 0, s>>>(p);
    return hipGetLastError();
  }
  const Shape* sh = find_shape(c);
  if (!sh) return hipErrorInvalidValue;
  const int total = grid * (nq > 0 ? nq : 1);
  if (sh->e.maxw == 1) {  // a merged launch with a single group
    SinkMerge m{};
    m.p = p;
    if (qs) m.qs = *qs;
    m.ngroups = 1;
    m.end[0] = total;
    m.ndocs[0] = p.ndocs;
    void* args[] = {&m};
    return hipLaunchKernel(kernel_for(*sh, p), dim3(total), dim3(256), args, 0, s);
  }
  SinkParams a = p;
  SinkQuerySet q{};
  if (qs) q = *qs;
  void* args[] = {&a, &q};
  return hipLaunchKernel(kernel_for(*sh, p), dim3(total), dim3(sink_block(c)), args, lds_bytes(c), s);
}

namespace {

// Rows per lane a one-wave item of 2^lg_cg column lanes needs for `cap` words.
int tr_needed(int lg_cg, int cap) {
  const int rsw = 64 >> lg_cg;
  int tr = 1;
  while (rsw * tr < cap) tr *= 2;
  return tr;
}

// ipw: items per wave (2 for half-wave items, whose column sums span one
// lane bit fewer).
double merged_cost(const Shape& variant, const int* tr, const int* ipw, const int* nd, int n) {
  const SinkEntry& e = variant.e;
  const int regs = (variant.regs + 7) & ~7;
  int occ = 512 / regs;
  occ = occ > 8 ? 8 : occ;
  double issue = 0.0, imax = 0.0, waves = 0.0;
  for (int i = 0; i < n; ++i) {
    const int rbits = (ipw[i] == 2 ? 5 : 6) - e.lg_cg;
    const double I = 2.0 * tr[i] * e.tc + tr[i] * e.lg_cg + e.tc * rbits + 2.0 * tr[i] + 2.0 * e.tc;
    const double w = std::ceil((double)nd[i] / ipw[i]);
    issue += w * I * 4.0 / 1024.0;
    imax = I > imax ? I : imax;
    waves += w;
  }
  const double lat = std::ceil(waves / (1024.0 * occ)) * imax * 8.0;
  return issue > lat ? issue : lat;
}

}  // namespace

// One launch for the buckets of one query that one-wave items can hold.  A
// candidate is a compiled one-wave shape (tc, TRMAX, lg_cg) whose columns
// cover S with the fewest padded columns: the buckets needing at most TRMAX
// rows per lane join (at least one needing exactly TRMAX), each with the
// smallest of TRMAX, TRMAX/2, TRMAX/4 that holds it; the others keep launches
// of their own.  A bucket that fits in half a wave at no more than TRMAX rows
// per lane runs as half-wave items (lg_cg <= 4): two documents per wave and
// one lane bit fewer in every column sum, which costs less per document.  The candidate holding the most buckets wins, the lowest
// modelled time (the separate launches included) among equals.  Measured on
// single queries, one launch over every bucket beat splitting them even where
// the model preferred a split: the short items fill in behind the long ones.
bool plan_merge(int S, const int* cap, const int* ndocs, int nb, MergePlan* out) {
  double best = 0.0;
  bool found = false;
  std::vector<double> alone((size_t)nb, -1.0);
  for (const Shape& sh : shapes()) {
    const SinkEntry& e = sh.e;
    if (e.maxw != 1 || sh.spills) continue;
    const int CG = 1 << e.lg_cg;
    if (e.tc * CG < S || (e.tc - 1) * CG >= S) continue;
    MergePlan p{};
    p.tc = e.tc; p.trmax = e.tr; p.lg_cg = e.lg_cg;
    int trs[kMergeMax], nds[kMergeMax], ipws[kMergeMax];
    bool exact = false;
    double rest = 0.0;
    for (int i = 0; i < nb; ++i) {
      const int t = tr_needed(e.lg_cg, cap[i]);
      if (t > e.tr || p.n == kMergeMax) {
        if (alone[(size_t)i] < 0.0) {
          alone[(size_t)i] = 1e30;
          for (const Shape& o : shapes()) {
            if (o.spills) continue;
            const int nw = waves_for(o.e, S, cap[i]);
            if (!nw) continue;
            SinkConfig oc{o.e.tc, o.e.tr, o.e.lg_cg, nw, o.e.maxw > 1, false, o.e.maxw};
            if (lds_bytes(oc) > 65536) continue;
            alone[(size_t)i] = std::min(alone[(size_t)i], model_cost(o, nw, ndocs[i]));
          }
        }
        rest += alone[(size_t)i];
        continue;
      }
      const bool half = e.lg_cg <= 4 && 2 * t <= e.tr;  // half a wave needs twice the rows per lane
      const int th = half ? 2 * t : t;
      exact = exact || th == e.tr;
      int shift = 0;
      while (shift < 2 && (e.tr >> (shift + 1)) >= th) ++shift;
      p.member[p.n] = i;
      p.body[p.n] = shift | (half ? 4 : 0);
      trs[p.n] = e.tr >> shift;
      ipws[p.n] = half ? 2 : 1;
      nds[p.n] = ndocs[i];
      ++p.n;
    }
    if (p.n == 0 || !exact) continue;
    const double c = merged_cost(sh, trs, ipws, nds, p.n) + rest;
    if (!found || p.n > out->n || (p.n == out->n && c < best)) {
      best = c;
      *out = p;
      found = true;
    }
  }
  if (!found) return false;
  // longest documents first
  MergePlan& p = *out;
  for (int i = 1; i < p.n; ++i)
    for (int j = i; j > 0 && cap[p.member[j]] > cap[p.member[j - 1]]; --j) {
      std::swap(p.member[j], p.member[j - 1]);
      std::swap(p.body[j], p.body[j - 1]);
    }
  return true;
}

hipError_t launch_sink_merged(const SinkParams& p, const MergePlan& plan, const int* off, const int* ndocs,
                              hipStream_t s, int* grid_out, const SinkQuerySet* qs) {
  SinkConfig c{plan.tc, plan.trmax, plan.lg_cg, 1, false, false, 1};
  const Shape* sh = find_shape(c);
  const int nq = qs ? qs->nq : 0;
  if (!sh || plan.n < 1 || plan.n > kMergeMax || nq < 0 || nq > kMaxLaunchQueries) return hipErrorInvalidValue;
  SinkMerge m{};
  m.p = p;
  if (qs) m.qs = *qs;
  m.ngroups = plan.n;
  int grid = 0;
  for (int g = 0; g < plan.n; ++g) {
    const int per_block = (plan.body[g] & 4) ? 8 : 4;  // items per block of four waves
    grid += (nq > 0 ? nq : 1) * ((ndocs[g] + per_block - 1) / per_block);
    m.end[g] = grid;
    m.off[g] = off[g];
    m.ndocs[g] = ndocs[g];
    m.body[g] = plan.body[g];
  }
  *grid_out = grid;
  if (grid == 0) return hipSuccess;
  void* args[] = {&m};
  return hipLaunchKernel(kernel_for(*sh, p), dim3(grid), dim3(256), args, 0, s);
}

}  // namespace wmd
