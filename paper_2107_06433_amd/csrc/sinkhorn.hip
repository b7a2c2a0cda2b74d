// Fused SDDMM-SpMM Sinkhorn-Knopp iterations and the final distance pass
// (Algorithm 1 loop and last line; Section III-C, SDDMM_SpMM type 1 and 2).
//
// Work item = one (query, target document) pair.  Documents are independent
// through the whole loop: x_k depends only on u_k, the K^T rows of document
// k's words and c_k.  Each item therefore owns a private group of lanes, the
// doc-major layout needs no atomics (the paper's row split does), and every
// sum has a fixed order, so results are deterministic.
//
// Lane grid of an item: 2^lg_cg "column" lanes x RS "row" lanes.  Column lane
// cg holds the query words cg, cg+CG, ... (TC of them); row lane rs holds the
// document words rs, rs+RS, ... (TR of them).  Each lane keeps its TR x TC
// block of the gathered K^T rows in registers, so one pass per iteration reads
// every element twice -- once for the dot product s_j = K_j . u (SDDMM) and once
// for the update acc += K_j w_j (SpMM) -- which is the paper's fusion.
//
//   s_j   = sum over the item's column lanes of the lane-local dot products
//   w_j   = c_jk / s_j                              (only where c_jk > 0)
//   acc_i = sum over the item's row lanes of K_ji w_j
//   u_i   = r_i / acc_i                             (x = acc / r, u = 1/x)
//
// Final pass: s_j as above, t_j = (K .* M)_j . u, d_k = sum_j c_jk t_j / s_j,
// which equals sum(u .* ((K .* M) v)) with v_j = c_jk / s_j.
//
// Items spanning more than one wave (2^lg_l > 64) finish the acc sums through
// LDS, one barrier per iteration (double-buffered by iteration parity).
#include "lanes.h"
#include "wmd_internal.h"

namespace wmd {

namespace {

template <int TC, int TR, bool MW>
__global__ void __launch_bounds__(MW ? 1024 : 256) sink_kernel(SinkParams p) {
  extern __shared__ float lds[];
  const int lg_cg = p.lg_cg, lg_l = p.lg_l;
  const int CG = 1 << lg_cg;
  const int L = 1 << lg_l;
  const int RS = L >> lg_cg;
  const int lid = threadIdx.x & (L - 1);
  const int cg = lid & (CG - 1);
  const int rs = lid >> lg_cg;
  const int items = MW ? 1 : (int)(blockDim.x >> lg_l);
  const int slot = MW ? 0 : (int)(threadIdx.x >> lg_l);
  const int wbits = lg_l < 6 ? lg_l : 6;          // lane bits of an item inside one wave
  const int wave = threadIdx.x >> 6;
  const int nwaves = MW ? (L >> 6) : 1;
  const int cw_stride = CG * TC;                  // LDS floats per wave and buffer
  const int S = p.S;
  const int vr = *p.vr;

  for (int base = blockIdx.x * items; base < p.ndocs; base += gridDim.x * items) {
    const int item = base + slot;
    const bool active = item < p.ndocs;
    const int k = active ? p.docs[item] : 0;
    const int64_t beg = p.doc_ptr[k];
    const int n = active ? (int)(p.doc_ptr[k + 1] - beg) : 0;

    // ---- gather: this lane's words of document k and their K^T entries
    int wid[TR];
    float cw[TR];
    float K[TR][TC];
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      const int j = rs + RS * t;
      wid[t] = j < n ? p.wl[beg + j] : -1;
      cw[t] = j < n ? p.wn[beg + j] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      const float* row = p.kt + (size_t)(wid[t] < 0 ? 0 : wid[t]) * S;
#pragma unroll
      for (int e = 0; e < TC; ++e) {
        const int col = cg + CG * e;
        const float v = row[col < S ? col : S - 1];  // clamped: never reads past the row
        K[t][e] = (wid[t] >= 0 && col < S) ? v : 0.f;
      }
    }
    float rv[TC], u[TC];
#pragma unroll
    for (int e = 0; e < TC; ++e) {
      const int col = cg + CG * e;
      rv[e] = col < S ? p.r[col] : 0.f;
      if (p.load_u)
        u[e] = (active && col < S) ? p.u[(size_t)k * S + col] : 0.f;
      else
        u[e] = rv[e] > 0.f ? (float)vr : 0.f;  // x = 1/v_r
    }
    float wv[TR];
    if (p.load_w) {
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const int j = rs + RS * t;
        wv[t] = j < n ? p.w[beg + j] : 0.f;
      }
    }

    // ---- Sinkhorn-Knopp iterations
    for (int it = 0; it < p.iters; ++it) {
      if (!p.load_w) {
        float s[TR];
#pragma unroll
        for (int t = 0; t < TR; ++t) {
          float a = 0.f;
#pragma unroll
          for (int e = 0; e < TC; ++e) a = fmaf(K[t][e], u[e], a);
          s[t] = sum_low_bits(a, lg_cg);
        }
#pragma unroll
        for (int t = 0; t < TR; ++t) wv[t] = cw[t] > 0.f ? __fdividef(cw[t], s[t]) : 0.f;
        if (p.store_w) {
          if (cg == 0 && active) {
#pragma unroll
            for (int t = 0; t < TR; ++t) {
              const int j = rs + RS * t;
              if (j < n) p.w[beg + j] = wv[t];
            }
          }
          continue;
        }
      }
      float acc[TC];
#pragma unroll
      for (int e = 0; e < TC; ++e) {
        float a = 0.f;
#pragma unroll
        for (int t = 0; t < TR; ++t) a = fmaf(K[t][e], wv[t], a);
        acc[e] = sum_mid_bits(a, lg_cg, wbits);
      }
      if (MW) {
        float* buf = lds + (it & 1) * nwaves * cw_stride;
        if ((threadIdx.x & 63) < CG) {
#pragma unroll
          for (int e = 0; e < TC; ++e) buf[wave * cw_stride + cg + CG * e] = acc[e];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < TC; ++e) {
          float a = 0.f;
          for (int w = 0; w < nwaves; ++w) a += buf[w * cw_stride + cg + CG * e];
          acc[e] = a;
        }
      }
#pragma unroll
      for (int e = 0; e < TC; ++e) u[e] = rv[e] > 0.f ? __fdividef(rv[e], acc[e]) : 0.f;
    }

    if (p.store_u && rs == 0 && active) {
#pragma unroll
      for (int e = 0; e < TC; ++e) {
        const int col = cg + CG * e;
        if (col < S) p.u[(size_t)k * S + col] = u[e];
      }
    }

    // ---- final pass: d_k = sum_j c_jk ((K.*M)_j . u) / (K_j . u)
    if (p.do_final) {
      float part = 0.f;
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const float* row = p.kmt + (size_t)(wid[t] < 0 ? 0 : wid[t]) * S;
        float a = 0.f, b = 0.f;
#pragma unroll
        for (int e = 0; e < TC; ++e) {
          const int col = cg + CG * e;
          const float kv = row[col < S ? col : S - 1];
          const float km = (wid[t] >= 0 && col < S) ? kv : 0.f;
          a = fmaf(K[t][e], u[e], a);
          b = fmaf(km, u[e], b);
        }
        a = sum_low_bits(a, lg_cg);
        b = sum_low_bits(b, lg_cg);
        if (cw[t] > 0.f) part += cw[t] * __fdividef(b, a);
      }
      part = cg == 0 ? part : 0.f;
      part = sum_low_bits(part, wbits);
      if (MW) {
        __syncthreads();  // the iteration buffers may still be read
        if ((threadIdx.x & 63) == 0) lds[wave] = part;
        __syncthreads();
        float a = 0.f;
        for (int w = 0; w < nwaves; ++w) a += lds[w];
        part = a;
        __syncthreads();
      }
      if (lid == 0 && active) p.out[k] = vr > 0 ? part : __int_as_float(0x7FC00000);
    }
  }
}

// Fallback for items whose K^T block does not fit in registers (very wide
// queries against very long documents): one 256-thread block per item, u and
// w in LDS, the K^T rows re-read from memory on every pass.  Phase 1: each
// wave takes rows j = wave, wave+4, ...; its lanes split the row's columns,
// and a wave sum gives s_j, then w_j.  Phase 2: the same rows, lanes own
// columns, partial sums per wave go through LDS and are added in wave order.
constexpr int kStreamMaxS = 2048;
__global__ void __launch_bounds__(256) sink_stream_kernel(SinkParams p) {
  __shared__ float su[kStreamMaxS];
  __shared__ float sw[kMaxDocLen];
  __shared__ float sacc[4][kStreamMaxS / 2];
  __shared__ float sred[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = p.S;
  const int vr = *p.vr;
  for (int item = blockIdx.x; item < p.ndocs; item += gridDim.x) {
    const int k = p.docs[item];
    const int64_t beg = p.doc_ptr[k];
    const int n = (int)(p.doc_ptr[k + 1] - beg);
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
          a = sum_low_bits(a, 6);
          const float cj = p.wn[beg + j];
          if (lane == 0) {
            const float wj = cj > 0.f ? __fdividef(cj, a) : 0.f;
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
          su[c] = rc > 0.f ? __fdividef(rc, a) : 0.f;
        }
        __syncthreads();
      }
    }
    if (p.store_u)
      for (int c = threadIdx.x; c < S; c += 256) p.u[(size_t)k * S + c] = su[c];
    if (p.do_final) {
      float part = 0.f;
      for (int j = wave; j < n; j += 4) {
        const float* row = p.kt + (size_t)p.wl[beg + j] * S;
        const float* rowm = p.kmt + (size_t)p.wl[beg + j] * S;
        float a = 0.f, b = 0.f;
        for (int c = lane; c < S; c += 64) {
          a = fmaf(row[c], su[c], a);
          b = fmaf(rowm[c], su[c], b);
        }
        a = sum_low_bits(a, 6);
        b = sum_low_bits(b, 6);
        const float cj = p.wn[beg + j];
        if (cj > 0.f) part += cj * __fdividef(b, a);
      }
      if (lane == 0) sred[wave] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        const float tot = ((sred[0] + sred[1]) + sred[2]) + sred[3];
        p.out[k] = vr > 0 ? tot : __int_as_float(0x7FC00000);
      }
    }
    __syncthreads();
  }
}

using KernelFn = void (*)(SinkParams);

// Instantiated (TC, TR) shapes.  Single-wave items allow up to 96 register
// cells per lane; multi-wave items (1024-thread blocks) up to 64.
#define WMD_TC_LIST(X, TR) X(1, TR) X(2, TR) X(3, TR) X(4, TR) X(5, TR) X(6, TR) X(8, TR) X(12, TR) X(16, TR)
#define WMD_TR_LIST(X) WMD_TC_LIST(X, 1) WMD_TC_LIST(X, 2) WMD_TC_LIST(X, 3) WMD_TC_LIST(X, 4) \
  WMD_TC_LIST(X, 6) WMD_TC_LIST(X, 8) WMD_TC_LIST(X, 12) WMD_TC_LIST(X, 16)

struct Entry { int tc, tr; KernelFn sw, mw; };

// Only instantiate what the register budget allows.
template <int TC, int TR, bool MW, bool OK = (TC * TR <= (MW ? 64 : 96))>
struct Pick { static KernelFn get() { return nullptr; } };
template <int TC, int TR, bool MW>
struct Pick<TC, TR, MW, true> { static KernelFn get() { return (KernelFn)sink_kernel<TC, TR, MW>; } };

#define WMD_ENTRY2(TC, TR) {TC, TR, Pick<TC, TR, false>::get(), Pick<TC, TR, true>::get()},

const Entry* table(int* n) {
  static const Entry t[] = {WMD_TR_LIST(WMD_ENTRY2)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

KernelFn find(const SinkConfig& c) {
  int n;
  const Entry* t = table(&n);
  for (int i = 0; i < n; ++i)
    if (t[i].tc == c.tc && t[i].tr == c.tr) return c.multiwave ? t[i].mw : t[i].sw;
  return nullptr;
}

const int kTC[] = {1, 2, 3, 4, 5, 6, 8, 12, 16};
const int kTR[] = {1, 2, 3, 4, 6, 8, 12, 16};

}  // namespace

bool sink_config_supported(const SinkConfig& c) { return c.stream ? c.tc <= kStreamMaxS : find(c) != nullptr; }

int sink_block(const SinkConfig& c) { return c.stream ? 256 : c.multiwave ? (1 << c.lg_l) : 256; }

int sink_grid(const SinkConfig& c, int ndocs) {
  const int items = (c.stream || c.multiwave) ? 1 : 256 >> c.lg_l;
  int g = (ndocs + items - 1) / items;
  return g < 1 ? 1 : g;
}

// Cost model: VALU instructions per item and iteration, per wave, times the
// waves an item occupies, divided by the items sharing a wave.  Two FMAs per
// register cell, one DPP step per summed lane bit, a few instructions per row
// and column for the divisions and masks, and an LDS round per column for
// multi-wave items.
bool choose_sink_config(int S, int cap, SinkConfig* out) {
  double best = 1e300;
  bool found = false;
  for (int lg_l = 4; lg_l <= 10; ++lg_l) {
    for (int lg_cg = 0; lg_cg <= 6 && lg_cg <= lg_l; ++lg_cg) {
      const int CG = 1 << lg_cg, RS = (1 << lg_l) >> lg_cg;
      int tc = 0, tr = 0;
      for (int v : kTC) if (v * CG >= S) { tc = v; break; }
      for (int v : kTR) if (v * RS >= cap) { tr = v; break; }
      if (!tc || !tr) continue;
      const bool mw = lg_l > 6;
      SinkConfig c{tc, tr, lg_cg, lg_l, mw, false};
      if (!find(c)) continue;
      if (mw && 2 * ((1 << lg_l) >> 6) * (CG * tc) * sizeof(float) > 65536) continue;
      const int wbits = lg_l < 6 ? lg_l : 6;
      const double per_wave = 2.0 * tc * tr + tr * (lg_cg + 4) + tc * (wbits - lg_cg + 4) +
                              (mw ? tc * ((1 << lg_l) >> 6) * 1.5 + 16 : 0);
      const double waves = lg_l >= 6 ? (double)((1 << lg_l) >> 6) : (double)(1 << lg_l) / 64.0;
      const double cost = per_wave * waves;
      if (cost < best - 1e-9) { best = cost; *out = c; found = true; }
    }
  }
  if (!found && S <= kStreamMaxS && cap <= kMaxDocLen) {
    *out = SinkConfig{S, cap, 6, 8, false, true};
    found = true;
  }
  return found;
}

hipError_t launch_sink(const SinkParams& p, const SinkConfig& c, int grid, hipStream_t s) {
  if (c.stream) {
    if (p.S > kStreamMaxS) return hipErrorInvalidValue;
    sink_stream_kernel<<<grid, 256, 0, s>>>(p);
    return hipGetLastError();
  }
  KernelFn fn = find(c);
  if (!fn) return hipErrorInvalidValue;
  const int block = sink_block(c);
  const size_t lds = c.multiwave ? sizeof(float) * (size_t)2 * ((1 << c.lg_l) >> 6) * ((1 << c.lg_cg) * c.tc) : 0;
  SinkParams q = p;
  q.lg_cg = c.lg_cg;
  q.lg_l = c.lg_l;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, q);
  return hipGetLastError();
}

}  // namespace wmd
