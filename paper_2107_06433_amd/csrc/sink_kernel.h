// Fused SDDMM-SpMM Sinkhorn-Knopp iterations and the final distance pass
// (Algorithm 1 loop and last line; Section III-C, SDDMM_SpMM type 1 and 2).
//
// Work item = one (query, target document) pair.  Documents are independent
// through the whole loop: x_k depends only on u_k, the K^T rows of document
// k's words and c_k.  Each item therefore owns private lanes, the doc-major
// layout needs no atomics (the paper's row split does), and every sum has a
// fixed order, so results are deterministic.
//
// Lane grid of an item: CG = 2^LG_CG column lanes x RS row lanes, one wave
// (64 lanes) or `nwaves` waves of one block (MW).  Column lane cg holds the
// query words cg, cg+CG, ... (TC of them); row lane rs holds the document
// words rs, rs+RS, ... (TR of them).  Each lane keeps its TR x TC block of the
// gathered K^T rows in registers, so every iteration reads each element
// twice -- for the dot product s_j = K_j . u (SDDMM) and for the update
// acc += K_j w_j (SpMM) -- the paper's fusion, with no sparse intermediate:
//
//   s_j   = sum over the column lanes of the lane-local dot products
//   w_j   = c_jk / s_j                              (only where c_jk > 0)
//   acc_i = sum over the row lanes of K_ji w_j
//   u_i   = r_i / acc_i                             (x = acc / r, u = 1/x)
//
// The final pass computes s_j and t_j = (K.*M)_j . u and
// d_k = sum_j c_jk t_j / s_j = sum(u .* ((K.*M) v)) with v_j = c_jk / s_j,
// recovering each M entry from the K entry it already holds.
// The lane geometry is compile-time so every cross-lane sum is a fixed
// sequence of DPP / permlane steps the compiler can interleave across rows.
#pragma once

#include "lanes.h"
#include "wmd_internal.h"

namespace wmd {

// Sum over lane bits [0, NB) of every element of x, step by step across the
// array so independent DPP chains interleave.  Lower bits first: the mirror
// patterns flip several bits at once and are only sums once the lower bits
// hold equal values.
template <int NB, int N>
__device__ __forceinline__ void sum_low(float (&x)[N]) {
  if constexpr (NB > 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppXor1>(x[i]);
  }
  if constexpr (NB > 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppXor2>(x[i]);
  }
  if constexpr (NB > 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppHalfMirror>(x[i]);
  }
  if constexpr (NB > 3) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppMirror>(x[i]);
  }
  if constexpr (NB > 4) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = add_xor16(x[i]);
  }
  if constexpr (NB > 5) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = add_xor32(x[i]);
  }
}

// Sum over lane bits [LO, 6) of a wave; bits below LO address different values.
// Bits 2 and 3 together are row_ror:8 then row_ror:4 (a clean 4-lane sum only
// when both are summed, which holds since the range always ends at bit 6).
template <int LO, int N, bool PERM = true>
__device__ __forceinline__ void sum_high(float (&x)[N]) {
  if constexpr (LO <= 3) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppRor8>(x[i]);
  }
  if constexpr (LO <= 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppRor4>(x[i]);
  }
  if constexpr (LO <= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppXor2>(x[i]);
  }
  if constexpr (LO <= 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += dpp<kDppXor1>(x[i]);
  }
  if constexpr (PERM && LO <= 4) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = add_xor16(x[i]);
  }
  if constexpr (PERM && LO <= 5) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = add_xor32(x[i]);
  }
}

// x[e] / (sum over the permlane bits of den[e]) for e < N, where the bits are
// bit 4 (M = 1), bit 5 (M = 2) or both (M = 3) and every other lane bit has
// been summed already or addresses different values.  Instead of a full
// reduction per element, 4 (M = 3) or 2 elements share one register: each
// 16-lane group (half) ends up with the total of a different element, one
// reciprocal serves them all, and the quotients are gathered back.  The
// numerators come packed the same way (pack_high, once per item).
template <int M, int N>
struct HighPack {
  static constexpr int NQ = M == 3 ? N / 4 : 0;               // groups of four elements
  static constexpr int NP = M == 3 ? (N % 4) / 2 : N / 2;     // pairs
  static constexpr int N1 = N % 2;                            // a last single element
  static constexpr int P = NQ + NP + N1;
};

// sel ? b : a as a bit blend.  A plain select between two elements of one
// register array can be turned into a load at a lane-dependent index, which
// would move the whole array to scratch memory.
__device__ __forceinline__ float pick(bool sel, float a, float b) {
  const int m = -(int)sel;
  return __int_as_float((__float_as_int(a) & ~m) | (__float_as_int(b) & m));
}

template <int M, int N>
__device__ __forceinline__ void pack_high(const float (&x)[N], float (&xp)[HighPack<M, N>::P], int lane) {
  using H = HighPack<M, N>;
  const int g = (lane >> 4) & 3;
#pragma unroll
  for (int q = 0; q < H::NQ; ++q)
    xp[q] = pick(g & 2, pick(g & 1, x[4 * q], x[4 * q + 1]), pick(g & 1, x[4 * q + 2], x[4 * q + 3]));
#pragma unroll
  for (int i = 0; i < H::NP; ++i) {
    const int a = 4 * H::NQ + 2 * i;
    const int sel = M == 2 ? (lane >> 5) & 1 : g & 1;
    xp[H::NQ + i] = pick(sel, x[a], x[a + 1]);
  }
  if constexpr (H::N1 > 0) xp[H::NQ + H::NP] = x[N - 1];
}

// LO < 4: the sums also run over lane bits [LO, 4), added with DPP after the
// packing, so once per register instead of once per element (every 16-lane
// row holds one element then, and row_ror / quad_perm keep the bits below LO
// apart).
template <int LO>
__device__ __forceinline__ float sum_row_bits(float z) {
  if constexpr (LO <= 3) z += dpp<kDppRor8>(z);
  if constexpr (LO <= 2) z += dpp<kDppRor4>(z);
  if constexpr (LO <= 1) z += dpp<kDppXor2>(z);
  if constexpr (LO <= 0) z += dpp<kDppXor1>(z);
  return z;
}

template <int M, int N, int LO = 4>
__device__ __forceinline__ void high_div(const float (&np)[HighPack<M, N>::P], const float (&den)[N], float (&out)[N]) {
  using H = HighPack<M, N>;
#pragma unroll
  for (int q = 0; q < H::NQ; ++q) {
    const int a = 4 * q;
    const float z = sum_row_bits<LO>(
        sum_scatter32(sum_scatter16(den[a], den[a + 1]), sum_scatter16(den[a + 2], den[a + 3])));
    const float v = fast_div(np[q], z);
    float lo, hi;
    gather32(v, lo, hi);
    gather16(lo, out[a], out[a + 1]);
    gather16(hi, out[a + 2], out[a + 3]);
  }
#pragma unroll
  for (int i = 0; i < H::NP; ++i) {
    const int a = 4 * H::NQ + 2 * i;
    if constexpr (M == 2) {
      const float v = fast_div(np[H::NQ + i], sum_row_bits<LO>(sum_scatter32(den[a], den[a + 1])));
      gather32(v, out[a], out[a + 1]);
    } else {
      float z = sum_scatter16(den[a], den[a + 1]);
      if constexpr (M == 3) z = add_xor32(z);
      const float v = fast_div(np[H::NQ + i], sum_row_bits<LO>(z));
      gather16(v, out[a], out[a + 1]);
    }
  }
  if constexpr (H::N1 > 0) {
    float z = sum_row_bits<LO>(den[N - 1]);
    if constexpr (M & 1) z = add_xor16(z);
    if constexpr (M & 2) z = add_xor32(z);
    out[N - 1] = fast_div(np[H::NQ + H::NP], z);
  }
}

// The same idea inside a lane quad, with DPP: x[e] / (sum over lane bit 0
// (L = 1) or bits 0 and 1 (L = 2) of den[e]), optionally also summed over
// lane bits 2 and 3 (HI23) and then over bit 4 (HB >= 1) and bit 5 (HB = 2)
// with permlane swaps.  The rows come in groups of four (L = 2), then pairs,
// then a last single row; quad lane q ends up with the total of row a + q of
// a group (a + (q & 1) of a pair), divides once, and quad permutations give
// every lane all the quotients.
//
// Two forms.  In natural slots (PERM false) every lane holds row t in slot
// t, and each reduce-scatter step picks which element to keep and which to
// hand over with two selects.  With permuted slots (PERM) slot a + s of quad
// lane q holds row a + (s ^ q) of a group of four, row a + (s ^ (q & 1)) of a
// pair (row_slot): then for every lane the bit-0 step is its slot a plus its
// partner's slot a + 1 (and slots a + 2, a + 3 alike), the bit-1 step its
// first partial plus its bit-1 partner's second, one DPP add each and no
// selects; the row a lane keeps is the row in its slot a, so its numerator
// is slot a of x, and slot a of the quotients needs no move.  Both forms add
// the same two operands at every step.
template <int L, int N>
struct LowPack {
  static constexpr int NQ = L == 2 ? N / 4 : 0;
  static constexpr int NP = L == 2 ? (N % 4) / 2 : N / 2;
  static constexpr int N1 = N % 2;
  static constexpr int P = NQ + NP + N1;
};

// Register slot t of quad lane q holds row row_slot(t) of the lane's rows
// (a permutation inside each group; q = lane & 3, or lane & 1 for L = 1).
template <int L, int N>
__device__ __forceinline__ int row_slot(int t, int q) {
  using H = LowPack<L, N>;
  return t < 4 * H::NQ ? t ^ q : t < 4 * H::NQ + 2 * H::NP ? t ^ (q & 1) : t;
}

// The numerators of the rows whose totals this lane will hold.
template <int L, int N, bool PERM>
__device__ __forceinline__ void pack_low(const float (&x)[N], float (&xp)[LowPack<L, N>::P], int lane) {
  using H = LowPack<L, N>;
  const int q = lane & 3;
#pragma unroll
  for (int i = 0; i < H::NQ; ++i)
    xp[i] = PERM ? x[4 * i]
                 : pick(q & 2, pick(q & 1, x[4 * i], x[4 * i + 1]), pick(q & 1, x[4 * i + 2], x[4 * i + 3]));
#pragma unroll
  for (int i = 0; i < H::NP; ++i) {
    const int a = 4 * H::NQ + 2 * i;
    xp[H::NQ + i] = PERM ? x[a] : pick(q & 1, x[a], x[a + 1]);
  }
  if constexpr (H::N1 > 0) xp[H::NQ + H::NP] = x[N - 1];
}

template <int L, bool HI23, int HB, int N, bool PERM>
__device__ __forceinline__ void low_div(const float (&np)[LowPack<L, N>::P], const float (&den)[N], float (&out)[N],
                                        int lane) {
  using H = LowPack<L, N>;
  const bool b0 = lane & 1, b1 = lane & 2;
  // natural slots: lane parity b0 keeps element (b0 ? b : a) and hands its
  // partner the other
  auto pair0 = [&](float a, float b) {
    // opaque copies: a select between two elements of one register array can
    // become a load at a lane-dependent index (see pick)
    asm("" : "+v"(a), "+v"(b));
    return (b0 ? b : a) + dpp<kDppXor1>(b0 ? a : b);
  };
  auto hi23 = [&](float z) {
    if constexpr (HI23) {
      z += dpp<kDppRor8>(z);
      z += dpp<kDppRor4>(z);
    }
    if constexpr (HB > 0) z = add_xor16(z);
    if constexpr (HB > 1) z = add_xor32(z);
    return z;
  };
#pragma unroll
  for (int i = 0; i < H::NQ; ++i) {
    const int a = 4 * i;
    if constexpr (PERM) {
      const float z0 = den[a] + dpp<kDppXor1>(den[a + 1]);
      const float z2 = den[a + 2] + dpp<kDppXor1>(den[a + 3]);
      const float v = fast_div(np[i], hi23(z0 + dpp<kDppXor2>(z2)));
      out[a] = v;
      out[a + 1] = dpp<kDppXor1>(v);
      out[a + 2] = dpp<kDppXor2>(v);
      out[a + 3] = dpp<kDppXor3>(v);
    } else {
      const float pab = pair0(den[a], den[a + 1]), pcd = pair0(den[a + 2], den[a + 3]);
      const float z = hi23((b1 ? pcd : pab) + dpp<kDppXor2>(b1 ? pab : pcd));
      const float v = fast_div(np[i], z);
      out[a] = dpp<0x00>(v);      // quad_perm [0,0,0,0]
      out[a + 1] = dpp<0x55>(v);  // quad_perm [1,1,1,1]
      out[a + 2] = dpp<0xAA>(v);  // quad_perm [2,2,2,2]
      out[a + 3] = dpp<0xFF>(v);  // quad_perm [3,3,3,3]
    }
  }
#pragma unroll
  for (int i = 0; i < H::NP; ++i) {
    const int a = 4 * H::NQ + 2 * i;
    float z = PERM ? den[a] + dpp<kDppXor1>(den[a + 1]) : pair0(den[a], den[a + 1]);
    if constexpr (L == 2) z += dpp<kDppXor2>(z);
    const float v = fast_div(np[H::NQ + i], hi23(z));
    if constexpr (PERM) {
      out[a] = v;
      out[a + 1] = dpp<kDppXor1>(v);
    } else {
      out[a] = dpp<0xA0>(v);      // quad_perm [0,0,2,2]
      out[a + 1] = dpp<0xF5>(v);  // quad_perm [1,1,3,3]
    }
  }
  if constexpr (H::N1 > 0) {
    float z = den[N - 1];
    z += dpp<kDppXor1>(z);
    if constexpr (L == 2) z += dpp<kDppXor2>(z);
    out[N - 1] = fast_div(np[H::NQ + H::NP], hi23(z));
  }
}

// Maximum over lane bits [0, NB), lower bits first (as sum_low).
template <int NB>
__device__ __forceinline__ float max_low(float x) {
  if constexpr (NB > 0) x = fmaxf(x, dpp<kDppXor1>(x));
  if constexpr (NB > 1) x = fmaxf(x, dpp<kDppXor2>(x));
  if constexpr (NB > 2) x = fmaxf(x, dpp<kDppHalfMirror>(x));
  if constexpr (NB > 3) x = fmaxf(x, dpp<kDppMirror>(x));
  if constexpr (NB > 4) x = max_xor16(x);
  if constexpr (NB > 5) x = max_xor32(x);
  return x;
}

// The cost M of a kernel entry K = exp(-lambda (M - m_j)) of a row-scaled row
// is m_j - ln(K) / lambda = m_j + log2(K) * (-ln 2 / lambda).  The final pass
// sums K u log2(K) per row and applies the constant once per lane.  The smallest normal float is added first: it
// leaves every K >= 2^-102 unchanged (K = 1, a padding entry, gives exactly
// 0) and turns K = 0 (an underflowed entry) into K u * (-126) = 0 instead of
// 0 * inf.  One add, where a clamp with fmaxf costs two instructions.
__device__ __forceinline__ float log2_gibbs(float k) {
  return __builtin_amdgcn_logf(k + 1.17549435e-38f);
}
constexpr float kNegLn2 = -0.693147180559945309f;

// A document with words always ends with a finite distance in exact
// arithmetic.  In float32 a row of K underflows to 0 once lambda M exceeds
// about 87-103 for every query word of that document word; its dot product is
// then 0, w = c / 0 is infinite and the sums turn NaN.  Such a distance is
// reported as +Inf, which keeps it apart from the NaN of an empty document or
// an invalid query.
__device__ __forceinline__ float flag_range(float d) {
  return fabsf(d) <= 3.40282347e38f ? d : __int_as_float(0x7F800000);
}

__device__ __forceinline__ int64_t rec_begin(const int4& r) {
  return (int64_t)(uint32_t)r.x | ((int64_t)r.y << 32);
}

// One launch group's share of the work: block `blk` of `nblk` blocks walks
// the items blk, blk + nblk, ... of p's documents.  RES: the resident
// schedule only (u and w neither loaded nor stored, every iteration and the
// final pass in this launch), so the code for the other schedules and the
// registers it needs are left out.  HALF (one-wave items, lg_cg <= 4): an
// item spans 32 lanes and a wave holds two; no sum crosses lane bit 5.
// first: this block's first document record, when the caller has read it.
template <int TC, int TR, int LG_CG, int MAXW, bool RES, bool HALF = false>
__device__ __forceinline__ void sink_body(const SinkParams& p, int blk, int nblk, const int4* first = nullptr) {
  static_assert(!HALF || (MAXW == 1 && LG_CG <= 4), "half-wave items are one-wave shapes");
  const bool load_u = !RES && p.load_u, store_u = !RES && p.store_u;
  const bool load_w = !RES && p.load_w, store_w = !RES && p.store_w;
  constexpr bool MW = MAXW > 1;                   // an item spans several waves of one block
  constexpr int CG = 1 << LG_CG;
  constexpr int IL = HALF ? 32 : 64;              // lanes per item (within a wave)
  constexpr int RSW = IL >> LG_CG;                // row lanes per wave and item
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = MW ? (int)(blockDim.x >> 6) : 1;
  const int il = lane & (IL - 1);                 // lane within the item
  const int cg = il & (CG - 1);
  const int rs = (MW ? wave * RSW : 0) + (il >> LG_CG);
  const int RS = nwaves * RSW;
  const int items = MW ? 1 : (int)(blockDim.x >> 6) * (64 / IL);
  const int slot = MW ? 0 : wave * (64 / IL) + (HALF ? lane >> 5 : 0);
  constexpr int cw_stride = CG * TC;              // LDS floats per wave and buffer
  const int S = p.S;
  const int vr = *p.vr;
  float* rvs = lds + 2 * nwaves * cw_stride + 2 * cw_stride;  // multi-wave items only
  // Row sums over 2, 4, 16, 32 or 64 column lanes divide packed within
  // quads (lane bits 0 and 1), the quads' totals summed over the remaining
  // column-lane bits first; 8 column lanes (lg_cg 3) sum each row plainly.
  // One-wave items of at most 40 cells with 2 or 4 column lanes keep their
  // rows in permuted register slots (PERM, see low_div): once the rows are
  // gathered, slot t of this lane holds row slot_row(t) of its row lane, and
  // the w loads and stores of the other schedules follow it.  The
  // permutation is a few exec-masked swaps per item against two selects per
  // reduce-scatter step in every iteration.  Elsewhere the swaps cost more
  // registers than they save: larger blocks, wider column groups and
  // multi-wave items lose a wave per SIMD with them (compiled register
  // counts), which costs the batched workloads more than the selects.
  constexpr bool ROWQ = LG_CG != 0 && LG_CG != 3;
  constexpr int LQ = LG_CG == 1 ? 1 : 2;
  constexpr bool PERM = ROWQ && !MW && LG_CG <= 2 && TR * TC <= 40;
  const int qid = lane & (LQ == 1 ? 1 : 3);
  auto slot_row = [&](int t) { return PERM ? row_slot<LQ, TR>(t, qid) : t; };

  for (int base = blk * items; base < p.ndocs; base += nblk * items) {
    const int item = base + slot;
    const bool active = item < p.ndocs;
    const int4 rec = first && base == blk * items ? *first : active ? p.drec[item] : make_int4(0, 0, 0, 0);
    const int64_t beg = rec_begin(rec);
    const int n = rec.z, k = rec.w;

    // ---- gather this lane's words of document k and their K^T entries.
    // Padding -- a row slot with no word (or a zero weight), a column slot
    // with no query word (r = 0: the cost-matrix kernel stores K = 1 there,
    // and slots past S are set here) -- holds K = 1.  A
    // padding row then has a positive dot product (the item's real u), so its
    // w = 0 * rcp(.) = 0 and it adds nothing to any column; a padding column
    // sums the item's w (> 0 for a document with mass), so its u =
    // 0 * rcp(.) = 0 and it adds nothing to any row.  In the final pass
    // log2(1) = 0.
    int wid[TR];
    float cw[TR];
    float K[TR][TC];
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      const int j = rs + RS * t;
      const int id = j < n ? p.wl[beg + j] : -1;
      const float c = j < n ? p.wn[beg + j] : 0.f;
      wid[t] = c > 0.f ? id : -1;
      cw[t] = c > 0.f ? c : 0.f;
    }

    // sum_j c_j m_j over the item's rows: the part of d_k that the row
    // scaling of K^T took out of the stored rows (M_ij = m_j - ln(K_ij) /
    // lambda).  The CG column lanes of a row lane share its rows, so row t is
    // loaded and added by column lane t mod CG only: ceil(TR / CG) loads per
    // lane, issued with the rows of K^T (loads return in order, so they wait
    // for nothing the first iteration does not need anyway) and summed before
    // the iterations.
    float cm = 0.f;
    auto shift_sum = [&](auto load) {
      constexpr int PER = (TR + CG - 1) / CG;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        int id = -1;
        float c = 0.f;
#pragma unroll
        for (int t = i * CG; t < TR && t < (i + 1) * CG; ++t) {
          const bool mine = t - i * CG == cg;
          id = mine ? wid[t] : id;
          c = mine ? cw[t] : c;
        }
        cm = fmaf(c, load(p.km + (id < 0 ? 0 : id)), cm);
      }
    };
    if constexpr (MW) {
      // rows t = cg, cg + CG, ...: their entries read again (cache hits) rather
      // than picked out of the row registers, which would need a mask per row
      constexpr int PER = (TR + CG - 1) / CG;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int t = cg + CG * i, j = rs + RS * t;
        const bool ok = t < TR && j < n;
        const int id = ok ? p.wl[beg + j] : 0;
        const float c = ok ? p.wn[beg + j] : 0.f;
        cm = fmaf(c > 0.f ? c : 0.f, p.km[id], cm);
      }
    }
    // Columns of lane cg: the 4-column chunks cg, cg + CG, ... (4 TC4 columns,
    // one 16-byte load per row each: S and every K^T row start are multiples
    // of 4 floats) and then the single columns 4 CG TC4 + cg, ... + CG, ...
    constexpr int TC4 = TC / 4;
    auto col_of = [&](int e) {
      return e < 4 * TC4 ? 4 * (cg + CG * (e >> 2)) + (e & 3) : 4 * CG * TC4 + cg + CG * (e - 4 * TC4);
    };
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      const float* row = p.kt + (size_t)(wid[t] < 0 ? 0 : wid[t]) * S;
#pragma unroll
      for (int c = 0; c < TC4; ++c) {
        const int c0 = col_of(4 * c);
        const float4 v = *(const float4*)(row + (c0 < S ? c0 : S - 4));  // clamped inside the row
        const bool ok = wid[t] >= 0 && c0 < S;
        K[t][4 * c] = ok ? v.x : 1.f;
        K[t][4 * c + 1] = ok ? v.y : 1.f;
        K[t][4 * c + 2] = ok ? v.z : 1.f;
        K[t][4 * c + 3] = ok ? v.w : 1.f;
      }
#pragma unroll
      for (int e = 4 * TC4; e < TC; ++e) {
        const int col = col_of(e);
        const float v = row[col < S ? col : S - 1];  // clamped: never reads past the row
        K[t][e] = (wid[t] >= 0 && col < S) ? v : 1.f;
      }
    }
    if constexpr (!MW) shift_sum([](const float* a) { return *a; });
    // cm is complete here, with nothing waited for that the rows do not need
    // (this keeps the compiler from carrying the loaded values, or the row
    // ids, into the iterations)
    asm volatile("" : "+v"(cm));
    // The rows were read in their natural slots (the lanes of a quad reading
    // the same K^T row, so that a load touches a row's lines once); PERM
    // wants them in slot_row order.  Swapping slot pairs by lane bit 0 and
    // then slot pairs two apart by lane bit 1 takes slot t to row t ^ q in
    // groups of four and t ^ (q & 1) in pairs.
    if constexpr (PERM) {
      using LP = LowPack<LQ, TR>;
      constexpr int G4 = 4 * LP::NQ, G2 = G4 + 2 * LP::NP;
      // swaps in the lanes whose bit is set only (exec-masked moves, no
      // selects and no second copy of the block)
      auto swap = [](auto& a, auto& b) {
        const auto t = a;
        a = b;
        b = t;
      };
      if (qid & 1) {
#pragma unroll
        for (int t = 0; t < G2; t += 2) {
#pragma unroll
          for (int e = 0; e < TC; ++e) swap(K[t][e], K[t + 1][e]);
          swap(cw[t], cw[t + 1]);
          swap(wid[t], wid[t + 1]);
        }
      }
      if (qid & 2) {
#pragma unroll
        for (int t = 0; t < G4; t += 4) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int e = 0; e < TC; ++e) swap(K[t + h][e], K[t + h + 2][e]);
            swap(cw[t + h], cw[t + h + 2]);
            swap(wid[t + h], wid[t + h + 2]);
          }
        }
      }
    }
    float rv[TC], u[TC];
#pragma unroll
    for (int e = 0; e < TC; ++e) {
      const int col = col_of(e);
      rv[e] = col < S ? p.r[col] : 0.f;
      if (load_u)
        u[e] = (active && col < S) ? p.u[(size_t)k * S + col] : 0.f;
      else
        u[e] = rv[e] > 0.f ? (float)vr : 0.f;  // x = 1/v_r
    }
    // multi-wave items: r of every (column lane, column) for the column
    // threads; the same for every item of the launch, written before the
    // first item's first barrier
    if constexpr (MW) {
      if (base == blk * items && wave == 0 && lane < CG) {
#pragma unroll
        for (int e = 0; e < TC; ++e) rvs[cg + CG * e] = rv[e];
      }
    }
    // Column sums that cross the permlane bits (lane bits 4 and 5) divide in
    // packed form when the row lanes reach them (one-wave items, lg_cg <= 5).
    constexpr bool COLP = !MW && LG_CG <= 5;
    constexpr int MC = HALF ? 1 : LG_CG <= 4 ? 3 : 2;  // half-wave items: bit 4 only
    float rpk[HighPack<MC, TC>::P];
    if constexpr (COLP) pack_high<MC, TC>(rv, rpk, lane);
    constexpr int RHB = LG_CG > 4 ? LG_CG - 4 : 0;
    float cqk[LowPack<LQ, TR>::P];
    if constexpr (ROWQ) pack_low<LQ, TR, PERM>(cw, cqk, lane);
    // w_j = c_j / s_j for this lane's rows, from partial dot products s
    // (summed over the column lanes here), in every column lane of the row
    auto row_div = [&](float (&sp)[TR], float (&q)[TR]) {
      if constexpr (ROWQ) {
        low_div<LQ, (LG_CG >= 4), RHB, TR, PERM>(cqk, sp, q, lane);
      } else {
        sum_low<LG_CG>(sp);
#pragma unroll
        for (int t = 0; t < TR; ++t) q[t] = fast_div(cw[t], sp[t]);
      }
    };
    float wv[TR];
    if (load_w) {
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const int j = rs + RS * slot_row(t);
        wv[t] = (j < n && wid[t] >= 0) ? p.w[beg + j] : 0.f;
      }
    }

    // ---- Sinkhorn-Knopp iterations
    int ran = p.iters;
    bool done = !active;  // half-wave items under a tolerance: this item has stopped
    for (int it = 0; it < p.iters; ++it) {
      if (!load_w) {
        float s[TR];
#pragma unroll
        for (int t = 0; t < TR; ++t) {
          float a = 0.f;
#pragma unroll
          for (int e = 0; e < TC; ++e) a = fmaf(K[t][e], u[e], a);
          s[t] = a;
        }
        row_div(s, wv);
        if (store_w) {
          if (cg == 0 && active) {
#pragma unroll
            for (int t = 0; t < TR; ++t) {
              const int j = rs + RS * slot_row(t);
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
        acc[e] = a;
      }
      // The new column scalings go straight into u (nothing below reads the
      // old u but the tolerance test, which keeps its own copy): a separate
      // array would cost a move per column and iteration to carry it back.
      const bool chk = p.tol > 0.f;
      float uprev[TC];
      if (chk) {
#pragma unroll
        for (int e = 0; e < TC; ++e) uprev[e] = u[e];
      }
      float (&un)[TC] = u;
      if constexpr (COLP) {
        high_div<MC, TC, LG_CG>(rpk, acc, un);
      } else {
        if constexpr (!MW) sum_high<LG_CG>(acc);
        if constexpr (MW) {
          // cross-wave sum in two phases: every wave posts its column partials,
          // one thread per column adds them in wave order, every lane reads back
          // its columns.  Both arrays alternate by iteration parity, so two
          // barriers per iteration suffice.  (Measured faster than one barrier
          // with every lane adding all waves' partials of its columns, even
          // for 4 waves.)  The in-wave sum over row-lane bits 4 and 5 is a
          // reduce-scatter: each 16-lane group (half) posts a different column,
          // and the row-lane bits below 4 are added after the packing.
          float* part = lds + (it & 1) * nwaves * cw_stride;
          float* tot = lds + 2 * nwaves * cw_stride + (it & 1) * cw_stride;
          float* wp = part + wave * cw_stride + cg;
          constexpr int MB = LG_CG <= 4 ? 3 : LG_CG == 5 ? 2 : 0;
          if constexpr (MB == 0) {
#pragma unroll
            for (int e = 0; e < TC; ++e) wp[CG * e] = acc[e];
          } else {
            // every lane takes part in the cross-lane sums (DPP reads of a
            // disabled lane are not defined to give its value); only lanes
            // whose in-row row-lane bits are 0 post
            using H = HighPack<MB, TC>;
            const int G = (lane >> 4) & 3, half = lane >> 5;
            const bool poster = (lane & 15) < CG;
            float z[H::P];
#pragma unroll
            for (int q = 0; q < H::NQ; ++q) {
              const int a = 4 * q;
              z[q] = sum_row_bits<LG_CG>(
                  sum_scatter32(sum_scatter16(acc[a], acc[a + 1]), sum_scatter16(acc[a + 2], acc[a + 3])));
            }
#pragma unroll
            for (int i = 0; i < H::NP; ++i) {
              const int a = 4 * H::NQ + 2 * i;
              if constexpr (MB == 2)
                z[H::NQ + i] = sum_row_bits<LG_CG>(sum_scatter32(acc[a], acc[a + 1]));
              else
                z[H::NQ + i] = sum_row_bits<LG_CG>(add_xor32(sum_scatter16(acc[a], acc[a + 1])));
            }
            if constexpr (H::N1 > 0) {
              float y = sum_row_bits<LG_CG>(acc[TC - 1]);
              if constexpr (MB & 1) y = add_xor16(y);
              z[H::P - 1] = add_xor32(y);
            }
            if (poster) {
#pragma unroll
              for (int q = 0; q < H::NQ; ++q) wp[CG * (4 * q + G)] = z[q];
#pragma unroll
              for (int i = 0; i < H::NP; ++i) {
                const int a = 4 * H::NQ + 2 * i;
                if constexpr (MB == 2)
                  wp[CG * (a + half)] = z[H::NQ + i];
                else if (G < 2)
                  wp[CG * (a + G)] = z[H::NQ + i];
              }
              if constexpr (H::N1 > 0) {
                if (MB == 2 ? half == 0 : G == 0) wp[CG * (TC - 1)] = z[H::P - 1];
              }
            }
          }
          __syncthreads();
          // the column thread adds the waves' partials in wave order and
          // divides: r over the total, once per column instead of in every
          // lane.  (The guarded adds compile to one LDS round trip per wave;
          // loading every wave's partial first measured no faster at the
          // batched workload, whose waves keep the SIMDs busy meanwhile, and
          // costs 16-wave blocks a wave per SIMD in registers.)
          for (int c = threadIdx.x; c < cw_stride; c += blockDim.x) {
            float a = 0.f;
#pragma unroll
            for (int w = 0; w < MAXW; ++w)
              if (w < nwaves) a += part[w * cw_stride + c];
            tot[c] = fast_div(rvs[c], a);
          }
          __syncthreads();
#pragma unroll
          for (int e = 0; e < TC; ++e) un[e] = tot[cg + CG * e];
        } else {
#pragma unroll
          for (int e = 0; e < TC; ++e) un[e] = fast_div(rv[e], acc[e]);
        }
      }
      if (chk) {
        // x = 1/u, so the relative change |x_new - x| / x_new is
        // |u - u_new| / u; padding columns (u = 0) are skipped.  Every lane of
        // the item holds the same u, so the decision is uniform over the
        // item's waves.
        float dm = 0.f;
#pragma unroll
        for (int e = 0; e < TC; ++e) {
          if (uprev[e] > 0.f) dm = fmaxf(dm, fabsf(uprev[e] - u[e]) * __builtin_amdgcn_rcpf(uprev[e]));
        }
        dm = max_low<LG_CG>(dm);
        if constexpr (HALF) {
          // two items per wave: an item that has stopped keeps the u of the
          // iteration it stopped after (restored here), and the wave leaves
          // the loop once both have stopped
          if (done) {
#pragma unroll
            for (int e = 0; e < TC; ++e) u[e] = uprev[e];
          } else if (!(dm > p.tol)) {
            ran = it + 1;
            done = true;
          }
          if (__ballot(!done) == 0) break;
          continue;
        }
        // uniform over the wave (one item per wave, or the same value in every
        // wave of a multi-wave item): a scalar branch, so the loop stays free
        // of divergent-exit bookkeeping
        const float dmu = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(dm)));
        if (!(dmu > p.tol)) {
          ran = it + 1;
          break;
        }
        continue;
      }
    }

    if (store_u && rs == 0 && active) {
#pragma unroll
      for (int e = 0; e < TC; ++e) {
        const int col = col_of(e);
        if (col < S) p.u[(size_t)k * S + col] = u[e];
      }
    }

    // ---- final pass: d_k = sum_j c_jk ((K.*M)_j . u) / (K_j . u), with the
    // costs recovered from the K entries held in registers.  c_j / (K_j . u)
    // is the w of the final u, divided as in an iteration; every lane then
    // adds w_j times its own columns' share of (K.*M)_j . u, so one sum over
    // all lanes gives d_k.
    if (p.do_final) {
      float sa[TR], sb[TR], wf[TR];
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        float a = 0.f, b = 0.f;
#pragma unroll
        for (int e = 0; e < TC; ++e) {
          const float ku = K[t][e] * u[e];
          a += ku;
          b = fmaf(ku, log2_gibbs(K[t][e]), b);
        }
        sa[t] = a;
        sb[t] = b;
      }
      row_div(sa, wf);
      float part[1] = {0.f};
#pragma unroll
      for (int t = 0; t < TR; ++t) part[0] = fmaf(wf[t], sb[t], part[0]);
      part[0] = fmaf(part[0], kNegLn2 * p.inv_lam, cm);
      sum_low<HALF ? 5 : 6>(part);
      float tot = part[0];
      if constexpr (MW) {
        __syncthreads();  // the last iteration's totals may still be read
        if (lane == 0) lds[wave] = tot;
        __syncthreads();
        float a = 0.f;
        for (int w = 0; w < nwaves; ++w) a += lds[w];
        tot = a;
        __syncthreads();
      }
      if (il == 0 && (MW ? wave == 0 : true) && active) {
        p.out[k] = vr > 0 ? flag_range(tot) : __int_as_float(0x7FC00000);
        if (p.iters_out) p.iters_out[k] = ran;
      }
    }
  }
}

// Multi-wave items: one item per block of up to MAXW waves.  When the grid
// has a block per document, a block whose document fits in 3/4 of its rows
// runs a body of 3TR/4 rows per lane (see sink_body_fit); the choice is the
// same for every wave of the block, so its barriers stay matched.
// With a query set the grid is nq runs of the per-query grid.
template <int TC, int TR, int LG_CG, int MAXW, bool RES>
__global__ void __launch_bounds__(64 * MAXW) sink_kernel(SinkParams p, SinkQuerySet qs) {
  int blk = blockIdx.x, nblk = gridDim.x;
  if (qs.nq > 0) {
    const int per = nblk / qs.nq;
    const int qi = blk / per;
    blk -= qi * per;
    nblk = per;
    p = for_query(p, qs, qi);
  }
  if constexpr (TR >= 4) {
    if (nblk >= p.ndocs) {
      constexpr int T3 = 3 * TR / 4;
      const int item = blk;
      const int4 rec = item < p.ndocs ? p.drec[item] : make_int4(0, 0, 0, 0);
      const int rows = (int)(blockDim.x >> 6) * (64 >> LG_CG) * T3;
      if (rec.z <= rows) {
        sink_body<TC, T3, LG_CG, MAXW, RES>(p, blk, nblk, &rec);
      } else {
        sink_body<TC, TR, LG_CG, MAXW, RES>(p, blk, nblk, &rec);
      }
      return;
    }
  }
  sink_body<TC, TR, LG_CG, MAXW, RES>(p, blk, nblk);
}

// T rows per lane hold documents of up to (lanes per item >> lg_cg) * T
// words.  A wave whose documents all fit in 3/4 of that runs a body of 3T/4
// rows: the power-of-two length buckets leave the upper quarter of the rows
// empty for most of their documents, and every row costs its cells' FMAs in
// every iteration.  The choice is per wave (no sum crosses waves here), from
// the document records the body would read first anyway.
template <int TC, int T, int LG_CG, bool RES, bool HALF>
__device__ __forceinline__ void sink_body_fit(const SinkParams& p, int blk, int nblk) {
  if constexpr (T >= 4) {
    constexpr int IL = HALF ? 32 : 64;
    constexpr int T3 = 3 * T / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int items = (int)(blockDim.x >> 6) * (64 / IL);
    const int item = blk * items + wave * (64 / IL) + (HALF ? lane >> 5 : 0);
    const int4 rec = item < p.ndocs ? p.drec[item] : make_int4(0, 0, 0, 0);
    int nmax = __builtin_amdgcn_readfirstlane(rec.z);
    if constexpr (HALF) nmax = max(nmax, __builtin_amdgcn_readlane(rec.z, 32));
    // only when the grid takes every document in one pass (the body keeps
    // its row count for all the items it walks)
    if (nmax <= (IL >> LG_CG) * T3 && nblk * items >= p.ndocs) {
      sink_body<TC, T3, LG_CG, 1, RES, HALF>(p, blk, nblk, &rec);
    } else {
      sink_body<TC, T, LG_CG, 1, RES, HALF>(p, blk, nblk, &rec);
    }
  } else {
    sink_body<TC, T, LG_CG, 1, RES, HALF>(p, blk, nblk);
  }
}

// One-wave items, four per block (eight as half-wave items), for several
// length buckets of one query (or of each query of a set) in a single launch.
// Group g holds blocks [end[g-1], end[g]) -- with a query set, nq equal runs,
// one per query -- and documents drec[off[g]] ... drec[off[g] + ndocs[g] - 1];
// body[g] & 3 = 0, 1, 2 gives its rows per lane TRMAX, TRMAX/2 or TRMAX/4, and
// body[g] & 4 makes its items half-wave (two per wave, 32 lanes each).
// Groups come longest documents first, so the longest items start first and
// the short ones fill in behind them.  The other fields of p are shared.
template <int TC, int TRMAX, int LG_CG, bool RES>
__global__ void __launch_bounds__(256) sink_merge_kernel(SinkMerge m) {
  const int b = blockIdx.x;
  int g = 0, b0 = 0;
#pragma unroll
  for (int i = 0; i + 1 < kMergeMax; ++i)
    if (i + 1 < m.ngroups && b >= m.end[i]) {
      g = i + 1;
      b0 = m.end[i];
    }
  int off = 0, nd = 0, body = 0, b1 = 0;
#pragma unroll
  for (int i = 0; i < kMergeMax; ++i)
    if (i == g) {
      off = m.off[i];
      nd = m.ndocs[i];
      body = m.body[i];
      b1 = m.end[i];
    }
  SinkParams p = m.p;
  int blk = b - b0, nblk = b1 - b0;
  if (m.qs.nq > 0) {
    const int per = nblk / m.qs.nq;  // this group's blocks for one query
    const int qi = blk / per;
    blk -= qi * per;
    nblk = per;
    p = for_query(p, m.qs, qi);
  }
  p.drec += off;
  p.ndocs = nd;
  const bool half = (body & 4) != 0;
  const int shift = body & 3;
  if constexpr (LG_CG <= 4) {
    if (half) {
      if (shift == 0) {
        sink_body_fit<TC, TRMAX, LG_CG, RES, true>(p, blk, nblk);
      } else if constexpr (TRMAX >= 2) {
        if (shift == 1) {
          sink_body_fit<TC, TRMAX / 2, LG_CG, RES, true>(p, blk, nblk);
        } else if constexpr (TRMAX >= 4) {
          sink_body_fit<TC, TRMAX / 4, LG_CG, RES, true>(p, blk, nblk);
        }
      }
      return;
    }
  }
  if (shift == 0) {
    sink_body_fit<TC, TRMAX, LG_CG, RES, false>(p, blk, nblk);
  } else if constexpr (TRMAX >= 2) {
    if (shift == 1) {
      sink_body_fit<TC, TRMAX / 2, LG_CG, RES, false>(p, blk, nblk);
    } else if constexpr (TRMAX >= 4) {
      sink_body_fit<TC, TRMAX / 4, LG_CG, RES, false>(p, blk, nblk);
    }
  }
}

struct SinkEntry {
  int tc, tr, lg_cg;
  int maxw;       // 1: one wave per item (sink_merge_kernel, TRMAX = tr); 4, 8 or 16: waves per block at most
  const void* fn;        // resident schedule only
  const void* fn_sched;  // every schedule (u / w loaded and stored as the launch says)
};

// Register budget per lane of the K^T block: up to 128 cells in blocks of at
// most 4 or 8 waves (512 or 256 VGPRs per lane), up to 64 cells in 16-wave
// blocks (128 VGPRs per lane).  Shapes that still spill are never chosen.
template <int TC, int TR, int MAXW>
constexpr bool kSinkFits = TC * TR <= (MAXW == 16 ? 64 : 128);

#define WMD_SINK_SW_TR(X, TC, LG) X(TC, 1, LG, 1) X(TC, 2, LG, 1) X(TC, 4, LG, 1) X(TC, 8, LG, 1) X(TC, 16, LG, 1)
#define WMD_SINK_MW_TR(X, TC, LG) X(TC, 8, LG, 4) X(TC, 16, LG, 4) X(TC, 8, LG, 8) X(TC, 4, LG, 16) X(TC, 8, LG, 16)
#define WMD_SINK_TC(X, TC, LG) WMD_SINK_SW_TR(X, TC, LG) WMD_SINK_MW_TR(X, TC, LG)

template <int TC, int TR, int LG_CG, int MAXW, bool OK = kSinkFits<TC, TR, MAXW>>
struct SinkPick {
  static SinkEntry get() { return SinkEntry{TC, TR, LG_CG, MAXW, nullptr, nullptr}; }
};
template <int TC, int TR, int LG_CG, int MAXW>
struct SinkPick<TC, TR, LG_CG, MAXW, true> {
  static SinkEntry get() {
    if constexpr (MAXW == 1)
      return SinkEntry{TC, TR, LG_CG, MAXW, (const void*)sink_merge_kernel<TC, TR, LG_CG, true>,
                       (const void*)sink_merge_kernel<TC, TR, LG_CG, false>};
    else
      return SinkEntry{TC, TR, LG_CG, MAXW, (const void*)sink_kernel<TC, TR, LG_CG, MAXW, true>,
                       (const void*)sink_kernel<TC, TR, LG_CG, MAXW, false>};
  }
};

#define WMD_SINK_ENTRY(TC, TR, LG, MAXW) SinkPick<TC, TR, LG, MAXW>::get(),

// Tables of the instantiated shapes, one per translation unit (column-lane width).
const SinkEntry* sink_table_cg0(int* n);
const SinkEntry* sink_table_cg1(int* n);
const SinkEntry* sink_table_cg2(int* n);
const SinkEntry* sink_table_cg3(int* n);
const SinkEntry* sink_table_cg4(int* n);
const SinkEntry* sink_table_cg5(int* n);
const SinkEntry* sink_table_cg6(int* n);

}  // namespace wmd
