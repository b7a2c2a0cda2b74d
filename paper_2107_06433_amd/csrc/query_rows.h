// Query selection and the embedding rows of the selected words (Algorithm 1,
// first step: the query side of the cost matrix), shared by the selection
// kernel and the cost-matrix kernel that selects a short query itself.
#pragma once

#include "lanes.h"

namespace wmd {

// Lane lane8 (0..7) of a row's 8 lanes reads the 4-float chunks starting at
// k = 4 (lane8 + 8 i) (+ 512 per round) of embedding row q, hands each chunk
// inside the padded width dp to put(k, chunk) (zeros past d, or for q < 0),
// and returns its partial sum of squares in double, added chunk by chunk in
// k order.  The loads of NC chunks are issued before the first of them is
// used (NC = 16: a whole round; fewer keep fewer registers live, with the
// same sum).  The caller adds the 8 partials with a fixed butterfly, so the
// norm is the same on every path.
// Floats k..k+3 of embedding row q (zeros past d, or for q < 0).
__device__ __forceinline__ float4 query_chunk(const float* emb, int d, int q, int k) {
  const float* src = emb + (size_t)(q < 0 ? 0 : q) * d;
  const bool vec = (d & 3) == 0 && ((uintptr_t)emb & 15) == 0;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (q >= 0 && k < d) {
    if (vec) {
      v = *(const float4*)(src + k);
    } else {
      v.x = src[k];
      v.y = k + 1 < d ? src[k + 1] : 0.f;
      v.z = k + 2 < d ? src[k + 2] : 0.f;
      v.w = k + 3 < d ? src[k + 3] : 0.f;
    }
  }
  return v;
}

// The chunk's squares added to a row's partial norm, in double.
__device__ __forceinline__ double add_squares(double nrm, float4 v) {
  return nrm + ((double)v.x * (double)v.x + (double)v.y * (double)v.y + (double)v.z * (double)v.z +
                (double)v.w * (double)v.w);
}

template <int NC = 16, class Put>
__device__ __forceinline__ double query_row(const float* emb, int d, int dp, int q, int lane8, Put&& put) {
  static_assert(16 % NC == 0, "chunks per batch");
  double nrm = 0.0;
  for (int k0 = 0; k0 < dp; k0 += 512) {
#pragma unroll
    for (int h = 0; h < 16; h += NC) {
      float4 x[NC];
#pragma unroll
      for (int i = 0; i < NC; ++i) x[i] = query_chunk(emb, d, q, k0 + 4 * (lane8 + 8 * (h + i)));
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        const int k = k0 + 4 * (lane8 + 8 * (h + i));
        if (k < dp) {
          put(k, x[i]);
          nrm = add_squares(nrm, x[i]);
        }
      }
    }
  }
  return nrm;
}

// the 8 lanes' partial norms, added in a fixed order: partners at lane
// distance 1 and 2, then the other quad of the 8 (row_half_mirror pairs the
// quads once each holds its sum), by DPP moves of both halves
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double sum_row_lanes(double x) {
  x += dpp_f64<kDppXor1>(x);
  x += dpp_f64<kDppXor2>(x);
  x += dpp_f64<kDppHalfMirror>(x);
  return x;
}

// four floats as bf16 (round to nearest even) in one 8-byte word
__device__ __forceinline__ uint2 pack_bf16x4(float4 v) {
  const uint32_t lo = (uint32_t)f32_to_bf16(v.x) | ((uint32_t)f32_to_bf16(v.y) << 16);
  const uint32_t hi = (uint32_t)f32_to_bf16(v.z) | ((uint32_t)f32_to_bf16(v.w) << 16);
  return make_uint2(lo, hi);
}

// Sum of a double over the 64 lanes, every lane receiving the same total:
// DPP moves of both halves within 16-lane rows (lower bits first, so the
// mirror patterns pair lanes holding equal partial sums), then the permlane
// swaps across rows.
__device__ __forceinline__ double sum_wave_f64(double x) {
  x += dpp_f64<kDppXor1>(x);
  x += dpp_f64<kDppXor2>(x);
  x += dpp_f64<kDppHalfMirror>(x);
  x += dpp_f64<kDppMirror>(x);
  auto cross = [&](bool half) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    auto pl = half ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                   : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto ph = half ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                   : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    x = __longlong_as_double((long long)(((uint64_t)ph[0] << 32) | pl[0])) +
        __longlong_as_double((long long)(((uint64_t)ph[1] << 32) | pl[1]));
  };
  cross(false);
  cross(true);
  return x;
}

// Selection (Algorithm 1, first step) for a query of at most 64 entries, by
// one wave with one entry per lane: repeats are merged by broadcasting each entry in turn (readlane), so
// the merge needs no LDS round trips and no barriers.  Same results as the
// general path: each first occurrence sums its repeats in entry order, slots
// follow entry order.  Writes s_id/s_m for the entries, s_slot for the S
// slots and the query's error code, word count and total weight.
__device__ __forceinline__ void select_small(const int32_t* q_ids, const float* q_w, int64_t V, int64_t beg, int n,
                                             int S, int lane, int* s_id, double* s_m, int* s_slot, int* s_err,
                                             int* s_vr, double* s_tot) {
  const bool in = lane < n;
  const int id = in ? q_ids[beg + lane] : -1;
  const float x = in ? q_w[beg + lane] : 0.f;
  const bool bad_id = in && (id < 0 || id >= V);
  const bool bad_w = in && (!(x >= 0.f) || isinf(x));
  const bool f1 = __ballot(bad_id) != 0, f2 = __ballot(bad_w) != 0;
  bool first = true;
  double m = 0.0;
  for (int j = 0; j < n; ++j) {
    const int idj = __builtin_amdgcn_readlane(id, j);
    const float wj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
    const bool eq = idj == id;
    first = first && !(eq && j < lane);
    m += (eq && j >= lane) ? (double)wj : 0.0;  // adding +0.0 leaves m unchanged
  }
  const bool sel = in && first && m > 0.0;
  const unsigned long long mask = __ballot(sel);
  const int c = __popcll(mask);
  if (sel) s_slot[__popcll(mask & ((1ull << lane) - 1))] = lane;
  if (lane >= c && lane < S) s_slot[lane] = -1;
  if (in) {
    s_id[lane] = id;
    s_m[lane] = first ? m : 0.0;
  }
  const double tot = sum_wave_f64(sel ? m : 0.0);
  if (lane == 0) {
    int e = (f1 ? 1 : 0) | (f2 ? 2 : 0);
    if (e == 0 && c == 0) e = 8;
    *s_err = e;
    *s_vr = e ? 0 : c;
    *s_tot = tot;
  }
}

}  // namespace wmd
