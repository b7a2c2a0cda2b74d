// Embedding rows of selected query words (Algorithm 1, first step: the query
// side of the cost matrix), read by 8 lanes per row.
#pragma once

#include "lanes.h"

namespace wmd {

// Lane lane8 (0..7) of a row's 8 lanes reads the 4-float chunks starting at
// k = 4 (lane8 + 8 i) (+ 512 per round) of embedding row q, hands each chunk
// inside the padded width dp to put(k, chunk) (zeros past d, or for q < 0),
// and returns its partial sum of squares in double.  All loads of a round are
// issued before the first chunk is used.  The caller adds the 8 partials with
// a fixed butterfly, so the norm is the same on every path.
template <class Put>
__device__ __forceinline__ double query_row(const float* emb, int d, int dp, int q, int lane8, Put&& put) {
  const float* src = emb + (size_t)(q < 0 ? 0 : q) * d;
  const bool vec = (d & 3) == 0 && ((uintptr_t)emb & 15) == 0;
  double nrm = 0.0;
  for (int k0 = 0; k0 < dp; k0 += 512) {
    float4 x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = k0 + 4 * (lane8 + 8 * i);
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
      x[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = k0 + 4 * (lane8 + 8 * i);
      if (k < dp) {
        put(k, x[i]);
        nrm += (double)x[i].x * (double)x[i].x + (double)x[i].y * (double)x[i].y +
               (double)x[i].z * (double)x[i].z + (double)x[i].w * (double)x[i].w;
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

}  // namespace wmd
