// Cross-lane sums inside a 64-wide gfx950 wavefront.
//
// Lane bits 0-3 address the 16 lanes of a DPP row, bit 4 the row pair and
// bit 5 the wave half.  Within a row the sums use DPP modifiers fused into
// v_add_f32 (no LDS traffic); across rows they use the gfx950 permlane swaps.
#pragma once

#include <hip/hip_runtime.h>

namespace wmd {

enum : int {
  kDppXor1 = 0xB1,        // quad_perm [1,0,3,2]
  kDppXor2 = 0x4E,        // quad_perm [2,3,0,1]
  kDppXor3 = 0x1B,        // quad_perm [3,2,1,0]
  kDppRor4 = 0x124,       // row_ror:4
  kDppRor8 = 0x128,       // row_ror:8
  kDppMirror = 0x140,     // row_mirror      (lane l <- 15-l)
  kDppHalfMirror = 0x141  // row_half_mirror (lane l <- 7-l within 8)
};

// Value of x in the lane selected by a DPP control word.  Every pattern used
// here reads a valid lane, so bound_ctrl is set and no `old` operand is needed,
// which lets the compiler fold the move into the consuming v_add_f32_dpp.
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

// a / b through the hardware reciprocal (v_rcp_f32, about 1 ulp) and one
// multiply: a few ulp in total, far inside the 1e-4 relative target, against
// ~10 instructions for the IEEE division sequence.
__device__ __forceinline__ float fast_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// max(x[l], x[l ^ 16]) and max(x[l], x[l ^ 32])
__device__ __forceinline__ float max_xor16(float x) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(p[0]), __uint_as_float(p[1]));
}
__device__ __forceinline__ float max_xor32(float x) {
  auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(p[0]), __uint_as_float(p[1]));
}

// x[l] + x[l ^ 16]
__device__ __forceinline__ float add_xor16(float x) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// x[l] + x[l ^ 32]
__device__ __forceinline__ float add_xor32(float x) {
  auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// Reduce-scatter and gather over the permlane bits.  Lane bit 4 selects the
// 16-lane group inside a half wave, bit 5 the half.  permlane16_swap(x, y)
// returns x with its odd groups replaced by y's even groups and y with its
// even groups replaced by x's odd groups, so the sum of the two results holds
// x summed over bit 4 in the even groups and y summed over bit 4 in the odd
// ones; permlane32_swap does the same for the halves.

// [a + a^16 in groups 0 and 2, b + b^16 in groups 1 and 3]
__device__ __forceinline__ float sum_scatter16(float a, float b) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
// [a + a^32 in lanes 0-31, b + b^32 in lanes 32-63]
__device__ __forceinline__ float sum_scatter32(float a, float b) {
  auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
// inverse of the scatters: v holds a in even groups (lower half) and b in odd
// groups (upper half); every lane receives both
__device__ __forceinline__ void gather16(float v, float& a, float& b) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  a = __uint_as_float(p[0]);
  b = __uint_as_float(p[1]);
}
__device__ __forceinline__ void gather32(float v, float& a, float& b) {
  auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  a = __uint_as_float(p[0]);
  b = __uint_as_float(p[1]);
}

// Sum over lane bits [0, nbits), every lane of the group receiving the total.
// Lower bits are summed first, so once bits 0..b-1 are uniform the mirror
// patterns (which flip several bits at once) pair lanes that hold equal
// partial sums in those bits.
__device__ __forceinline__ float sum_low_bits(float x, int nbits) {
  if (nbits > 0) x += dpp<kDppXor1>(x);
  if (nbits > 1) x += dpp<kDppXor2>(x);
  if (nbits > 2) x += dpp<kDppHalfMirror>(x);
  if (nbits > 3) x += dpp<kDppMirror>(x);
  if (nbits > 4) x = add_xor16(x);
  if (nbits > 5) x = add_xor32(x);
  return x;
}

// Sum over lane bits [lo, hi) while the bits below lo address different
// values that must not mix.  Requires hi >= 4 (groups of at least 16 lanes):
// the 4-lane sum over bits 2 and 3 is row_ror:8 followed by row_ror:4, which
// is only a clean sum when both bits are reduced.
__device__ __forceinline__ float sum_mid_bits(float x, int lo, int hi) {
  if (lo <= 3 && hi > 3) x += dpp<kDppRor8>(x);
  if (lo <= 2 && hi > 2) x += dpp<kDppRor4>(x);
  if (lo <= 1 && hi > 1) x += dpp<kDppXor2>(x);
  if (lo <= 0 && hi > 0) x += dpp<kDppXor1>(x);
  if (lo <= 4 && hi > 4) x = add_xor16(x);
  if (lo <= 5 && hi > 5) x = add_xor32(x);
  return x;
}

// Minimum over lane bits [0, NB) (NB <= 4), lower bits first, every lane of
// the group receiving it.
template <int NB>
__device__ __forceinline__ float min_low(float x) {
  if constexpr (NB > 0) x = fminf(x, dpp<kDppXor1>(x));
  if constexpr (NB > 1) x = fminf(x, dpp<kDppXor2>(x));
  if constexpr (NB > 2) x = fminf(x, dpp<kDppHalfMirror>(x));
  if constexpr (NB > 3) x = fminf(x, dpp<kDppMirror>(x));
  static_assert(NB <= 4, "within a 16-lane row");
  return x;
}

// float -> bf16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

}  // namespace wmd
