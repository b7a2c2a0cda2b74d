// Measurement kernels: the achievable ceilings the hot path is judged
// against (the paper models the fused SDDMM-SpMM as bound by memory
// bandwidth, Section III-E; its Table II quotes the machine's bandwidths).
// None of them is part of the method; they measure the GPU:
//   - a streaming read and a streaming copy of a large buffer (HBM bandwidth),
//   - a gather of K^T-shaped rows (S floats, 16-byte pieces) in the order of a
//     corpus's own word-id stream (the access pattern of the Sinkhorn
//     kernels' row gather, served by L2 / MALL / HBM as the ids repeat),
//   - independent float32 FMA chains, and the same with the hardware
//     reciprocal and with DPP cross-lane adds (the VALU rates the iteration
//     is made of).
#include "wmd_bench.h"

#include <hip/hip_runtime.h>

#include "lanes.h"

namespace {

using wmd::dpp;

// Stream: grid-stride over float4 pieces, four in flight per thread.  The
// read-only mode keeps a running sum that is stored only if it equals a
// value no input produces here (so the loads cannot be dropped).
__global__ void __launch_bounds__(256) stream_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    size_t n, int copy, float* sink) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.f;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    if (copy) {
      dst[i] = a;
      dst[i + stride] = b;
      dst[i + 2 * stride] = c;
      dst[i + 3 * stride] = d;
    } else {
      acc += (a.x + b.y) + (c.z + d.w);
    }
  }
  for (; i < n; i += stride) {
    const float4 a = src[i];
    if (copy) dst[i] = a;
    else acc += a.x;
  }
  if (!copy && acc == -1.2345678e30f) *sink = acc;
}

// Row tiles in MFMA operand order (each lane loading its own operand pieces).  Rows of row_bytes
// (a multiple of 64); each wave owns 16 consecutive rows and, per step, lane l
// reads bytes [64 i + 16 (l >> 4), +16) of row l & 15, all steps of the row
// issued at once; one wave per 16 rows, blocks of four waves.
__global__ void __launch_bounds__(256) tile_kernel(const unsigned char* __restrict__ src, size_t rows, int row_bytes,
                                                  float* sink) {
  const int lane = threadIdx.x & 63;
  const size_t r0 = ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (r0 >= rows) return;
  const size_t row = r0 + (lane & 15) < rows ? r0 + (lane & 15) : rows - 1;
  const unsigned char* base = src + row * (size_t)row_bytes + 16 * (lane >> 4);
  const int steps = row_bytes / 64;
  float acc = 0.f;
  int i = 0;
  for (; i + 8 <= steps; i += 8) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = *(const float4*)(base + (size_t)(i + u) * 64);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u].x + v[u].w;
  }
  for (; i < steps; ++i) {
    const float4 v = *(const float4*)(base + (size_t)i * 64);
    acc += v.x + v.w;
  }
  if (acc == -1.2345678e30f) *sink = acc;
}

// Gather, issued the way the Sinkhorn kernels gather their K^T rows: L =
// 2^l lanes per row, each reading two 16-byte pieces (pieces past the row
// are skipped), 64 / L rows per wave and load step, and eight such steps per
// pass, every load of a pass in flight before any value is used.  Each row's
// values are summed and one float per row is written (4 bytes against the
// 4 S read).  ids are read with clamped indices, so every read stays inside
// ids[0 .. nids) and the rows they name.
__global__ void __launch_bounds__(256) gather_kernel(const float* __restrict__ table, int S,
                                                    const int* __restrict__ ids, size_t nids, float* __restrict__ out) {
  constexpr int T = 8;  // load steps per pass
  const int n4 = S >> 2;
  int lg = 0;
  while ((2 << lg) < n4) ++lg;
  const int L = 1 << lg, R = 64 >> lg;
  const int lane = threadIdx.x & 63;
  const int sub = lane & (L - 1), rw = lane >> lg;
  const size_t waves = (size_t)gridDim.x * (blockDim.x >> 6);
  const size_t per = (size_t)R * T;
  for (size_t g = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); g * per < nids; g += waves) {
    int id[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const size_t k = g * per + rw + (size_t)R * t;
      id[t] = ids[k < nids ? k : nids - 1];
    }
    float4 v[T][2];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float4* row = (const float4*)(table + (size_t)id[t] * S);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int c = sub + L * i;
        v[t][i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < n4) v[t][i] = row[c];
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      float acc = (v[t][0].x + v[t][0].y) + (v[t][0].z + v[t][0].w) + (v[t][1].x + v[t][1].y) +
                  (v[t][1].z + v[t][1].w);
      for (int o = 1; o < L; o <<= 1) acc += __shfl_xor(acc, o);
      const size_t k = g * per + rw + (size_t)R * t;
      if (k < nids && sub == 0) out[k] = acc;
    }
  }
}

// VALU rates: 16 independent chains per lane (enough to cover the latency of
// a dependent FMA at one wave per SIMD), `iters` rounds of 16 instructions.
// mode 0: v_fma_f32 (2 flops per lane); 1: v_rcp_f32; 2: v_add_f32 with a
// DPP row rotation operand.  The result is stored so nothing is dropped.
__global__ void __launch_bounds__(256) valu_kernel(float* out, int iters, int mode, float a, float b) {
  float x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = a + (float)(threadIdx.x + i);
  if (mode == 0) {
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = fmaf(x[i], b, a);
    }
  } else if (mode == 1) {
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = __builtin_amdgcn_rcpf(x[i]);
    }
  } else {
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] += dpp<wmd::kDppRor4>(x[i]);  // grows to inf: rate only
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += x[i];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" {

int wmd_bench_stream(const void* src, void* dst, size_t bytes, int32_t copy, int32_t blocks, float* sink,
                     void* stream) {
  if (!src || (copy && !dst) || (!copy && !sink) || bytes % 16 || blocks < 1) return 1;
  stream_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const float4*>(src), static_cast<float4*>(dst), bytes / 16, copy, sink);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int wmd_bench_tiles(const void* src, size_t rows, int32_t row_bytes, float* sink, void* stream) {
  if (!src || !sink || rows < 1 || row_bytes < 64 || row_bytes % 64) return 1;
  const size_t blocks = (rows + 63) / 64;
  tile_kernel<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const unsigned char*>(src), rows, row_bytes, sink);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int wmd_bench_gather(const float* table, int32_t S, const int32_t* ids, size_t nids, float* out, int32_t blocks,
                     void* stream) {
  if (!table || !ids || !out || S < 4 || S > 512 || S % 4 || blocks < 1) return 1;
  gather_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(table, S, ids, nids, out);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int wmd_bench_valu(float* out, int32_t blocks, int32_t iters, int32_t mode, void* stream) {
  if (!out || blocks < 1 || iters < 1 || mode < 0 || mode > 2) return 1;
  valu_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(out, iters, mode, 0.5f, 0.999f);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

}  // extern "C"
