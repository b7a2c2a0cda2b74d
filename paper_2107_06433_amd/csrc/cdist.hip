// Cost matrix and Gibbs kernel for all queries of a call (Algorithm 1, first
// line; Table I's cdist and exp).
//
// G = E_c Q^T on MFMA, with E_c the U x dp compacted vocabulary embeddings and
// Q the C x dp query-word embeddings of every query (C = sum of padded query
// widths).  The epilogue turns each G[t][n] into
//     M = sqrt(max(0, |e_t|^2 + |q_n|^2 - 2 G)),  M = 0 when word t IS query word n,
//     K = exp(-lambda M),
// and stores K transposed per query: row t of query b is S_b contiguous floats,
// the row the fused SDDMM-SpMM gathers for every nonzero.  K.*M is not stored:
// the final pass recovers M = -ln(K) / lambda from the K values it holds.
//
// FP32 inputs use v_mfma_f32_16x16x4_f32; BF16 inputs use gfx950's
// v_mfma_f32_16x16x32_bf16; accumulation is float32 in both.  Both operands
// are k-contiguous rows staged through LDS with double buffering.  Within one
// instruction the assignment of k indices to lane groups is immaterial as long
// as A and B use the same one, so each lane feeds a run of consecutive k
// values read with one 16-byte LDS load.
#include "lanes.h"
#include "query_rows.h"
#include "wmd_internal.h"

namespace wmd {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int WM, bool BF16, int BK_>
struct Tile {
  static constexpr int WN = 4 / WM;
  static constexpr int TM = BM / WM, TN = BN / WN;
  static constexpr int FM = TM / 16, FN = TN / 16;
  static constexpr int BK = BK_;                     // k elements per stage
  static constexpr int ESZ = BF16 ? 2 : 4;           // bytes per element
  static constexpr int PAD = 16 / ESZ;               // one 16-byte pad per row
  static constexpr int LDK = BK + PAD;               // LDS row length (elements)
  static constexpr int VEC = 16 / ESZ;               // elements per 16-byte load
  static constexpr int NA = BM * BK / VEC / 256;     // 16-byte loads per thread
  static constexpr int NB = BN * BK / VEC / 256;
  static constexpr int VPR = BK / VEC;               // 16-byte loads per row
  static constexpr size_t STAGE = (size_t)2 * (BM + BN) * LDK * ESZ;  // double-buffered A and B
  // then the epilogue's per-row (|e|^2, word id) and per-column (query word
  // id, |q|^2, column base and width) data
  static constexpr size_t LDS = STAGE + (size_t)BM * 8 + (size_t)BN * 16;
  static_assert(FM >= 1 && FN >= 1 && NA >= 1 && NB >= 1, "tile");
  static_assert(BM * BK % (VEC * 256) == 0 && BN * BK % (VEC * 256) == 0, "loads");
  static_assert(BK % (BF16 ? 32 : 16) == 0 && 64 % BK == 0, "k step");
  static_assert(LDS <= 65536, "lds");
};

template <int BM, int BN, int WM, bool BF16, int BK>
__global__ void __launch_bounds__(256) cdist_kernel(CdistParams p) {
  using T = Tile<BM, BN, WM, BF16, BK>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned char* As = smem;
  unsigned char* Bs = smem + (size_t)2 * BM * T::LDK * T::ESZ;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int64_t n0 = (int64_t)blockIdx.y * BN;
  const unsigned char* Ag = BF16 ? (const unsigned char*)p.e16 : (const unsigned char*)p.e32;
  const unsigned char* Bg = BF16 ? (const unsigned char*)p.q16 : (const unsigned char*)p.q32;
  const size_t row_bytes = (size_t)p.dp * T::ESZ;

  uint4 ra[T::NA], rb[T::NB];
  auto load = [&](int kt) {
    const size_t kb = (size_t)kt * T::BK * T::ESZ;
#pragma unroll
    for (int j = 0; j < T::NA; ++j) {
      const int i = tid + 256 * j, row = i / T::VPR, v = i % T::VPR;
      const int64_t g = m0 + row;
      ra[j] = g < p.U ? *(const uint4*)(Ag + (size_t)g * row_bytes + kb + 16 * v) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < T::NB; ++j) {
      const int i = tid + 256 * j, row = i / T::VPR, v = i % T::VPR;
      const int64_t g = n0 + row;
      rb[j] = g < p.C ? *(const uint4*)(Bg + (size_t)g * row_bytes + kb + 16 * v) : make_uint4(0, 0, 0, 0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < T::NA; ++j) {
      const int i = tid + 256 * j, row = i / T::VPR, v = i % T::VPR;
      *(uint4*)(As + ((size_t)(buf * BM + row) * T::LDK) * T::ESZ + 16 * v) = ra[j];
    }
#pragma unroll
    for (int j = 0; j < T::NB; ++j) {
      const int i = tid + 256 * j, row = i / T::VPR, v = i % T::VPR;
      *(uint4*)(Bs + ((size_t)(buf * BN + row) * T::LDK) * T::ESZ + 16 * v) = rb[j];
    }
  };

  f32x4 acc[T::FM][T::FN];
#pragma unroll
  for (int a = 0; a < T::FM; ++a)
#pragma unroll
    for (int b = 0; b < T::FN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // the epilogue's row and column data go to LDS, fetched ahead of the first
  // stage (indices clamped; rows past U and columns past C are never stored)
  float* s_en = (float*)(smem + T::STAGE);
  int* s_used = (int*)(s_en + BM);
  int2* s_ci = (int2*)(s_used + BM);
  int* s_qid = (int*)(s_ci + BN);
  float* s_qn = (float*)(s_qid + BN);
  float e_en = 0.f, e_qn = 0.f;
  int e_used = 0, e_qid = 0;
  int2 e_ci = make_int2(0, 0);
  if (tid < BM) {
    const int64_t m = m0 + tid;
    const int64_t mc = m < p.U ? m : p.U - 1;
    e_en = p.en[mc];
    e_used = p.used[mc];
  }
  if (tid < BN) {
    const int64_t n = n0 + tid;
    const int64_t nc = n < p.C ? n : p.C - 1;
    e_qid = p.qid[nc];
    e_qn = p.qn[nc];
    e_ci = p.cinfo[nc];
  }
  const int nk = p.dp / T::BK;
  load(0);
  if (tid < BM) {
    s_en[tid] = e_en;
    s_used[tid] = e_used;
  }
  if (tid < BN) {
    s_qid[tid] = e_qid;
    s_qn[tid] = e_qn;
    s_ci[tid] = e_ci;
  }
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
    const unsigned char* Ab = As + (size_t)cur * BM * T::LDK * T::ESZ;
    const unsigned char* Bb = Bs + (size_t)cur * BN * T::LDK * T::ESZ;
    if constexpr (!BF16) {
#pragma unroll
      for (int kk = 0; kk < T::BK / 16; ++kk) {
        const int kofs = kk * 16 + 4 * (lane >> 4);
        f32x4 av[T::FM], bv[T::FN];
#pragma unroll
        for (int a = 0; a < T::FM; ++a)
          av[a] = *(const f32x4*)(Ab + ((size_t)(wm * T::TM + a * 16 + (lane & 15)) * T::LDK + kofs) * 4);
#pragma unroll
        for (int b = 0; b < T::FN; ++b)
          bv[b] = *(const f32x4*)(Bb + ((size_t)(wn * T::TN + b * 16 + (lane & 15)) * T::LDK + kofs) * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int a = 0; a < T::FM; ++a)
#pragma unroll
            for (int b = 0; b < T::FN; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][i], bv[b][i], acc[a][b], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < T::BK / 32; ++kk) {
        const int kofs = kk * 32 + 8 * (lane >> 4);
        bf16x8 av[T::FM], bv[T::FN];
#pragma unroll
        for (int a = 0; a < T::FM; ++a)
          av[a] = *(const bf16x8*)(Ab + ((size_t)(wm * T::TM + a * 16 + (lane & 15)) * T::LDK + kofs) * 2);
#pragma unroll
        for (int b = 0; b < T::FN; ++b)
          bv[b] = *(const bf16x8*)(Bb + ((size_t)(wn * T::TN + b * 16 + (lane & 15)) * T::LDK + kofs) * 2);
#pragma unroll
        for (int a = 0; a < T::FM; ++a)
#pragma unroll
          for (int b = 0; b < T::FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // Epilogue.  Accumulator register i of lane l holds row 4*(l/16)+i, column l%16
  // of each 16x16 tile.  The row and column data come from LDS: a store
  // counts against the same memory counter as a global load, so a global
  // load consumed between two stores would wait for the first store.
  int qc[T::FN];
  float qnc[T::FN];
  int2 cic[T::FN];
#pragma unroll
  for (int b = 0; b < T::FN; ++b) {
    const int c = wn * T::TN + b * 16 + (lane & 15);
    qc[b] = s_qid[c];
    qnc[b] = s_qn[c];
    cic[b] = s_ci[c];
  }
#pragma unroll
  for (int a = 0; a < T::FM; ++a) {
    float enr[4];
    int usr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * T::TM + a * 16 + 4 * (lane >> 4) + i;
      enr[i] = s_en[r];
      usr[i] = s_used[r];
    }
#pragma unroll
    for (int b = 0; b < T::FN; ++b) {
      const int64_t n = n0 + wn * T::TN + b * 16 + (lane & 15);
      float* kt = p.kt + (size_t)cic[b].x * (size_t)p.U + (n - cic[b].x);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + wm * T::TM + a * 16 + 4 * (lane >> 4) + i;
        const float m2 = enr[i] + qnc[b] - 2.f * acc[a][b][i];
        const float dist = usr[i] == qc[b] ? 0.f : sqrtf(fmaxf(m2, 0.f));
        // distances; gibbs_rows_kernel turns them into the row-scaled K (an
        // unused query slot, +inf here, becomes K = 1: padding for the
        // Sinkhorn kernels)
        const float kv = qc[b] >= 0 ? dist : __int_as_float(0x7F800000);
        if (n < p.C && m < p.U) kt[(size_t)m * cic[b].y] = kv;
      }
    }
  }
}

template <int BM, int BN, int WM, bool BF16, int BK>
hipError_t run(const CdistParams& p, hipStream_t s) {
  using T = Tile<BM, BN, WM, BF16, BK>;
  dim3 grid((unsigned)((p.U + BM - 1) / BM), (unsigned)((p.C + BN - 1) / BN));
  cdist_kernel<BM, BN, WM, BF16, BK><<<grid, 256, T::LDS, s>>>(p);
  return hipGetLastError();
}


// Few query columns (C <= 32): the GEMM is a stream over the U x dp vocabulary
// rows.  Each wave owns 16 rows and reads them straight from memory into the
// MFMA operand registers -- for every 16 (f32) or 32 (bf16) k values, the four
// lane quads of a row read one contiguous 64-byte piece.  All loads of a row
// (CH steps) are issued at once, so one memory latency covers the whole row.
//
// NT tiles of 16 query columns use 16x16 MFMAs.  F32 inputs may add N4 groups
// of 4 columns on v_mfma_f32_4x4x1_16b_f32, whose 16 blocks here are 4 row
// quads x 4 k slices of the same operand registers (lane l: row l & 15, k
// slice l >> 4, as for the 16x16 shape), so a 4-column group costs a quarter
// of a 16-column tile.  The k slices are summed once at the end.
//
// SEL: the query (one, of at most 64 entries) is selected here instead of by
// the selection kernel: while the row's loads are in flight, wave 0 selects
// it, then 8 lanes per slot read its embedding rows straight into the Q tile
// with the selection kernel's own row reader (same values, same norms), and
// block 0 writes the selection's outputs for the kernels that follow.
template <int NT, int N4, bool BF16, int CH, bool SEL>
__global__ void __launch_bounds__(256) cdist_skinny_kernel(CdistParams p) {
  static_assert(!BF16 || N4 == 0, "4-column groups are an f32 path");
  static_assert(NT + N4 > 0, "no columns");
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int KS = BF16 ? 32 : 16;        // k values per 16-byte-per-lane load step
  // CH = dp / KS load steps: the whole row, a compile-time count, and every
  // load unconditional (rows past U read row 0 and are never stored), so the
  // MFMA of step i waits only for load i
  constexpr int ROWB = CH * KS * ESZ;       // bytes per embedding row (64 per step)
  constexpr int LDQ = ROWB + 16;            // LDS row pitch in bytes (one 16-byte pad)
  constexpr int VPR = ROWB / 16;            // 16-byte pieces per row
  constexpr int QROWS = NT * 16 + N4 * 4;   // Q rows staged in LDS
  constexpr int QTOT = QROWS * VPR;         // pieces of the Q tile
  constexpr int QPT = (QTOT + 255) / 256;   // per thread
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const int64_t myrow = m0 + (lane & 15);
  const bool row_ok = myrow < p.U;
  (void)row_ok;
  // The wave's 16 rows are read in full 128-byte lines: per chunk of two load
  // steps (128 bytes of every row), load j covers rows 8j .. 8j+7, 8 lanes per
  // row, each lane 16 bytes.  (Reading the MFMA operand layout directly -- 16
  // rows x 64 bytes per load -- touches half a line per row and load and
  // streams at ~3.1 TB/s against ~4.7 TB/s for the same bytes read whole.)
  // A per-wave LDS stage then hands every lane its MFMA operand: row l & 15,
  // bytes 64 s + 16 (l >> 4) of step s, as before.
  static_assert(CH % 2 == 0, "whole 128-byte chunks");
  const unsigned char* Eg = BF16 ? (const unsigned char*)p.e16 : (const unsigned char*)p.e32;
  const unsigned char* Ag0;
  const unsigned char* Ag1;
  {
    const int64_t r0 = m0 + (lane >> 3), r1 = m0 + 8 + (lane >> 3);  // rows past U read row 0
    Ag0 = Eg + (size_t)(r0 < p.U ? r0 : 0) * ROWB + 16 * (lane & 7);
    Ag1 = Eg + (size_t)(r1 < p.U ? r1 : 0) * ROWB + 16 * (lane & 7);
  }
  constexpr int STR = 144;  // stage row pitch in bytes: 128 + 16 (rows fall on distinct banks)
  __shared__ __attribute__((aligned(16))) unsigned char stage[4][16 * STR];
  unsigned char* st = stage[wave];
  f32x4 acc[NT > 0 ? NT : 1], acc4[N4 > 0 ? N4 : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < N4; ++u) acc4[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Q: QROWS rows go to LDS through registers.  Its loads are issued first
  // and its LDS stores come after the vocabulary row's loads: loads retire in
  // order, so the stores wait for the Q pieces alone while the row is already
  // in flight.  Rows past C repeat row C - 1: each output column depends on its
  // own Q row only, and the epilogue never stores those columns.
  const unsigned char* Qg = BF16 ? (const unsigned char*)p.q16 : (const unsigned char*)p.q32;
  uint4 qv[QPT];
#pragma unroll
  for (int j = 0; j < (SEL ? 0 : QPT); ++j) {
    const int i = QTOT % 256 == 0 ? j * 256 + tid : min(j * 256 + tid, QTOT - 1);
    const int row = i / VPR;
    qv[j] = *(const uint4*)(Qg + (size_t)min(row, (int)p.C - 1) * ROWB + 16 * (i - row * VPR));
  }
  uint4 buf[CH];
  float en_r[4];
  int used_r[4];
  auto load_rows = [&]() {
#pragma unroll
    for (int c = 0; c < CH / 2; ++c) {
      buf[2 * c] = *(const uint4*)(Ag0 + (size_t)c * 128);
      buf[2 * c + 1] = *(const uint4*)(Ag1 + (size_t)c * 128);
    }
    // the epilogue's per-row and per-column data, fetched early for the same
    // reason (indices clamped)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t m = m0 + 4 * (lane >> 4) + i;
      const int64_t mc = m < p.U ? m : p.U - 1;
      en_r[i] = p.en[mc];
      used_r[i] = p.used[mc];
    }
  };
  // SEL, f32: wave 0 selects first and reads its rows afterwards (loads
  // return in order: the selection's would otherwise wait behind the row's).
  // With bf16 rows (half the bytes) starting wave 0's rows late cost more
  // than the wait (measured), so there every wave reads its rows first.
  constexpr bool SEL_FIRST = SEL && !BF16;
  if (!SEL_FIRST || wave != 0) load_rows();
  constexpr int NTA = NT > 0 ? NT : 1;
  int q_c[NTA];
  float qn_c[NTA];
  int2 ci_c[NTA];
#pragma unroll
  for (int t = 0; t < (SEL ? 0 : NT); ++t) {
    const int64_t n = t * 16 + (lane & 15);
    const int64_t nc = n < p.C ? n : p.C - 1;
    q_c[t] = p.qid[nc];
    qn_c[t] = p.qn[nc];
    ci_c[t] = p.cinfo[nc];
  }
  // 4-column groups: lane l ends with row 4 ((l >> 2) & 3) + (l >> 4) of the
  // wave's 16 and column 4 u + (l & 3) of group u
  const int64_t m4 = m0 + 4 * ((lane >> 2) & 3) + (lane >> 4);
  float en_4 = 0.f;
  int used_4 = 0;
  int q_4[N4 > 0 ? N4 : 1];
  float qn_4[N4 > 0 ? N4 : 1];
  int2 ci_4[N4 > 0 ? N4 : 1];
  if constexpr (N4 > 0) {
    const int64_t mc = m4 < p.U ? m4 : p.U - 1;
    en_4 = p.en[mc];
    used_4 = p.used[mc];
  }
#pragma unroll
  for (int u = 0; u < (SEL ? 0 : N4); ++u) {
    const int64_t n = NT * 16 + 4 * u + (lane & 3);
    const int64_t nc = n < p.C ? n : p.C - 1;
    q_4[u] = p.qid[nc];
    qn_4[u] = p.qn[nc];
    ci_4[u] = p.cinfo[nc];
  }
  // An empty asm that takes and returns the Q pieces keeps their LDS stores
  // (and the waits for them) below every load above, which the scheduler
  // would otherwise interleave with the row's loads.  It keeps the pieces live
  // across the row's loads, so only where the registers allow three waves
  // per SIMD.
  if constexpr (!SEL && 4 * (CH + QPT) <= 108) {
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
      u32x4 t = __builtin_bit_cast(u32x4, qv[j]);
      asm volatile("" : "+v"(t));
      qv[j] = __builtin_bit_cast(uint4, t);
    }
  }
  // threads past the tile repeat the last piece (same value, same address):
  // every store is unconditional, so none waits for more than its own load
#pragma unroll
  for (int j = 0; j < (SEL ? 0 : QPT); ++j) {
    const int i = QTOT % 256 == 0 ? j * 256 + tid : min(j * 256 + tid, QTOT - 1);
    const int row = i / VPR;
    *(uint4*)(smem + row * LDQ + 16 * (i - row * VPR)) = qv[j];
  }
  if constexpr (SEL) {
    static_assert(QROWS <= 32, "at most 32 slots");
    __shared__ int s_id[64], s_slot[64], s_qid[32];
    __shared__ double s_m[64];
    __shared__ float s_qn[32];
    __shared__ int s_err, s_vr;
    __shared__ double s_tot;
    const int S = (int)p.C;
    // Q row g = slot g's embedding row (zeros past the words), 8 lanes per
    // row, as the selection kernel reads them: the same chunks per lane, the
    // same norm order
    constexpr int DPC = CH * KS;                // padded width
    constexpr int NCH = (DPC + 31) / 32;        // chunks per lane and row
    const int lane8 = lane & 7;
    auto row_of = [&](int g) {
      const int e = g < s_vr ? s_slot[g] : -1;
      return e >= 0 ? s_id[e] : -1;
    };
    auto fetch = [&](int q, float4(&xr)[NCH]) {
#pragma unroll
      for (int i = 0; i < NCH; ++i) xr[i] = query_chunk(p.emb, p.d, q, 4 * (lane8 + 8 * i));
    };
    auto emit = [&](int g, int q, const float4(&xr)[NCH]) {
      double nrm = 0.0;
#pragma unroll
      for (int i = 0; i < NCH; ++i) {
        const int k = 4 * (lane8 + 8 * i);
        if (k < DPC) {
          if (g < QROWS) {
            if constexpr (BF16)
              *(uint2*)(smem + g * LDQ + 2 * k) = pack_bf16x4(xr[i]);
            else
              *(float4*)(smem + g * LDQ + 4 * k) = xr[i];
          }
          nrm = add_squares(nrm, xr[i]);
        }
      }
      nrm = sum_row_lanes(nrm);
      if (g < QROWS && lane8 == 0) {
        s_qn[g] = (float)nrm;
        s_qid[g] = q;
      }
    };
    if (wave == 0) {
      select_small(p.q_ids, p.q_w, p.V, 0, p.sel_n, S, lane, s_id, s_m, s_slot, &s_err, &s_vr, &s_tot);
      __builtin_amdgcn_wave_barrier();
      const int vr = s_vr;
      if (blockIdx.x == 0) {
        if (lane == 0) {
          const int err = s_err;
          p.err[0] = err & 1 ? 1 : err & 2 ? 2 : err & 4 ? 4 : err & 8 ? 3 : 0;
          p.vr[0] = vr;
        }
        if (lane < S) {
          const int i = lane < vr ? s_slot[lane] : -1;
          p.qid_out[lane] = i >= 0 ? s_id[i] : -1;
          p.r[lane] = i >= 0 ? (float)(s_m[i] / s_tot) : 0.f;
          p.cinfo_out[lane] = make_int2(0, S);
        }
      }
      if constexpr (SEL_FIRST) {
        // wave 0 alone, 8 rows per pass, every pass's loads in flight at once
        // when the registers allow; its own rows after that
        constexpr int PASSES = (QROWS + 7) / 8;
        constexpr bool BATCH = PASSES * NCH <= 32;
        float4 x[BATCH ? PASSES : 1][NCH];
        int qr[PASSES];
#pragma unroll
        for (int r = 0; r < PASSES; ++r) qr[r] = row_of(8 * r + (lane >> 3));
        if constexpr (BATCH) {
#pragma unroll
          for (int r = 0; r < PASSES; ++r) fetch(qr[r], x[r]);
#pragma unroll
          for (int r = 0; r < PASSES; ++r) emit(8 * r + (lane >> 3), qr[r], x[r]);
        } else {
#pragma unroll
          for (int r = 0; r < PASSES; ++r) {
            fetch(qr[r], x[0]);
            emit(8 * r + (lane >> 3), qr[r], x[0]);
          }
        }
        load_rows();
      }
    }
    if constexpr (!SEL_FIRST) {
      // every wave's rows are in flight already: all 32 groups of 8 lanes
      // read one Q row each
      __syncthreads();
      const int g = tid >> 3;
      const int q = row_of(g);
      float4 x[NCH];
      fetch(q, x);
      emit(g, q, x);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 16 + (lane & 15);
      const int nc = n < S ? n : S - 1;
      q_c[t] = s_qid[nc];
      qn_c[t] = s_qn[nc];
      ci_c[t] = make_int2(0, S);
    }
#pragma unroll
    for (int u = 0; u < N4; ++u) {
      const int n = NT * 16 + 4 * u + (lane & 3);
      const int nc = n < S ? n : S - 1;
      q_4[u] = s_qid[nc];
      qn_4[u] = s_qn[nc];
      ci_4[u] = make_int2(0, S);
    }
  } else {
    __syncthreads();
  }
  {
    uint4 op = make_uint4(0, 0, 0, 0);  // this lane's operand of the current step
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (i % 2 == 0) {
        // stage chunk i / 2 (rows 8j + (l >> 3), bytes 16 (l & 7)) and read
        // this lane's operands of steps i and i + 1 back
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        *(uint4*)(st + (lane >> 3) * STR + 16 * (lane & 7)) = buf[i];
        *(uint4*)(st + (8 + (lane >> 3)) * STR + 16 * (lane & 7)) = buf[i + 1];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        op = *(const uint4*)(st + (lane & 15) * STR + 16 * (lane >> 4));
        buf[i + 1] = *(const uint4*)(st + (lane & 15) * STR + 64 + 16 * (lane >> 4));
      } else {
        op = buf[i];
      }
      const int kb = i * 64 + 16 * (lane >> 4);  // byte offset of this lane's k run
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const uint4 q = *(const uint4*)(smem + (t * 16 + (lane & 15)) * LDQ + kb);
        if constexpr (BF16) {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, op),
                                                          __builtin_bit_cast(bf16x8, q), acc[t], 0, 0, 0);
        } else {
          const f32x4 a = __builtin_bit_cast(f32x4, op);
          const f32x4 b = __builtin_bit_cast(f32x4, q);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], acc[t], 0, 0, 0);
        }
      }
      if constexpr (!BF16) {
#pragma unroll
        for (int u = 0; u < N4; ++u) {
          const uint4 q = *(const uint4*)(smem + (NT * 16 + 4 * u + (lane & 3)) * LDQ + kb);
          const f32x4 a = __builtin_bit_cast(f32x4, op);
          const f32x4 b = __builtin_bit_cast(f32x4, q);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc4[u] = __builtin_amdgcn_mfma_f32_4x4x1f32(a[j], b[j], acc4[u], 0, 0, 0);
        }
      }
    }
  }
  // 4-column groups: register i of lane l holds row 4 ((l >> 2) & 3) + i,
  // column l & 3, summed over k slice l >> 4; a reduce-scatter over the k
  // slices leaves lane l the total of register l >> 4
  float k4[N4 > 0 ? N4 : 1];
#pragma unroll
  for (int u = 0; u < N4; ++u)
    k4[u] = sum_scatter32(sum_scatter16(acc4[u][0], acc4[u][1]), sum_scatter16(acc4[u][2], acc4[u][3]));
  // epilogue: register i of lane l holds row 4*(l/16)+i, column l%16 of each
  // tile.  All values first, then the stores (a store counts against the
  // same memory counter as a load; nothing waits on them).
  constexpr float kInf = __builtin_huge_valf();
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float m2 = en_r[i] + qn_c[t] - 2.f * acc[t][i];
      const float dist = used_r[i] == q_c[t] ? 0.f : sqrtf(fmaxf(m2, 0.f));
      // an unused query slot: +inf; so is a column past C (never stored, and
      // with a selected query its Q row is zero, not a copy of a real one),
      // which keeps both out of the row minima below
      acc[t][i] = q_c[t] >= 0 && t * 16 + (lane & 15) < p.C ? dist : kInf;
    }
#pragma unroll
  for (int u = 0; u < N4; ++u) {
    const float m2 = en_4 + qn_4[u] - 2.f * k4[u];
    const float dist = used_4 == q_4[u] ? 0.f : sqrtf(fmaxf(m2, 0.f));
    k4[u] = q_4[u] >= 0 && NT * 16 + 4 * u + (lane & 3) < p.C ? dist : kInf;
  }
  // One query in the call: every column belongs to it, so each row's shift
  // m_j is the minimum over the row's columns (over the tiles, then over the
  // 16 lanes that hold a tile row; over the 4-column groups, then over the 4
  // lanes that hold a group row), the two layouts exchanging their row minima
  // through lane reads.  Rows then hold K = exp(-lambda (M - m_j)) and an
  // unused slot K = 1.  Otherwise the distances are stored as they are.
  const bool shift = p.one_query != 0;
  float rmin[4] = {kInf, kInf, kInf, kInf};  // tile layout: row 4 (l >> 4) + i
  float rmin4 = kInf;                        // group layout: row 4 ((l >> 2) & 3) + (l >> 4)
  if (shift) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int t = 0; t < NT; ++t) rmin[i] = fminf(rmin[i], acc[t][i]);
      if constexpr (NT > 0) rmin[i] = min_low<4>(rmin[i]);
    }
#pragma unroll
    for (int u = 0; u < N4; ++u) rmin4 = fminf(rmin4, k4[u]);
    if constexpr (N4 > 0) rmin4 = min_low<2>(rmin4);
    if constexpr (NT > 0 && N4 > 0) {
      // tile row 4g + i is group row (a, b) = (g, i), held by lane 16 i + 4 g;
      // group row (a, b) is tile row 4a + b, register b of lane 16 a
      const int g = lane >> 4, a = (lane >> 2) & 3;
      float from4[4], fromt[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        from4[i] = __shfl(rmin4, 16 * i + 4 * g);
        fromt[i] = __shfl(rmin[i], 16 * a);
      }
      const float tb = g == 0 ? fromt[0] : g == 1 ? fromt[1] : g == 2 ? fromt[2] : fromt[3];
#pragma unroll
      for (int i = 0; i < 4; ++i) rmin[i] = fminf(rmin[i], from4[i]);
      rmin4 = fminf(rmin4, tb);
    }
    // a row with no used column (an invalid query): no shift, K = 1
#pragma unroll
    for (int i = 0; i < 4; ++i) rmin[i] = rmin[i] < kInf ? rmin[i] : 0.f;
    rmin4 = rmin4 < kInf ? rmin4 : 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[t][i] = acc[t][i] < kInf ? expf(-p.lam * (acc[t][i] - rmin[i])) : 1.f;
#pragma unroll
    for (int u = 0; u < N4; ++u) k4[u] = k4[u] < kInf ? expf(-p.lam * (k4[u] - rmin4)) : 1.f;
  }
#pragma unroll
  for (int u = 0; u < N4; ++u) {
    const int64_t n = NT * 16 + 4 * u + (lane & 3);
    if (n < p.C && m4 < p.U)
      p.kt[(size_t)ci_4[u].x * (size_t)p.U + (n - ci_4[u].x) + (size_t)m4 * ci_4[u].y] = k4[u];
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int64_t n = t * 16 + (lane & 15);
    float* kt = p.kt + (size_t)ci_c[t].x * (size_t)p.U + (n - ci_c[t].x);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t m = m0 + 4 * (lane >> 4) + i;
      if (n < p.C && m < p.U) kt[(size_t)m * ci_c[t].y] = acc[t][i];
    }
  }
  if (shift) {
    if constexpr (NT > 0) {
      if ((lane & 15) == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t m = m0 + 4 * (lane >> 4) + i;
          if (m < p.U) p.km[m] = rmin[i];
        }
      }
    } else {
      if ((lane & 3) == 0 && m4 < p.U) p.km[m4] = rmin4;
    }
  }
}

size_t skinny_lds(int nt, int n4, int dp, bool bf16) {
  return (size_t)(nt * 16 + n4 * 4) * (size_t)(dp * (bf16 ? 2 : 4) + 16);
}

template <int NT, int N4, bool BF16, int CH>
hipError_t run_skinny_ch(const CdistParams& p, hipStream_t s) {
  const unsigned grid = (unsigned)((p.U + 63) / 64);
  if (p.sel_n > 0)
    cdist_skinny_kernel<NT, N4, BF16, CH, true><<<grid, 256, skinny_lds(NT, N4, p.dp, BF16), s>>>(p);
  else
    cdist_skinny_kernel<NT, N4, BF16, CH, false><<<grid, 256, skinny_lds(NT, N4, p.dp, BF16), s>>>(p);
  return hipGetLastError();
}

// the skinny kernel instantiated for this row length (dp / (16 / elem bytes)
// load steps), or hipErrorInvalidValue when there is none
template <int NT, int N4, bool BF16>
hipError_t run_skinny(const CdistParams& p, hipStream_t s) {
  const int steps = p.dp / (BF16 ? 32 : 16);
  switch (steps) {
    case 4: return run_skinny_ch<NT, N4, BF16, 4>(p, s);
    case 8: return run_skinny_ch<NT, N4, BF16, 8>(p, s);
    case 12: return run_skinny_ch<NT, N4, BF16, 12>(p, s);
    case 16: return run_skinny_ch<NT, N4, BF16, 16>(p, s);
    case 20: return run_skinny_ch<NT, N4, BF16, 20>(p, s);
    case 24: return run_skinny_ch<NT, N4, BF16, 24>(p, s);
    default: break;
  }
  if constexpr (BF16) {
    switch (steps) {
      case 2: return run_skinny_ch<NT, N4, BF16, 2>(p, s);
      case 6: return run_skinny_ch<NT, N4, BF16, 6>(p, s);
      case 10: return run_skinny_ch<NT, N4, BF16, 10>(p, s);
      case 14: return run_skinny_ch<NT, N4, BF16, 14>(p, s);
      case 18: return run_skinny_ch<NT, N4, BF16, 18>(p, s);
      case 22: return run_skinny_ch<NT, N4, BF16, 22>(p, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// F32, C <= 32: the fewest MFMA cycles per 16 rows -- 16-column tiles (32
// cycles per k step of 4) and 4-column groups (8 cycles) -- covering C
hipError_t run_skinny_f32(const CdistParams& p, hipStream_t s, const char** name) {
  switch ((p.C + 3) / 4) {
    case 1: *name = "cdist_skinny_kernel<0,1,0>"; return run_skinny<0, 1, false>(p, s);
    case 2: *name = "cdist_skinny_kernel<0,2,0>"; return run_skinny<0, 2, false>(p, s);
    case 3: *name = "cdist_skinny_kernel<0,3,0>"; return run_skinny<0, 3, false>(p, s);
    case 4: *name = "cdist_skinny_kernel<1,0,0>"; return run_skinny<1, 0, false>(p, s);
    case 5: *name = "cdist_skinny_kernel<1,1,0>"; return run_skinny<1, 1, false>(p, s);
    case 6: *name = "cdist_skinny_kernel<1,2,0>"; return run_skinny<1, 2, false>(p, s);
    case 7: *name = "cdist_skinny_kernel<1,3,0>"; return run_skinny<1, 3, false>(p, s);
    default: *name = "cdist_skinny_kernel<2,0,0>"; return run_skinny<2, 0, false>(p, s);
  }
}

bool skinny_steps_ok(int dp, bool bf16) {
  const int steps = dp / (bf16 ? 32 : 16);
  return steps >= (bf16 ? 2 : 4) && steps <= 24 && steps % (bf16 ? 2 : 4) == 0;
}

}  // namespace

// the skinny kernel whenever its Q tile (at most 32 rows), the row stages
// (9 KiB) and the selection's arrays (under 2 KiB) fit in 64 KiB of LDS
static bool skinny_fits(const CdistParams& p, bool bf16) {
  return skinny_steps_ok(p.dp, bf16) && skinny_lds(2, 0, p.dp, bf16) + 9216 + 2048 <= 65536 && p.C <= 32;
}

bool cdist_fuses_select(const CdistParams& p, bool bf16) { return p.U > 0 && p.C > 0 && skinny_fits(p, bf16); }

hipError_t launch_cdist(const CdistParams& p, bool bf16, hipStream_t s, const char** name, bool* shifted) {
  *shifted = false;
  if (p.U <= 0 || p.C <= 0) return hipSuccess;
  if (p.sel_n > 0 && (!cdist_fuses_select(p, bf16) || p.sel_n > 64 || p.C != ((p.sel_n + 3) & ~3) ||
                      !p.one_query))
    return hipErrorInvalidValue;
  const bool skinny = skinny_fits(p, bf16);
  *shifted = skinny && p.one_query;
  if (skinny && !bf16 && p.C <= 32) return run_skinny_f32(p, s, name);
  if (skinny && p.C <= 16) {
    *name = "cdist_skinny_kernel<1,0,1>";
    return run_skinny<1, 0, true>(p, s);
  }
  if (skinny && p.C <= 32) {
    *name = "cdist_skinny_kernel<2,0,1>";
    return run_skinny<2, 0, true>(p, s);
  }
  if (p.C <= 32) {
    *name = bf16 ? "cdist_kernel<64,32,4,1,64>" : "cdist_kernel<64,32,4,0,32>";
    return bf16 ? run<64, 32, 4, true, 64>(p, s) : run<64, 32, 4, false, 32>(p, s);
  }
  if (p.C <= 64) {
    *name = bf16 ? "cdist_kernel<128,64,2,1,64>" : "cdist_kernel<128,64,2,0,32>";
    return bf16 ? run<128, 64, 2, true, 64>(p, s) : run<128, 64, 2, false, 32>(p, s);
  }
  *name = bf16 ? "cdist_kernel<128,128,2,1,32>" : "cdist_kernel<128,128,2,0,16>";
  return bf16 ? run<128, 128, 2, true, 32>(p, s) : run<128, 128, 2, false, 16>(p, s);
}

// Row shift for calls whose cost-matrix kernel stored plain distances (see
// CdistParams): per query b and row j, m_j = min over the query's columns,
// K = exp(-lambda (M - m_j)), +inf (an unused slot) -> 1.  A row of S floats
// takes L = S/4 lanes rounded up to a power of two (at most 64), one 16-byte
// piece per lane and step, 64 / L rows per wave.  The waves of a query's
// blocks stride over its row groups, four groups at a time so that four
// loads per lane are in flight; the first two pieces of every lane stay in
// registers between the minimum and the rewrite (longer rows, S > 512, read
// the rest twice).
__global__ void __launch_bounds__(256) gibbs_rows_kernel(float* kt, float* km, const int2* qinfo, int64_t U,
                                                        float lam) {
  constexpr int G = 4;  // row groups per pass
  const int b = blockIdx.y;
  const int2 qi = qinfo[b];
  const int S = qi.y;
  const int n4 = S >> 2;
  int lg = 0;
  while ((1 << lg) < n4 && lg < 6) ++lg;
  const int L = 1 << lg, R = 64 >> lg;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane & (L - 1), rw = lane >> lg;
  constexpr float kInf = __builtin_huge_valf();
  float* blk = kt + (size_t)qi.x * (size_t)U;
  const int64_t step = (int64_t)gridDim.x * 4 * R;  // rows between a wave's consecutive groups
  for (int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * R; r0 < U; r0 += G * step) {
    float4 v0[G], v1[G];
    float mn[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t row = r0 + g * step + rw;
      float4* rp = (float4*)(blk + (size_t)(row < U ? row : 0) * S);
      v0[g] = v1[g] = make_float4(kInf, kInf, kInf, kInf);
      if (sub < n4) v0[g] = rp[sub];
      if (sub + L < n4) v1[g] = rp[sub + L];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t row = r0 + g * step + rw;
      float4* rp = (float4*)(blk + (size_t)(row < U ? row : 0) * S);
      float m = fminf(fminf(fminf(v0[g].x, v0[g].y), fminf(v0[g].z, v0[g].w)),
                      fminf(fminf(v1[g].x, v1[g].y), fminf(v1[g].z, v1[g].w)));
      for (int c = sub + 2 * L; c < n4; c += L) {
        const float4 v = rp[c];
        m = fminf(m, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
      }
      for (int o = 1; o < L; o <<= 1) m = fminf(m, __shfl_xor(m, o));
      mn[g] = m < kInf ? m : 0.f;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t row = r0 + g * step + rw;
      if (row >= U) continue;
      float4* rp = (float4*)(blk + (size_t)row * S);
      const float m = mn[g];
      auto gibbs = [&](float4 v) {
        v.x = v.x < kInf ? expf(-lam * (v.x - m)) : 1.f;
        v.y = v.y < kInf ? expf(-lam * (v.y - m)) : 1.f;
        v.z = v.z < kInf ? expf(-lam * (v.z - m)) : 1.f;
        v.w = v.w < kInf ? expf(-lam * (v.w - m)) : 1.f;
        return v;
      };
      if (sub < n4) rp[sub] = gibbs(v0[g]);
      if (sub + L < n4) rp[sub + L] = gibbs(v1[g]);
      for (int c = sub + 2 * L; c < n4; c += L) rp[c] = gibbs(rp[c]);
      if (sub == 0) km[(size_t)b * (size_t)U + row] = m;
    }
  }
}

hipError_t launch_gibbs_rows(float* kt, float* km, const int2* qinfo, int64_t U, int B, int max_S, float lam,
                             hipStream_t s) {
  if (U <= 0 || B <= 0) return hipSuccess;
  int lg = 0;
  while ((1 << lg) < (max_S >> 2) && lg < 6) ++lg;
  // about 8192 blocks in all, at most one row group per wave of the widest query
  const int64_t need = (U + 4 * (64 >> lg) - 1) / (4 * (64 >> lg));
  int64_t gx = (8192 + B - 1) / B;
  gx = gx < need ? gx : need;
  dim3 grid((unsigned)(gx < 1 ? 1 : gx), (unsigned)B);
  gibbs_rows_kernel<<<grid, 256, 0, s>>>(kt, km, qinfo, U, lam);
  return hipGetLastError();
}

}  // namespace wmd
