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
#include "wmd_internal.h"

namespace wmd {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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
        // an unused query slot holds K = 1: padding for the Sinkhorn kernels
        const float kv = qc[b] >= 0 ? expf(-p.lam * dist) : 1.f;
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
template <int NT, bool BF16, int CH>
__global__ void __launch_bounds__(256) cdist_skinny_kernel(CdistParams p) {
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int KS = BF16 ? 32 : 16;        // k values per 16-byte-per-lane load step
  // CH = dp / KS load steps: the whole row, a compile-time count, and every
  // load unconditional (rows past U read row 0 and are never stored), so the
  // MFMA of step i waits only for load i
  constexpr int ROWB = CH * KS * ESZ;       // bytes per embedding row (64 per step)
  constexpr int LDQ = ROWB + 16;            // LDS row pitch in bytes (one 16-byte pad)
  constexpr int VPR = ROWB / 16;            // 16-byte pieces per row
  constexpr int QTOT = NT * 16 * VPR;       // pieces of the Q tile
  constexpr int QPT = (QTOT + 255) / 256;   // per thread
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const int64_t myrow = m0 + (lane & 15);
  const bool row_ok = myrow < p.U;
  const unsigned char* Ag = (BF16 ? (const unsigned char*)p.e16 : (const unsigned char*)p.e32) +
                            (size_t)(row_ok ? myrow : 0) * ROWB + 16 * (lane >> 4);
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Q: NT*16 rows go to LDS through registers.  Its loads are issued first
  // and its LDS stores come after the vocabulary row's loads: loads retire in
  // order, so the stores wait for the Q pieces alone while the row is already
  // in flight.  Rows past C repeat Q's first piece: each output column depends
  // on its own Q row only, and the epilogue never stores those columns.
  const unsigned char* Qg = BF16 ? (const unsigned char*)p.q16 : (const unsigned char*)p.q32;
  uint4 qv[QPT];
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int i = j * 256 + tid;
    const int row = i / VPR;
    const bool ok = (QTOT % 256 == 0 || i < QTOT) && row < p.C;
    qv[j] = *(const uint4*)(Qg + (ok ? (size_t)row * ROWB + 16 * (i - row * VPR) : 0));
  }
  uint4 buf[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) buf[i] = *(const uint4*)(Ag + (size_t)i * 64);
  // the epilogue's per-row and per-column data, fetched early for the same
  // reason (indices clamped)
  float en_r[4];
  int used_r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + 4 * (lane >> 4) + i;
    const int64_t mc = m < p.U ? m : p.U - 1;
    en_r[i] = p.en[mc];
    used_r[i] = p.used[mc];
  }
  int q_c[NT];
  float qn_c[NT];
  int2 ci_c[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int64_t n = t * 16 + (lane & 15);
    const int64_t nc = n < p.C ? n : p.C - 1;
    q_c[t] = p.qid[nc];
    qn_c[t] = p.qn[nc];
    ci_c[t] = p.cinfo[nc];
  }
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int i = j * 256 + tid;
    const int row = i / VPR;
    if (QTOT % 256 == 0 || i < QTOT) *(uint4*)(smem + row * LDQ + 16 * (i - row * VPR)) = qv[j];
  }
  __syncthreads();
  {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int kb = i * 64 + 16 * (lane >> 4);  // byte offset of this lane's k run
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const uint4 q = *(const uint4*)(smem + (t * 16 + (lane & 15)) * LDQ + kb);
        if constexpr (BF16) {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, buf[i]),
                                                          __builtin_bit_cast(bf16x8, q), acc[t], 0, 0, 0);
        } else {
          const f32x4 a = __builtin_bit_cast(f32x4, buf[i]);
          const f32x4 b = __builtin_bit_cast(f32x4, q);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], acc[t], 0, 0, 0);
        }
      }
    }
  }
  // epilogue: register i of lane l holds row 4*(l/16)+i, column l%16 of each
  // tile.  All K values first, then the stores (a store counts against the
  // same memory counter as a load; nothing waits on them).
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float m2 = en_r[i] + qn_c[t] - 2.f * acc[t][i];
      const float dist = used_r[i] == q_c[t] ? 0.f : sqrtf(fmaxf(m2, 0.f));
      // an unused query slot holds K = 1: padding for the Sinkhorn kernels
      acc[t][i] = q_c[t] >= 0 ? expf(-p.lam * dist) : 1.f;
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
}

template <int NT, bool BF16, int CH>
hipError_t run_skinny_ch(const CdistParams& p, hipStream_t s) {
  const size_t lds = (size_t)NT * 16 * (p.dp * (BF16 ? 2 : 4) + 16);
  const unsigned grid = (unsigned)((p.U + 63) / 64);
  cdist_skinny_kernel<NT, BF16, CH><<<grid, 256, lds, s>>>(p);
  return hipGetLastError();
}

// the skinny kernel instantiated for this row length (dp / (16 / elem bytes)
// load steps), or hipErrorInvalidValue when there is none
template <int NT, bool BF16>
hipError_t run_skinny(const CdistParams& p, hipStream_t s) {
  const int steps = p.dp / (BF16 ? 32 : 16);
  switch (steps) {
    case 4: return run_skinny_ch<NT, BF16, 4>(p, s);
    case 8: return run_skinny_ch<NT, BF16, 8>(p, s);
    case 12: return run_skinny_ch<NT, BF16, 12>(p, s);
    case 16: return run_skinny_ch<NT, BF16, 16>(p, s);
    case 20: return run_skinny_ch<NT, BF16, 20>(p, s);
    case 24: return run_skinny_ch<NT, BF16, 24>(p, s);
    default: break;
  }
  if constexpr (BF16) {
    switch (steps) {
      case 2: return run_skinny_ch<NT, BF16, 2>(p, s);
      case 6: return run_skinny_ch<NT, BF16, 6>(p, s);
      case 10: return run_skinny_ch<NT, BF16, 10>(p, s);
      case 14: return run_skinny_ch<NT, BF16, 14>(p, s);
      case 18: return run_skinny_ch<NT, BF16, 18>(p, s);
      case 22: return run_skinny_ch<NT, BF16, 22>(p, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

bool skinny_steps_ok(int dp, bool bf16) {
  const int steps = dp / (bf16 ? 32 : 16);
  return steps >= (bf16 ? 2 : 4) && steps <= 24 && steps % (bf16 ? 2 : 4) == 0;
}

}  // namespace

hipError_t launch_cdist(const CdistParams& p, bool bf16, hipStream_t s, const char** name) {
  if (p.U <= 0 || p.C <= 0) return hipSuccess;
  const size_t skinny_lds = (size_t)32 * (p.dp * (bf16 ? 2 : 4) + 16);
  const bool skinny = skinny_steps_ok(p.dp, bf16);
  if (skinny && p.C <= 16 && skinny_lds / 2 <= 65536) {
    *name = bf16 ? "cdist_skinny_kernel<1,1>" : "cdist_skinny_kernel<1,0>";
    return bf16 ? run_skinny<1, true>(p, s) : run_skinny<1, false>(p, s);
  }
  if (skinny && p.C <= 32 && skinny_lds <= 65536) {
    *name = bf16 ? "cdist_skinny_kernel<2,1>" : "cdist_skinny_kernel<2,0>";
    return bf16 ? run_skinny<2, true>(p, s) : run_skinny<2, false>(p, s);
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

}  // namespace wmd
