/*
 * wmd_bench.h -- measurement kernels of libwmd.so.
 *
 * Not part of the method: they measure the ceilings the hot path is measured
 * against.  The paper models its fused SDDMM-SpMM as bound by memory bandwidth
 * (Section III-E) and quotes the machine's bandwidths in Table II; on a GPU
 * the Sinkhorn kernels' bytes come from two places -- a stream of the corpus
 * entries from HBM, and a gather of K^T rows whose ids follow the corpus's
 * Zipf word distribution (mostly cache hits) -- and with the K^T block kept in
 * registers the iterations are bound by the VALU instead.  Each function
 * enqueues one kernel on `stream` (a hipStream_t, NULL = default) and returns
 * 0, 1 for an invalid argument, or 3 if the launch failed; the caller times it
 * (HIP events on the same stream).  All pointers are device pointers owned by
 * the caller.
 */
#ifndef WMD_BENCH_H
#define WMD_BENCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Streams `bytes` (a multiple of 16) through `blocks` blocks of 256 threads:
 * copy = 0 reads src only (HBM read bandwidth; `sink` receives one float that
 * is written only in a case that cannot occur), copy = 1 copies src to dst
 * (bytes read + bytes written). */
int wmd_bench_stream(const void* src, void* dst, size_t bytes, int32_t copy, int32_t blocks, float* sink,
                     void* stream);

/* Reads `rows` rows of row_bytes (a multiple of 64) in MFMA operand order: a
 * wave per 16 consecutive rows, each load step reading a 64-byte piece of
 * every one of the 16 rows (16 bytes per lane, each load instruction touching
 * 16 lines), all steps of a row in flight together.  Set beside a plain
 * stream of the same bytes it prices that read order, which the cost-matrix
 * kernel avoids by reading whole 128-byte lines and re-laying them out in
 * LDS. */
int wmd_bench_tiles(const void* src, size_t rows, int32_t row_bytes, float* sink, void* stream);

/* Reads row ids[k] (S floats, S a multiple of 4 from 4 to 512) of `table`
 * for every k < nids and writes each row's sum to out[k]: 4 S bytes read per
 * id.  Rows are read as the Sinkhorn kernels read their K^T rows: 16-byte
 * pieces, two per lane, eight rows per lane with all their loads in flight
 * together.  Every ids[k] must name a row of `table`.  With the corpus's
 * entry stream as `ids` and a table of the K^T shape (U rows of S floats)
 * this is the Sinkhorn row gather on its own. */
int wmd_bench_gather(const float* table, int32_t S, const int32_t* ids, size_t nids, float* out, int32_t blocks,
                     void* stream);

/* VALU issue rate: every thread of `blocks` blocks of 256 runs `iters` rounds
 * of 16 independent instructions and writes one float to out[thread]:
 * mode 0 = float32 FMA (2 flops each), 1 = hardware reciprocal, 2 = add with a
 * DPP cross-lane operand. */
int wmd_bench_valu(float* out, int32_t blocks, int32_t iters, int32_t mode, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WMD_BENCH_H */
