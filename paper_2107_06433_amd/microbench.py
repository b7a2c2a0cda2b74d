"""Achievable ceilings of one MI355X, measured with the library's measurement
kernels (include/wmd_bench.h): HBM read and copy bandwidth, the bandwidth of a
K^T-shaped row gather in a corpus's own word-id order, and the VALU issue
rates of float32 FMA, the hardware reciprocal and DPP cross-lane adds.

    python -m paper_2107_06433_amd.microbench [--workload single] [--S 20]

prints one JSON line.  bench.py calls measure() to report each kernel's
fraction of these ceilings next to its fraction of the published peaks.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from paper_2107_06433_amd import wmd

CUS = 256              # MI355X compute units
SIMDS = 4 * CUS
CLOCK_GHZ = 2.4        # peak engine clock


def _time(fn, reps: int) -> float:
    """Median of `reps` event-timed runs of fn (ms), after one warm-up run."""
    fn()
    s = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def _ok(rc: int):
    if rc != 0:
        raise RuntimeError(f"measurement kernel failed to launch (code {rc})")


def hbm(nbytes: int = 2 << 30, reps: int = 5) -> dict:
    lib = wmd.lib()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    best = {}
    for blocks in (2048, 4096, 8192, 16384):
        r = _time(lambda: _ok(lib.wmd_bench_stream(src.data_ptr(), None, nbytes, 0, blocks, sink.data_ptr(), sh)), reps)
        c = _time(lambda: _ok(lib.wmd_bench_stream(src.data_ptr(), dst.data_ptr(), nbytes, 1, blocks, None, sh)), reps)
        best["read"] = max(best.get("read", 0.0), nbytes / (r * 1e-3) / 1e9)
        best["copy"] = max(best.get("copy", 0.0), 2 * nbytes / (c * 1e-3) / 1e9)
    del src, dst
    return {"read_GBps": best["read"], "copy_GBps": best["copy"], "bytes": nbytes}


def tiles(rows: int, row_bytes: int, reps: int = 10) -> dict:
    """The cost-matrix kernel's read pattern over rows x row_bytes (16-row
    tiles, 64-byte pieces) next to a plain stream of the same bytes."""
    lib = wmd.lib()
    nbytes = rows * row_bytes
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    t_tile = _time(lambda: _ok(lib.wmd_bench_tiles(src.data_ptr(), rows, row_bytes, sink.data_ptr(), sh)), reps)
    t_stream = min(_time(lambda: _ok(lib.wmd_bench_stream(src.data_ptr(), None, nbytes, 0, b, sink.data_ptr(), sh)),
                         reps) for b in (673, 2048, 8192))
    return {"rows": rows, "row_bytes": row_bytes, "bytes": nbytes, "tile_us": t_tile * 1e3,
            "tile_GBps": nbytes / (t_tile * 1e-3) / 1e9, "stream_us": t_stream * 1e3,
            "stream_GBps": nbytes / (t_stream * 1e-3) / 1e9}


def gather(ids: torch.Tensor, U: int, S: int, reps: int = 10, min_rows: int = 1 << 22) -> dict:
    """Rows of S floats from a U-row table, in the order of `ids` (device
    int32), the id stream repeated to at least min_rows rows: a single pass
    over one corpus's entries (tens of MB) is over in a few microseconds, and
    its time would be mostly the launch's own."""
    lib = wmd.lib()
    if ids.numel() < min_rows:
        ids = ids.repeat(-(-min_rows // ids.numel()))
    table = torch.rand(U * S, dtype=torch.float32, device="cuda")
    out = torch.empty(ids.numel(), dtype=torch.float32, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    best = 0.0
    for blocks in (1024, 2048, 4096, 8192):
        t = _time(lambda: _ok(lib.wmd_bench_gather(table.data_ptr(), S, ids.data_ptr(), ids.numel(), out.data_ptr(),
                                                   blocks, sh)), reps)
        best = max(best, ids.numel() * S * 4 / (t * 1e-3) / 1e9)
    return {"GBps": best, "rows": int(ids.numel()), "S": S, "table_rows": U}


def valu(reps: int = 5) -> dict:
    lib = wmd.lib()
    blocks, iters = 2 * SIMDS, 8192  # 8 waves per SIMD
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    res = {}
    for mode, name in ((0, "fma"), (1, "rcp"), (2, "dpp_add")):
        t = _time(lambda: _ok(lib.wmd_bench_valu(out.data_ptr(), blocks, iters, mode, sh)), reps)
        inst = blocks * 4 * iters * 16  # wave instructions
        res[name + "_wave_inst_per_simd_cycle"] = inst / (t * 1e-3) / (SIMDS * CLOCK_GHZ * 1e9)
        if mode == 0:
            res["fma_TFLOPs"] = blocks * 256 * iters * 16 * 2 / (t * 1e-3) / 1e12
    return res


def measure(ids: torch.Tensor | None = None, U: int = 0, S: int = 20) -> dict:
    r = {"hbm": hbm(), "valu": valu()}
    if ids is not None and U > 0:
        r["gather"] = gather(ids, U, S)
        r["cost_matrix_stream"] = tiles(U, 1280)  # the compacted f32 table, d = 300 padded to 320
    return r


def corpus_ids(word_ids: np.ndarray) -> tuple[np.ndarray, int]:
    """The corpus's entry stream as compacted row ids (rows of the used words
    in ascending vocabulary order, as the library numbers them)."""
    uniq, inv = np.unique(np.asarray(word_ids), return_inverse=True)
    return inv.astype(np.int32), len(uniq)


def main():
    from paper_2107_06433_amd import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="single", choices=["tiny", "single", "batched", "serving"])
    ap.add_argument("--S", type=int, default=20, help="floats per gathered row (the padded query width)")
    args = ap.parse_args()
    w = synth.make_workload(args.workload, n_queries=1 if args.workload == "serving" else None)
    ids, U = corpus_ids(w.corpus.word_ids)
    res = measure(torch.from_numpy(ids).cuda(), U, args.S)
    res["workload"] = args.workload
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
