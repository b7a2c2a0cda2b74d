"""Python binding of libwmd.so (the C ABI in include/wmd.h).

Argument marshalling only: this module turns torch tensors into device
pointers and the current HIP stream into a handle, allocates the workspaces the
library asks for (torch owns all device memory), and calls the library.  Every
step of the computation runs in the library's HIP kernels.  If the shared
library is missing the import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from dataclasses import dataclass, field

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwmd.so")

WMD_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "device error", 4: "not supported"}
CDIST = {"fp32": 0, "bf16": 1}
SCHEDULE = {"auto": 0, "resident": 1, "per_iteration": 2, "unfused": 3}
QUERY_GRAPH = 1
QUERY_PER_QUERY_LAUNCHES = 2
MAX_QUERY_LEN = 2048     # raw entries per query the library accepts
MAX_DOC_LEN = 4096       # entries per document
QUERY_ERRORS = {0: "ok", 1: "query word id out of range", 2: "query weight negative or not finite",
                3: "query has no positive weight", 4: "query too long"}

EXPORTS = [
    "wmd_corpus_workspace_bytes", "wmd_create_corpus", "wmd_get_corpus_info", "wmd_destroy",
    "wmd_query_workspace_bytes", "wmd_query", "wmd_query_errors", "wmd_set_timing", "wmd_get_timing",
    "wmd_get_launches", "wmd_sink_candidates", "wmd_set_sink_shape", "wmd_set_merge", "wmd_last_error",
    "wmd_query_static", "wmd_query_static_capacity",
]
# include/wmd_bench.h: measurement kernels (not part of the method)
BENCH_EXPORTS = ["wmd_bench_stream", "wmd_bench_tiles", "wmd_bench_gather", "wmd_bench_valu"]
MERGE = {"all": 0, "none": 1}
TUNING_FILE = os.path.join(_PKG, "tuning", "gfx950_sink_shapes.json")


class CorpusDesc(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_int64), ("d", ctypes.c_int32), ("emb", ctypes.c_void_p),
        ("N", ctypes.c_int64), ("nnz", ctypes.c_int64), ("doc_ptr", ctypes.c_void_p),
        ("word_ids", ctypes.c_void_p), ("weights", ctypes.c_void_p),
        ("compact_vocab", ctypes.c_int32), ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class CorpusInfo(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_int64), ("N", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("d", ctypes.c_int32), ("d_padded", ctypes.c_int32), ("U", ctypes.c_int64),
        ("empty_docs", ctypes.c_int64), ("n_buckets", ctypes.c_int32),
        ("bucket_docs", ctypes.c_int64 * 16), ("bucket_cap", ctypes.c_int32 * 16),
    ]


class QueryDesc(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int32), ("q_ptr_host", ctypes.c_void_p), ("q_ptr", ctypes.c_void_p),
        ("q_ids", ctypes.c_void_p), ("q_weights", ctypes.c_void_p), ("lam", ctypes.c_float),
        ("max_iter", ctypes.c_int32), ("cdist", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("tol", ctypes.c_float), ("iters", ctypes.c_void_p), ("flags", ctypes.c_int32),
    ]


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 96), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
        ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
    ]


class LaunchRec(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 96), ("query", ctypes.c_int32), ("S", ctypes.c_int32),
        ("cap", ctypes.c_int32), ("ndocs", ctypes.c_int32), ("ms", ctypes.c_double),
    ]


class SinkShape(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("tc", "tr", "lg_cg", "maxw", "nwaves", "stream")]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2107_06433_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.wmd_corpus_workspace_bytes.argtypes = [i64, i32, i64, i64]
    lib.wmd_corpus_workspace_bytes.restype = sz
    lib.wmd_create_corpus.argtypes = [ctypes.POINTER(CorpusDesc), vp, ctypes.POINTER(vp)]
    lib.wmd_create_corpus.restype = i32
    lib.wmd_get_corpus_info.argtypes = [vp, ctypes.POINTER(CorpusInfo)]
    lib.wmd_get_corpus_info.restype = i32
    lib.wmd_destroy.argtypes = [vp]
    lib.wmd_destroy.restype = i32
    lib.wmd_query_workspace_bytes.argtypes = [vp, i32, vp, i32]
    lib.wmd_query_workspace_bytes.restype = sz
    lib.wmd_query.argtypes = [vp, ctypes.POINTER(QueryDesc), vp, vp, sz, vp]
    lib.wmd_query.restype = i32
    lib.wmd_query_static.argtypes = [vp, ctypes.POINTER(QueryDesc), vp, vp]
    lib.wmd_query_static.restype = i32
    lib.wmd_query_static_capacity.argtypes = []
    lib.wmd_query_static_capacity.restype = sz
    lib.wmd_query_errors.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), vp]
    lib.wmd_query_errors.restype = i32
    lib.wmd_set_timing.argtypes = [vp, i32]
    lib.wmd_set_timing.restype = i32
    lib.wmd_get_timing.argtypes = [vp, ctypes.POINTER(KernelStat), i32, ctypes.POINTER(ctypes.c_int32)]
    lib.wmd_get_timing.restype = i32
    lib.wmd_get_launches.argtypes = [vp, ctypes.POINTER(LaunchRec), i32, ctypes.POINTER(ctypes.c_int32)]
    lib.wmd_get_launches.restype = i32
    lib.wmd_sink_candidates.argtypes = [vp, i32, i32, ctypes.POINTER(SinkShape), i32, ctypes.POINTER(ctypes.c_int32)]
    lib.wmd_sink_candidates.restype = i32
    lib.wmd_set_sink_shape.argtypes = [vp, i32, i32, ctypes.POINTER(SinkShape)]
    lib.wmd_set_sink_shape.restype = i32
    lib.wmd_set_merge.argtypes = [vp, i32]
    lib.wmd_set_merge.restype = i32
    lib.wmd_last_error.argtypes = []
    lib.wmd_last_error.restype = ctypes.c_char_p
    lib.wmd_bench_stream.argtypes = [vp, vp, sz, i32, i32, vp, vp]
    lib.wmd_bench_stream.restype = ctypes.c_int
    lib.wmd_bench_tiles.argtypes = [vp, sz, i32, vp, vp]
    lib.wmd_bench_tiles.restype = ctypes.c_int
    lib.wmd_bench_gather.argtypes = [vp, i32, vp, sz, vp, i32, vp]
    lib.wmd_bench_gather.restype = ctypes.c_int
    lib.wmd_bench_valu.argtypes = [vp, i32, i32, i32, vp]
    lib.wmd_bench_valu.restype = ctypes.c_int
    return lib


_LIB: ctypes.CDLL | None = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class WMDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status: int):
    if status != WMD_OK:
        raise WMDError(status, lib().wmd_last_error().decode())


def _stream_handle(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


@dataclass
class QueryBatch:
    """Queries marshalled for the library: offsets on host and device, ids and weights on device."""
    q_ptr_host: np.ndarray      # int64 [B+1]
    q_ptr: torch.Tensor         # int64 [B+1], device
    ids: torch.Tensor           # int32 [T], device
    weights: torch.Tensor       # float32 [T], device
    _ws_bytes: dict = field(default_factory=dict, repr=False)  # (corpus id, schedule) -> bytes

    @property
    def B(self) -> int:
        return len(self.q_ptr_host) - 1

    @staticmethod
    def from_arrays(q_ptr, ids, weights, device="cuda") -> "QueryBatch":
        q_ptr = np.ascontiguousarray(np.asarray(q_ptr, dtype=np.int64))
        return QueryBatch(
            q_ptr_host=q_ptr,
            q_ptr=torch.from_numpy(q_ptr).to(device),
            ids=torch.as_tensor(np.asarray(ids, dtype=np.int32)).to(device),
            weights=torch.as_tensor(np.asarray(weights, dtype=np.float32)).to(device),
        )

    @staticmethod
    def from_list(queries, device="cuda") -> "QueryBatch":
        lens = [len(q[0]) for q in queries]
        ptr = np.zeros(len(queries) + 1, dtype=np.int64)
        ptr[1:] = np.cumsum(lens)
        ids = np.concatenate([np.asarray(q[0], dtype=np.int32) for q in queries])
        w = np.concatenate([np.asarray(q[1], dtype=np.float32) for q in queries])
        return QueryBatch.from_arrays(ptr, ids, w, device)


class Corpus:
    """A resident corpus: embeddings (V x d) and documents in CSC form, on one GPU."""

    def __init__(self, emb: torch.Tensor, doc_ptr: torch.Tensor, word_ids: torch.Tensor,
                 weights: torch.Tensor, compact_vocab: bool = True, stream=None,
                 tuning: str | None = TUNING_FILE):
        if not emb.is_cuda:
            raise ValueError("emb must be a device tensor")
        self.emb = emb.contiguous().to(torch.float32)
        self.doc_ptr = doc_ptr.contiguous().to(device=emb.device, dtype=torch.int64)
        self.word_ids = word_ids.contiguous().to(device=emb.device, dtype=torch.int32)
        self.weights = weights.contiguous().to(device=emb.device, dtype=torch.float32)
        self.device = emb.device
        V, d = self.emb.shape
        N = self.doc_ptr.numel() - 1
        nnz = self.word_ids.numel()
        nbytes = lib().wmd_corpus_workspace_bytes(V, d, N, nnz)
        if nbytes == 0:
            raise WMDError(1, "invalid corpus sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=emb.device)
        desc = CorpusDesc(V=V, d=d, emb=_ptr(self.emb), N=N, nnz=nnz, doc_ptr=_ptr(self.doc_ptr),
                          word_ids=_ptr(self.word_ids), weights=_ptr(self.weights),
                          compact_vocab=1 if compact_vocab else 0,
                          workspace=_ptr(self.workspace), workspace_bytes=nbytes)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().wmd_create_corpus(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(handle)))
        self._h = handle
        self.V, self.d, self.N, self.nnz = V, d, N, nnz
        self.pinned = 0
        if tuning and os.path.exists(tuning):
            self.load_tuning(tuning)

    @classmethod
    def from_numpy(cls, emb, doc_ptr, word_ids, weights, device="cuda", compact_vocab=True,
                   tuning: str | None = TUNING_FILE):
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        return cls(t(emb, torch.float32), t(doc_ptr, torch.int64), t(word_ids, torch.int32),
                   t(weights, torch.float32), compact_vocab=compact_vocab, tuning=tuning)

    # ---- kernel shapes (measured tuning)
    def sink_candidates(self, S: int, cap: int) -> list[dict]:
        arr = (SinkShape * 512)()
        n = ctypes.c_int32()
        _check(lib().wmd_sink_candidates(self._h, S, cap, arr, 512, ctypes.byref(n)))
        return [arr[i].as_dict() for i in range(min(n.value, 512))]

    def set_sink_shape(self, S: int, cap: int, shape: dict | None) -> None:
        if shape is None:
            _check(lib().wmd_set_sink_shape(self._h, S, cap, None))
        else:
            _check(lib().wmd_set_sink_shape(self._h, S, cap, ctypes.byref(SinkShape(**shape))))

    def set_merge(self, mode: str) -> None:
        """How length buckets share Sinkhorn launches: "all" (default) or "none"."""
        _check(lib().wmd_set_merge(self._h, MERGE[mode]))

    def load_tuning(self, path: str) -> int:
        """Pin shapes from a measured tuning table; returns how many were applied.

        Entries are keyed by (S, bucket capacity, log2 of the bucket's document
        count); for each (S, cap) the entry tuned on the nearest document count
        to this corpus's bucket is used.
        """
        import json
        import math
        with open(path) as f:
            table = json.load(f)
        info = self.info()
        docs = dict(zip(info["bucket_cap"], info["bucket_docs"]))
        best = {}
        for ent in table.get("entries", []):
            key = (int(ent["S"]), int(ent["cap"]))
            nd = docs.get(key[1], 0)
            if nd <= 0:
                continue
            dist = abs(int(ent.get("ndocs_log2", 0)) - int(math.floor(math.log2(nd))))
            if key not in best or dist < best[key][0]:
                best[key] = (dist, ent["shape"])
        n = 0
        for (S, cap), (_, shape) in best.items():
            try:
                self.set_sink_shape(S, cap, shape)
                n += 1
            except WMDError:
                pass  # a shape the library cannot run for that key: keep the model's choice
        self.pinned = n
        return n

    def launches(self) -> list[dict]:
        cap = 1 << 16
        arr = (LaunchRec * cap)()
        n = ctypes.c_int32()
        _check(lib().wmd_get_launches(self._h, arr, cap, ctypes.byref(n)))
        return [dict(name=arr[i].name.decode(), query=arr[i].query, S=arr[i].S, cap=arr[i].cap,
                     ndocs=arr[i].ndocs, ms=arr[i].ms) for i in range(min(n.value, cap))]

    def info(self) -> dict:
        info = CorpusInfo()
        _check(lib().wmd_get_corpus_info(self._h, ctypes.byref(info)))
        nb = info.n_buckets
        return dict(V=info.V, N=info.N, nnz=info.nnz, d=info.d, d_padded=info.d_padded, U=info.U,
                    empty_docs=info.empty_docs, bucket_docs=list(info.bucket_docs[:nb]),
                    bucket_cap=list(info.bucket_cap[:nb]))

    def close(self):
        if getattr(self, "_h", None):
            lib().wmd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, batch: QueryBatch, schedule: str = "auto") -> int:
        key = (id(self), schedule)
        n = batch._ws_bytes.get(key)
        if n is None:
            n = lib().wmd_query_workspace_bytes(self._h, batch.B, batch.q_ptr_host.ctypes.data,
                                                SCHEDULE[schedule])
            if n == 0:
                raise WMDError(1, lib().wmd_last_error().decode() or "invalid query batch")
            batch._ws_bytes[key] = n
        return n

    def query(self, batch: QueryBatch, lam: float, max_iter: int, cdist: str = "fp32",
              schedule: str = "auto", out: torch.Tensor | None = None,
              workspace: torch.Tensor | None = None, stream=None, check: bool = True,
              tol: float = 0.0, iters: torch.Tensor | None = None, graph: bool = False,
              per_query_launches: bool = False) -> torch.Tensor:
        """Distances of every query to every document: float32 [B, N] on the device.

        With ``check`` the call waits for the stream and raises ValueError if a
        query held an invalid id or weight (its row is NaN either way); it also
        counts the distances that came back +Inf (float32 K underflowed for a
        whole row of a document at this lambda) into ``last_out_of_range`` and
        warns when there are any.

        With ``graph`` the launch sequence is captured into a HIP graph the
        first time and replayed by later calls whose arguments are identical
        (same out / workspace / query tensors and offsets, lambda, iterations,
        options); the device contents of the query tensors may change between
        calls.  Pass ``out`` and ``workspace`` to reuse a graph.  Needs a
        stream other than the legacy default stream.

        ``per_query_launches`` gives every query its own Sinkhorn launches
        instead of sharing launches between queries with identical plans.
        """
        B = batch.B
        if out is None:
            out = torch.empty((B, self.N), dtype=torch.float32, device=self.device)
        need = self.workspace_bytes(batch, schedule)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        if iters is not None and (iters.dtype != torch.int32 or iters.numel() < B * self.N or not iters.is_cuda):
            raise ValueError("iters must be a device int32 tensor of B*N elements")
        desc = QueryDesc(B=B, q_ptr_host=batch.q_ptr_host.ctypes.data, q_ptr=_ptr(batch.q_ptr),
                         q_ids=_ptr(batch.ids), q_weights=_ptr(batch.weights), lam=float(lam),
                         max_iter=int(max_iter), cdist=CDIST[cdist], schedule=SCHEDULE[schedule],
                         tol=float(tol), iters=_ptr(iters),
                         flags=(QUERY_GRAPH if graph else 0) | (QUERY_PER_QUERY_LAUNCHES if per_query_launches else 0))
        sh = _stream_handle(stream)
        with torch.cuda.device(self.device):
            _check(lib().wmd_query(self._h, ctypes.byref(desc), _ptr(out), _ptr(workspace),
                                   workspace.numel(), sh))
        self.last_workspace = workspace
        if check:
            codes = self.query_errors(workspace, B, stream)
            bad = [(b, QUERY_ERRORS.get(int(c), int(c))) for b, c in enumerate(codes) if c]
            if bad:
                raise ValueError(f"invalid queries: {bad[:8]}")
            self.last_out_of_range = int(torch.isposinf(out).sum().item())
            if self.last_out_of_range:
                warnings.warn(f"{self.last_out_of_range} distances are +Inf: float32 K = exp(-lambda M) "
                              f"underflowed for a whole row at lambda={lam:g}", RuntimeWarning, stacklevel=2)
        return out

    def query_static(self, batch: QueryBatch, lam: float, max_iter: int, out: torch.Tensor,
                     cdist: str = "fp32", schedule: str = "auto", stream=None, tol: float = 0.0,
                     iters: torch.Tensor | None = None) -> torch.Tensor:
        """wmd_query_static: the same distances into the caller's ``out`` (float32
        [B, N] on the device) with the library's static device scratch as the
        query workspace -- no device allocation by this call."""
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() < batch.B * self.N:
            raise ValueError("out must be a device float32 tensor of B*N elements")
        if iters is not None and (iters.dtype != torch.int32 or iters.numel() < batch.B * self.N or not iters.is_cuda):
            raise ValueError("iters must be a device int32 tensor of B*N elements")
        desc = QueryDesc(B=batch.B, q_ptr_host=batch.q_ptr_host.ctypes.data, q_ptr=_ptr(batch.q_ptr),
                         q_ids=_ptr(batch.ids), q_weights=_ptr(batch.weights), lam=float(lam),
                         max_iter=int(max_iter), cdist=CDIST[cdist], schedule=SCHEDULE[schedule],
                         tol=float(tol), iters=_ptr(iters), flags=0)
        with torch.cuda.device(self.device):
            _check(lib().wmd_query_static(self._h, ctypes.byref(desc), _ptr(out), _stream_handle(stream)))
        return out

    def set_timing(self, enable: bool):
        """Record HIP events around every kernel launch of later queries."""
        _check(lib().wmd_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> list[dict]:
        """Per-kernel launches, summed duration (ms) and algorithmic flops / bytes."""
        cap = 64
        arr = (KernelStat * cap)()
        n = ctypes.c_int32()
        _check(lib().wmd_get_timing(self._h, arr, cap, ctypes.byref(n)))
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                     flops=arr[i].flops, bytes=arr[i].bytes) for i in range(min(n.value, cap))]

    def query_errors(self, workspace: torch.Tensor, B: int, stream=None) -> np.ndarray:
        codes = np.zeros(B, dtype=np.int32)
        _check(lib().wmd_query_errors(_ptr(workspace), B,
                                      codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      _stream_handle(stream)))
        return codes
