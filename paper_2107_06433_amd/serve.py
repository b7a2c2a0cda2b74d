"""Continuous-batching query server over a resident corpus.

Requests (a query document: word ids and weights) arrive at arbitrary times.
The scheduler keeps them in FIFO order and, whenever an execution slot is free,
admits the longest prefix of the queue whose device memory (the query
workspace: K^T for every query word over the corpus vocabulary, plus the
output rows) fits in what the memory budget has left, up to `max_batch`
queries.  The admitted batch is one wmd_query call on one of several HIP
streams, so batches admitted while others are still on the GPU run
concurrently; their memory returns to the budget as they complete.  A request
that alone exceeds the whole budget is rejected.

The scheduler is host logic only; an executor does the device work.  The GPU
executor (GpuExecutor) calls the library; tests drive the scheduler with a
stand-in executor on the CPU.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


class RejectedError(RuntimeError):
    """The request can never be admitted (its memory exceeds the whole budget)."""


@dataclass
class Request:
    ids: np.ndarray
    weights: np.ndarray
    arrival: float                       # seconds on the scheduler's clock
    future: Future = field(default_factory=Future)
    rid: int = -1
    admitted: float = float("nan")
    done: float = float("nan")


@dataclass
class Batch:
    requests: list
    nbytes: int
    handle: object = None
    launched: float = float("nan")


class Scheduler:
    """FIFO admission by memory budget and free execution slots."""

    def __init__(self, executor, mem_budget: int, max_batch: int = 64, max_inflight: int = 3):
        self.ex = executor
        self.budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.pending: collections.deque[Request] = collections.deque()
        self.inflight: list[Batch] = []
        self.used = 0
        self.completed: list[Request] = []
        self.rejected: list[Request] = []
        self.peak_used = 0
        self.batches = 0
        self._next = 0

    def submit(self, req: Request) -> Future:
        req.rid = self._next
        self._next += 1
        self.pending.append(req)
        return req.future

    def poll(self, now: float) -> int:
        """Resolve finished batches; returns how many requests completed.

        A batch whose executor fails (while asking whether it is done or for
        its results) resolves every one of its requests with that exception;
        its memory returns to the budget either way.
        """
        n = 0
        still = []
        for b in self.inflight:
            try:
                if not self.ex.done(b.handle):
                    still.append(b)
                    continue
                results = self.ex.results(b.handle)
            except Exception as e:  # noqa: BLE001 - handed to the callers' futures
                results = [e] * len(b.requests)
            for req, res in zip(b.requests, results):
                req.done = now
                if isinstance(res, Exception):
                    req.future.set_exception(res)
                else:
                    req.future.set_result(res)
                self.completed.append(req)
                n += 1
            try:
                self.ex.release(b.handle)
            finally:
                self.used -= b.nbytes
        self.inflight = still
        return n

    def _fail(self, req: Request, now: float, exc: Exception) -> None:
        req.done = now
        req.future.set_exception(exc)
        self.rejected.append(req)

    def admit(self, now: float) -> int:
        """Launch batches while slots and memory allow; returns requests admitted.

        A request whose cost the executor cannot compute (an invalid query) is
        rejected with that exception; a batch whose launch fails resolves its
        requests with the launch's exception and takes no memory.
        """
        admitted = 0
        while self.pending and len(self.inflight) < self.max_inflight:
            take, nbytes = [], 0
            while self.pending and len(take) < self.max_batch:
                cand = take + [self.pending[0]]
                try:
                    need = self.ex.cost(cand)
                except Exception as e:  # noqa: BLE001
                    if take:
                        try:  # is the newcomer the problem? check it alone
                            self.ex.cost(cand[-1:])
                        except Exception as e1:  # noqa: BLE001
                            self._fail(self.pending.popleft(), now, e1)
                            continue
                        break  # it is valid alone: launch what we have, retry it next time
                    self._fail(self.pending.popleft(), now, e)
                    continue
                if need > self.budget and not take:
                    req = self.pending.popleft()  # can never fit, even alone
                    self._fail(req, now, RejectedError(
                        f"request {req.rid} needs {need} bytes, budget is {self.budget}"))
                    continue
                if self.used + need > self.budget:
                    break
                take.append(self.pending.popleft())
                nbytes = need
            if not take:
                break
            for r in take:
                r.admitted = now
            b = Batch(requests=take, nbytes=nbytes, launched=now)
            try:
                b.handle = self.ex.launch(take)
            except Exception as e:  # noqa: BLE001
                for r in take:
                    self._fail(r, now, e)
                continue
            self.inflight.append(b)
            self.used += nbytes
            self.peak_used = max(self.peak_used, self.used)
            self.batches += 1
            admitted += len(take)
        return admitted

    def drain(self, clock, sleep: float = 0.0) -> None:
        while self.pending or self.inflight:
            now = clock()
            self.poll(now)
            self.admit(now)
            if sleep:
                time.sleep(sleep)


class GpuExecutor:
    """Runs admitted batches with wmd_query on a pool of HIP streams."""

    def __init__(self, corpus, lam: float, max_iter: int, cdist: str = "bf16", streams: int = 3,
                 to_host: bool = True):
        import torch

        from . import wmd
        self.torch = torch
        self.wmd = wmd
        self.corpus = corpus
        self.lam, self.max_iter, self.cdist = lam, max_iter, cdist
        self.streams = [torch.cuda.Stream(device=corpus.device) for _ in range(streams)]
        self._rr = 0
        self.to_host = to_host
        self._cost_cache: dict = {}

    def _ptr(self, reqs):
        lens = [len(r.ids) for r in reqs]
        ptr = np.zeros(len(reqs) + 1, dtype=np.int64)
        ptr[1:] = np.cumsum(lens)
        return ptr

    def cost(self, reqs) -> int:
        for r in reqs:
            if len(r.ids) > self.wmd.MAX_QUERY_LEN:
                raise self.wmd.WMDError(4, f"a query has {len(r.ids)} entries, at most "
                                           f"{self.wmd.MAX_QUERY_LEN} are supported")
        ptr = self._ptr(reqs)
        key = (len(reqs), int(((np.diff(ptr) + 3) // 4).sum()))  # workspace depends on B and sum of widths
        n = self._cost_cache.get(key)
        if n is None:
            batch = self.wmd.QueryBatch(q_ptr_host=ptr, q_ptr=None, ids=None, weights=None)
            n = self.corpus.workspace_bytes(batch) + 4 * len(reqs) * self.corpus.N
            if len(self._cost_cache) < 100000:
                self._cost_cache[key] = n
        return n

    def launch(self, reqs):
        torch = self.torch
        s = self.streams[self._rr % len(self.streams)]
        self._rr += 1
        ptr = self._ptr(reqs)
        ids = np.concatenate([r.ids for r in reqs]).astype(np.int32)
        w = np.concatenate([r.weights for r in reqs]).astype(np.float32)
        with torch.cuda.stream(s):
            dev = self.corpus.device
            h_ptr = torch.from_numpy(ptr).pin_memory()
            h_ids = torch.from_numpy(ids).pin_memory()
            h_w = torch.from_numpy(w).pin_memory()
            batch = self.wmd.QueryBatch(q_ptr_host=ptr, q_ptr=h_ptr.to(dev, non_blocking=True),
                                        ids=h_ids.to(dev, non_blocking=True), weights=h_w.to(dev, non_blocking=True))
            out = torch.empty((len(reqs), self.corpus.N), dtype=torch.float32, device=dev)
            ws = torch.empty(self.corpus.workspace_bytes(batch), dtype=torch.uint8, device=dev)
            self.corpus.query(batch, self.lam, self.max_iter, cdist=self.cdist, out=out, workspace=ws,
                              stream=s, check=False)
            err = torch.empty(len(reqs), dtype=torch.int32, pin_memory=True)
            err.copy_(ws[:4 * len(reqs)].view(torch.int32), non_blocking=True)
            host = None
            if self.to_host:
                host = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)
                host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # keep every buffer alive until the event has passed
        return dict(ev=ev, out=out, ws=ws, err=err, host=host, keep=(batch, h_ptr, h_ids, h_w))

    def done(self, h) -> bool:
        return h["ev"].query()

    def results(self, h):
        res = []
        rows = h["host"] if h["host"] is not None else h["out"]
        for b, code in enumerate(h["err"].tolist()):
            if code:
                res.append(ValueError(self.wmd.QUERY_ERRORS.get(code, str(code))))
            else:
                res.append(rows[b])
        return res

    def release(self, h) -> None:
        h.clear()


class Server:
    """Background-thread server: submit() returns a Future of the distances."""

    def __init__(self, corpus, lam: float, max_iter: int, cdist: str = "bf16", mem_budget: int = 8 << 30,
                 max_batch: int = 64, max_inflight: int = 3, executor=None, max_query_len: int = 2048):
        # executor: a stand-in for the GPU executor (tests); corpus is then unused
        self.ex = executor if executor is not None else GpuExecutor(corpus, lam, max_iter, cdist,
                                                                    streams=max_inflight)
        self.max_query_len = int(max_query_len)
        self.sched = Scheduler(self.ex, mem_budget, max_batch, max_inflight)
        self._lock = threading.Lock()
        self._stop = threading.Event()
        self._t0 = time.perf_counter()
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    def _clock(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, ids, weights) -> Future:
        """Queue one query; malformed or oversized queries get a failed Future."""
        ids = np.asarray(ids, dtype=np.int32).ravel()
        weights = np.asarray(weights, dtype=np.float32).ravel()
        if ids.size == 0 or ids.shape != weights.shape:
            f: Future = Future()
            f.set_exception(ValueError("a query needs matching, non-empty ids and weights"))
            return f
        if ids.size > self.max_query_len:
            f = Future()
            f.set_exception(ValueError(f"a query has {ids.size} entries, at most {self.max_query_len} "
                                       "are supported"))
            return f
        req = Request(ids=ids, weights=weights, arrival=self._clock())
        with self._lock:
            return self.sched.submit(req)

    def _loop(self):
        while not self._stop.is_set() or self.sched.pending or self.sched.inflight:
            with self._lock:
                now = self._clock()
                try:
                    self.sched.poll(now)
                    self.sched.admit(now)
                except Exception as e:  # noqa: BLE001 - keep serving; fail what is queued
                    while self.sched.pending:
                        self.sched._fail(self.sched.pending.popleft(), now, e)
                idle = not self.sched.pending and not self.sched.inflight
            time.sleep(0.001 if idle else 0.00005)

    def close(self) -> None:
        """Stop accepting work and finish everything already submitted."""
        self._stop.set()
        self._thread.join()


def run_trace(sched: Scheduler, requests: list, arrivals: np.ndarray, warmup: int = 0, sleep: float = 0.0):
    """Open-loop replay: request i enters the queue at arrivals[i] seconds.

    Latency is completion (observed by the polling loop) minus scheduled
    arrival.  Statistics cover the requests after the first `warmup`.
    """
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0  # noqa: E731
    i, n = 0, len(requests)
    while i < n or sched.pending or sched.inflight:
        now = clock()
        while i < n and arrivals[i] <= now:
            requests[i].arrival = float(arrivals[i])
            sched.submit(requests[i])
            i += 1
        sched.poll(now)
        sched.admit(now)
        if sleep:
            time.sleep(sleep)
    wall = clock()
    meas = [r for r in requests[warmup:] if not np.isnan(r.done)]
    lat = np.array([r.done - r.arrival for r in meas])
    ok = [r for r in meas if r.future.exception() is None]
    t_first = min(r.arrival for r in meas) if meas else 0.0
    t_last = max(r.done for r in meas) if meas else 0.0
    return {
        "completed": len(ok), "rejected": len(sched.rejected), "batches": sched.batches,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else float("nan"),
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else float("nan"),
        "mean_ms": float(lat.mean() * 1e3) if len(lat) else float("nan"),
        "window_s": t_last - t_first, "wall_s": wall, "peak_mem_bytes": sched.peak_used,
        "offered_qps": (len(arrivals) / arrivals[-1]) if len(arrivals) else 0.0,
        "served_qps": len(ok) / max(1e-9, t_last - t_first),
    }
