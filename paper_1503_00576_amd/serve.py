"""Serving loop: exact triangle counts for a stream of graph requests on one GPU.

Continuous batching: a scheduler thread admits waiting requests whenever their HBM footprint
(edge array + workspace + outputs) fits the free part of the memory budget and an execution
slot is free.  Small graphs admitted together are packed into one batched launch
(tc_count_batched); larger graphs run tc_count on their own stream, so several requests'
kernels overlap on the device.  A finished request's memory returns to the budget, except the
prepared CSR of a graph that carries a key, which stays resident (least recently used first
out) so that the next request for the same key only runs the counting kernel.

Every result is exact and independent of what else is in flight (each request has its own
outputs and workspace), so a result alone and in the mix are equal."""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import torch

from . import api, synth

_EDGE_BYTES = 8


@dataclass
class Request:
    edges: torch.Tensor          # int32 [m, 2], host (ideally pinned) or device
    n: int
    key: object = None           # graphs with a key keep their prepared CSR resident
    arrival: float = field(default_factory=time.perf_counter)


@dataclass(eq=False)  # flights compare by identity (they hold tensors)
class _Flight:
    reqs: list
    futures: list
    event: torch.cuda.Event
    result: object               # api.Result or api.BatchResult
    nbytes: int
    stream: torch.cuda.Stream
    keep: list                   # tensors that must live until the event
    kind: str
    resident: object = None      # (key, Prepared) to cache after completion
    busy_key: object = None      # resident key this flight uses


class Server:
    def __init__(self, device="cuda:0", budget_bytes: int = 32 << 30, streams: int = 4,
                 small_edges: int = 1 << 18, batch_graphs: int = 512, max_inflight: int = 8,
                 resident_bytes: int = 8 << 30):
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.resident_budget = int(resident_bytes)
        self.small_edges = int(small_edges)
        self.batch_graphs = int(batch_graphs)
        self.max_inflight = int(max_inflight)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self._next_stream = 0
        self._pending: collections.deque = collections.deque()
        self._inflight: list[_Flight] = []
        self._resident: collections.OrderedDict = collections.OrderedDict()  # key -> (Prepared, bytes)
        self._busy: collections.Counter = collections.Counter()  # resident keys in flight
        self._used = 0
        self._resident_used = 0
        self._cv = threading.Condition()
        self._stop = False
        self._failed = None
        self.stats = collections.Counter()
        self._thread = threading.Thread(target=self._loop, name="tc-serve", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------------ public

    def submit(self, req: Request) -> Future:
        fut: Future = Future()
        with self._cv:
            if self._failed is not None:
                fut.set_exception(RuntimeError(f"tc-serve scheduler failed: {self._failed!r}"))
                return fut
            self._pending.append((req, fut))
            self._cv.notify()
        return fut

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify()
        self._thread.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ footprint

    def footprint(self, req: Request) -> int:
        m = int(req.edges.shape[0])
        if req.key is not None and req.key in self._resident:
            return 64
        if m <= self.small_edges:
            # packed symmetric CSR (row_ptr + 2m col) + batched workspace share
            return 16 * m + 12 * req.n + 4096
        return _EDGE_BYTES * m + api.workspace_size(req.n, m) + 64

    # ------------------------------------------------------------------ scheduler

    def _stream(self) -> torch.cuda.Stream:
        s = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        return s

    def _evict_resident(self, need: int):
        for key in list(self._resident):
            if self._used + need <= self.budget:
                break
            if self._busy[key]:
                continue  # in use by a request in flight
            prep, nb = self._resident.pop(key)
            self._used -= nb
            self._resident_used -= nb
            self.stats["evicted"] += 1
            del prep

    def _loop(self):
        try:
            self._schedule()
        except BaseException as exc:  # never leave a caller waiting on a dead scheduler
            with self._cv:
                self._failed = exc
                futs = [f for _, f in self._pending] + [f for fl in self._inflight
                                                         for f in fl.futures]
                self._pending.clear()
                self._inflight.clear()
            for f in futs:
                if not f.done():
                    f.set_exception(RuntimeError(f"tc-serve scheduler failed: {exc!r}"))
            raise

    def _schedule(self):
        torch.cuda.set_device(self.device)
        while True:
            with self._cv:
                self._complete_ready()
                if self._stop and not self._pending and not self._inflight:
                    return
                admitted_small, admitted_large = [], []
                # admit in arrival order while memory and slots allow
                while self._pending and len(self._inflight) + len(admitted_large) + \
                        (1 if admitted_small else 0) < self.max_inflight:
                    req, fut = self._pending[0]
                    need = self.footprint(req)
                    if self._used + need > self.budget:
                        self._evict_resident(need)
                    if self._used + need > self.budget:
                        if not self._inflight and not admitted_small and not admitted_large:
                            self._pending.popleft()
                            fut.set_exception(MemoryError(
                                f"request needs {need} B, budget {self.budget} B"))
                            self.stats["rejected"] += 1
                            continue
                        break  # wait for memory to free up
                    self._pending.popleft()
                    self._used += need
                    hit = req.key is not None and req.key in self._resident
                    if not hit and int(req.edges.shape[0]) <= self.small_edges:
                        admitted_small.append((req, fut, need))
                        if len(admitted_small) >= self.batch_graphs:
                            break
                    else:
                        admitted_large.append((req, fut, need))
                if not admitted_small and not admitted_large:
                    self._cv.wait(timeout=0.0002)
                    continue
            for req, fut, need in admitted_large:
                self._launch_single(req, fut, need)
            if admitted_small:
                self._launch_batch(admitted_small)

    def _complete_ready(self) -> bool:
        done = [f for f in self._inflight if f.event.query()]
        for f in done:
            self._inflight.remove(f)
            self._finish(f)
        return bool(done)

    def _finish(self, f: _Flight):
        now = time.perf_counter()
        try:
            if f.kind == "batch":
                st = f.result.status.cpu()
                tot = f.result.totals.cpu()
                for i, (req, fut) in enumerate(zip(f.reqs, f.futures)):
                    if int(st[i]):
                        fut.set_exception(api.TCError(int(st[i]), "request"))
                    else:
                        fut.set_result((int(tot[i]) & 0xFFFFFFFFFFFFFFFF, now - req.arrival))
            else:
                st = int(f.result.status.item())
                req, fut = f.reqs[0], f.futures[0]
                if st:
                    fut.set_exception(api.TCError(st, "request"))
                else:
                    fut.set_result((int(f.result.total.item()) & 0xFFFFFFFFFFFFFFFF,
                                    now - req.arrival))
        except Exception as exc:  # never leave a future pending
            for fut in f.futures:
                if not fut.done():
                    fut.set_exception(exc)
        self.stats["completed"] += len(f.reqs)
        if f.busy_key is not None:
            self._busy[f.busy_key] -= 1
        released = f.nbytes
        if f.resident is not None:
            key, prep = f.resident
            nb = int(prep.workspace.numel())
            if nb <= self.resident_budget - self._resident_used and key not in self._resident:
                self._resident[key] = (prep, nb)
                self._resident_used += nb
                released -= min(released, nb)
        with self._cv:
            self._used -= released
            self._cv.notify()

    def _launch_single(self, req: Request, fut: Future, need: int):
        s = self._stream()
        keep = []
        with torch.cuda.stream(s):
            res = api.Result(torch.empty(1, dtype=torch.int64, device=self.device),
                             torch.empty(1, dtype=torch.int32, device=self.device))
            resident, busy = None, None
            if req.key is not None and req.key in self._resident:
                prep, _ = self._resident[req.key]
                self._resident.move_to_end(req.key)
                self._busy[req.key] += 1
                busy = req.key
                prep.count_async(out=res)
                self.stats["resident_hits"] += 1
                kind = "resident"
            else:
                e = req.edges.to(self.device, non_blocking=True)
                keep.append(e)
                prep = api.Prepared(e, req.n)
                prep.count_async(out=res)
                if req.key is not None:
                    resident = (req.key, prep)
                keep.append(prep.workspace)
                kind = "single"
            ev = torch.cuda.Event()
            ev.record(s)
        self._inflight.append(_Flight([req], [fut], ev, res, need, s, keep, kind, resident, busy))
        self.stats[kind] += 1

    def _launch_batch(self, items):
        s = self._stream()
        reqs = [r for r, _, _ in items]
        futs = [f for _, f, _ in items]
        with torch.cuda.stream(s):
            graphs = [(r.edges.to(self.device, non_blocking=True), r.n) for r in reqs]
            packed = synth.pack_symmetric(graphs, device=self.device)
            b = api.Batch(packed["vtx_off"], packed["adj_off"], packed["row_ptr"],
                          packed["col"], packed["G"], packed["n_total"], packed["adj_total"])
            res = api.count_batched_async(b)
            ev = torch.cuda.Event()
            ev.record(s)
        keep = [g for g, _ in graphs] + [packed, res]
        self._inflight.append(_Flight(reqs, futs, ev, res, sum(n for _, _, n in items), s, keep,
                                      "batch"))
        self.stats["batches"] += 1
        self.stats["batched_requests"] += len(items)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]
