"""Serving loop: exact triangle counts for a stream of graph requests on one GPU.

Continuous batching: a scheduler thread admits waiting requests whenever their HBM footprint
(edge array + workspace + outputs) fits the free part of the memory budget and an execution
slot is free.  Small graphs admitted together are packed into one batched input on the device
(tc_batched_pack) and counted by one batched launch (tc_count_batched); larger graphs run
tc_preprocess + tc_count_prepared on their own stream, so several requests' kernels overlap
on the device.  A finished request's memory returns to the budget, except the prepared CSR of
a graph that carries a key, which stays resident (least recently used first out) so that the
next request for the same key only runs the counting kernel.

A key names one graph: a request whose key is resident but whose graph differs (vertex count,
edge count or a sample of its edges) is counted from scratch and replaces the resident entry.
Counts on one resident workspace are enqueued on the stream that prepared it, so they run one
after another on the device (they share the workspace's work-queue counters).

Every result is exact and independent of what else is in flight (each request has its own
outputs), so a result alone and in the mix are equal.  This module only moves data and
marshals calls: every step of the counting runs in libtc's HIP kernels."""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import torch

from . import api

_EDGE_BYTES = 8
_SIG_SAMPLES = 64


def graph_signature(edges: torch.Tensor, n: int) -> tuple:
    """(n, m, a sample of edges at evenly spaced rows): what a resident-key hit must match."""
    m = int(edges.shape[0])
    if m == 0:
        return (int(n), 0, ())
    idx = torch.linspace(0, m - 1, min(m, _SIG_SAMPLES)).round().to(torch.int64)
    sample = edges[idx.to(edges.device)].to("cpu").flatten().tolist()
    return (int(n), m, tuple(sample))


@dataclass
class Request:
    edges: torch.Tensor          # int32 [m, 2], host (ideally pinned) or device
    n: int
    key: object = None           # graphs with a key keep their prepared CSR resident
    arrival: float = field(default_factory=time.perf_counter)
    signature: tuple = None      # filled in by Server.submit for keyed requests


@dataclass(eq=False)  # flights compare by identity (they hold tensors)
class _Flight:
    reqs: list
    futures: list
    event: torch.cuda.Event
    result: object               # api.Result, or (api.BatchResult, pack status)
    nbytes: int
    stream: torch.cuda.Stream
    keep: list                   # tensors that must live until the event
    kind: str
    resident: object = None      # _Resident to cache after completion
    busy_key: object = None      # resident key this flight uses


@dataclass(eq=False)
class _Resident:
    prep: api.Prepared
    nbytes: int
    stream: torch.cuda.Stream    # every count on this workspace is enqueued here
    signature: tuple


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
        self._resident: collections.OrderedDict = collections.OrderedDict()  # key -> _Resident
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
        if req.key is not None and req.signature is None:
            req.signature = graph_signature(req.edges, req.n)
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

    def _hit(self, req: Request) -> bool:
        if req.key is None:
            return False
        r = self._resident.get(req.key)
        return r is not None and r.signature == req.signature

    def footprint(self, req: Request) -> int:
        m = int(req.edges.shape[0])
        if self._hit(req):
            return 64
        if m <= self.small_edges:
            # edge array, packed symmetric CSR (row_ptr + 2m col), the pack's sort keys and
            # the batched workspace's share
            return 48 * m + 24 * req.n + 4096
        return _EDGE_BYTES * m + api.workspace_size(req.n, m) + 64

    # ------------------------------------------------------------------ scheduler

    def _stream(self) -> torch.cuda.Stream:
        s = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        return s

    def _drop_resident(self, key):
        r = self._resident.pop(key)
        self._used -= r.nbytes
        self._resident_used -= r.nbytes
        self.stats["evicted"] += 1

    def _evict_resident(self, need: int):
        for key in list(self._resident):
            if self._used + need <= self.budget:
                break
            if self._busy[key]:
                continue  # a request in flight (or admitted in this round) uses it
            self._drop_resident(key)

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
                    hit = self._hit(req)
                    if hit:
                        # held from admission on, so that no later admission evicts it
                        self._busy[req.key] += 1
                        admitted_large.append((req, fut, need, True))
                    elif int(req.edges.shape[0]) <= self.small_edges:
                        admitted_small.append((req, fut, need))
                        if len(admitted_small) >= self.batch_graphs:
                            break
                    else:
                        admitted_large.append((req, fut, need, False))
                if not admitted_small and not admitted_large:
                    self._cv.wait(timeout=0.0002)
                    continue
            for req, fut, need, hit in admitted_large:
                self._launch_single(req, fut, need, hit)
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
                res, pack_status = f.result
                pst = pack_status.cpu().tolist()
                st = res.status.cpu().tolist()
                tot = res.totals.cpu().tolist()
                for i, (req, fut) in enumerate(zip(f.reqs, f.futures)):
                    code = pst[i] or st[i]  # the pack's finding first
                    if code:
                        fut.set_exception(api.TCError(code, "request"))
                    else:
                        fut.set_result((tot[i] & 0xFFFFFFFFFFFFFFFF, now - req.arrival))
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
        with self._cv:
            if f.busy_key is not None:
                self._busy[f.busy_key] -= 1
            released = f.nbytes
            if f.resident is not None and int(f.result.status.item()) == 0:
                key, r = f.resident
                old = self._resident.get(key)
                if old is not None and old.signature != r.signature and not self._busy[key]:
                    self._drop_resident(key)  # the key now names another graph
                    old = None
                if old is None and r.nbytes <= self.resident_budget - self._resident_used:
                    self._resident[key] = r
                    self._resident_used += r.nbytes
                    released -= min(released, r.nbytes)
            self._used -= released
            self._cv.notify()

    def _launch_single(self, req: Request, fut: Future, need: int, hit: bool):
        keep = []
        resident, busy = None, None
        if hit:
            r = self._resident[req.key]
            self._resident.move_to_end(req.key)
            s = r.stream  # after every earlier count on this workspace
            busy = req.key
            with torch.cuda.stream(s):
                res = api.Result(torch.empty(1, dtype=torch.int64, device=self.device),
                                 torch.empty(1, dtype=torch.int32, device=self.device))
                r.prep.count_async(out=res)
                ev = torch.cuda.Event()
                ev.record(s)
            kind = "resident"
            self.stats["resident_hits"] += 1
        else:
            s = self._stream()
            with torch.cuda.stream(s):
                res = api.Result(torch.empty(1, dtype=torch.int64, device=self.device),
                                 torch.empty(1, dtype=torch.int32, device=self.device))
                e = req.edges.to(self.device, non_blocking=True)
                keep.append(e)
                prep = api.Prepared(e, req.n)
                prep.count_async(out=res)
                if req.key is not None:
                    resident = (req.key, _Resident(prep, int(prep.workspace.numel()), s,
                                                   req.signature))
                keep.append(prep.workspace)
                ev = torch.cuda.Event()
                ev.record(s)
            kind = "single"
        self._inflight.append(_Flight([req], [fut], ev, res, need, s, keep, kind, resident, busy))
        self.stats[kind] += 1

    def _launch_batch(self, items):
        s = self._stream()
        reqs = [r for r, _, _ in items]
        futs = [f for _, f, _ in items]
        ns = [int(r.n) for r in reqs]
        ms = [int(r.edges.shape[0]) for r in reqs]
        vo, eo = [0], [0]
        for n, m in zip(ns, ms):
            vo.append(vo[-1] + n)
            eo.append(eo[-1] + m)
        G, N, M = len(reqs), vo[-1], eo[-1]
        keep = []
        with torch.cuda.stream(s):
            # one upload of the offsets and one of the concatenated edge arrays
            offs_h = torch.tensor(vo + eo, dtype=torch.int64).pin_memory()
            if all(not r.edges.is_cuda for r in reqs):
                edges_h = torch.empty((M, 2), dtype=torch.int32, pin_memory=True)
                if M:
                    torch.cat([r.edges for r in reqs], out=edges_h)
                edges = edges_h.to(self.device, non_blocking=True)
                keep.append(edges_h)
            else:
                edges = torch.cat([r.edges.to(self.device, non_blocking=True) for r in reqs])
            offs = offs_h.to(self.device, non_blocking=True)
            packed = api.pack_edges_async(edges, offs[:G + 1], offs[G + 1:], N)
            res = api.count_batched_async(packed.batch)
            ev = torch.cuda.Event()
            ev.record(s)
        keep += [offs_h, offs, edges, packed, res]
        self._inflight.append(_Flight(reqs, futs, ev, (res, packed.status),
                                      sum(n for _, _, n in items), s, keep, "batch"))
        self.stats["batches"] += 1
        self.stats["batched_requests"] += len(items)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]
