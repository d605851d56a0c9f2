"""Python binding of libtc.so: argument marshalling only (every step of the path runs in the
library's HIP kernels).  Device memory comes from torch; the work is enqueued on torch's
current stream of the edge tensor's device."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _native

OK, E_ARG, E_RANGE, E_SELF_LOOP, E_DUP_EDGE, E_ASYMMETRIC, E_UNSORTED, E_WORKSPACE, \
    E_TOO_LARGE, E_HIP, E_MISMATCH, E_SCRATCH = range(12)
STATUS_NAMES = {OK: "ok", E_ARG: "arg", E_RANGE: "range", E_SELF_LOOP: "self_loop",
                E_DUP_EDGE: "dup_edge", E_ASYMMETRIC: "asymmetric", E_UNSORTED: "unsorted",
                E_WORKSPACE: "workspace", E_TOO_LARGE: "too_large", E_HIP: "hip",
                E_MISMATCH: "mismatch", E_SCRATCH: "scratch"}

EDGES_ONCE = 0
EDGES_BOTH = 1


class TCError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        msg = _native.lib().tc_strerror(code).decode()
        super().__init__(f"{where}: {msg} (status {code})" if where else msg)
        self.code = code
        self.name = STATUS_NAMES.get(code, "?")


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check_edges(edges: torch.Tensor) -> torch.Tensor:
    if not isinstance(edges, torch.Tensor) or not edges.is_cuda:
        raise TypeError("edges must be a CUDA (HIP) tensor")
    if edges.dtype != torch.int32:
        raise TypeError("edges must be int32")
    if edges.dim() != 2 or edges.shape[1] != 2:
        raise ValueError("edges must have shape [m, 2]")
    return edges.contiguous()


def _flags(both: bool) -> int:
    return EDGES_BOTH if both else EDGES_ONCE


OPTION_NAMES = tuple(name for name, _ in _native.TcOptions._fields_ if name != "size")


def default_options() -> dict:
    """The library's defaults for the single-graph options (struct tc_options)."""
    o = _native.TcOptions()
    _raise(_native.lib().tc_options_init(ctypes.byref(o)), "tc_options_init")
    return {k: int(getattr(o, k)) for k in OPTION_NAMES}


def _opts(options: dict | None):
    """struct tc_options for a dict of overrides (None: the library's defaults, NULL)."""
    if not options:
        return None
    o = _native.TcOptions()
    _raise(_native.lib().tc_options_init(ctypes.byref(o)), "tc_options_init")
    for k, v in options.items():
        if k not in OPTION_NAMES:
            raise KeyError(f"unknown option {k!r}")
        setattr(o, k, int(v))
    return ctypes.byref(o)


def workspace_size(n: int, m: int, both: bool = False, options: dict | None = None) -> int:
    s = _native.lib().tc_workspace_size(int(n), int(m), _flags(both), _opts(options))
    if s == 0:
        raise TCError(E_ARG, "tc_workspace_size")
    return s


def alloc_workspace(n: int, m: int, both: bool = False, device=None,
                    options: dict | None = None) -> torch.Tensor:
    return torch.empty(workspace_size(n, m, both, options), dtype=torch.uint8, device=device)


def _raise(code: int, where: str):
    if code != OK:
        raise TCError(code, where)


@dataclass
class Result:
    total: torch.Tensor        # uint64 as int64 [1] on the device
    status: torch.Tensor       # int32 [1] on the device
    per_vertex: torch.Tensor | None = None  # uint64 as int64 [n]

    def check(self) -> "Result":
        st = int(self.status.item())
        if st != OK:
            raise TCError(st, "device")
        return self


def count_async(edges: torch.Tensor, n: int, both: bool = False, per_vertex: bool = False,
                workspace: torch.Tensor | None = None, out: Result | None = None,
                options: dict | None = None) -> Result:
    """Enqueue tc_count (or tc_count_per_vertex) on the current stream; no synchronisation."""
    edges = _check_edges(edges)
    dev = edges.device
    m = edges.shape[0]
    ws = workspace if workspace is not None else alloc_workspace(n, m, both, dev, options)
    op = _opts(options)
    if out is None:
        out = Result(torch.empty(1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int32, device=dev),
                     torch.empty(n, dtype=torch.int64, device=dev) if per_vertex else None)
    L = _native.lib()
    if per_vertex:
        code = L.tc_count_per_vertex(_ptr(edges), n, m, _flags(both), op, _ptr(ws), ws.numel(),
                                     _stream(dev), _ptr(out.total), _ptr(out.per_vertex),
                                     _ptr(out.status))
    else:
        code = L.tc_count(_ptr(edges), n, m, _flags(both), op, _ptr(ws), ws.numel(),
                          _stream(dev), _ptr(out.total), _ptr(out.status))
    _raise(code, "tc_count")
    return out


def count(edges: torch.Tensor, n: int, both: bool = False, options: dict | None = None) -> int:
    """Exact number of triangles of the graph given as an int32 [m, 2] edge array."""
    r = count_async(edges, n, both, options=options).check()
    return int(r.total.item()) & 0xFFFFFFFFFFFFFFFF


def count_per_vertex(edges: torch.Tensor, n: int, both: bool = False,
                     options: dict | None = None):
    """(total, per-vertex counts as int64 [n] on the device)."""
    r = count_async(edges, n, both, per_vertex=True, options=options).check()
    return int(r.total.item()) & 0xFFFFFFFFFFFFFFFF, r.per_vertex


def layout(n: int, m: int, both: bool = False, options: dict | None = None) -> _native.TcLayout:
    lay = _native.TcLayout()
    _raise(_native.lib().tc_workspace_layout(n, m, _flags(both), _opts(options),
                                             ctypes.byref(lay)), "tc_workspace_layout")
    return lay


class Prepared:
    """A graph preprocessed on the device (tc_preprocess): its workspace stays resident and
    can be counted again with count_prepared()."""

    def __init__(self, edges: torch.Tensor, n: int, both: bool = False,
                 workspace: torch.Tensor | None = None, options: dict | None = None):
        edges = _check_edges(edges)
        self.device = edges.device
        self.n, self.m, self.both = int(n), int(edges.shape[0]), bool(both)
        self.options = dict(options) if options else None
        self.workspace = (workspace if workspace is not None
                          else alloc_workspace(self.n, self.m, self.both, self.device,
                                               self.options))
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        _raise(_native.lib().tc_preprocess(_ptr(edges), self.n, self.m, _flags(self.both),
                                           _opts(self.options), _ptr(self.workspace),
                                           self.workspace.numel(), _stream(self.device),
                                           _ptr(self.status)), "tc_preprocess")

    def count_async(self, per_vertex: bool = False, out: Result | None = None) -> Result:
        dev = self.device
        if out is None:
            out = Result(torch.empty(1, dtype=torch.int64, device=dev),
                         torch.empty(1, dtype=torch.int32, device=dev),
                         torch.empty(self.n, dtype=torch.int64, device=dev) if per_vertex else None)
        _raise(_native.lib().tc_count_prepared(
            self.n, self.m, _flags(self.both), _opts(self.options), _ptr(self.workspace),
            self.workspace.numel(), _stream(dev), _ptr(out.total),
            _ptr(out.per_vertex) if per_vertex else None, _ptr(out.status)),
            "tc_count_prepared")
        return out

    def count(self) -> int:
        return int(self.count_async().check().total.item()) & 0xFFFFFFFFFFFFFFFF

    def arrays(self) -> dict:
        """Views of the preprocessing arrays: deg, perm, rank (int32 [n]), row_ptr
        (int32 [n+1]), col (int32 [m_fwd]); raises on a data error."""
        st = int(self.status.item())
        if st:
            raise TCError(st, "device")
        lay = layout(self.n, self.m, self.both, self.options)
        ws = self.workspace

        def view(off, count):
            return ws[off: off + 4 * count].view(torch.int32)

        return {"deg": view(lay.deg, self.n), "perm": view(lay.perm, self.n),
                "rank": view(lay.rank, self.n), "row_ptr": view(lay.row_ptr, self.n + 1),
                "col": view(lay.col, lay.m_fwd), "src": view(lay.src, lay.m_fwd),
                "col_padded": view(lay.col, lay.m_fwd + 16), "id_bits": lay.id_bits}


def preprocess(edges: torch.Tensor, n: int, both: bool = False,
               options: dict | None = None) -> dict:
    """Run the preprocessing phase only and return views of its arrays (see Prepared)."""
    p = Prepared(edges, n, both, options=options)
    out = p.arrays()
    out["prepared"] = p
    return out


def sort_u64(keys: torch.Tensor, bits: int) -> torch.Tensor:
    """Sort int64 storage of uint64 keys in place on their low `bits` bits (stable)."""
    if not keys.is_cuda or keys.dtype != torch.int64 or not keys.is_contiguous():
        raise TypeError("keys must be a contiguous int64 CUDA tensor")
    dev = keys.device
    n = keys.numel()
    tmp = torch.empty_like(keys)
    L = _native.lib()
    ws = torch.empty(max(L.tc_sort_workspace_size(n), 256), dtype=torch.uint8, device=dev)
    _raise(L.tc_sort_u64(_ptr(keys), _ptr(tmp), n, bits, _ptr(ws), ws.numel(), _stream(dev)),
           "tc_sort_u64")
    return keys


# ------------------------------------------------------------------ graphs beyond the GPU

def _host_edges(edges):
    """int32 [m, 2] edges in host memory as a contiguous numpy array."""
    import numpy as np
    if isinstance(edges, torch.Tensor):
        if edges.is_cuda:
            raise TypeError("split counting takes the edge array in host memory")
        edges = edges.numpy()
    a = np.ascontiguousarray(edges)
    if a.dtype != np.int32 or a.ndim != 2 or (a.size and a.shape[1] != 2):
        raise TypeError("edges must be int32 [m, 2]")
    return a


class Split:
    """A graph prepared for counting in subgraphs (tc_split_prepare: host only).  The edges
    stay in host memory; the host workspace holds them bucketed by block of the vertex
    partition and is pinned when a GPU is present, so that tc_split_count's copies overlap
    the counting.  parts = 0 picks the smallest number of parts whose device workspace fits
    device_budget bytes (default: 90% of the free device memory)."""

    def __init__(self, edges, n: int, both: bool = False, parts: int = 0,
                 device_budget: int | None = None, options: dict | None = None,
                 pin: bool | None = None):
        e = _host_edges(edges)
        self.n, self.m, self.both = int(n), int(e.shape[0]), bool(both)
        self.options = dict(options) if options else None
        L = _native.lib()
        hsz = L.tc_split_host_workspace_size(self.n, self.m, _flags(self.both))
        if hsz == 0:
            raise TCError(E_ARG, "tc_split_host_workspace_size")
        if pin is None:
            pin = torch.cuda.is_available()
        self.host_ws = torch.empty(hsz + 64, dtype=torch.uint8, pin_memory=bool(pin))
        # 64-byte alignment inside the buffer
        skip = (-self.host_ws.data_ptr()) % 64
        self.host_ws = self.host_ws[skip: skip + hsz]
        if parts == 0 and device_budget is None:
            free, _ = torch.cuda.mem_get_info()
            device_budget = int(free * 0.9)
        info = _native.TcSplitInfo()
        _raise(L.tc_split_prepare(e.ctypes.data_as(ctypes.c_void_p) if e.size else None,
                                  self.n, self.m, _flags(self.both), int(parts),
                                  int(device_budget or 0), _opts(self.options),
                                  _ptr(self.host_ws), hsz, ctypes.byref(info)),
               "tc_split_prepare")
        self.info = {k: int(getattr(info, k)) for k, _ in info._fields_}

    def subgraph(self, i: int):
        """(info dict, local edge array int32 [m_i, 2], global id of every local vertex) of
        subgraph i, exactly as the device counts it."""
        import numpy as np
        L = _native.lib()
        si = _native.TcSplitSubgraph()
        _raise(L.tc_split_subgraph(_ptr(self.host_ws), int(i), ctypes.byref(si)),
               "tc_split_subgraph")
        d = {"n": si.n, "m": si.m, "coef": si.coef, "parts": list(si.parts)[: si.nparts]}
        e = np.empty((si.m, 2), dtype=np.int32)
        v = np.empty(si.n, dtype=np.int32)
        _raise(L.tc_split_subgraph_edges(_ptr(self.host_ws), int(i),
                                         e.ctypes.data_as(ctypes.c_void_p),
                                         v.ctypes.data_as(ctypes.c_void_p)),
               "tc_split_subgraph_edges")
        return d, e, v

    def count_async(self, device=None, per_vertex: bool = False, overlap: bool = True,
                    workspace: torch.Tensor | None = None) -> Result:
        """Enqueue tc_split_count on the device's current stream (the copies on a second
        stream when overlap is set)."""
        dev = torch.device(device if device is not None else "cuda")
        ws = workspace if workspace is not None else torch.empty(
            max(self.info["device_bytes"], 256), dtype=torch.uint8, device=dev)
        out = Result(torch.empty(1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int32, device=dev),
                     torch.empty(self.n, dtype=torch.int64, device=dev) if per_vertex else None)
        cs = None
        if overlap:
            self._copy_stream = torch.cuda.Stream(dev)  # default priority
            cs = ctypes.c_void_p(self._copy_stream.cuda_stream)
        _raise(_native.lib().tc_split_count(
            _ptr(self.host_ws), _opts(self.options), _ptr(ws), ws.numel(), _stream(dev), cs,
            _ptr(out.total), _ptr(out.per_vertex) if per_vertex else None, _ptr(out.status)),
            "tc_split_count")
        out.workspace = ws  # kept until the work has run
        return out

    def count(self, device=None, overlap: bool = True) -> int:
        return int(self.count_async(device, overlap=overlap).check().total.item()) & \
            0xFFFFFFFFFFFFFFFF

    def count_per_vertex(self, device=None, overlap: bool = True):
        r = self.count_async(device, per_vertex=True, overlap=overlap).check()
        return int(r.total.item()) & 0xFFFFFFFFFFFFFFFF, r.per_vertex


def count_split(edges, n: int, both: bool = False, parts: int = 0,
                device_budget: int | None = None, per_vertex: bool = False,
                options: dict | None = None, device=None):
    """Triangle count of a graph held in host memory, counted in subgraphs that fit the
    device (tc_split_prepare + tc_split_count).  Returns the total, or (total, per-vertex)."""
    sp = Split(edges, n, both, parts, device_budget, options)
    if per_vertex:
        return sp.count_per_vertex(device)
    return sp.count(device)


# ------------------------------------------------------------------ derived quantities

def clustering(per_vertex, degree):
    """Local clustering coefficient C(v) = 2 T(v) / (deg(v) (deg(v) - 1)), 0 when deg < 2,
    computed in float64 on the host from exact integer counts."""
    import numpy as np
    t = np.asarray(per_vertex.cpu() if hasattr(per_vertex, "cpu") else per_vertex, dtype=np.float64)
    d = np.asarray(degree.cpu() if hasattr(degree, "cpu") else degree, dtype=np.float64)
    den = d * (d - 1.0)
    out = np.zeros_like(t)
    np.divide(2.0 * t, den, out=out, where=d >= 2)
    return out


def transitivity(total: int, degree) -> float:
    """3 * T / (number of paths of length two) = 3T / sum_v C(deg v, 2); 0 if no such path."""
    import numpy as np
    d = np.asarray(degree.cpu() if hasattr(degree, "cpu") else degree, dtype=np.int64)
    wedges = int((d * (d - 1) // 2).sum())
    return 0.0 if wedges == 0 else 3.0 * total / wedges


# ------------------------------------------------------------------ batched counting

@dataclass
class Batch:
    """Concatenated symmetric CSRs of G graphs on the device (see tc.h, batched counting)."""
    vtx_off: torch.Tensor   # int64 [G+1]
    adj_off: torch.Tensor   # int64 [G+1]
    row_ptr: torch.Tensor   # int32 [n_total + G]
    col: torch.Tensor       # int32 [adj_total]
    G: int
    n_total: int
    adj_total: int


@dataclass
class BatchResult:
    totals: torch.Tensor            # uint64 as int64 [G]
    status: torch.Tensor            # int32 [G]
    per_vertex: torch.Tensor | None = None   # uint64 as int64 [n_total]

    def check(self) -> "BatchResult":
        bad = torch.nonzero(self.status).flatten()
        if bad.numel():
            g = int(bad[0])
            raise TCError(int(self.status[g]), f"graph {g}")
        return self


def batched_workspace_size(g_cap: int, n_cap: int, adj_cap: int) -> int:
    s = _native.lib().tc_batched_workspace_size(int(g_cap), int(n_cap), int(adj_cap))
    if s == 0:
        raise TCError(E_ARG, "tc_batched_workspace_size")
    return s


class BatchPlan:
    """A captured launch sequence for batches within (g_cap, n_cap, adj_cap), bound to its own
    workspace; run() replays it on the current stream."""

    def __init__(self, g_cap: int, n_cap: int, adj_cap: int, tuning: dict | None = None,
                 device=None):
        import json
        self.device = torch.device(device if device is not None else "cuda")
        self.caps = (int(g_cap), int(n_cap), int(adj_cap))
        self.workspace = torch.empty(batched_workspace_size(*self.caps), dtype=torch.uint8,
                                     device=self.device)
        self.tuning = dict(tuning or {})
        js = json.dumps(self.tuning).encode() if self.tuning else None
        h = ctypes.c_void_p()
        _raise(_native.lib().tc_batched_plan_create(*self.caps, 0, js, _ptr(self.workspace),
                                                    self.workspace.numel(), ctypes.byref(h)),
               "tc_batched_plan_create")
        self._h = h

    def run_async(self, b: Batch, per_vertex: bool = False,
                  out: BatchResult | None = None) -> BatchResult:
        dev = self.device
        if out is None:
            out = BatchResult(torch.empty(b.G, dtype=torch.int64, device=dev),
                              torch.empty(b.G, dtype=torch.int32, device=dev),
                              torch.empty(b.n_total, dtype=torch.int64, device=dev)
                              if per_vertex else None)
        _raise(_native.lib().tc_batched_plan_run(
            self._h, b.G, _ptr(b.vtx_off), _ptr(b.adj_off), _ptr(b.row_ptr), _ptr(b.col),
            b.n_total, b.adj_total, _stream(dev), _ptr(out.totals),
            _ptr(out.per_vertex) if per_vertex else None, _ptr(out.status)),
            "tc_batched_plan_run")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            _native.lib().tc_batched_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count_batched_async(b: Batch, per_vertex: bool = False,
                        workspace: torch.Tensor | None = None) -> BatchResult:
    """Enqueue a one-shot batched count (no graph capture) on the current stream."""
    dev = b.vtx_off.device
    ws = workspace if workspace is not None else torch.empty(
        batched_workspace_size(b.G, b.n_total, b.adj_total), dtype=torch.uint8, device=dev)
    out = BatchResult(torch.empty(b.G, dtype=torch.int64, device=dev),
                      torch.empty(b.G, dtype=torch.int32, device=dev),
                      torch.empty(b.n_total, dtype=torch.int64, device=dev) if per_vertex else None)
    _raise(_native.lib().tc_count_batched(
        b.G, _ptr(b.vtx_off), _ptr(b.adj_off), _ptr(b.row_ptr), _ptr(b.col), b.n_total,
        b.adj_total, _ptr(ws), ws.numel(), _stream(dev), _ptr(out.totals),
        _ptr(out.per_vertex) if per_vertex else None, _ptr(out.status)), "tc_count_batched")
    out.workspace = ws  # keep alive until the work has run
    return out


def count_batched(b: Batch, per_vertex: bool = False) -> BatchResult:
    """One-shot batched count (no graph capture); returns checked results."""
    return count_batched_async(b, per_vertex).check()


@dataclass
class Packed:
    """Result of tc_batched_pack: the batched input plus the pack's per-graph status."""
    batch: Batch
    status: torch.Tensor        # int32 [G]: range / self-loop / offset errors found by the pack
    workspace: torch.Tensor     # the sort's workspace (kept until the work has run)


def pack_edges_async(edges: torch.Tensor, vtx_off: torch.Tensor, edge_off: torch.Tensor,
                     n_total: int) -> Packed:
    """Enqueue tc_batched_pack on the current stream: G graphs' edge arrays, concatenated
    (int32 [m_total, 2] of local ids, graph g's at rows edge_off[g] .. edge_off[g+1]), with
    int64 [G+1] vertex and edge offsets, all on the device -> the batched input format."""
    edges = _check_edges(edges)
    dev = edges.device
    G = int(vtx_off.numel()) - 1
    M = int(edges.shape[0])
    for t in (vtx_off, edge_off):
        if t.device != dev or t.dtype != torch.int64 or t.numel() != G + 1 or \
                not t.is_contiguous():
            raise TypeError("offsets must be contiguous int64 [G+1] tensors on the edges' device")
    L = _native.lib()
    wsz = L.tc_batched_pack_workspace_size(G, int(n_total), M)
    if wsz == 0:
        raise TCError(E_TOO_LARGE if G > 0 else E_ARG, "tc_batched_pack_workspace_size")
    ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    adj_off = torch.empty(G + 1, dtype=torch.int64, device=dev)
    row_ptr = torch.empty(int(n_total) + G, dtype=torch.int32, device=dev)
    col = torch.empty(max(2 * M, 1), dtype=torch.int32, device=dev)
    status = torch.empty(G, dtype=torch.int32, device=dev)
    _raise(L.tc_batched_pack(G, _ptr(vtx_off), _ptr(edge_off), _ptr(edges), int(n_total), M,
                             _ptr(ws), ws.numel(), _stream(dev), _ptr(adj_off), _ptr(row_ptr),
                             _ptr(col), _ptr(status)), "tc_batched_pack")
    return Packed(Batch(vtx_off, adj_off, row_ptr, col, G, int(n_total), 2 * M), status, ws)
