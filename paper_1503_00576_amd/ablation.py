"""Python binding of libtc_ablation.so (include/tc_ablation.h): the yardstick kernels for
timing the paper's own counting design (Section 3.3: one thread per oriented edge, two-pointer
merge) and the variants of its Section 3.4 optimisations on this GPU.  Argument marshalling
only; the counting path never uses this module."""
from __future__ import annotations

import ctypes
import os

import torch

from . import api

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtc_ablation.so")
EXPORTS = ["tca_edge_merge", "tca_zip_edges", "tca_sort_temp_bytes", "tca_sort", "tca_gather"]

TWO_READS, AOS, PLAIN_PTRS, HALF_WAVE = 1, 2, 4, 8
SORT_PAIRS_COMPARE, SORT_PAIRS_RADIX, SORT_PACKED_RADIX = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libtc_ablation.so not found at {LIB_PATH}: build it first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                             ctypes.c_size_t)
    L.tca_edge_merge.argtypes = [vp, vp, vp, vp, vp, i64, u32, i32, i32, vp, vp]
    L.tca_edge_merge.restype = ctypes.c_int
    L.tca_zip_edges.argtypes = [vp, vp, i64, vp, vp]
    L.tca_zip_edges.restype = ctypes.c_int
    L.tca_sort_temp_bytes.argtypes = [i32, i64, i32]
    L.tca_sort_temp_bytes.restype = sz
    L.tca_sort.argtypes = [i32, i64, i32, vp, vp, vp, vp, vp, sz, vp]
    L.tca_sort.restype = ctypes.c_int
    L.tca_gather.argtypes = [vp, i64, i32, i64, u32, vp, vp]
    L.tca_gather.restype = ctypes.c_int
    _lib = L
    return L


class EdgeMerge:
    """The thread-per-edge merge over a prepared graph's oriented CSR (rank space)."""

    def __init__(self, prepared: api.Prepared):
        a = prepared.arrays()
        self.prepared = prepared  # keeps the workspace alive
        self.row_ptr, self.col = a["row_ptr"], a["col_padded"]
        self.src, self.dst = a["src"], a["col"]
        self.mf = int(self.dst.numel())
        self.dev = prepared.device
        self.pairs = None
        self.total = torch.empty(1, dtype=torch.int64, device=self.dev)

    def zip(self):
        if self.pairs is None:
            self.pairs = torch.empty(2 * max(self.mf, 1), dtype=torch.int32, device=self.dev)
            api._raise(lib().tca_zip_edges(api._ptr(self.src), api._ptr(self.dst), self.mf,
                                           api._ptr(self.pairs), api._stream(self.dev)),
                       "tca_zip_edges")
        return self.pairs

    def run_async(self, flags: int = 0, threads: int = 64, blocks: int | None = None):
        """Enqueue one count; blocks default to 8 per compute unit (the paper's tuned shape
        was 64 threads x 8 blocks per multiprocessor)."""
        if blocks is None:
            blocks = 8 * torch.cuda.get_device_properties(self.dev).multi_processor_count
        pairs = self.zip() if flags & AOS else None
        api._raise(lib().tca_edge_merge(api._ptr(self.row_ptr), api._ptr(self.col),
                                        api._ptr(self.src), api._ptr(self.dst), api._ptr(pairs),
                                        self.mf, flags, threads, blocks, api._ptr(self.total),
                                        api._stream(self.dev)), "tca_edge_merge")
        return self.total

    def count(self, flags: int = 0, threads: int = 64, blocks: int | None = None) -> int:
        return int(self.run_async(flags, threads, blocks).item()) & 0xFFFFFFFFFFFFFFFF


def sort_async(method: int, bits: int, a: torch.Tensor, b: torch.Tensor | None = None,
               a_alt: torch.Tensor | None = None, b_alt: torch.Tensor | None = None,
               temp: torch.Tensor | None = None) -> torch.Tensor:
    """Enqueue one library sort of edges (see tc_ablation.h); returns the temp buffer."""
    count = a.numel() // (2 if method == SORT_PAIRS_COMPARE else 1)
    L = lib()
    need = L.tca_sort_temp_bytes(method, count, bits)
    if temp is None or temp.numel() < need:
        temp = torch.empty(max(need, 1), dtype=torch.uint8, device=a.device)
    api._raise(L.tca_sort(method, count, bits, api._ptr(a), api._ptr(b), api._ptr(a_alt),
                          api._ptr(b_alt), api._ptr(temp), temp.numel(), api._stream(a.device)),
               "tca_sort")
    return temp


def gather_async(table: torch.Tensor, elem_bytes: int, count: int, seed: int,
                 sink: torch.Tensor) -> None:
    api._raise(lib().tca_gather(api._ptr(table), table.numel() * table.element_size(),
                                elem_bytes, count, seed, api._ptr(sink),
                                api._stream(table.device)), "tca_gather")
