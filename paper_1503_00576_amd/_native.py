"""ctypes loader for libtc.so (the HIP library).  There is no fallback: if the library is
missing or fails to load, every entry point raises."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TC_LIB", os.path.join(HERE, "libtc.so"))

EXPORTS = [
    "tc_strerror", "tc_options_init", "tc_workspace_size", "tc_count", "tc_count_per_vertex",
    "tc_count_noalloc",
    "tc_workspace_layout", "tc_preprocess", "tc_count_prepared", "tc_sort_workspace_size",
    "tc_sort_u64", "tc_batched_workspace_size", "tc_batched_plan_create", "tc_batched_plan_run",
    "tc_batched_plan_destroy", "tc_count_batched", "tc_batched_pack_workspace_size",
    "tc_batched_pack", "tc_split_host_workspace_size", "tc_split_prepare", "tc_split_count",
    "tc_split_subgraph", "tc_split_subgraph_edges",
]


class TcOptions(ctypes.Structure):
    """struct tc_options (include/tc.h); fill with tc_options_init."""
    _fields_ = [(name, ctypes.c_uint32) for name in (
        "size", "panel_ranks", "hub_ranks", "row_blocks", "wave_item_edges", "block_item_edges",
        "wave_bitmap_span", "wave_list_max", "block_bitmap_span", "block_list_max",
        "degree_partition", "sort_onesweep", "high_ranks", "row_sort")]


class TcLayout(ctypes.Structure):
    _fields_ = [("deg", ctypes.c_size_t), ("perm", ctypes.c_size_t), ("rank", ctypes.c_size_t),
                ("row_ptr", ctypes.c_size_t), ("col", ctypes.c_size_t),
                ("m_fwd", ctypes.c_int64), ("id_bits", ctypes.c_int32),
                ("src", ctypes.c_size_t)]


class TcSplitInfo(ctypes.Structure):
    """struct tc_split_info (include/tc.h)."""
    _fields_ = [("parts", ctypes.c_uint32), ("subgraphs", ctypes.c_uint32),
                ("m_kept", ctypes.c_int64), ("max_sub_n", ctypes.c_int64),
                ("max_sub_m", ctypes.c_int64), ("device_bytes", ctypes.c_size_t),
                ("host_bytes", ctypes.c_size_t)]


class TcSplitSubgraph(ctypes.Structure):
    """struct tc_split_subgraph_info (include/tc.h)."""
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("coef", ctypes.c_int64),
                ("nparts", ctypes.c_uint32), ("parts", ctypes.c_uint32 * 3)]


_lib = None


def lib():
    """The loaded library (raises RuntimeError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libtc.so not found at {LIB_PATH}: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    L.tc_strerror.argtypes = [ctypes.c_int]
    L.tc_strerror.restype = ctypes.c_char_p
    op = ctypes.POINTER(TcOptions)
    L.tc_options_init.argtypes = [op]
    L.tc_options_init.restype = ctypes.c_int
    L.tc_workspace_size.argtypes = [i64, i64, u32, op]
    L.tc_workspace_size.restype = sz
    L.tc_count.argtypes = [vp, i64, i64, u32, op, vp, sz, vp, vp, vp]
    L.tc_count.restype = ctypes.c_int
    L.tc_count_per_vertex.argtypes = [vp, i64, i64, u32, op, vp, sz, vp, vp, vp, vp]
    L.tc_count_per_vertex.restype = ctypes.c_int
    L.tc_count_noalloc.argtypes = [vp, i64, i64, u32, op, vp, vp, vp]
    L.tc_count_noalloc.restype = ctypes.c_int
    L.tc_workspace_layout.argtypes = [i64, i64, u32, op, ctypes.POINTER(TcLayout)]
    L.tc_workspace_layout.restype = ctypes.c_int
    L.tc_preprocess.argtypes = [vp, i64, i64, u32, op, vp, sz, vp, vp]
    L.tc_preprocess.restype = ctypes.c_int
    L.tc_count_prepared.argtypes = [i64, i64, u32, op, vp, sz, vp, vp, vp, vp]
    L.tc_count_prepared.restype = ctypes.c_int
    L.tc_sort_workspace_size.argtypes = [i64]
    L.tc_sort_workspace_size.restype = sz
    L.tc_sort_u64.argtypes = [vp, vp, i64, ctypes.c_int32, vp, sz, vp]
    L.tc_sort_u64.restype = ctypes.c_int
    i32 = ctypes.c_int32
    L.tc_batched_workspace_size.argtypes = [i32, i64, i64]
    L.tc_batched_workspace_size.restype = sz
    L.tc_batched_plan_create.argtypes = [i32, i64, i64, u32, ctypes.c_char_p, vp, sz,
                                         ctypes.POINTER(vp)]
    L.tc_batched_plan_create.restype = ctypes.c_int
    L.tc_batched_plan_run.argtypes = [vp, i32, vp, vp, vp, vp, i64, i64, vp, vp, vp, vp]
    L.tc_batched_plan_run.restype = ctypes.c_int
    L.tc_batched_plan_destroy.argtypes = [vp]
    L.tc_batched_plan_destroy.restype = None
    L.tc_count_batched.argtypes = [i32, vp, vp, vp, vp, i64, i64, vp, sz, vp, vp, vp, vp]
    L.tc_count_batched.restype = ctypes.c_int
    L.tc_batched_pack_workspace_size.argtypes = [i32, i64, i64]
    L.tc_batched_pack_workspace_size.restype = sz
    L.tc_batched_pack.argtypes = [i32, vp, vp, vp, i64, i64, vp, sz, vp, vp, vp, vp, vp]
    L.tc_batched_pack.restype = ctypes.c_int
    L.tc_split_host_workspace_size.argtypes = [i64, i64, u32]
    L.tc_split_host_workspace_size.restype = sz
    L.tc_split_prepare.argtypes = [vp, i64, i64, u32, u32, sz, op, vp, sz,
                                   ctypes.POINTER(TcSplitInfo)]
    L.tc_split_prepare.restype = ctypes.c_int
    L.tc_split_count.argtypes = [vp, op, vp, sz, vp, vp, vp, vp, vp]
    L.tc_split_count.restype = ctypes.c_int
    L.tc_split_subgraph.argtypes = [vp, u32, ctypes.POINTER(TcSplitSubgraph)]
    L.tc_split_subgraph.restype = ctypes.c_int
    L.tc_split_subgraph_edges.argtypes = [vp, u32, vp, vp]
    L.tc_split_subgraph_edges.restype = ctypes.c_int
    _lib = L
    return L
