"""CPU oracle for exact triangle counting -- TEST INFRASTRUCTURE, not part of the product.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It wraps ``forward.c`` (plain single-threaded C, see that file's header for what
each routine follows in the paper) through ctypes.  It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "forward.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_RANGE, E_SELF_LOOP, E_DUP_EDGE, E_ASYMMETRIC, E_NOMEM, E_UNSORTED = range(8)
ERROR_NAMES = {
    E_ARG: "arg", E_RANGE: "range", E_SELF_LOOP: "self_loop", E_DUP_EDGE: "dup_edge",
    E_ASYMMETRIC: "asymmetric", E_NOMEM: "nomem", E_UNSORTED: "unsorted",
}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code} ({ERROR_NAMES.get(code, '?')})")
        self.code = code
        self.name = ERROR_NAMES.get(code, "?")


def build(extra_flags: tuple[str, ...] = (), out: str | None = None) -> str:
    """Compile forward.c with gcc into a shared library; returns its path."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", *extra_flags, _SRC, "-o", out]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def _load(path: str | None = None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        build(out=p)
    lib = ctypes.CDLL(p)
    i64, p_ = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_degrees.argtypes = [i64, i64, p_, ctypes.c_int, p_]
    lib.oracle_oriented_csr.argtypes = [i64, i64, p_, ctypes.c_int, ctypes.c_int, p_, p_, i64, p_]
    lib.oracle_count.argtypes = [i64, i64, p_, ctypes.c_int, ctypes.c_int, p_, p_]
    lib.oracle_count_sym_csr.argtypes = [i64, p_, p_, p_, p_]
    lib.oracle_vertex_triangles.argtypes = [i64, i64, p_, i64, p_, p_]
    for f in (lib.oracle_degrees, lib.oracle_oriented_csr, lib.oracle_count,
              lib.oracle_count_sym_csr, lib.oracle_vertex_triangles):
        f.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _edges_np(edges) -> np.ndarray:
    if hasattr(edges, "detach"):
        edges = edges.detach().cpu().numpy()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    return e


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Bound to one compiled copy of forward.c (tests may load deliberately broken copies)."""

    def __init__(self, lib_path: str | None = None):
        self.lib = _load(lib_path)

    def degrees(self, edges, n: int, both: bool = False) -> np.ndarray:
        e = _edges_np(edges)
        deg = np.zeros(max(n, 1), dtype=np.int64)
        st = self.lib.oracle_degrees(n, e.shape[0], _ptr(e), int(both), _ptr(deg))
        if st:
            raise OracleError(st)
        return deg[:n]

    def oriented_csr(self, edges, n: int, both: bool = False, order: int = 0):
        """(row_ptr int64[n+1], col int32[m_fwd]) of the forward-oriented sorted lists."""
        e = _edges_np(edges)
        rp = np.zeros(n + 1, dtype=np.int64)
        mf = np.zeros(1, dtype=np.int64)
        cap = e.shape[0]
        col = np.zeros(max(cap, 1), dtype=np.int32)
        st = self.lib.oracle_oriented_csr(n, e.shape[0], _ptr(e), int(both), order, _ptr(rp),
                                          _ptr(col), cap, _ptr(mf))
        if st:
            raise OracleError(st)
        return rp, col[: int(mf[0])]

    def count(self, edges, n: int, both: bool = False, order: int = 0,
              per_vertex: bool = False):
        """Total (int) or (total, per-vertex uint64[n]) when per_vertex is set."""
        e = _edges_np(edges)
        tot = np.zeros(1, dtype=np.uint64)
        pv = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
        st = self.lib.oracle_count(n, e.shape[0], _ptr(e), int(both), order, _ptr(tot), _ptr(pv))
        if st:
            raise OracleError(st)
        if per_vertex:
            return int(tot[0]), pv[:n]
        return int(tot[0])

    def count_sym_csr(self, row_ptr, col, n: int, per_vertex: bool = False):
        rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
        c = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
        if c.size == 0:
            c = np.zeros(1, dtype=np.int32)
        tot = np.zeros(1, dtype=np.uint64)
        pv = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
        st = self.lib.oracle_count_sym_csr(n, _ptr(rp), _ptr(c), _ptr(tot), _ptr(pv))
        if st:
            raise OracleError(st)
        if per_vertex:
            return int(tot[0]), pv[:n]
        return int(tot[0])

    def vertex_triangles(self, edges, n: int, queries) -> np.ndarray:
        e = _edges_np(edges)
        q = np.ascontiguousarray(np.asarray(queries, dtype=np.int32))
        out = np.zeros(max(q.size, 1), dtype=np.uint64)
        st = self.lib.oracle_vertex_triangles(n, e.shape[0], _ptr(e), q.size, _ptr(q), _ptr(out))
        if st:
            raise OracleError(st)
        return out[: q.size]


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def count(edges, n, **kw):
    return default().count(edges, n, **kw)


def oriented_csr(edges, n, **kw):
    return default().oriented_csr(edges, n, **kw)


def degrees(edges, n, **kw):
    return default().degrees(edges, n, **kw)


def vertex_triangles(edges, n, queries):
    return default().vertex_triangles(edges, n, queries)


def count_sym_csr(row_ptr, col, n, **kw):
    return default().count_sym_csr(row_ptr, col, n, **kw)
