"""Host-side checks of libtc.so (no GPU needed): the library loads, exports every function
include/tc.h declares, and rejects bad arguments before enqueuing anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1503_00576_amd import _native
    return _native.lib()


def test_exports_every_declared_symbol(lib):
    from paper_1503_00576_amd import _native
    names = header_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_native.EXPORTS) == names


def test_strerror(lib):
    for code in range(10):
        assert lib.tc_strerror(code)
    assert lib.tc_strerror(0) == b"ok"


def test_workspace_size_arithmetic(lib):
    s0 = lib.tc_workspace_size(0, 0, 0)
    assert s0 > 0
    s1 = lib.tc_workspace_size(1000, 10000, 0)
    s2 = lib.tc_workspace_size(1000, 20000, 0)
    assert s2 > s1 > s0
    # about 16 B of sort buffers + 16 B of lists per edge, plus per-vertex arrays
    assert 40 * 10000 < s1 < 200 * 10000 + 200 * 1000
    assert lib.tc_workspace_size(-1, 0, 0) == 0
    assert lib.tc_workspace_size(10, -1, 0) == 0
    assert lib.tc_workspace_size(1 << 31, 0, 0) == 0
    assert lib.tc_workspace_size(10, 1 << 32, 0) == 0
    assert lib.tc_workspace_size(10, 10, 4) == 0
    both = lib.tc_workspace_size(1000, 20000, 1)
    assert both > 0


def test_host_validation_before_launch(lib):
    """Every rejected call returns before touching the device (works without a GPU)."""
    from paper_1503_00576_amd import api
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: the checks fail first
    ws = ctypes.c_void_p(0x10000)
    big = 1 << 40
    out = ctypes.c_void_p(0x2000)
    # negative sizes, bad flags
    assert lib.tc_count(fake, -1, 3, 0, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(fake, 5, -3, 0, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(fake, 5, 3, 8, ws, big, None, out, None) == api.E_ARG
    # too large
    assert lib.tc_count(fake, 1 << 31, 3, 0, ws, big, None, out, None) == api.E_TOO_LARGE
    assert lib.tc_count(fake, 5, 1 << 32, 0, ws, big, None, out, None) == api.E_TOO_LARGE
    # n = 0 with edges, null or misaligned edge pointer
    assert lib.tc_count(fake, 0, 3, 0, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(None, 5, 3, 0, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(ctypes.c_void_p(0x1004), 5, 3, 0, ws, big, None, out, None) == api.E_ARG
    # two-direction format with an odd number of entries
    assert lib.tc_count(fake, 5, 3, 1, ws, big, None, out, None) == api.E_ASYMMETRIC
    # workspace: null, misaligned, short
    need = lib.tc_workspace_size(5, 3, 0)
    assert lib.tc_count(fake, 5, 3, 0, None, big, None, out, None) == api.E_WORKSPACE
    assert lib.tc_count(fake, 5, 3, 0, ctypes.c_void_p(0x10010), big, None, out, None) == api.E_WORKSPACE
    assert lib.tc_count(fake, 5, 3, 0, ws, need - 1, None, out, None) == api.E_WORKSPACE
    # missing outputs
    assert lib.tc_count(fake, 5, 3, 0, ws, big, None, None, None) == api.E_ARG
    assert lib.tc_count_per_vertex(fake, 5, 3, 0, ws, big, None, out, None, None) == api.E_ARG
    assert lib.tc_count_prepared(5, 3, 0, ws, need - 1, None, out, None, None) == api.E_WORKSPACE
    assert lib.tc_count_prepared(5, 3, 0, ws, big, None, None, None, None) == api.E_ARG
    assert lib.tc_preprocess(fake, 5, 3, 2, ws, big, None, None) == api.E_ARG
    # sort
    assert lib.tc_sort_u64(fake, fake, 10, 0, ws, big, None) == api.E_ARG
    assert lib.tc_sort_u64(fake, fake, 10, 65, ws, big, None) == api.E_ARG
    assert lib.tc_sort_u64(fake, fake, 10, 8, ws, 0, None) == api.E_WORKSPACE
    lay = api._native.TcLayout()
    assert lib.tc_workspace_layout(-1, 0, 0, ctypes.byref(lay)) == api.E_ARG


def test_layout(lib):
    from paper_1503_00576_amd import api
    lay = api.layout(1000, 9000)
    assert lay.m_fwd == 9000 and lay.id_bits == 10
    assert len({lay.deg, lay.perm, lay.rank, lay.row_ptr, lay.col}) == 5
    assert all(x % 256 == 0 for x in (lay.deg, lay.perm, lay.rank, lay.row_ptr, lay.col))
    assert max(lay.deg, lay.perm, lay.rank, lay.row_ptr, lay.col) < lib.tc_workspace_size(1000, 9000, 0)
    assert api.layout(1000, 9000, both=True).m_fwd == 4500
    assert api.layout(1 << 23, 10).id_bits == 23
    assert api.layout((1 << 23) + 1, 10).id_bits == 24


def test_clustering_transitivity_helpers():
    import numpy as np
    from paper_1503_00576_amd import api
    # K4: every vertex in 3 triangles, degree 3 -> C = 1; transitivity 1
    c = api.clustering(np.array([3, 3, 3, 3]), np.array([3, 3, 3, 3]))
    assert np.allclose(c, 1.0)
    assert api.transitivity(4, np.array([3, 3, 3, 3])) == 1.0
    # star: no triangles; leaves degree 1 -> 0
    assert np.allclose(api.clustering(np.zeros(4), np.array([3, 1, 1, 1])), 0.0)
    assert api.transitivity(0, np.array([3, 1, 1, 1])) == 0.0
    assert api.transitivity(0, np.array([1, 1])) == 0.0
