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
    s0 = lib.tc_workspace_size(0, 0, 0, None)
    assert s0 > 0
    s1 = lib.tc_workspace_size(1000, 10000, 0, None)
    s2 = lib.tc_workspace_size(1000, 20000, 0, None)
    assert s2 > s1 > s0
    # about 16 B of sort buffers + 16 B of lists per edge, plus per-vertex arrays
    assert 40 * 10000 < s1 < 200 * 10000 + 200 * 1000
    assert lib.tc_workspace_size(-1, 0, 0, None) == 0
    assert lib.tc_workspace_size(10, -1, 0, None) == 0
    assert lib.tc_workspace_size(1 << 31, 0, 0, None) == 0
    assert lib.tc_workspace_size(10, 1 << 32, 0, None) == 0
    assert lib.tc_workspace_size(10, 10, 4, None) == 0
    both = lib.tc_workspace_size(1000, 20000, 1, None)
    assert both > 0


def test_host_validation_before_launch(lib):
    """Every rejected call returns before touching the device (works without a GPU)."""
    from paper_1503_00576_amd import api
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: the checks fail first
    ws = ctypes.c_void_p(0x10000)
    big = 1 << 40
    out = ctypes.c_void_p(0x2000)
    # negative sizes, bad flags
    assert lib.tc_count(fake, -1, 3, 0, None, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(fake, 5, -3, 0, None, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(fake, 5, 3, 8, None, ws, big, None, out, None) == api.E_ARG
    # too large
    assert lib.tc_count(fake, 1 << 31, 3, 0, None, ws, big, None, out, None) == api.E_TOO_LARGE
    assert lib.tc_count(fake, 5, 1 << 32, 0, None, ws, big, None, out, None) == api.E_TOO_LARGE
    # n = 0 with edges, null or misaligned edge pointer
    assert lib.tc_count(fake, 0, 3, 0, None, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(None, 5, 3, 0, None, ws, big, None, out, None) == api.E_ARG
    assert lib.tc_count(ctypes.c_void_p(0x1004), 5, 3, 0, None, ws, big, None, out, None) == api.E_ARG
    # two-direction format with an odd number of entries
    assert lib.tc_count(fake, 5, 3, 1, None, ws, big, None, out, None) == api.E_ASYMMETRIC
    # workspace: null, misaligned, short
    need = lib.tc_workspace_size(5, 3, 0, None)
    assert lib.tc_count(fake, 5, 3, 0, None, None, big, None, out, None) == api.E_WORKSPACE
    assert lib.tc_count(fake, 5, 3, 0, None, ctypes.c_void_p(0x10010), big, None, out, None) == api.E_WORKSPACE
    assert lib.tc_count(fake, 5, 3, 0, None, ws, need - 1, None, out, None) == api.E_WORKSPACE
    # missing outputs
    assert lib.tc_count(fake, 5, 3, 0, None, ws, big, None, None, None) == api.E_ARG
    assert lib.tc_count_per_vertex(fake, 5, 3, 0, None, ws, big, None, out, None, None) == api.E_ARG
    assert lib.tc_count_prepared(5, 3, 0, None, ws, need - 1, None, out, None, None) == api.E_WORKSPACE
    assert lib.tc_count_prepared(5, 3, 0, None, ws, big, None, None, None, None) == api.E_ARG
    assert lib.tc_preprocess(fake, 5, 3, 2, None, ws, big, None, None) == api.E_ARG
    # sort
    assert lib.tc_sort_u64(fake, fake, 10, 0, ws, big, None) == api.E_ARG
    assert lib.tc_sort_u64(fake, fake, 10, 65, ws, big, None) == api.E_ARG
    assert lib.tc_sort_u64(fake, fake, 10, 8, ws, 0, None) == api.E_WORKSPACE
    lay = api._native.TcLayout()
    assert lib.tc_workspace_layout(-1, 0, 0, None, ctypes.byref(lay)) == api.E_ARG


def test_layout(lib):
    from paper_1503_00576_amd import api
    lay = api.layout(1000, 9000)
    assert lay.m_fwd == 9000 and lay.id_bits == 10
    assert len({lay.deg, lay.perm, lay.rank, lay.row_ptr, lay.col}) == 5
    assert all(x % 256 == 0 for x in (lay.deg, lay.perm, lay.rank, lay.row_ptr, lay.col))
    assert max(lay.deg, lay.perm, lay.rank, lay.row_ptr, lay.col) < lib.tc_workspace_size(1000, 9000, 0, None)
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


@pytest.mark.parametrize("graph", ["er_1000", "rmat10", "ba", "ws"])
def test_clustering_transitivity_vs_networkx(graph):
    """The derived quantities from exact per-vertex counts (here the oracle's, on the host)
    against networkx's own clustering and transitivity of the same graph."""
    import networkx as nx
    import numpy as np

    import oracle
    from paper_1503_00576_amd import api, synth
    if graph == "er_1000":
        e, n = synth.er_1000()
    elif graph == "rmat10":
        e, n = synth.rmat_graph(10, 8, seed=2)
    elif graph == "ba":
        e, n = synth.barabasi_albert(800, 5, 3), 800
    else:
        e, n = synth.watts_strogatz(700, 4, 0.1, 5), 700
    e = e.numpy()
    total, pv = oracle.count(e, n, per_vertex=True)
    deg = oracle.degrees(e, n)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(map(tuple, e.tolist()))
    c = api.clustering(pv, deg)
    want = nx.clustering(G)
    assert np.allclose(c, [want[v] for v in range(n)], rtol=1e-12, atol=0)
    assert abs(float(np.mean(c)) - nx.average_clustering(G)) < 1e-12
    assert abs(api.transitivity(total, deg) - nx.transitivity(G)) < 1e-12


def test_options(lib):
    """struct tc_options: defaults, validation of every field, and the fields that change the
    workspace layout (host arithmetic only)."""
    from paper_1503_00576_amd import _native, api
    d = api.default_options()
    assert d == {"panel_ranks": 32736, "hub_ranks": 0, "row_blocks": 1, "wave_item_edges": 512,
                 "block_item_edges": 65536, "wave_bitmap_span": 65504, "wave_list_max": 2048,
                 "block_bitmap_span": 1048544, "block_list_max": 32768, "degree_partition": 1,
                 "sort_onesweep": 0, "high_ranks": 65536, "row_sort": 1}
    assert lib.tc_options_init(None) == api.E_ARG
    base = api.workspace_size(1000, 9000)
    assert api.workspace_size(1000, 9000, options=d) == base
    fake = ctypes.c_void_p(0x1000)
    ws, out = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x2000)
    bad = [("panel_ranks", 32737), ("hub_ranks", 65537), ("row_blocks", 0), ("row_blocks", 9),
           ("wave_item_edges", 15), ("wave_item_edges", 65537), ("block_item_edges", 15),
           ("block_item_edges", (1 << 20) + 1), ("wave_bitmap_span", 65505),
           ("wave_list_max", 2049), ("block_bitmap_span", 1048545), ("block_list_max", 32769),
           ("degree_partition", 2), ("sort_onesweep", 2), ("high_ranks", 65537),
           ("row_sort", 2)]
    for k, v in bad:
        assert lib.tc_workspace_size(1000, 9000, 0, api._opts({k: v})) == 0, k
        assert lib.tc_count(fake, 5, 3, 0, api._opts({k: v}), ws, 1 << 40, None, out,
                            None) == api.E_ARG, k
        assert lib.tc_count_prepared(5, 3, 0, api._opts({k: v}), ws, 1 << 40, None, out, None,
                                     None) == api.E_ARG, k
    o = _native.TcOptions()
    assert lib.tc_options_init(ctypes.byref(o)) == api.OK
    o.size = 4
    assert lib.tc_workspace_size(1000, 9000, 0, ctypes.byref(o)) == 0
    # every extreme that is valid is accepted
    for k, v in [("panel_ranks", 0), ("hub_ranks", 65536), ("row_blocks", 8),
                 ("wave_item_edges", 16), ("block_item_edges", 1 << 20),
                 ("wave_bitmap_span", 0), ("wave_list_max", 0), ("block_bitmap_span", 0),
                 ("block_list_max", 0), ("degree_partition", 0), ("sort_onesweep", 1),
                 ("high_ranks", 0), ("row_sort", 0)]:
        assert api.workspace_size(1000, 9000, options={k: v}) > 0, k
    # the layout grows with hubs (two byte matrices), row blocks (lists per block) and smaller
    # items (more item slots)
    assert api.workspace_size(1000, 9000, options={"hub_ranks": 128}) >= base + 2 * 128 * 128 - 512
    assert api.workspace_size(1000, 9000, options={"row_blocks": 4}) > base
    assert api.workspace_size(1000, 9000, options={"wave_item_edges": 16}) > base
    with pytest.raises(KeyError):
        api._opts({"bogus": 1})


def test_single_tuner_prefers_defaults_on_ties(lib):
    """The single-graph tuner keeps the library defaults when they time within its tie margin
    of the fastest candidate, and the fastest candidate otherwise (host logic)."""
    from paper_1503_00576_amd import api, autotune
    d = api.default_options()
    dflt = {k: d[k] for k in ("panel_ranks", "wave_item_edges", "block_item_edges")}
    other = dict(dflt, wave_item_edges=1024)
    slow = dict(dflt, panel_ranks=0)
    assert autotune._prefer_defaults([(slow, 40.0), (other, 32.0), (dflt, 32.05)]) == dflt
    assert autotune._prefer_defaults([(slow, 40.0), (other, 32.0), (dflt, 33.0)]) == other
    assert autotune._prefer_defaults([(slow, 40.0), (other, 32.0)]) == other


def ablation_header_functions():
    src = open(os.path.join(ROOT, "include", "tc_ablation.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tca_[a-z0-9_]+)\s*\(", src)))


def test_ablation_library_exports_and_validation():
    from paper_1503_00576_amd import ablation, api
    L = ablation.lib()
    names = ablation_header_functions()
    assert names == sorted(ablation.EXPORTS)
    for name in names:
        assert hasattr(L, name), name
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x2000)
    # bad shapes and flags are rejected before anything is enqueued
    assert L.tca_edge_merge(fake, fake, fake, fake, None, 10, 0, 96, 1, out, None) == api.E_ARG
    assert L.tca_edge_merge(fake, fake, fake, fake, None, 10, 16, 64, 1, out, None) == api.E_ARG
    assert L.tca_edge_merge(fake, fake, fake, fake, None, 10, 0, 64, 0, out, None) == api.E_ARG
    assert L.tca_edge_merge(fake, fake, fake, fake, None, 10, ablation.AOS, 64, 1, out,
                            None) == api.E_ARG
    assert L.tca_sort(3, 10, 8, fake, fake, fake, fake, fake, 1 << 20, None) == api.E_ARG
    assert L.tca_sort(0, 10, 33, fake, fake, fake, fake, fake, 1 << 20, None) == api.E_ARG
    assert L.tca_gather(fake, 1 << 20, 12, 10, 0, out, None) == api.E_ARG
    assert L.tca_gather(fake, 2, 4, 10, 0, out, None) == api.E_ARG
