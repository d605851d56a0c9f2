"""tc_count_noalloc (the entry point with its workspace in a static device array, for callers
that cannot allocate) through the C ABI, against tc_count with a caller workspace: two calls
in a row, the second on a smaller graph, data errors, and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1503_00576_amd import _native, api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LIMIT = 64 << 20


def noalloc(e, n, options=None):
    L = _native.lib()
    tot = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    code = L.tc_count_noalloc(api._ptr(e), n, int(e.shape[0]), 0, api._opts(options),
                              api._stream(torch.device(DEV)), api._ptr(tot), api._ptr(st))
    torch.cuda.synchronize()
    return code, int(tot.item()), int(st.item())


def with_workspace(e, n, options=None):
    L = _native.lib()
    ws = api.alloc_workspace(n, int(e.shape[0]), False, DEV, options)
    tot = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    st = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    code = L.tc_count(api._ptr(e), n, int(e.shape[0]), 0, api._opts(options), api._ptr(ws),
                      ws.numel(), api._stream(torch.device(DEV)), api._ptr(tot), api._ptr(st))
    torch.cuda.synchronize()
    return code, int(tot.item()), int(st.item())


def test_noalloc_equals_tc_count_two_calls():
    big = synth.rmat_graph(16, 14, seed=31, device=DEV)
    small = synth.er_1000(device=DEV)
    assert api.workspace_size(big[1], big[0].shape[0]) <= LIMIT
    assert small[0].shape[0] < big[0].shape[0]
    for e, n in [big, small, big]:
        want = oracle.count(e.cpu().numpy(), n)
        got = noalloc(e, n)
        assert got == with_workspace(e, n) == (api.OK, want, api.OK)


def test_noalloc_options_and_errors():
    e, n = synth.rmat_graph(13, 16, seed=32, device=DEV)
    want = oracle.count(e.cpu().numpy(), n)
    opt = {"panel_ranks": 100, "wave_item_edges": 64}
    assert noalloc(e, n, opt) == with_workspace(e, n, opt) == (api.OK, want, api.OK)
    bad = torch.tensor([(0, 1), (1, 2), (2, 2)], dtype=torch.int32, device=DEV)
    code, _, st = noalloc(bad, 5)
    assert code == api.OK and st == api.E_SELF_LOOP == with_workspace(bad, 5)[2]
    # the shared array keeps the failed call's contents; the next call starts clean
    assert noalloc(e, n) == (api.OK, want, api.OK)


def test_noalloc_rejects_graphs_beyond_the_scratch():
    n, m = 1 << 20, 4_000_000
    assert api.workspace_size(n, m) > LIMIT
    L = _native.lib()
    tot = torch.full((1,), 7, dtype=torch.int64, device=DEV)
    st = torch.full((1,), 7, dtype=torch.int32, device=DEV)
    # rejected on the host before anything is enqueued (the edge pointer is never read)
    code = L.tc_count_noalloc(ctypes.c_void_p(0x1000), n, m, 0, None,
                              api._stream(torch.device(DEV)), api._ptr(tot), api._ptr(st))
    torch.cuda.synchronize()
    assert code == api.E_SCRATCH
    assert int(tot.item()) == 7 and int(st.item()) == 7
    assert b"static scratch" in L.tc_strerror(api.E_SCRATCH)
