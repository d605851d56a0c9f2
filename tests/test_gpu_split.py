"""GPU parity of the split path for graphs beyond device memory (tc_split_prepare on the host,
tc_split_count on the device) against the oracle: totals and per-vertex counts, with the
copies overlapped on a second stream and without, both input formats, the number of parts
picked from a device budget, repeated-edge reports, and R-MAT scale 20 against the oracle's
stored total and per-vertex digest."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1503_00576_amd import api, synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
DEV = "cuda:0"


def _check(e, n, K, both=False, overlap=True, options=None):
    print(f"split: n={n} m={len(e)} K={K} both={both} overlap={overlap}", flush=True)
    sp = api.Split(e, n, both=both, parts=K, device_budget=0, options=options)
    want_t, want_pv = oracle.count(e, n, both=both, per_vertex=True)
    assert sp.count(DEV, overlap=overlap) == want_t
    t, pv = sp.count_per_vertex(DEV, overlap=overlap)
    assert t == want_t
    assert np.array_equal(pv.cpu().numpy().astype(np.uint64), want_pv)
    return sp


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_split_rmat_vs_oracle(K):
    e, n = synth.rmat_graph(13, 16, seed=4)
    _check(e.numpy(), n, K)


@pytest.mark.parametrize("overlap", [False, True])
def test_split_copy_stream(overlap):
    e, n = synth.rmat_graph(14, 16, seed=9)
    _check(e.numpy(), n, 4, overlap=overlap)


def test_split_small_graphs():
    e, n = synth.er_1000()
    _check(e.numpy(), n, 3)
    tri = np.array([[0, 1], [1, 2], [0, 2]], dtype=np.int32)
    for K in (1, 3, 64):
        _check(tri, 3, K)
    sp = api.Split(np.zeros((0, 2), dtype=np.int32), 5, parts=3, device_budget=0)
    t, pv = sp.count_per_vertex(DEV)
    assert t == 0 and pv.cpu().tolist() == [0] * 5


@pytest.mark.parametrize("K", [1, 4])
def test_split_two_direction(K):
    e, n = synth.rmat_graph(12, 16, seed=6)
    e = e.numpy()
    both = np.concatenate([e, e[:, ::-1]])
    both = np.ascontiguousarray(both[np.random.default_rng(2).permutation(len(both))])
    sp = _check(both, n, K, both=True)
    assert sp.info["m_kept"] == len(e)


def test_split_with_options():
    """Subgraphs counted through every workgroup form and without panels."""
    e, n = synth.rmat_graph(13, 16, seed=8)
    _check(e.numpy(), n, 3, options={"panel_ranks": 0, "wave_bitmap_span": 0,
                                      "wave_list_max": 0, "block_bitmap_span": 0})


def test_split_budget():
    e, n = synth.rmat_graph(15, 16, seed=3)
    e = e.numpy()
    full = api.Split(e, n, parts=1, device_budget=0).info["device_bytes"]
    sp = api.Split(e, n, parts=0, device_budget=full // 4)
    assert sp.info["parts"] >= 3 and sp.info["device_bytes"] <= full // 4
    ws = torch.empty(sp.info["device_bytes"], dtype=torch.uint8, device=DEV)
    r = sp.count_async(DEV, per_vertex=True, workspace=ws).check()
    want_t, want_pv = oracle.count(e, n, per_vertex=True)
    assert int(r.total.item()) == want_t
    assert np.array_equal(r.per_vertex.cpu().numpy().astype(np.uint64), want_pv)
    # a workspace one byte short is refused before anything is enqueued
    with pytest.raises(api.TCError) as ex:
        sp.count_async(DEV, workspace=ws[: sp.info["device_bytes"] - 256])
    assert ex.value.code == api.E_WORKSPACE


def test_split_duplicate_edge_reported():
    e, n = synth.rmat_graph(11, 8, seed=1)
    e = e.numpy()
    dup = np.ascontiguousarray(np.concatenate([e, e[5:6, ::-1]]))
    for K in (1, 3):
        r = api.Split(dup, n, parts=K, device_budget=0).count_async(DEV)
        torch.cuda.synchronize()
        assert int(r.status.item()) == api.E_DUP_EDGE, K


def test_split_rmat20_golden():
    """R-MAT scale 20 in 6 parts: total and the whole per-vertex array against the oracle's
    stored values."""
    with open(os.path.join(HERE, "golden", "workloads.json")) as f:
        g = json.load(f)["rmat_s20_ef16_s0"]
    e, n = synth.rmat_graph(20, 16, seed=0)
    assert synth.edges_sha256(e) == g["sha256"]
    sp = api.Split(e.numpy(), n, parts=6, device_budget=0)
    assert sp.info["max_sub_m"] < len(e) // 3
    t, pv = sp.count_per_vertex(DEV)
    assert t == g["total"]
    pvh = np.ascontiguousarray(pv.cpu().numpy(), dtype="<u8")
    assert hashlib.sha256(pvh.tobytes()).hexdigest() == g["per_vertex_sha256"]
