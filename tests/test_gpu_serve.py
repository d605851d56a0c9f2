"""Serving loop on the GPU: every result equals the oracle's and is the same alone and in a
mix of concurrent requests (exact integers, tolerance 0), with memory-budget queueing,
batching of small graphs, overlapping large graphs and resident-CSR reuse."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1503_00576_amd import api, serve, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make_requests():
    reqs = []
    rng = np.random.default_rng(3)
    for i in range(60):
        s = int(rng.choice([8, 9, 10, 11, 12]))
        e, n = synth.rmat_graph(s, 16, seed=100 + i)
        reqs.append((e.pin_memory(), n, None))
    for i in range(6):
        # a key names one graph: requests 3..5 repeat 0..2 and are served from resident CSRs
        e, n = synth.rmat_graph(15, 16, seed=200 + i % 3)
        reqs.append((e.pin_memory(), n, ("big", i % 3)))
    e, n = synth.er_1000()
    reqs.append((e.pin_memory(), n, None))
    return reqs


def test_alone_equals_mix_equals_oracle():
    reqs = make_requests()
    want = [oracle.count(e, n) for e, n, _ in reqs]
    # alone: one request at a time
    alone = []
    with serve.Server(DEV, max_inflight=1) as srv:
        for e, n, key in reqs:
            alone.append(srv.submit(serve.Request(e, n, key)).result(timeout=120)[0])
        hits = srv.stats["resident_hits"]
    assert alone == want
    assert hits == 3
    # mix: everything at once, budget small enough that requests queue, small ones batched,
    # large ones overlapping on several streams, repeated keys served from resident CSRs
    budget = 2 * api.workspace_size(1 << 15, 600000) + (64 << 20)
    with serve.Server(DEV, budget_bytes=budget, streams=4, small_edges=1 << 16,
                      batch_graphs=16, max_inflight=6, resident_bytes=budget // 2) as srv:
        futs = [srv.submit(serve.Request(e, n, key)) for e, n, key in reqs]
        mix = [f.result(timeout=300)[0] for f in futs]
        stats = dict(srv.stats)
    assert mix == want
    assert stats.get("batches", 0) >= 2
    assert stats.get("completed", 0) == len(reqs)


def test_request_larger_than_budget_is_rejected():
    e, n = synth.rmat_graph(12, 16, seed=1)
    with serve.Server(DEV, budget_bytes=4096, small_edges=0) as srv:
        f = srv.submit(serve.Request(e, n))
        with pytest.raises(MemoryError):
            f.result(timeout=60)
        assert srv.stats["rejected"] == 1


def test_bad_request_reports_error():
    bad = torch.tensor([(0, 1), (1, 1)], dtype=torch.int32)
    good, n = synth.er_1000()
    with serve.Server(DEV, small_edges=1 << 20) as srv:
        fb = srv.submit(serve.Request(bad, 4))
        fg = srv.submit(serve.Request(good, n))
        with pytest.raises(api.TCError):
            fb.result(timeout=60)
        assert fg.result(timeout=60)[0] == oracle.count(good, n)


def test_resident_key_concurrent_and_reused():
    """The same resident key submitted many times with several requests in flight (counts
    on one workspace run in stream order), and a key reused for another graph (counted from
    scratch, then resident in its place): every result equals the oracle's."""
    g1, n1 = synth.rmat_graph(14, 16, seed=301)
    g2, n2 = synth.rmat_graph(14, 16, seed=302)
    w1, w2 = oracle.count(g1, n1), oracle.count(g2, n2)
    g1, g2 = g1.pin_memory(), g2.pin_memory()
    with serve.Server(DEV, small_edges=1 << 10, max_inflight=6, streams=3) as srv:
        assert srv.submit(serve.Request(g1, n1, "k")).result(timeout=120)[0] == w1
        futs = [srv.submit(serve.Request(g1, n1, "k")) for _ in range(12)]
        other, _ = synth.rmat_graph(10, 16, seed=5)
        futs += [srv.submit(serve.Request(other.pin_memory(), 1 << 10)) for _ in range(4)]
        assert [f.result(timeout=120)[0] for f in futs[:12]] == [w1] * 12
        for f in futs[12:]:
            f.result(timeout=120)
        assert srv.stats["resident_hits"] >= 12
        # the key now names another graph
        assert srv.submit(serve.Request(g2, n2, "k")).result(timeout=120)[0] == w2
        futs = [srv.submit(serve.Request(g2, n2, "k")) for _ in range(6)]
        assert [f.result(timeout=120)[0] for f in futs] == [w2] * 6
        # and back
        assert srv.submit(serve.Request(g1, n1, "k")).result(timeout=120)[0] == w1


def test_bad_ids_in_a_batch_fail_only_their_request():
    """Small requests packed together: one with an id outside [0, n) (first, middle and last
    position of the batch) fails alone; the others' counts are exact."""
    goods = [synth.rmat_graph(9, 8, seed=400 + i) for i in range(7)]
    want = [oracle.count(e, n) for e, n in goods]
    for pos in (0, 3, 7):
        bad = torch.tensor([[0, 1], [1, 9]], dtype=torch.int32)
        reqs = [serve.Request(e.pin_memory(), n) for e, n in goods]
        reqs.insert(pos, serve.Request(bad.pin_memory(), 4))
        with serve.Server(DEV, small_edges=1 << 20, batch_graphs=64, max_inflight=2) as srv:
            futs = [srv.submit(r) for r in reqs]
            with pytest.raises(api.TCError) as ei:
                futs[pos].result(timeout=120)
            assert ei.value.name == "range"
            got = [f.result(timeout=120)[0] for i, f in enumerate(futs) if i != pos]
        assert got == want


def test_serving_workload_pool():
    """The serving workload's request mix at its own sizes: every graph of the request pool
    (R-MAT scales 10-14, 17-19 and 21, edgefactor 16) submitted at once, in the trace's
    order of scales, plus a slice of the Poisson trace; every count equals the oracle's
    stored one."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "serve_pool.json")) as f:
        ref = json.load(f)
    pool = {}
    for sc, k in synth.SERVE_POOL.items():
        pool[sc] = []
        for i in range(k):
            e, n = synth.serve_pool_graph(sc, i, device=DEV)
            assert synth.edges_sha256(e) == ref[str(sc)][i]["sha256"]
            pool[sc].append((e.cpu().pin_memory(), n))
    _, u = synth.poisson_trace(200.0, 2.0, 0)
    picks = [(sc, i) for sc, k in synth.SERVE_POOL.items() for i in range(k)]
    picks += [synth.serve_pick(j, x) for j, x in enumerate(u.tolist())]
    with serve.Server(DEV, budget_bytes=32 << 30, streams=4, small_edges=1 << 18,
                      batch_graphs=512, max_inflight=8) as srv:
        futs = [srv.submit(serve.Request(*pool[sc][i])) for sc, i in picks]
        got = [f.result(timeout=240)[0] for f in futs]
        stats = dict(srv.stats)
    assert got == [ref[str(sc)][i]["total"] for sc, i in picks]
    assert stats.get("batches", 0) >= 1 and stats.get("single", 0) >= 1
