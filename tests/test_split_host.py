"""Host half of the split path for graphs beyond device memory (tc_split_prepare): the
partition, the block bucketing, the pre-filter of two-direction input (Section 3.4) and the
inclusion-exclusion over subgraphs, checked on the CPU.  Every subgraph that the device would
count is taken out of the host workspace exactly as tc_split_count uploads it and counted by
the oracle; the signed sum must equal the oracle's count of the whole graph, in total and
vertex by vertex."""
import numpy as np
import pytest

import oracle
from paper_1503_00576_amd import api, synth


def _graphs():
    e, n = synth.er_1000()
    yield "G(1000,0.02)", e.numpy(), n
    e, n = synth.rmat_graph(10, 16, seed=3)
    yield "R-MAT(10,16)", e.numpy(), n
    # isolated vertices above every id in use, and a dense corner
    e = synth.erdos_renyi(60, 0.5, seed=11).numpy()
    yield "G(60,0.5)+isolated", e, 200


GRAPHS = list(_graphs())


def _combine(sp, n):
    total = 0
    pv = np.zeros(n, dtype=np.int64)
    for i in range(sp.info["subgraphs"]):
        d, e, v = sp.subgraph(i)
        assert e.shape == (d["m"], 2) and v.shape == (d["n"],)
        if d["m"]:
            assert e.min() >= 0 and e.max() < d["n"]
        t, p = oracle.count(e, d["n"], per_vertex=True)
        total += d["coef"] * t
        np.add.at(pv, v, d["coef"] * p.astype(np.int64))
    return total, pv


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_subgraphs_sum_to_the_count(gi, K):
    name, e, n = GRAPHS[gi]
    sp = api.Split(e, n, parts=K, device_budget=0, pin=False)
    assert sp.info["parts"] == K
    want_t, want_pv = oracle.count(e, n, per_vertex=True)
    t, pv = _combine(sp, n)
    assert t == want_t, (name, K)
    assert np.array_equal(pv, want_pv.astype(np.int64)), (name, K)
    # subgraph count: C(K,3) + C(K,2) + K (minus empty ones); K = 2 has no one-part terms
    full = K * (K - 1) * (K - 2) // 6 + K * (K - 1) // 2 + (K if K != 2 else 0)
    assert sp.info["subgraphs"] <= (1 if K == 1 else full)


@pytest.mark.parametrize("K", [1, 3, 6])
def test_blocks_hold_every_edge_once(K):
    """The blocks partition the edge set: the one-part and two-part subgraphs of every pair of
    parts, mapped back to global ids, cover each undirected edge exactly once when each block
    is taken once."""
    e, n = synth.rmat_graph(9, 8, seed=5)
    e = e.numpy()
    sp = api.Split(e, n, parts=K, device_budget=0, pin=False)
    seen = {}
    for i in range(sp.info["subgraphs"]):
        d, el, v = sp.subgraph(i)
        if len(d["parts"]) == 1 or K == 1:
            g = v[el]
            for a, b in g:
                key = (min(a, b), max(a, b))
                seen[key] = seen.get(key, 0) + 1
    # edges within a part (blocks E_aa) appear in their one-part subgraph
    parts_of = {}
    for i in range(sp.info["subgraphs"]):
        d, el, v = sp.subgraph(i)
        if len(d["parts"]) == 1:
            for x in v:
                parts_of[int(x)] = d["parts"][0]
    canon = {(min(a, b), max(a, b)) for a, b in e}
    if K == 1:
        assert set(seen) == canon and all(c == 1 for c in seen.values())
    else:
        inner = {k for k in canon if k[0] in parts_of and k[1] in parts_of
                 and parts_of[k[0]] == parts_of[k[1]]}
        assert set(seen) == inner and all(c == 1 for c in seen.values())


def test_local_ids_follow_the_parts():
    e, n = synth.rmat_graph(10, 8, seed=2)
    sp = api.Split(e.numpy(), n, parts=4, device_budget=0, pin=False)
    for i in range(sp.info["subgraphs"]):
        d, el, v = sp.subgraph(i)
        # every global vertex at most once, parts' vertices in id order within each part
        assert len(np.unique(v)) == len(v)
    # one-part subgraphs together hold every vertex that has an edge inside its part
    allv = np.concatenate([sp.subgraph(i)[2] for i in range(sp.info["subgraphs"])
                           if len(sp.subgraph(i)[0]["parts"]) == 1])
    assert len(np.unique(allv)) == len(allv)


@pytest.mark.parametrize("K", [1, 3, 4])
def test_two_direction_prefilter(K):
    """Section 3.4: the host keeps only the forward entries of the paper's two-direction
    format; the kept half counts the same triangles."""
    e, n = synth.rmat_graph(10, 8, seed=7)
    e = e.numpy()
    both = np.concatenate([e, e[:, ::-1]], axis=0)
    rng = np.random.default_rng(1)
    both = np.ascontiguousarray(both[rng.permutation(len(both))])
    sp = api.Split(both, n, both=True, parts=K, device_budget=0, pin=False)
    assert sp.info["m_kept"] == len(e)
    want_t, want_pv = oracle.count(e, n, per_vertex=True)
    t, pv = _combine(sp, n)
    assert t == want_t and np.array_equal(pv, want_pv.astype(np.int64))


def test_host_errors():
    e = np.array([[0, 1], [1, 2], [2, 0]], dtype=np.int32)
    with pytest.raises(api.TCError) as ex:
        api.Split(np.array([[0, 1], [1, 5]], dtype=np.int32), 3, parts=1, device_budget=0,
                  pin=False)
    assert ex.value.code == api.E_RANGE
    with pytest.raises(api.TCError) as ex:
        api.Split(np.array([[0, 1], [2, 2]], dtype=np.int32), 3, parts=1, device_budget=0,
                  pin=False)
    assert ex.value.code == api.E_SELF_LOOP
    with pytest.raises(api.TCError) as ex:
        api.Split(np.array([[0, 1], [-1, 2]], dtype=np.int32), 3, parts=3, device_budget=0,
                  pin=False)
    assert ex.value.code == api.E_RANGE
    # two-direction input with a missing mirror entry
    both = np.concatenate([e, e[:, ::-1]])[:-1]
    with pytest.raises(api.TCError) as ex:
        api.Split(np.ascontiguousarray(both), 3, both=True, parts=1, device_budget=0, pin=False)
    assert ex.value.code == api.E_ASYMMETRIC
    both = np.concatenate([e, e[:, ::-1]])
    both[-1] = [1, 0]  # even count, but (0, 2) has no mirror and (1, 0) is doubled
    with pytest.raises(api.TCError) as ex:
        api.Split(np.ascontiguousarray(both), 3, both=True, parts=1, device_budget=0, pin=False)
    assert ex.value.code == api.E_ASYMMETRIC
    with pytest.raises(api.TCError) as ex:
        api.Split(e, 3, parts=65, device_budget=0, pin=False)
    assert ex.value.code == api.E_ARG


def test_budget_picks_the_smallest_fitting_parts():
    e, n = synth.rmat_graph(12, 16, seed=1)
    e = e.numpy()
    one = api.Split(e, n, parts=1, device_budget=0, pin=False).info
    assert one["subgraphs"] == 1 and one["max_sub_m"] == len(e)
    prev_k = 1
    for frac in (1.0, 0.6, 0.35, 0.2):
        budget = int(one["device_bytes"] * frac)
        info = api.Split(e, n, parts=0, device_budget=budget, pin=False).info
        assert info["device_bytes"] <= budget
        assert info["parts"] != 2 and info["parts"] >= prev_k
        prev_k = info["parts"]
        if frac == 1.0:
            assert info["parts"] == 1
        # the chosen K is the smallest fitting one: every smaller K (but 2) needs more
        for k in range(1, info["parts"]):
            if k != 2:
                assert api.Split(e, n, parts=k, device_budget=0,
                                 pin=False).info["device_bytes"] > budget
    assert prev_k > 3
    with pytest.raises(api.TCError) as ex:
        api.Split(e, n, parts=0, device_budget=1 << 16, pin=False)
    assert ex.value.code == api.E_TOO_LARGE


def test_empty_and_edge_cases():
    sp = api.Split(np.zeros((0, 2), dtype=np.int32), 0, parts=0, device_budget=1 << 30,
                   pin=False)
    assert sp.info["subgraphs"] == 0
    sp = api.Split(np.zeros((0, 2), dtype=np.int32), 10, parts=3, device_budget=0, pin=False)
    assert sp.info["subgraphs"] == 0
    # a single triangle split over many parts
    e = np.array([[0, 1], [1, 2], [0, 2]], dtype=np.int32)
    for K in (1, 2, 3, 7, 64):
        sp = api.Split(e, 3, parts=K, device_budget=0, pin=False)
        t, pv = _combine(sp, 3)
        assert t == 1 and list(pv) == [1, 1, 1], K
