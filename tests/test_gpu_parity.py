"""GPU parity: the HIP path (through libtc.so's C ABI) against the CPU oracle, bit-exact.

Integer results, so the bar is equality: totals, per-vertex counts, the degree array, the
order, the oriented sorted lists, the sort.  Sizes span several tiles and ragged tails; the
full-size R-MAT case is checked against the oracle's stored total and sampled per-vertex
values computed one vertex at a time from the definition."""
import hashlib
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1503_00576_amd import api, synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
DEV = "cuda:0"


def golden():
    with open(os.path.join(HERE, "golden", "workloads.json")) as f:
        return json.load(f)


def gpu_counts(edges_np, n, both=False, per_vertex=True, options=None):
    e = torch.as_tensor(np.ascontiguousarray(np.asarray(edges_np, dtype=np.int32).reshape(-1, 2)),
                        device=DEV)
    if per_vertex:
        tot, pv = api.count_per_vertex(e, n, both, options=options)
        return tot, pv.cpu().numpy().astype(np.uint64)
    return api.count(e, n, both, options=options), None


def check_vs_oracle(edges_np, n, both=False, options=None, prepared_pv=False):
    """Totals and per-vertex counts of the one-shot calls (and, with prepared_pv, per-vertex
    counts of tc_preprocess + tc_count_prepared, which keep the panels) against the oracle."""
    e = np.asarray(edges_np, dtype=np.int32).reshape(-1, 2)
    ot, opv = oracle.count(e, n, both=both, per_vertex=True)
    gt, gpv = gpu_counts(e, n, both, options=options)
    assert gt == ot
    assert np.array_equal(gpv, opv)
    assert api.count(torch.as_tensor(e, device=DEV), n, both, options=options) == ot
    if prepared_pv:
        p = api.Prepared(torch.as_tensor(e, device=DEV), n, both, options=options)
        r = p.count_async(per_vertex=True).check()
        assert int(r.total.item()) == ot
        assert np.array_equal(r.per_vertex.cpu().numpy().astype(np.uint64), opv)
    return ot


def complete(k):
    return [(i, j) for i in range(k) for j in range(i + 1, k)]


# ------------------------------------------------------------------ small / closed forms

def test_closed_forms_and_named():
    for k in [0, 1, 2, 3, 4, 5, 17, 64, 65, 130]:
        assert check_vs_oracle(complete(k) or np.zeros((0, 2)), k) == math.comb(k, 3)
    for n in [5, 6, 100, 1000]:
        rim = list(range(1, n))
        e = [(0, r) for r in rim] + [(rim[i], rim[(i + 1) % len(rim)]) for i in range(len(rim))]
        assert check_vs_oracle(e, n) == n - 1
    e = [(a, b) for a in range(40) for b in range(40, 90)]
    assert check_vs_oracle(e, 90) == 0
    with open(os.path.join(HERE, "golden", "named_graphs.json")) as f:
        for name, g in json.load(f).items():
            assert check_vs_oracle(g["edges"], g["n"]) == g["total"], name


def test_empty_and_isolated():
    assert check_vs_oracle(np.zeros((0, 2)), 10) == 0
    assert check_vs_oracle([(3, 7)], 1000) == 0
    # n = 0, m = 0
    tot, _ = gpu_counts(np.zeros((0, 2)), 0, per_vertex=False)
    assert tot == 0


def test_random_small_graphs():
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(2, 300))
        p = float(rng.choice([0.01, 0.05, 0.2, 0.6]))
        iu = np.triu_indices(n, 1)
        keep = rng.random(iu[0].size) < p
        e = np.stack([iu[0][keep], iu[1][keep]], 1)
        e = e[rng.permutation(len(e))]
        flip = rng.random(len(e)) < 0.5
        e[flip] = e[flip][:, ::-1]
        check_vs_oracle(e, n)


def test_er_1000_golden():
    g = golden()["er_1000_p0.02_s0"]
    e, n = synth.er_1000(device=DEV)
    assert synth.edges_sha256(e) == g["sha256"]
    tot, pv = api.count_per_vertex(e, n)
    assert tot == g["total"]
    pv = pv.cpu().numpy()
    for v, want in g["per_vertex_sample"].items():
        assert pv[int(v)] == want
    check_vs_oracle(e.cpu().numpy(), n)


@pytest.mark.parametrize("scale,ef,seed", [(8, 8, 1), (10, 16, 2), (12, 16, 3), (14, 16, 4), (16, 16, 0)])
def test_rmat_vs_oracle(scale, ef, seed):
    e, n = synth.rmat_graph(scale, ef, seed=seed, device=DEV)
    check_vs_oracle(e.cpu().numpy(), n)


@pytest.mark.parametrize("kind,n,k", [(0, 5000, 8), (1, 5000, 8), (0, 20000, 16), (1, 20000, 2)])
def test_ba_ws_vs_oracle(kind, n, k):
    e = synth.batch_graph(kind, n, k, seed=11, device=DEV)
    check_vs_oracle(e.cpu().numpy(), n)


def test_two_direction_format():
    e, n = synth.rmat_graph(12, 16, seed=7)
    en = e.numpy()
    both = np.concatenate([en, en[:, ::-1]])[np.random.default_rng(1).permutation(2 * len(en))]
    t = check_vs_oracle(both, n, both=True)
    assert t == oracle.count(en, n)


def test_repeat_runs_identical():
    e, n = synth.rmat_graph(14, 16, seed=9, device=DEV)
    outs = [gpu_counts(e.cpu().numpy(), n) for _ in range(3)]
    for t, pv in outs[1:]:
        assert t == outs[0][0] and np.array_equal(pv, outs[0][1])


@pytest.mark.parametrize("blocks", [3, 8])
def test_row_blocks_forced(blocks):
    """In-edge lists split into row blocks (counted one block after another)."""
    opt = {"row_blocks": blocks}
    for e, n in [synth.rmat_graph(16, 16, seed=2, device=DEV), synth.er_1000(device=DEV),
                 synth.rmat_graph(12, 16, seed=3, device=DEV)]:
        check_vs_oracle(e.cpu().numpy(), n, options=opt, prepared_pv=True)


@pytest.mark.parametrize("n", [(1 << 24) - 3, (1 << 25) + 7])
def test_degree_partition_wide_ids(n):
    """The degree partition on id ranges whose 256 buckets hold 2^16 ids (endpoints kept as
    2-byte offsets, two LDS windows per bucket) and 2^17 ids (4-byte offsets, four windows):
    degrees and counts against the oracle on a sparse graph spread over the whole id range
    with a dense cluster at its top (its ids fall in the last, ragged bucket)."""
    rng = np.random.default_rng(n % 1000)
    a = rng.integers(0, n, 300_000)
    b = rng.integers(0, n, 300_000)
    top = n - 1 - np.arange(60)
    ci, cj = np.triu_indices(60, 1)
    e = np.concatenate([np.stack([a, b], 1), np.stack([top[ci], top[cj]], 1)])
    e = e[e[:, 0] != e[:, 1]]
    key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    _, first = np.unique(key, return_index=True)
    e = np.ascontiguousarray(e[np.sort(first)].astype(np.int32))
    out = api.preprocess(torch.as_tensor(e, device=DEV), n)
    assert np.array_equal(out["deg"].cpu().numpy().astype(np.int64), oracle.degrees(e, n))
    assert check_vs_oracle(e, n) >= math.comb(60, 3)


@pytest.mark.parametrize("both", [False, True])
def test_degree_atomic_path(both):
    """Degrees by one atomic per endpoint and orientation in input order (the path of graphs
    beyond the bucket partition's limits), both input formats, with an invalid input."""
    opt = {"degree_partition": 0}
    for e, n in [synth.er_1000(), synth.rmat_graph(14, 16, seed=5),
                 (synth.barabasi_albert(3000, 12, 2), 3000)]:
        e = e.numpy()
        if both:
            e = np.concatenate([e, e[:, ::-1]])
        check_vs_oracle(e, n, both=both, options=opt)
    for k in [3, 40, 130]:
        assert check_vs_oracle(complete(k), k, options=opt) == math.comb(k, 3)
    for edges, name in [([(0, 1), (1, 2), (2, 2)], "self_loop"), ([(0, 1), (1, 5)], "range"),
                        ([(0, 1), (1, 2), (1, 0)], "dup_edge")]:
        with pytest.raises(api.TCError) as ei:
            api.count(torch.tensor(edges, dtype=torch.int32, device=DEV), 5, options=opt)
        assert ei.value.name == name


@pytest.mark.parametrize("ranks", [0, 1, 31, 33, 517, 4000])
def test_panel_thresholds(ranks):
    """The top-ranks panel region of every size: off (per-vertex lists only), one partial
    panel, one panel plus a ragged one, and many panels over graphs of every family, for totals
    and for per-vertex counts (one-shot and on a prepared graph: the per-vertex panel kernel)."""
    opt = {"panel_ranks": ranks}
    for e, n in [synth.er_1000(), (synth.barabasi_albert(2000, 8, 2), 2000),
                 (synth.watts_strogatz(1500, 6, 0.1, 3), 1500), synth.rmat_graph(11, 8, seed=4),
                 synth.rmat_graph(14, 16, seed=6)]:
        check_vs_oracle(e.numpy(), n, options=opt, prepared_pv=True)
    for k in [3, 40, 130]:
        assert check_vs_oracle(complete(k), k, options=opt, prepared_pv=True) == math.comb(k, 3)


def test_wide_panels_per_vertex():
    """Per-vertex counts with more panel ranks than one window of the per-vertex panel kernel
    holds: the lower panels take their ranks in two windows (every segment streamed once per
    window), the upper ones in one; both on a prepared graph and in the one-shot call, with
    the suffixes read as 16-bit offsets and, without a 16-bit region, as 32-bit ranks."""
    e, n = synth.rmat_graph(15, 16, seed=12)
    assert n > 16384 + 64
    for ranks in (32736, 20000):
        check_vs_oracle(e.numpy(), n, options={"panel_ranks": ranks}, prepared_pv=True)
    check_vs_oracle(e.numpy(), n, options={"panel_ranks": 32736, "high_ranks": 0},
                    prepared_pv=True)


@pytest.mark.parametrize("row_sort", [1, 0])
def test_single_sweep_sort(row_sort):
    """The single-sweep radix variant (look-back instead of a histogram pass) in the sort of
    the oriented edges (by source, its passes before the unzipping one; by (source, target),
    all six) of graphs above its 2^20-key threshold, with ragged last tiles."""
    opt = {"sort_onesweep": 1, "row_sort": row_sort}
    for e, n in [synth.rmat_graph(17, 16, seed=21), synth.rmat_graph(18, 6, seed=22)]:
        assert e.shape[0] >= (1 << 20) and e.shape[0] % 4096
        check_vs_oracle(e.numpy(), n, options=opt)


def hub_fan(L, seed, dup=False):
    """L hubs (ids 2 .. L + 1) forming a clique, and vertices 0 and 1 joined to every hub:
    0 and 1 have degree L and the hubs L + 1, so in the order of Section 2.2 the oriented list
    of 0 (and of 1) holds all L hubs and hub i's list the hubs above it, lengths 0 .. L - 1.
    Edges in random order and orientation; dup repeats the edge (0, 2) (reversed), which puts
    a repeated entry in the list of 0, then of L + 1 entries."""
    hi, hj = np.triu_indices(L, 1)
    e = [np.stack([hi + 2, hj + 2], 1), np.stack([np.zeros(L, np.int64), np.arange(2, L + 2)], 1),
         np.stack([np.ones(L, np.int64), np.arange(2, L + 2)], 1)]
    if dup:
        e.append(np.array([[2, 0]]))
    e = np.concatenate(e)
    rng = np.random.default_rng(seed)
    flip = rng.random(len(e)) < 0.5
    e[flip] = e[flip][:, ::-1]
    return np.ascontiguousarray(e[rng.permutation(len(e))].astype(np.int32)), L + 2


@pytest.mark.parametrize("row_sort", [1, 0])
def test_row_sort_lengths(row_sort):
    """Oriented lists of every length class of the in-place row sort (per lane up to 16
    entries, per wave up to 1024 and up to 2048, per workgroup above), and the full sort of
    the oriented edges (row_sort 0), on hub fans checked against closed forms: C(L, 3) +
    2 C(L, 2) triangles, each hub in C(L - 1, 2) + 2 (L - 1), vertices 0 and 1 in C(L, 2).  A
    repeated edge in a list of each class is reported, and so is a list of more than 32768
    entries (possible only with repeated edges below 2^29 oriented edges)."""
    opt = {"row_sort": row_sort}
    for L in (10, 40, 100, 700, 1500, 2600):
        e, n = hub_fan(L, seed=L)
        tot, pv = gpu_counts(e, n, options=opt)
        want = np.full(n, math.comb(L - 1, 2) + 2 * (L - 1), dtype=np.uint64)
        want[:2] = math.comb(L, 2)
        assert tot == math.comb(L, 3) + 2 * math.comb(L, 2), L
        assert np.array_equal(pv, want), L
        e, n = hub_fan(L, seed=L + 1, dup=True)
        for pv_call in (api.count, api.count_per_vertex):
            with pytest.raises(api.TCError) as ei:
                pv_call(torch.as_tensor(e, device=DEV), n, options=opt)
            assert ei.value.name == "dup_edge", L
    e = torch.tensor([[0, 1]] * 33000, dtype=torch.int32, device=DEV)
    with pytest.raises(api.TCError) as ei:
        api.count(e, 2, options=opt)
    assert ei.value.name == "dup_edge"


@pytest.mark.parametrize("span", [0, 40, 600])
def test_wave_item_forms(span):
    """Wave items in both forms (bitmap below the span limit, sorted list above it) and
    workgroup items, reached on small graphs by lowering the limit, with panels off so that
    every list is a wave or workgroup item."""
    opt = {"panel_ranks": 0, "wave_bitmap_span": span}
    for e, n in [synth.er_1000(), (synth.barabasi_albert(3000, 12, 2), 3000),
                 synth.rmat_graph(12, 16, seed=8), (synth.erdos_renyi(1500, 0.9, 3), 1500)]:
        check_vs_oracle(e.numpy(), n, options=opt)
    for k in [3, 40, 130]:
        assert check_vs_oracle(complete(k), k, options=opt) == math.comb(k, 3)


# every form of every item, forced on small graphs through the options: wave items (bitmap,
# sorted LDS list), workgroup items (bitmap, sorted LDS list, sorted list in global memory),
# for totals, per-vertex counts and the per-vertex panel path, with items of 16 in-edges so
# that lists span many items
FORCED = {
    "wave_list": {"panel_ranks": 0, "wave_bitmap_span": 0, "wave_list_max": 40},
    "block_bitmap": {"panel_ranks": 0, "wave_bitmap_span": 0, "wave_list_max": 0},
    "block_lds_list": {"panel_ranks": 0, "wave_bitmap_span": 0, "wave_list_max": 0,
                       "block_bitmap_span": 0},
    "block_global_list": {"panel_ranks": 0, "wave_bitmap_span": 0, "wave_list_max": 0,
                          "block_bitmap_span": 0, "block_list_max": 0},
    "block_mixed": {"panel_ranks": 0, "wave_bitmap_span": 0, "wave_list_max": 10,
                    "block_bitmap_span": 100, "block_list_max": 30},
    "panels_global_pv": {"panel_ranks": 600, "block_list_max": 0},
    "small_items": {"panel_ranks": 300, "wave_item_edges": 16, "block_item_edges": 16,
                    "wave_list_max": 20, "block_list_max": 25},
}


@pytest.mark.parametrize("name", sorted(FORCED))
def test_forced_item_forms(name):
    opt = FORCED[name]
    for e, n in [synth.er_1000(), (synth.barabasi_albert(3000, 12, 2), 3000),
                 synth.rmat_graph(12, 16, seed=8), (synth.erdos_renyi(700, 0.9, 3), 700),
                 (synth.watts_strogatz(2500, 8, 0.1, 4), 2500)]:
        check_vs_oracle(e.numpy(), n, options=opt, prepared_pv=True)
    for k in [3, 40, 130]:
        assert check_vs_oracle(complete(k), k, options=opt, prepared_pv=True) == math.comb(k, 3)


@pytest.mark.parametrize("high", [0, 100])
@pytest.mark.parametrize("name", sorted(FORCED))
def test_forced_item_forms_high_region(name, high):
    """Every item form with the 16-bit region of the node array cut to the top `high` ranks
    (0: only the panel region), so that total counts stream suffixes that start in 32-bit
    entries and continue in 16-bit ones, or stay 32-bit throughout."""
    opt = dict(FORCED[name], high_ranks=high)
    for e, n in [synth.er_1000(), (synth.barabasi_albert(3000, 12, 2), 3000),
                 synth.rmat_graph(12, 16, seed=8), (synth.erdos_renyi(700, 0.9, 3), 700)]:
        check_vs_oracle(e.numpy(), n, options=opt)
    for k in [3, 40, 130]:
        assert check_vs_oracle(complete(k), k, options=opt) == math.comb(k, 3)


@pytest.mark.parametrize("high", [0, 1, 7, 33, 517, 4000])
def test_high_region_sizes(high):
    """16-bit region of every size against panel regions below, inside and above it: pieces
    whose 32-bit part ends mid-piece, one-entry 16-bit parts, and the region clamped to the
    panel region when that is larger."""
    for panels in (0, 64, 2000):
        opt = {"high_ranks": high, "panel_ranks": panels}
        for e, n in [synth.er_1000(), synth.rmat_graph(13, 16, seed=9),
                     (synth.barabasi_albert(2500, 10, 5), 2500)]:
            check_vs_oracle(e.numpy(), n, options=opt)


def test_prepared_options_mismatch():
    """tc_count_prepared with options (or sizes) other than the preprocessing's reports a
    mismatch on the device; the workspace stays usable with the right ones."""
    e, n = synth.rmat_graph(12, 16, seed=3, device=DEV)
    want = oracle.count(e.cpu().numpy(), n)
    # room for every layout below, so that only the device-side check can object
    ws = torch.empty(2 * api.workspace_size(n, e.shape[0]) + (1 << 20), dtype=torch.uint8,
                     device=DEV)
    p = api.Prepared(e, n, workspace=ws, options={"panel_ranks": 64})
    assert p.count() == want
    other = api.Prepared.__new__(api.Prepared)
    other.__dict__.update(p.__dict__)
    for opts in [None, {"panel_ranks": 32}, {"panel_ranks": 64, "wave_item_edges": 256}]:
        other.options = opts
        with pytest.raises(api.TCError) as ei:
            other.count()
        assert ei.value.name == "mismatch"
    other.options = {"panel_ranks": 64}
    other.m = p.m - 1
    with pytest.raises(api.TCError) as ei:
        other.count()
    assert ei.value.name == "mismatch"
    assert p.count() == want


@pytest.mark.parametrize("hubs", [0, 1, 63, 64, 100, 1000, 5000])
def test_hub_matrix_path(hubs):
    """Triangles among the top ranks counted as a masked int8 product on the matrix cores,
    the rest by the middle-vertex kernel, totals and per-vertex counts: no hubs, one hub, hub
    counts that are and are not multiples of the 64-wide tiles, and graphs that are all hubs."""
    opt = {"hub_ranks": hubs}
    for e, n in [synth.er_1000(), (synth.barabasi_albert(3000, 12, 2), 3000),
                 synth.rmat_graph(13, 16, seed=8), (synth.erdos_renyi(700, 0.5, 3), 700),
                 (synth.watts_strogatz(2500, 8, 0.1, 4), 2500)]:
        check_vs_oracle(e.numpy(), n, options=opt)
    for k in [3, 40, 130]:
        assert check_vs_oracle(complete(k), k, options=opt) == math.comb(k, 3)


def test_prepared_recount():
    """A resident preprocessed graph counted repeatedly, with and without per-vertex counts."""
    e, n = synth.rmat_graph(13, 16, seed=12, device=DEV)
    ot, opv = oracle.count(e.cpu().numpy(), n, per_vertex=True)
    p = api.Prepared(e, n)
    for _ in range(3):
        assert p.count() == ot
        r = p.count_async(per_vertex=True).check()
        assert int(r.total.item()) == ot
        assert np.array_equal(r.per_vertex.cpu().numpy().astype(np.uint64), opv)


# ------------------------------------------------------------------ intermediate stages

@pytest.mark.parametrize("row_sort", [1, 0])
def test_preprocess_stages(row_sort):
    """Degrees, the order, and the oriented CSR against the oracle, through both sorts of the
    oriented edges (by source, then each row in place; by (source, target)), which must give
    the same arrays, the per-entry source array included."""
    opt = {"row_sort": row_sort}
    for e, n in [synth.er_1000(), synth.rmat_graph(13, 16, seed=5),
                 (synth.watts_strogatz(5000, 6, 0.1, 2), 5000), synth.rmat_graph(16, 24, seed=9)]:
        en = e.numpy()
        out = api.preprocess(e.to(DEV), n, options=opt)
        other = api.preprocess(e.to(DEV), n, options={"row_sort": 1 - row_sort})
        for k in ("deg", "perm", "rank", "row_ptr", "col", "src"):
            assert torch.equal(out[k], other[k]), k
        rp_ = out["row_ptr"].cpu().numpy().astype(np.int64)
        src_ = out["src"].cpu().numpy().astype(np.int64)
        assert np.array_equal(src_, np.repeat(np.arange(n), np.diff(rp_)))
        deg = out["deg"].cpu().numpy().astype(np.int64)
        assert np.array_equal(deg, oracle.degrees(en, n))
        perm = out["perm"].cpu().numpy().astype(np.int64)
        rank = out["rank"].cpu().numpy().astype(np.int64)
        # the order of Section 2.2: ascending (degree, id)
        keyed = deg[perm] * n + perm
        assert np.all(np.diff(keyed) > 0)
        assert np.array_equal(rank[perm], np.arange(n))
        rp = out["row_ptr"].cpu().numpy().astype(np.int64)
        col = out["col"].cpu().numpy().astype(np.int64)
        orp, ocol = oracle.oriented_csr(en, n)
        assert rp[-1] == len(en) == col.size
        for r in range(n):
            row = col[rp[r]:rp[r + 1]]
            assert np.all(np.diff(row) > 0)
            assert np.all(row > r)
            v = perm[r]
            assert sorted(perm[row].tolist()) == ocol[orp[v]:orp[v + 1]].tolist()


@pytest.mark.parametrize("count,bits", [(1, 8), (100, 7), (4096, 64), (4097, 40), (8192, 64),
                                        (8193, 12), (24575, 3), (100003, 46), (1 << 20, 20),
                                        (3_000_001, 33)])
def test_radix_sort(count, bits):
    g = torch.Generator().manual_seed(count + bits)
    keys = torch.randint(-(1 << 62), 1 << 62, (count,), generator=g, dtype=torch.int64)
    if bits < 20:
        keys = keys & 0xFF  # many equal low bits: stability matters
    ref = keys.numpy().view(np.uint64)
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(ref & mask, kind="stable")
    want = ref[order]
    got = api.sort_u64(keys.to(DEV), bits).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("count,bits", [(8192 * 3 + 77, 24), (1 << 20, 40), (300_001, 64)])
def test_radix_sort_skewed(count, bits):
    """Heavily repeated digits (most keys share one value on the sorted bits, the rest spread
    over a few values), as hub ranks and the unlisted in-edges produce: the histogram counts
    runs of equal digits with one atomic, and the sort must stay stable."""
    g = torch.Generator().manual_seed(count ^ bits)
    payload = torch.randint(0, 1 << 30, (count,), generator=g, dtype=torch.int64)
    common = torch.randint(0, 1 << 20, (1,), generator=g, dtype=torch.int64)
    rare = torch.randint(0, 1 << 20, (count,), generator=g, dtype=torch.int64) % 7
    pick = torch.rand(count, generator=g) < 0.9
    low = torch.where(pick, common.expand(count), rare)
    keys = payload << 20 | low  # the payload above the sorted bits shows the order of ties
    ref = keys.numpy().view(np.uint64)
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    want = ref[np.argsort(ref & mask, kind="stable")]
    got = api.sort_u64(keys.to(DEV), bits).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)


# ------------------------------------------------------------------ errors

@pytest.mark.parametrize("edges,n,both,name", [
    ([(0, 1), (1, 5)], 5, False, "range"),
    ([(0, 1), (-1, 2)], 5, False, "range"),
    ([(0, 1), (2, 2)], 5, False, "self_loop"),
    ([(0, 1), (1, 2), (1, 0)], 5, False, "dup_edge"),
    ([(0, 1), (1, 2), (0, 1)], 5, False, "dup_edge"),
    ([(0, 1), (1, 0), (1, 2), (3, 2)], 5, True, "asymmetric"),
])
def test_device_errors(edges, n, both, name):
    e = torch.tensor(edges, dtype=torch.int32, device=DEV)
    with pytest.raises(api.TCError) as ei:
        api.count(e, n, both)
    assert ei.value.name == name
    with pytest.raises(api.TCError) as ei:
        api.count_per_vertex(e, n, both)
    assert ei.value.name == name


def test_host_errors():
    e = torch.tensor([(0, 1), (1, 2), (0, 2)], dtype=torch.int32, device=DEV)
    ws = api.alloc_workspace(3, 3, device=DEV)
    short = ws[: ws.numel() - 256]
    with pytest.raises(api.TCError) as ei:
        api.count_async(e, 3, workspace=short)
    assert ei.value.name == "workspace"
    with pytest.raises(api.TCError) as ei:
        api.count_async(torch.tensor([(0, 1), (1, 0), (1, 2)], dtype=torch.int32, device=DEV), 3,
                        both=True)
    assert ei.value.name == "asymmetric"
    # a valid call after the errors still works
    assert api.count(e, 3) == 1


# ------------------------------------------------------------------ full-size workloads

def pv_digest(pv) -> str:
    """sha256 of per-vertex counts as little-endian uint64, the stored goldens' digest."""
    return hashlib.sha256(np.ascontiguousarray(pv, dtype="<u8").tobytes()).hexdigest()


def test_rmat20_golden():
    """R-MAT scale 20: total and the whole per-vertex array (digest) against the oracle's
    stored values, one-shot and through a prepared graph with panels."""
    g = golden()["rmat_s20_ef16_s0"]
    e, n = synth.rmat_graph(20, 16, seed=0, device=DEV)
    assert synth.edges_sha256(e) == g["sha256"]
    tot, pv = api.count_per_vertex(e, n)
    assert tot == g["total"]
    pv = pv.cpu().numpy()
    assert int(pv.sum()) == g["per_vertex_sum"] == 3 * tot
    for v, want in g["per_vertex_sample"].items():
        assert pv[int(v)] == want
    assert pv_digest(pv) == g["per_vertex_sha256"]
    assert api.count(e, n) == tot
    r = api.Prepared(e, n).count_async(per_vertex=True).check()
    assert int(r.total.item()) == tot
    assert pv_digest(r.per_vertex.cpu().numpy()) == g["per_vertex_sha256"]


def test_rmat23_full_size():
    """The headline workload at full size, as the benchmark launches it."""
    gd = golden().get("rmat_s23_ef24_s0")
    e, n = synth.rmat_graph(23, 24, seed=0, device=DEV)
    if gd is not None:
        assert synth.edges_sha256(e) == gd["sha256"]
    tot = api.count(e, n)
    tot2, pv = api.count_per_vertex(e, n)
    assert tot2 == tot
    assert int(pv.sum().item()) == 3 * tot
    if gd is not None:
        assert tot == gd["total"]
        pvh = pv.cpu().numpy()
        for v, want in gd["per_vertex_sample"].items():
            assert pvh[int(v)] == want
        assert pv_digest(pvh) == gd["per_vertex_sha256"]
    # sampled per-vertex counts from the definition, one vertex at a time
    pvh = pv.cpu().numpy()
    deg = api.preprocess(e, n)["deg"].cpu().numpy()
    rng = np.random.default_rng(0)
    cand = np.flatnonzero((deg >= 2) & (deg <= 2000))
    q = rng.choice(cand, size=min(64, cand.size), replace=False)
    want = oracle.vertex_triangles(e.cpu().numpy(), n, q)
    assert np.array_equal(pvh[q].astype(np.uint64), want)


def test_autotune_single(tmp_path):
    """The single-graph tuner times its candidates on the caller's graph, returns one of them,
    counts exactly with it, and answers later calls of the same size class from its cache."""
    from paper_1503_00576_amd import autotune
    e, n = synth.rmat_graph(13, 16, seed=14, device=DEV)
    want = oracle.count(e.cpu().numpy(), n)
    cands = [{"panel_ranks": 0, "wave_item_edges": 256, "block_item_edges": 4096},
             {"panel_ranks": 2048, "wave_item_edges": 512, "block_item_edges": 16384},
             {"panel_ranks": 8192, "wave_item_edges": 1024, "block_item_edges": 65536}]
    cache = str(tmp_path / "tune.json")
    best, timings = autotune.tune_single(e, n, reps=1, cache=cache, candidates=cands)
    assert best in cands and len(timings) == 3 and all(ms > 0 for _, ms in timings)
    assert api.count(e, n, options=best) == want
    again, _ = autotune.tune_single(e, n, cache=cache, candidates=cands[:1])
    assert again == best
