"""Pins for the CPU oracle (oracle/forward.c): checks against facts fixed by the paper and by
mathematics, never against the oracle itself.

  - brute force over all vertex triples (tiny graphs), and every labelled graph on 6 vertices;
  - trace(A^3)/6 and diag(A^3)/2 in float64 BLAS (exact: every partial sum is an integer
    below 2**53), networkx's triangle routine, a scipy.sparse product;
  - closed forms (complete, complete multipartite, wheel, cycles, trees, friendship graphs)
    and the named graphs of tests/golden/named_graphs.json;
  - invariants: sum of per-vertex counts = 3 * total, relabelling, edge order and
    orientation, identifier order instead of degree order (Section 2.2: any total order
    consistent with degrees works and the count does not depend on the order at all),
    disjoint-union additivity, the out-degree bound d+ < sqrt(2m) (Section 2.2);
  - properties of the oriented CSR (Sections 2.2 and 3.2): every undirected edge exactly once,
    oriented from the lower to the higher (degree, id), rows strictly ascending;
  - input errors of Section 3.1 (ids out of range, self-loops, repeated edges) are reported;
  - planted mistakes: copies of forward.c with one deliberate bug must fail these pins.
"""
import itertools
import json
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1503_00576_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------- helpers

def brute(n, edges):
    """Triangles by enumerating every vertex triple."""
    adj = set()
    for u, v in edges:
        adj.add((u, v))
        adj.add((v, u))
    tot = 0
    pv = [0] * n
    for a, b, c in itertools.combinations(range(n), 3):
        if (a, b) in adj and (b, c) in adj and (a, c) in adj:
            tot += 1
            pv[a] += 1
            pv[b] += 1
            pv[c] += 1
    return tot, pv


def dense_counts(n, edges):
    """trace(A^3)/6 and diag(A^3)/2 with float64 matrix products."""
    A = np.zeros((n, n), dtype=np.float64)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    A[e[:, 0], e[:, 1]] = 1.0
    A[e[:, 1], e[:, 0]] = 1.0
    A3 = A @ A @ A
    d = np.diag(A3)
    return int(round(d.sum())) // 6, np.rint(d).astype(np.int64) // 2


def rand_graph(n, p, rng):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    rng.shuffle(pairs)
    return [(j, i) if rng.random() < 0.5 else (i, j) for i, j in pairs]


def complete(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def multipartite(sizes):
    off = np.cumsum([0] + list(sizes))
    parts = [range(off[i], off[i + 1]) for i in range(len(sizes))]
    e = []
    for a, b in itertools.combinations(range(len(sizes)), 2):
        e += [(x, y) for x in parts[a] for y in parts[b]]
    return int(off[-1]), e


def wheel(n):
    """hub 0 joined to a cycle on vertices 1..n-1"""
    rim = list(range(1, n))
    e = [(0, r) for r in rim]
    e += [(rim[i], rim[(i + 1) % len(rim)]) for i in range(len(rim))]
    return e


def cycle(k):
    return [(i, (i + 1) % k) for i in range(k)]


def friendship(k):
    """k triangles sharing the centre 0"""
    e = []
    for i in range(k):
        a, b = 1 + 2 * i, 2 + 2 * i
        e += [(0, a), (0, b), (a, b)]
    return 2 * k + 1, e


def check_csr_properties(n, edges, rp, col, order=0):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    deg = np.bincount(e.ravel(), minlength=n) if e.size else np.zeros(n, np.int64)
    assert rp[0] == 0 and rp[-1] == len(e) == col.size
    assert np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(n), np.diff(rp))
    for s, t in zip(src.tolist(), col.tolist()):
        if order == 0:
            assert (deg[s], s) < (deg[t], t)
        else:
            assert s < t
    for x in range(n):
        row = col[rp[x]:rp[x + 1]]
        assert np.all(np.diff(row) > 0)
    got = sorted((min(s, t), max(s, t)) for s, t in zip(src.tolist(), col.tolist()))
    want = sorted((min(u, v), max(u, v)) for u, v in e.tolist())
    assert got == want


# ---------------------------------------------------------------------------- brute force

def test_brute_force_random_small(orc):
    rng = np.random.default_rng(12345)
    import random
    r = random.Random(7)
    for trial in range(300):
        n = int(rng.integers(0, 22))
        p = float(rng.choice([0.05, 0.2, 0.4, 0.7, 1.0]))
        e = rand_graph(n, p, r)
        tot, pv = orc.count(e, n, per_vertex=True)
        bt, bpv = brute(n, e)
        assert tot == bt, (trial, n, p)
        assert list(pv) == bpv


def test_exhaustive_six_vertices(orc):
    """Every one of the 2**15 labelled graphs on 6 vertices: total and per-vertex."""
    n = 6
    pairs = list(itertools.combinations(range(n), 2))
    triples = list(itertools.combinations(range(n), 3))
    pidx = {p: i for i, p in enumerate(pairs)}
    tmask = [(1 << pidx[(a, b)]) | (1 << pidx[(b, c)]) | (1 << pidx[(a, c)]) for a, b, c in triples]
    g = np.arange(1 << 15, dtype=np.int64)
    has = np.stack([(g & mk) == mk for mk in tmask], axis=1)  # [graphs, triples]
    want_tot = has.sum(1)
    memb = np.zeros((len(triples), n), dtype=np.int64)
    for i, t in enumerate(triples):
        memb[i, list(t)] = 1
    want_pv = has.astype(np.int64) @ memb
    for gi in range(1 << 15):
        e = [pairs[b] for b in range(15) if (gi >> b) & 1]
        tot, pv = orc.count(e, n, per_vertex=True)
        assert tot == want_tot[gi]
        assert np.array_equal(pv.astype(np.int64), want_pv[gi])


# ---------------------------------------------------------------------------- algebra / libraries

def test_dense_trace_er_1000(orc):
    e, n = synth.er_1000()
    tot, pv = orc.count(e, n, per_vertex=True)
    dt, dpv = dense_counts(n, e.numpy())
    assert tot == dt
    assert np.array_equal(pv.astype(np.int64), dpv)


def test_networkx_triangles(orc):
    nx = pytest.importorskip("networkx")
    graphs = [synth.er_1000(), (synth.rmat(synth.RmatSpec(10, 16, seed=3)), 1 << 10),
              (synth.barabasi_albert(800, 5, 11), 800), (synth.watts_strogatz(900, 6, 0.1, 5), 900)]
    for e, n in graphs:
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(e.numpy().tolist())
        tri = nx.triangles(G)
        want = np.array([tri[v] for v in range(n)], dtype=np.int64)
        tot, pv = orc.count(e, n, per_vertex=True)
        assert np.array_equal(pv.astype(np.int64), want)
        assert tot * 3 == int(want.sum())


def test_scipy_sparse_rmat14(orc):
    sp = pytest.importorskip("scipy.sparse")
    e, n = synth.rmat_graph(14, 16, seed=1)
    en = e.numpy().astype(np.int64)
    A = sp.coo_matrix((np.ones(len(en) * 2, dtype=np.int64),
                       (np.r_[en[:, 0], en[:, 1]], np.r_[en[:, 1], en[:, 0]])), shape=(n, n)).tocsr()
    pv_want = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() // 2
    tot, pv = orc.count(e, n, per_vertex=True)
    assert np.array_equal(pv.astype(np.int64), pv_want)
    assert tot == int(pv_want.sum()) // 3


# ---------------------------------------------------------------------------- closed forms

@pytest.mark.parametrize("k", list(range(0, 31)))
def test_complete(orc, k):
    tot, pv = orc.count(complete(k), k, per_vertex=True)
    assert tot == math.comb(k, 3)
    assert all(int(x) == math.comb(k - 1, 2) for x in pv)


@pytest.mark.parametrize("sizes", [(1, 1), (3, 4), (7, 9), (5, 5, 5), (2, 3, 4), (1, 6, 2), (3, 3, 3, 3)])
def test_multipartite(orc, sizes):
    n, e = multipartite(sizes)
    tot, pv = orc.count(e, n, per_vertex=True)
    want = sum(a * b * c for a, b, c in itertools.combinations(sizes, 3))
    assert tot == want
    off = np.cumsum([0] + list(sizes))
    for p, sz in enumerate(sizes):
        others = [s for i, s in enumerate(sizes) if i != p]
        per = sum(a * b for a, b in itertools.combinations(others, 2))
        assert all(int(x) == per for x in pv[off[p]:off[p + 1]])


@pytest.mark.parametrize("n", [4, 5, 6, 7, 10, 50, 257])
def test_wheel(orc, n):
    tot, pv = orc.count(wheel(n), n, per_vertex=True)
    if n == 4:  # hub + triangle rim = K4
        assert tot == 4
        return
    assert tot == n - 1
    assert int(pv[0]) == n - 1
    assert all(int(x) == 2 for x in pv[1:])


def test_cycles_trees_stars_paths_empty(orc):
    assert orc.count(cycle(3), 3) == 1
    for k in range(4, 40):
        assert orc.count(cycle(k), k) == 0
    rng = np.random.default_rng(3)
    for n in [1, 2, 10, 200]:
        tree = [(int(rng.integers(0, v)), v) for v in range(1, n)]
        assert orc.count(tree, n) == 0
        assert orc.count([(0, v) for v in range(1, n)], n) == 0
        assert orc.count([(v, v + 1) for v in range(n - 1)], n) == 0
    assert orc.count([], 0) == 0
    assert orc.count([], 17) == 0
    tot, pv = orc.count([], 5, per_vertex=True)
    assert tot == 0 and not pv.any()


@pytest.mark.parametrize("k", [1, 2, 3, 10, 100])
def test_friendship(orc, k):
    n, e = friendship(k)
    tot, pv = orc.count(e, n, per_vertex=True)
    assert tot == k and int(pv[0]) == k and all(int(x) == 1 for x in pv[1:])


def test_named_graphs(orc):
    with open(os.path.join(HERE, "golden", "named_graphs.json")) as f:
        named = json.load(f)
    for name, g in named.items():
        tot, pv = orc.count(g["edges"], g["n"], per_vertex=True)
        assert tot == g["total"], name
        if "per_vertex_all" in g:
            assert all(int(x) == g["per_vertex_all"] for x in pv), name


# ---------------------------------------------------------------------------- invariants

def _graphs():
    yield synth.er_1000()
    yield synth.rmat_graph(12, 16, seed=2)
    yield synth.barabasi_albert(3000, 7, 4), 3000
    yield synth.watts_strogatz(3000, 10, 0.1, 9), 3000


def test_invariants(orc):
    rng = np.random.default_rng(99)
    for e, n in _graphs():
        e = e.numpy()
        tot, pv = orc.count(e, n, per_vertex=True)
        assert int(pv.sum()) == 3 * tot
        # identifier order instead of degree order: same total
        assert orc.count(e, n, order=1) == tot
        # relabelling permutes per-vertex counts
        perm = rng.permutation(n).astype(np.int32)
        t2, pv2 = orc.count(perm[e], n, per_vertex=True)
        assert t2 == tot and np.array_equal(pv2[perm], pv)
        # edge order and orientation do not matter
        e3 = e[rng.permutation(len(e))].copy()
        flip = rng.random(len(e3)) < 0.5
        e3[flip] = e3[flip][:, ::-1]
        assert orc.count(e3, n) == tot
        # the paper's two-direction edge array gives the same result
        both = np.concatenate([e, e[:, ::-1]])[rng.permutation(2 * len(e))]
        t4, pv4 = orc.count(both, n, both=True, per_vertex=True)
        assert t4 == tot and np.array_equal(pv4, pv)
        # out-degree bound: d+ < sqrt(2m)
        rp, col = orc.oriented_csr(e, n)
        assert np.diff(rp).max(initial=0) ** 2 < 2 * max(len(e), 1)


def test_edge_iterator_identity(orc):
    """Sum over undirected edges of |N(u) & N(v)| counts every triangle three times."""
    for e, n in [synth.er_1000(), synth.rmat_graph(11, 16, seed=5)]:
        e = e.numpy()
        nb = [set() for _ in range(n)]
        for u, v in e.tolist():
            nb[u].add(v)
            nb[v].add(u)
        s = sum(len(nb[u] & nb[v]) for u, v in e.tolist())
        assert s == 3 * orc.count(e, n)


def test_disjoint_union_additive(orc):
    parts = [synth.er_1000(), synth.rmat_graph(10, 16, seed=8), (synth.barabasi_albert(500, 4, 2), 500)]
    off = 0
    allp = []
    tot = 0
    for e, n in parts:
        tot += orc.count(e, n)
        allp.append(e.numpy() + off)
        off += n
    assert orc.count(np.concatenate(allp), off) == tot


def test_oriented_csr_properties(orc):
    import random
    r = random.Random(1)
    for n, p in [(30, 0.3), (60, 0.1), (12, 1.0)]:
        e = rand_graph(n, p, r)
        for order in (0, 1):
            rp, col = orc.oriented_csr(e, n, order=order)
            check_csr_properties(n, e, rp, col, order)
    e, n = synth.rmat_graph(10, 8, seed=4)
    rp, col = orc.oriented_csr(e, n)
    check_csr_properties(n, e.numpy(), rp, col)
    rp2, col2 = orc.oriented_csr(np.concatenate([e.numpy(), e.numpy()[:, ::-1]]), n, both=True)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)


def test_degrees(orc):
    e, n = synth.rmat_graph(10, 8, seed=4)
    en = e.numpy()
    assert np.array_equal(orc.degrees(en, n), np.bincount(en.ravel(), minlength=n))


# ---------------------------------------------------------------------------- per-vertex definition, sym CSR

def test_vertex_triangles_definition(orc):
    import random
    r = random.Random(4)
    for n, p in [(15, 0.5), (25, 0.3)]:
        e = rand_graph(n, p, r)
        _, bpv = brute(n, e)
        assert list(orc.vertex_triangles(e, n, list(range(n)))) == bpv
    e, n = synth.rmat_graph(12, 16, seed=6)
    _, pv = orc.count(e, n, per_vertex=True)
    q = np.arange(0, n, 7)
    assert np.array_equal(orc.vertex_triangles(e, n, q), pv[q])


def test_sym_csr_matches_edge_array(orc):
    for e, n in [synth.er_1000(), (synth.watts_strogatz(700, 5, 0.1, 3), 700)]:
        rp, col = synth.symmetric_csr(e, n)
        assert orc.count_sym_csr(rp.numpy(), col.numpy(), n, per_vertex=True)[0] == orc.count(e, n)
    # unsorted row is reported
    rp = np.array([0, 2, 3, 4]); col = np.array([2, 1, 0, 0], dtype=np.int32)
    with pytest.raises(oracle.OracleError) as ei:
        orc.count_sym_csr(rp, col, 3)
    assert ei.value.name == "unsorted"


# ---------------------------------------------------------------------------- input errors

@pytest.mark.parametrize("edges,n,both,name", [
    ([(0, 1), (1, 5)], 5, False, "range"),
    ([(0, 1), (-1, 2)], 5, False, "range"),
    ([(0, 1), (2, 2)], 5, False, "self_loop"),
    ([(0, 1), (1, 2), (1, 0)], 5, False, "dup_edge"),
    ([(0, 1), (1, 2), (0, 1)], 5, False, "dup_edge"),
    ([(0, 1), (1, 0), (1, 2)], 5, True, "asymmetric"),
    ([(0, 1), (1, 0), (1, 2), (1, 2), (2, 1), (2, 1)], 5, True, "dup_edge"),
])
def test_input_errors(orc, edges, n, both, name):
    with pytest.raises(oracle.OracleError) as ei:
        orc.count(edges, n, both=both)
    assert ei.value.name == name


# ---------------------------------------------------------------------------- planted mistakes

MUTANTS = {
    # merge steps over the element after a match in the second list
    "merge_skips_after_match": ("++t;", "++t; ++j;"),
    # first out-edge of every row skipped
    "skip_first_edge": ("for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)",
                        "for (int64_t e = row_ptr[u] + 1; e < row_ptr[u + 1]; ++e)"),
    # the third vertex of a triangle not credited
    "per_vertex_drops_w": ("per_vertex[a] += 1;", ";"),
    # lists left unsorted
    "no_row_sort": ("if (len > 1) qsort", "if (len > 1 && 0) qsort"),
    # orientation against the degree order
    "order_reversed": ("return deg[u] < deg[v];", "return deg[u] > deg[v];"),
    # degree counts only first ends
    "degree_first_only": ("if (!both) deg[edges[2 * i + 1]] += 1;", ";"),
    # off-by-one range check
    "range_off_by_one": ("(int64_t)u >= n || (int64_t)v >= n", "(int64_t)u > n || (int64_t)v > n"),
}


def _mutant_fails(orc_m) -> bool:
    """Run a reduced pin battery; True if any pin fails."""
    import random
    try:
        r = random.Random(3)
        for _ in range(40):
            n = r.randint(3, 14)
            e = rand_graph(n, 0.5, r)
            tot, pv = orc_m.count(e, n, per_vertex=True)
            if (tot, list(pv)) != brute(n, e):
                return True
        e, n = synth.rmat_graph(9, 8, seed=4)
        rp, col = orc_m.oriented_csr(e, n)
        check_csr_properties(n, e.numpy(), rp, col)
        try:
            orc_m.count([(0, 1), (1, 5)], 5)
            return True
        except oracle.OracleError as err:
            if err.name != "range":
                return True
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "forward.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, name
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mut.c")
        so = os.path.join(d, "libmut.so")
        with open(c, "w") as f:
            f.write(src.replace(old, new, 1))
        subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", c, "-o", so], check=True)
        assert _mutant_fails(oracle.Oracle(so)), name


def test_unmutated_passes_battery(orc):
    assert not _mutant_fails(orc)
