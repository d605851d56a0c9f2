"""Seeded inputs: determinism, format contract (no loops, no duplicates, ids in range), the
hash-based generator against an independent integer implementation, and the batch packer."""
import json
import os

import numpy as np
import torch

from paper_1503_00576_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def lowbias32_ref(x: int) -> int:
    x &= 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def test_lowbias32_exact():
    xs = [0, 1, 2, 12345, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0xDEADBEEF]
    xs += list(np.random.default_rng(0).integers(0, 2**32, 1000, dtype=np.uint64).tolist())
    got = synth.lowbias32(torch.tensor(xs, dtype=torch.int64)).tolist()
    assert got == [lowbias32_ref(x) for x in xs]


def valid_edges(e, n):
    e = e.numpy().astype(np.int64)
    assert e.ndim == 2 and e.shape[1] == 2
    assert (e >= 0).all() and (e < n).all()
    assert (e[:, 0] != e[:, 1]).all()
    key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    assert np.unique(key).size == key.size


def test_generators_contract_and_determinism():
    cases = [lambda: synth.er_1000(), lambda: synth.rmat_graph(12, 16, seed=3),
             lambda: (synth.barabasi_albert(2000, 5, 1), 2000),
             lambda: (synth.watts_strogatz(2000, 4, 0.1, 1), 2000)]
    for mk in cases:
        e1, n = mk()
        e2, _ = mk()
        valid_edges(e1, n)
        assert torch.equal(e1, e2)


def test_golden_hashes():
    with open(os.path.join(HERE, "golden", "workloads.json")) as f:
        g = json.load(f)
    e, n = synth.er_1000()
    assert synth.edges_sha256(e) == g["er_1000_p0.02_s0"]["sha256"]
    e, n = synth.rmat_graph(16, 16, seed=0)
    assert synth.edges_sha256(e) == g["rmat_s16_ef16_s0"]["sha256"]


def test_er_density():
    e = synth.erdos_renyi(2000, 0.01, 5)
    expect = 0.01 * 2000 * 1999 / 2
    assert abs(e.shape[0] - expect) < 5 * np.sqrt(expect)


def test_ws_degree_and_ba_growth():
    e = synth.watts_strogatz(1000, 5, 0.0, 2).numpy()  # no rewiring: exact ring lattice
    deg = np.bincount(e.ravel(), minlength=1000)
    assert (deg == 10).all()
    e = synth.barabasi_albert(3000, 4, 2).numpy()
    deg = np.bincount(e.ravel(), minlength=3000)
    assert deg.max() > 5 * np.median(deg)   # preferential attachment makes hubs


def test_pack_symmetric_matches_per_graph_csr():
    gs = [synth.er_1000(), (synth.barabasi_albert(300, 3, 1), 300),
          (torch.zeros((0, 2), dtype=torch.int32), 5), (synth.watts_strogatz(50, 2, 0.1, 2), 50)]
    b = synth.pack_symmetric(gs)
    assert b["G"] == 4 and b["n_total"] == 1355
    assert b["adj_total"] == 2 * sum(int(e.shape[0]) for e, _ in gs)
    for g, (e, n) in enumerate(gs):
        v0 = int(b["vtx_off"][g])
        rp = b["row_ptr"][v0 + g: v0 + g + n + 1]
        a0, a1 = int(b["adj_off"][g]), int(b["adj_off"][g + 1])
        rp2, col2 = synth.symmetric_csr(e, n)
        assert torch.equal(rp, rp2) and torch.equal(b["col"][a0:a1], col2)


def test_batch_params():
    spec = synth.BatchSpec(graphs=512, seed=0)
    ps = synth.batch_graph_params(spec)
    ns = np.array([n for _, n, _, _ in ps])
    ks = np.array([k for _, _, k, _ in ps])
    kinds = np.array([kd for kd, _, _, _ in ps])
    assert ns.min() >= 50 and ns.max() <= 20000
    assert ks.min() >= 2 and ks.max() <= 16
    assert 0.4 < kinds.mean() < 0.6
    assert ps == synth.batch_graph_params(spec)


def test_poisson_trace():
    t, u = synth.poisson_trace(200.0, 60.0, 1)
    assert abs(t.numel() - 12000) < 5 * np.sqrt(12000)
    assert (torch.diff(t) > 0).all() and float(t[-1]) < 60.0
    assert 0.0 <= float(u.min()) and float(u.max()) < 1.0


def test_serve_pool_hashes():
    """The serving pool's small graphs regenerate the bytes whose counts are stored."""
    with open(os.path.join(HERE, "golden", "serve_pool.json")) as f:
        ref = json.load(f)
    for sc in (10, 12, 14):
        for i in (0, synth.SERVE_POOL[sc] - 1):
            e, n = synth.serve_pool_graph(sc, i)
            assert n == ref[str(sc)][i]["n"] and e.shape[0] == ref[str(sc)][i]["m"]
            assert synth.edges_sha256(e) == ref[str(sc)][i]["sha256"]


def test_serve_pick_mix():
    """Request i's scale follows the stated mix (90% scales 10-14, 9% 17-19, 1% 21)."""
    assert synth.serve_pick(0, 0.0) == (10, 0)
    assert synth.serve_pick(5, 0.899)[0] == 14
    assert synth.serve_pick(5, 0.9)[0] == 17
    assert synth.serve_pick(5, 0.989)[0] == 19
    assert synth.serve_pick(3, 0.995) == (21, 1)
    _, u = synth.poisson_trace(200.0, 60.0, 0)
    scales = np.array([synth.serve_pick(i, x)[0] for i, x in enumerate(u.tolist())])
    assert 11000 < scales.size < 13000
    assert abs((scales <= 14).mean() - 0.9) < 0.02
    assert abs((scales == 21).mean() - 0.01) < 0.005
