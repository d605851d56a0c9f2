"""GPU parity of the yardstick kernels (libtc_ablation.so): the paper's thread-per-edge merge in
every variant of its Section 3.4 optimisations counts exactly the oracle's triangles; the
library edge sorts order (u, v) pairs exactly as numpy does; the gather probe reads the
positions its hash names."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1503_00576_amd import ablation, api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def graphs():
    k = 130
    yield np.array([(i, j) for i in range(k) for j in range(i + 1, k)], dtype=np.int32), k
    yield synth.er_1000()[0].numpy(), 1000
    yield synth.rmat_graph(12, 16, seed=41)[0].numpy(), 1 << 12
    yield synth.barabasi_albert(3000, 12, 2).numpy(), 3000
    yield synth.watts_strogatz(2500, 8, 0.1, 4).numpy(), 2500
    yield np.zeros((0, 2), dtype=np.int32), 10


@pytest.mark.parametrize("flags", list(range(16)))
def test_edge_merge_variants(flags):
    for e, n in graphs():
        want = oracle.count(e, n)
        em = ablation.EdgeMerge(api.Prepared(torch.as_tensor(e, device=DEV), n))
        for threads, blocks in [(64, 8 * 256), (256, 3), (1024, 1)]:
            assert em.count(flags, threads, blocks) == want, (n, threads, blocks)


def test_edge_merge_rmat16():
    e, n = synth.rmat_graph(16, 16, seed=0, device=DEV)
    want = oracle.count(e.cpu().numpy(), n)
    em = ablation.EdgeMerge(api.Prepared(e, n))
    assert em.count() == want
    assert em.count(ablation.TWO_READS | ablation.AOS) == want


@pytest.mark.parametrize("count,bits", [(1, 5), (1000, 10), (300_001, 17), (2_000_003, 20)])
def test_library_edge_sorts(count, bits):
    g = np.random.default_rng(count)
    u = g.integers(0, 1 << bits, count, dtype=np.int64)
    v = g.integers(0, 1 << bits, count, dtype=np.int64)
    order = np.lexsort((v, u))
    want_u, want_v = u[order], v[order]
    # comparison sort of pairs
    pairs = torch.from_numpy(np.stack([u, v], 1).astype(np.int32).reshape(-1)).to(DEV)
    ablation.sort_async(ablation.SORT_PAIRS_COMPARE, bits, pairs)
    p = pairs.cpu().numpy().reshape(-1, 2)
    assert np.array_equal(p[:, 0], want_u) and np.array_equal(p[:, 1], want_v)
    # two radix passes over pairs of arrays
    a = torch.from_numpy(u.astype(np.int32)).to(DEV)
    b = torch.from_numpy(v.astype(np.int32)).to(DEV)
    ablation.sort_async(ablation.SORT_PAIRS_RADIX, bits, a, b, torch.empty_like(a),
                        torch.empty_like(b))
    assert np.array_equal(a.cpu().numpy(), want_u) and np.array_equal(b.cpu().numpy(), want_v)
    # packed 64-bit keys
    keys = torch.from_numpy((u << bits) | v).to(DEV)
    out = torch.empty_like(keys)
    ablation.sort_async(ablation.SORT_PACKED_RADIX, bits, keys, None, out)
    assert np.array_equal(out.cpu().numpy(), (want_u << bits) | want_v)


def fmix32(h):
    h = h.astype(np.uint64) & 0xFFFFFFFF
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    return h


@pytest.mark.parametrize("elem_bytes", [4, 8, 16])
def test_gather_probe(elem_bytes):
    words = elem_bytes // 4
    table = torch.randint(0, 1 << 30, (3001 * words,), dtype=torch.int32,
                          generator=torch.Generator().manual_seed(elem_bytes))
    count, seed = 50_000, 1234
    sink = torch.empty(1, dtype=torch.int64, device=DEV)
    ablation.gather_async(table.to(DEV), elem_bytes, count, seed, sink)
    i = np.arange(count, dtype=np.uint64)
    h = fmix32(i ^ fmix32(np.full(count, seed, dtype=np.uint64)))
    at = (h * np.uint64(3001)) >> np.uint64(32)
    t = table.numpy().view(np.uint32).reshape(-1, words).astype(np.uint64)
    x = t[at.astype(np.int64)]
    val = x[:, 0]
    for k in range(1, words):
        val = val ^ x[:, k]
    # per-lane sums wrap at 32 bits before the wave reduction; compare modulo 2^32
    assert int(sink.item()) % (1 << 32) == int(val.sum()) % (1 << 32)
