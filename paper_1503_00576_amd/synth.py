"""Seeded synthetic graph inputs (Erdos-Renyi, R-MAT, Barabasi-Albert, Watts-Strogatz,
Poisson request traces).

This module only produces inputs: it holds none of the triangle-counting arithmetic and is
the one piece of code that both the GPU path's tests/benchmarks and the CPU oracle's tests
use.  The paper evaluates on Kronecker (R-MAT) graphs, a Barabasi-Albert and a
Watts-Strogatz network (Section 4, Table 1); the generators below synthesise graphs of those
families with seeded randomness.

Every random number comes from one counter-based generator: Chris Wellons' published
``lowbias32`` integer hash ("hash prospector", 2018: xorshift 16, multiply 0x7feb352d,
xorshift 15, multiply 0x846ca68b, xorshift 16) applied to (seed, stream, index).  All
arithmetic is exact int64 tensor arithmetic (32x32-bit products are split into 16-bit halves
so no intermediate overflows), so the same call gives the same bytes on the CPU and on a GPU.

Output format: an int32 tensor of shape [m, 2] listing every undirected edge once, in a
shuffled order, each pair in a random orientation; no self-loops and no duplicates.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import torch

_M32 = 0xFFFFFFFF
_GOLDEN = 0x9E3779B9

# stream ids: keep every use of the generator on its own stream
_S_ER = 1
_S_RMAT = 2  # + level pair (< 64)
_S_PERM = 100
_S_SHUFFLE = 101
_S_SWAP = 102
_S_BA = 200
_S_WS_REWIRE = 300
_S_WS_TARGET = 301
_S_BATCH = 400
_S_TRACE = 500


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2**32 for x in [0, 2**32) held in int64, without int64 overflow."""
    lo = c & 0xFFFF
    hi = (c >> 16) & 0xFFFF
    return (x * lo + (((x * hi) & 0xFFFF) << 16)) & _M32


def lowbias32(x: torch.Tensor) -> torch.Tensor:
    """Wellons' lowbias32 mixer on int64 tensors holding 32-bit values."""
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def _lowbias32_int(x: int) -> int:
    x &= _M32
    x ^= x >> 16
    x = (x * 0x7FEB352D) & _M32
    x ^= x >> 15
    x = (x * 0x846CA68B) & _M32
    x ^= x >> 16
    return x


def _stream_key(seed: int, stream: int) -> int:
    return _lowbias32_int((seed & _M32) ^ _lowbias32_int((stream * _GOLDEN + 0x632BE5AB) & _M32))


def rand32(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """Uniform 32-bit values (int64 tensor) for counters ``idx`` (int64, 0 <= idx < 2**62)."""
    k = _stream_key(seed, stream)
    lo = idx & _M32
    hi = (idx >> 32) & _M32
    x = lowbias32(lo ^ k)
    x = lowbias32((x + _lowbias32_int(k ^ 0x5BD1E995)) & _M32 ^ lowbias32(hi))
    return x


def _counter(n: int, device) -> torch.Tensor:
    return torch.arange(n, dtype=torch.int64, device=device)


def _finish(lo: torch.Tensor, hi: torch.Tensor, n: int, seed: int, device) -> torch.Tensor:
    """Drop loops, deduplicate undirected pairs, shuffle, randomly orient; int32 [m, 2]."""
    a = torch.minimum(lo, hi)
    b = torch.maximum(lo, hi)
    keep = a != b
    key = a[keep] * n + b[keep]
    del a, b, keep
    key = torch.unique(key, sorted=True)
    m = key.numel()
    if m == 0:
        return torch.empty((0, 2), dtype=torch.int32, device=device)
    order = torch.argsort(rand32(seed, _S_SHUFFLE, _counter(m, device)), stable=True)
    key = key[order]
    del order
    u = torch.div(key, n, rounding_mode="floor")
    v = key - u * n
    del key
    swap = (rand32(seed, _S_SWAP, _counter(m, device)) & 1).bool()
    first = torch.where(swap, v, u)
    second = torch.where(swap, u, v)
    return torch.stack([first, second], dim=1).to(torch.int32)


def erdos_renyi(n: int, p: float, seed: int, device="cpu") -> torch.Tensor:
    """G(n, p): every pair {i, j}, i < j, kept independently with probability p."""
    if n < 2:
        return torch.empty((0, 2), dtype=torch.int32, device=device)
    thr = int(round(p * 2**32))
    i = torch.arange(n, dtype=torch.int64, device=device)
    ii, jj = torch.triu_indices(n, n, offset=1, device=device).to(torch.int64)
    pair = ii * n + jj
    keep = rand32(seed, _S_ER, pair) < thr
    return _finish(ii[keep], jj[keep], n, seed, device)


@dataclass(frozen=True)
class RmatSpec:
    scale: int
    edgefactor: int
    a: float = 0.57
    b: float = 0.19
    c: float = 0.19
    seed: int = 0

    @property
    def n(self) -> int:
        return 1 << self.scale

    @property
    def draws(self) -> int:
        return self.edgefactor << self.scale


def rmat(spec: RmatSpec, device="cpu", chunk: int = 1 << 24) -> torch.Tensor:
    """R-MAT (Kronecker) graph, Graph500 style.

    ``edgefactor * 2**scale`` directed draws; each draw picks one of the four adjacency
    quadrants per level (probabilities a, b, c, 1-a-b-c, quantised to 1/65536, MSB first,
    no parameter noise); then a seeded vertex-label permutation, symmetrisation, loop and
    duplicate removal, shuffle and random orientation.
    """
    s, n, M = spec.scale, spec.n, spec.draws
    ta = int(round(spec.a * 65536))
    tb = int(round((spec.a + spec.b) * 65536))
    tc = int(round((spec.a + spec.b + spec.c) * 65536))
    src = torch.empty(M, dtype=torch.int64, device=device)
    dst = torch.empty(M, dtype=torch.int64, device=device)
    for c0 in range(0, M, chunk):
        idx = torch.arange(c0, min(M, c0 + chunk), dtype=torch.int64, device=device)
        su = torch.zeros_like(idx)
        du = torch.zeros_like(idx)
        r = None
        for lvl in range(s):
            if lvl % 2 == 0:
                r = rand32(spec.seed, _S_RMAT + lvl // 2, idx)
                r16 = r & 0xFFFF
            else:
                r16 = r >> 16
            sb = (r16 >= tb).to(torch.int64)
            db = (((r16 >= ta) & (r16 < tb)) | (r16 >= tc)).to(torch.int64)
            su = su * 2 + sb
            du = du * 2 + db
        src[c0:c0 + idx.numel()] = su
        dst[c0:c0 + idx.numel()] = du
        del idx, su, du, r
    relabel = torch.argsort(rand32(spec.seed, _S_PERM, _counter(n, device)), stable=True)
    src = relabel[src]
    dst = relabel[dst]
    del relabel
    return _finish(src, dst, n, spec.seed, device)


def _uniform(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """float64 in [0, 1) from 32 random bits."""
    return rand32(seed, stream, idx).to(torch.float64) * (1.0 / 2**32)


def barabasi_albert(n: int, k: int, seed: int, device="cpu") -> torch.Tensor:
    """Preferential attachment (Batagelj-Brandes edge-copy form).

    A (k+1)-clique seeds the graph; every later vertex x adds k edges, each to the endpoint
    at a uniformly random position of the endpoint list of all earlier edges (so a target is
    chosen with probability proportional to its degree).  A draw that lands on a target slot
    of an earlier edge copies that edge's target; chains are resolved by pointer jumping.
    Repeated targets of one vertex collapse in deduplication.
    """
    k = max(1, int(k))
    if n <= k + 1:
        ii, jj = torch.triu_indices(n, n, offset=1, device=device).to(torch.int64)
        return _finish(ii, jj, n, seed, device)
    c = k + 1
    ci, cj = torch.triu_indices(c, c, offset=1, device=device).to(torch.int64)
    e0 = ci.numel()
    nadd = (n - c) * k
    E = e0 + nadd
    src = torch.empty(E, dtype=torch.int64, device=device)
    src[:e0] = ci
    src[e0:] = torch.arange(c, n, dtype=torch.int64, device=device).repeat_interleave(k)
    # tgt_ref >= 0: literal vertex; tgt_ref < 0: copy target of edge (-1 - tgt_ref)
    tgt_ref = torch.empty(E, dtype=torch.int64, device=device)
    tgt_ref[:e0] = cj
    e = torch.arange(e0, E, dtype=torch.int64, device=device)
    # vertex x's edges draw from endpoints of edges added before x (index < first edge of x)
    first_of_x = e0 + torch.div(e - e0, k, rounding_mode="floor") * k
    pos = (_uniform(seed, _S_BA, e) * (2 * first_of_x).to(torch.float64)).to(torch.int64)
    pos = torch.minimum(pos, 2 * first_of_x - 1)
    eref = torch.div(pos, 2, rounding_mode="floor")
    is_src = (pos & 1) == 0
    tgt_ref[e0:] = torch.where(is_src, src[eref], -1 - eref)
    del e, first_of_x, pos, is_src, eref
    while True:
        neg = tgt_ref < 0
        if not bool(neg.any()):
            break
        tgt_ref = torch.where(neg, tgt_ref[torch.clamp(-1 - tgt_ref, min=0)], tgt_ref)
    return _finish(src, tgt_ref, n, seed, device)


def watts_strogatz(n: int, k: int, beta: float, seed: int, device="cpu") -> torch.Tensor:
    """Ring lattice (every vertex joined to its k nearest neighbours on each side), each
    lattice edge's far end rewired with probability beta to a uniformly random vertex;
    loops and duplicates created by rewiring are dropped."""
    k = max(1, min(int(k), (n - 1) // 2))
    if n < 3:
        return torch.empty((0, 2), dtype=torch.int32, device=device)
    u = torch.arange(n, dtype=torch.int64, device=device).repeat_interleave(k)
    off = torch.arange(1, k + 1, dtype=torch.int64, device=device).repeat(n)
    v = (u + off) % n
    E = u.numel()
    idx = _counter(E, device)
    rew = _uniform(seed, _S_WS_REWIRE, idx) < beta
    tgt = (rand32(seed, _S_WS_TARGET, idx) % n)
    v = torch.where(rew, tgt, v)
    return _finish(u, v, n, seed, device)


@dataclass(frozen=True)
class BatchSpec:
    """A batch of independent small graphs: half Barabasi-Albert, half Watts-Strogatz."""
    graphs: int = 4096
    n_min: int = 50
    n_max: int = 20000
    deg_min: float = 4.0
    deg_max: float = 32.0
    beta: float = 0.1
    seed: int = 0


def batch_graph_params(spec: BatchSpec):
    """Per-graph (kind, n, k, seed): kind 0 = BA, 1 = WS; n log-uniform; k = round(d/2)."""
    g = _counter(spec.graphs, "cpu")
    un = _uniform(spec.seed, _S_BATCH, 3 * g)
    ud = _uniform(spec.seed, _S_BATCH, 3 * g + 1)
    uk = rand32(spec.seed, _S_BATCH, 3 * g + 2)
    out = []
    for i in range(spec.graphs):
        n = int(round(math.exp(math.log(spec.n_min) + float(un[i]) * (math.log(spec.n_max) - math.log(spec.n_min)))))
        d = spec.deg_min + float(ud[i]) * (spec.deg_max - spec.deg_min)
        k = max(1, int(round(d / 2)))
        out.append((int(uk[i]) & 1, n, k, spec.seed * 1000003 + i))
    return out


def batch_graph(kind: int, n: int, k: int, seed: int, beta: float = 0.1, device="cpu") -> torch.Tensor:
    if kind == 0:
        return barabasi_albert(n, k, seed, device)
    return watts_strogatz(n, k, beta, seed, device)


def symmetric_csr(edges: torch.Tensor, n: int):
    """Symmetric CSR (both directions, rows ascending) of an edge list: (row_ptr int32[n+1],
    col int32[2m]).  Input formatting for the batched entry point."""
    e = edges.to(torch.int64)
    u = torch.cat([e[:, 0], e[:, 1]])
    v = torch.cat([e[:, 1], e[:, 0]])
    key = torch.sort(u * n + v).values
    col = (key % n).to(torch.int32) if n > 0 else key.to(torch.int32)
    cnt = torch.bincount(torch.div(key, max(n, 1), rounding_mode="floor"), minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=edges.device)
    row_ptr[1:] = torch.cumsum(cnt, 0)
    return row_ptr.to(torch.int32), col


def pack_symmetric(graphs, device="cpu") -> dict:
    """Concatenate graphs [(edges int32 [m, 2], n), ...] into the batched input format: per
    graph a symmetric CSR (both directions, rows ascending, local ids), plus vertex and
    adjacency offsets.  Returns dict(vtx_off int64 [G+1], adj_off int64 [G+1],
    row_ptr int32 [N+G], col int32 [2 sum m], G, n_total, adj_total).  Runs on `device`
    without host synchronisation (sizes come from the host-side graph list)."""
    G = len(graphs)
    ns = [int(n) for _, n in graphs]
    ms = [int(e.shape[0]) for e, _ in graphs]
    offs = [0]
    for n in ns:
        offs.append(offs[-1] + n)
    N, M = offs[-1], sum(ms)
    vo = torch.tensor(offs, dtype=torch.int64, device=device)
    if M:
        E = torch.cat([e.to(device=device, dtype=torch.int64) + offs[g]
                       for g, (e, _) in enumerate(graphs) if e.shape[0]])
    else:
        E = torch.zeros((0, 2), dtype=torch.int64, device=device)
    src = torch.cat([E[:, 0], E[:, 1]])
    dst = torch.cat([E[:, 1], E[:, 0]])
    order = torch.argsort(src * max(N, 1) + dst)
    src, dst = src[order], dst[order]
    grow = torch.zeros(N + 1, dtype=torch.int64, device=device)
    grow.index_add_(0, src + 1, torch.ones_like(src))
    grow = torch.cumsum(grow, 0)
    adj_off = grow[vo]
    reps = torch.tensor([n + 1 for n in ns], dtype=torch.int64, device=device)
    gidx = torch.repeat_interleave(torch.arange(G, device=device), reps, output_size=N + G)
    pos = torch.arange(N + G, device=device) - gidx
    row_ptr = (grow[pos] - adj_off[gidx]).to(torch.int32)
    g_of = torch.searchsorted(vo[1:], src, right=True)
    col = (dst - vo[g_of]).to(torch.int32)
    return {"vtx_off": vo, "adj_off": adj_off, "row_ptr": row_ptr, "col": col, "G": G,
            "n_total": N, "adj_total": 2 * M}


def batch_graphs(spec: BatchSpec, device="cpu"):
    """The graphs of a BatchSpec as [(edges, n), ...]."""
    return [(batch_graph(kind, n, k, seed, spec.beta, device), n)
            for kind, n, k, seed in batch_graph_params(spec)]


def poisson_trace(rate: float, duration: float, seed: int):
    """Arrival times of a Poisson process (exponential gaps) plus one uniform draw per
    arrival for the caller's request mix; returns (times float64[k], u float64[k])."""
    expect = int(rate * duration * 1.5 + 64)
    idx = _counter(expect, "cpu")
    gaps = -torch.log1p(-_uniform(seed, _S_TRACE, 2 * idx)) / rate
    t = torch.cumsum(gaps, 0)
    keep = t < duration
    return t[keep], _uniform(seed, _S_TRACE, 2 * idx + 1)[keep]


# the serving workload's request mix -----------------------------------------------------

# Graphs are drawn from a seeded pool per R-MAT scale (edgefactor 16) so that generation time
# stays bounded: scale -> pool size.  90% of requests are scale 10-14, 9% scale 17-19 and
# 1% scale 21.
SERVE_POOL = {10: 16, 11: 16, 12: 16, 13: 16, 14: 16, 17: 6, 18: 4, 19: 3, 21: 2}
SERVE_EDGEFACTOR = 16


def serve_pool_seed(scale: int, i: int) -> int:
    return 1000 * scale + i


def serve_pool_graph(scale: int, i: int, device="cpu") -> tuple[torch.Tensor, int]:
    """Graph i of the serving pool at this scale."""
    return rmat_graph(scale, SERVE_EDGEFACTOR, seed=serve_pool_seed(scale, i), device=device)


def serve_pick(i: int, u: float) -> tuple[int, int]:
    """(scale, pool index) of request i, given its uniform draw u from poisson_trace."""
    if u < 0.9:
        sc = 10 + min(4, int(u / 0.9 * 5))
    elif u < 0.99:
        sc = 17 + min(2, int((u - 0.9) / 0.09 * 3))
    else:
        sc = 21
    return sc, i % SERVE_POOL[sc]


def edges_sha256(edges: torch.Tensor) -> str:
    return hashlib.sha256(edges.detach().to("cpu").contiguous().numpy().tobytes()).hexdigest()


# named workloads --------------------------------------------------------------------------

def er_1000(device="cpu") -> tuple[torch.Tensor, int]:
    """G(n=1000, p=0.02), seed 0."""
    return erdos_renyi(1000, 0.02, 0, device), 1000


def rmat_graph(scale: int, edgefactor: int, seed: int = 0, device="cpu") -> tuple[torch.Tensor, int]:
    spec = RmatSpec(scale, edgefactor, seed=seed)
    return rmat(spec, device), spec.n
