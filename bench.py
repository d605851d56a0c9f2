"""Benchmark: exact triangle counting of a synthetic R-MAT graph on one MI355X.

A step is one pass of the whole path over the device-resident edge array: degrees, order,
orientation, key sort, node array, in-edge lists (tc_preprocess) and the counting kernel
(tc_count_prepared) -- i.e. exactly what tc_count enqueues.  The headline workload is R-MAT
scale 23, edgefactor 24, (a, b, c) = (0.57, 0.19, 0.19), seed 0: about 1.9e8 undirected
edges.  `value` is oriented edges (one sorted-list intersection each) per second of step
time.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 int32 lanes/clk x 2.4 GHz = 39.3

WORKLOADS = {
    "rmat23": dict(kind="rmat", scale=23, ef=24, seed=0,
                   label="R-MAT scale 23, edgefactor 24, a=0.57 b=0.19 c=0.19, seed 0"),
    "rmat20": dict(kind="rmat", scale=20, ef=16, seed=0,
                   label="R-MAT scale 20, edgefactor 16, a=0.57 b=0.19 c=0.19, seed 0"),
    "er1000": dict(kind="er", label="Erdos-Renyi G(1000, 0.02), seed 0"),
}
GOLDEN_KEYS = {"rmat23": "rmat_s23_ef24_s0", "rmat20": "rmat_s20_ef16_s0",
               "er1000": "er_1000_p0.02_s0"}
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
# the sources whose change invalidates a committed counter summary of the counting kernel
# (the kernel itself, and the preprocessing that lays out its work items and segments)
COUNT_SOURCES = [os.path.join(ROOT, "paper_1503_00576_amd", "csrc", f)
                 for f in ("count.hip", "prep.hip", "api.hip", "internal.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_sha(paths=COUNT_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_counters(kernel: str, workload: str) -> dict | None:
    """key = value pairs of the committed rocprofv3 counter summary of a kernel on a workload
    (profiles/counters_<kernel>_<workload>.txt), or None when absent or taken on other
    sources than the current ones."""
    path = os.path.join(ROOT, "profiles", f"counters_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha") != sources_sha():
        return None
    out = {}
    for k, v in kv.items():
        try:
            out[k] = float(v)
        except ValueError:
            out[k] = v
    return out


def golden(name: str):
    path = os.path.join(GOLDEN_DIR, name)
    if not os.path.exists(path) or os.path.getsize(path) == 0:
        return None
    with open(path) as f:
        return json.load(f)


def pv_digest(pv) -> str:
    """sha256 of per-vertex counts as little-endian uint64 (the stored goldens' digest)."""
    return hashlib.sha256(pv.detach().cpu().numpy().astype("<u8").tobytes()).hexdigest()


def streamed_elements(row_ptr, col, p0: int, hbase: int, panel: int = 32):
    """Elements the counting kernel streams through its LDS structures, and its segments:
    for a middle vertex v below the panel region, the suffix of N+(u) after v for every
    in-edge u -> v (when N+(v) is not empty); in the panel region (ranks >= p0, panels of 32
    consecutive middle vertices), one suffix per (u, panel), after u's first panel vertex.
    Also the streamed elements below rank hbase (4 bytes each; the others are read as 16-bit
    offsets from hbase)."""
    import torch
    rp = row_ptr.to(torch.int64)
    c = col.to(torch.int64)
    n = rp.numel() - 1
    deg = rp[1:] - rp[:-1]
    src = torch.repeat_interleave(torch.arange(n, device=rp.device), deg)
    e = torch.arange(c.numel(), device=rp.device)
    row_end = rp[src + 1]
    suffix = row_end - e - 1
    mid = (c < p0) & (suffix > 0) & (deg[c] > 0)
    streamed = int(suffix[mid].sum().item())
    segments = int(mid.sum().item())
    # the first entry >= hbase of every row (the row end when there is none)
    first_high = rp[1:].clone()
    hi = c >= hbase
    first_high.scatter_reduce_(0, src[hi], e[hi], reduce="amin", include_self=True)
    low_end = torch.minimum(first_high[src], row_end)
    low = torch.clamp(low_end - e - 1, min=0)
    streamed_low = int(low[mid & (c < hbase)].sum().item())
    del mid, first_high, hi, low_end, low
    pan = c >= p0
    if bool(pan.any()):
        first = p0 + torch.div(c - p0, panel, rounding_mode="floor") * panel
        prev = torch.roll(c, 1)
        run_start = (e == rp[src]) | (prev < first)
        sel = pan & run_start & (suffix > 0)
        streamed += int(suffix[sel].sum().item())
        segments += int(sel.sum().item())
    return streamed, segments, streamed_low


def make_graph(name: str, dev):
    from paper_1503_00576_amd import synth
    w = WORKLOADS[name]
    if w["kind"] == "rmat":
        return synth.rmat_graph(w["scale"], w["ef"], seed=w["seed"], device=dev)
    return synth.er_1000(device=dev)


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(dev):
    """The oracle (single-threaded C, test infrastructure) on a bounded sample of the same
    workload family: R-MAT scale 19, edgefactor 24, same (a, b, c), seed 0.  The stored oracle
    run of the full headline graph (tests/golden/workloads.json) is reported beside it."""
    import oracle
    from paper_1503_00576_amd import synth
    e, n = synth.rmat_graph(19, 24, seed=0, device=dev)
    eh = e.cpu().numpy()
    m = eh.shape[0]
    t0 = time.perf_counter()
    tot = oracle.count(eh, n)
    dt = time.perf_counter() - t0
    out = {"value": m / dt, "unit": "oriented-edge intersections/s", "cores": 1,
           "kind": "oracle",
           "sample": f"R-MAT scale 19, edgefactor 24, seed 0 ({m} edges, {tot} triangles): "
                     f"oracle end to end (degrees, orientation, sorted lists, merges) "
                     f"in {dt:.2f} s on one host core ({host_cpu_model()}, "
                     f"{os.cpu_count()} logical CPUs visible)"}
    g = (golden("workloads.json") or {}).get("rmat_s23_ef24_s0")
    if g is not None:
        out["headline_graph_oracle"] = {
            "seconds": g["oracle_seconds"], "edges": g["m"],
            "intersections_per_s": g["m"] / g["oracle_seconds"],
            "note": "the stored oracle run of the full R-MAT scale 23 graph (total and "
                    "per-vertex counts), one core of the machine that wrote the goldens "
                    "(tests/golden/make_golden.py --c3), not of this host"}
    return out


def pcie_section(edges, n, m, total, ws, out, L, sp, op):
    """The paper's wall-clock protocol: edge array from (pinned) host memory, the step, the
    total back to the host; reported beside `value`, never as it (median of 3 runs)."""
    import torch
    from paper_1503_00576_amd import api
    wsz = ws.numel()
    host_edges = torch.empty(edges.shape, dtype=edges.dtype, pin_memory=True)
    host_edges.copy_(edges)
    dev_edges = torch.empty_like(edges)
    host_total = torch.empty(1, dtype=torch.int64, pin_memory=True)
    pcie = []
    for _ in range(3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dev_edges.copy_(host_edges, non_blocking=True)
        api._raise(L.tc_preprocess(api._ptr(dev_edges), n, m, 0, op, api._ptr(ws), wsz, sp,
                                   None), "tc_preprocess")
        api._raise(L.tc_count_prepared(n, m, 0, op, api._ptr(ws), wsz, sp, api._ptr(out.total),
                                       None, api._ptr(out.status)), "tc_count_prepared")
        host_total.copy_(out.total, non_blocking=True)
        torch.cuda.synchronize()
        pcie.append((time.perf_counter() - t1) * 1e3)
        assert int(host_total.item()) == total
    pcie_ms = sorted(pcie)[1]
    return {"ms": round(pcie_ms, 3), "intersections_per_s": m / (pcie_ms * 1e-3),
            "h2d_bytes": 8 * m, "runs": [round(x, 3) for x in pcie],
            "note": "median of 3: host-to-device copy of the edge array from pinned memory, the "
                    "step, the total back to the host"}


def batched_section(dev, steps: int, graphs_n: int = 4096, loop: bool = True):
    """4096 Barabasi-Albert / Watts-Strogatz graphs (50/50, n log-uniform in [50, 20000],
    average degree in [4, 32]) in one captured plan, tuned, against a loop of one tc_count
    call per graph on the same GPU; per-graph totals and the per-vertex digest checked against
    the oracle's stored values."""
    import torch
    from paper_1503_00576_amd import api, autotune, synth
    spec = synth.BatchSpec(graphs=graphs_n, seed=0)
    t0 = time.perf_counter()
    graphs = synth.batch_graphs(spec, device=dev)
    packed = synth.pack_symmetric(graphs, device=dev)
    b = api.Batch(packed["vtx_off"], packed["adj_off"], packed["row_ptr"], packed["col"],
                  packed["G"], packed["n_total"], packed["adj_total"])
    edges = packed["adj_total"] // 2
    torch.cuda.synchronize()
    log(f"batch: {b.G} graphs, {b.n_total} vertices, {edges} edges in "
        f"{time.perf_counter() - t0:.1f} s")
    log("tuning")
    best, timings = autotune.tune_batched(b)
    log(f"tuned: {best} ({min(t for _, t in timings):.3f} ms)")
    plan = api.BatchPlan(b.G, b.n_total, b.adj_total, best, device=dev)
    res = plan.run_async(b)
    torch.cuda.synchronize()
    res.check()
    totals = res.totals.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run_async(b, out=res)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3 / steps
    assert torch.equal(res.totals, totals)
    log(f"plan: {batch_ms:.3f} ms per batch")
    # per-vertex counts of the same batch (one replay of the per-vertex plan)
    pv_res = plan.run_async(b, per_vertex=True)
    torch.cuda.synchronize()
    pv_res.check()
    ref = golden("batch4096.json") if graphs_n == 4096 else None
    gmatch = None
    if ref is not None:
        gmatch = {"totals": totals.cpu().tolist() == ref["totals"],
                  "per_vertex_sha256": pv_digest(pv_res.per_vertex) == ref["per_vertex_sha256"]}
        log(f"batched golden match: {gmatch}")
    out = {"graphs": b.G, "vertices": b.n_total, "edges": edges,
           "triangles": int(totals.sum().item()), "ms_per_batch": round(batch_ms, 3),
           "graphs_per_s": b.G / (batch_ms * 1e-3), "edges_per_s": edges / (batch_ms * 1e-3),
           "golden_match": gmatch, "tuning": best,
           "tuning_ms": [[t, round(ms, 3)] for t, ms in timings]}
    if not loop:
        plan.close()
        return out
    # the plain per-graph loop: one tc_count per graph, workspace sized for the largest
    nmax = max(n for _, n in graphs)
    mmax = max(int(e.shape[0]) for e, _ in graphs)
    ws = api.alloc_workspace(nmax, mmax, False, dev)
    outs = [api.Result(torch.empty(1, dtype=torch.int64, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev)) for _ in graphs]
    for (e, n), o in zip(graphs, outs):
        api.count_async(e, n, workspace=ws, out=o)
    torch.cuda.synchronize()
    loop_totals = torch.cat([o.total for o in outs])
    assert torch.equal(loop_totals, totals), "batched and per-graph totals differ"
    t0 = time.perf_counter()
    for (e, n), o in zip(graphs, outs):
        api.count_async(e, n, workspace=ws, out=o)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3
    plan.close()
    out.update({"loop_ms": round(loop_ms, 3), "loop_graphs_per_s": b.G / (loop_ms * 1e-3),
                "speedup_vs_loop": round(loop_ms / batch_ms, 2)})
    return out


def serve_section(dev, duration: float, rate: float, seed: int = 0):
    """Poisson arrivals (rate per second, `duration` seconds); 90% R-MAT scale 10-14, 9% scale
    17-19, 1% scale 21, edgefactor 16, drawn from a seeded pool per scale (bounded generation
    time).  Each request carries its edge array in pinned host memory and is processed in full
    (copy to the device, preprocessing, count); every result is checked against the oracle's
    stored count of its pool graph."""
    import concurrent.futures as cf
    import threading
    import torch
    from paper_1503_00576_amd import serve, synth
    times, u = synth.poisson_trace(rate, duration, seed)
    times, u = times.tolist(), u.tolist()
    ref = golden("serve_pool.json")
    pool = {}
    t0 = time.perf_counter()
    for sc, k in synth.SERVE_POOL.items():
        pool[sc] = []
        for i in range(k):
            e, n = synth.serve_pool_graph(sc, i, device=dev)
            pool[sc].append((e.cpu().pin_memory(), n))
    torch.cuda.synchronize()
    log(f"serve: {len(times)} arrivals, pool generated in {time.perf_counter() - t0:.1f} s")
    picks = [synth.serve_pick(i, x) for i, x in enumerate(u)]
    reqs = [pool[sc][i] for sc, i in picks]
    futs = [None] * len(reqs)
    srv = serve.Server(dev, budget_bytes=32 << 30, streams=4, small_edges=1 << 18,
                       batch_graphs=512, max_inflight=8)
    start = time.perf_counter() + 0.5

    def producer():
        for i, ((e, n), t) in enumerate(zip(reqs, times)):
            delay = start + t - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            futs[i] = srv.submit(serve.Request(e, n, arrival=start + t))

    th = threading.Thread(target=producer)
    th.start()
    last_log = time.perf_counter()
    while th.is_alive():
        th.join(timeout=5.0)
        if time.perf_counter() - last_log > 10:
            log(f"serve: {srv.stats['completed']} completed")
            last_log = time.perf_counter()
    pending, waited = set(futs), 0.0
    while pending and waited < 240.0:
        done, pending = cf.wait(pending, timeout=10.0)
        waited += 10.0 if pending else 0.0
        log(f"serve: {len(futs) - len(pending)} of {len(futs)} finished")
    if pending:
        raise RuntimeError(f"serve: {len(pending)} requests unfinished after the trace")
    lat, ok, failed, checked, wrong = [], 0, 0, 0, 0
    for f, (sc, i) in zip(futs, picks):
        try:
            tot, l = f.result(timeout=0)
            lat.append(l)
            ok += 1
            if ref is not None:
                checked += 1
                wrong += int(tot != ref[str(sc)][i]["total"])
        except Exception:
            failed += 1
    makespan = time.perf_counter() - start
    stats = dict(srv.stats)
    srv.close()
    edges = sum(int(e.shape[0]) for e, _ in reqs)
    return {"requests": len(reqs), "completed": ok, "failed": failed,
            "golden_match": (wrong == 0 and checked == ok) if ref is not None else None,
            "checked": checked, "mismatches": wrong,
            "duration_s": duration, "rate_per_s": rate, "makespan_s": round(makespan, 3),
            "graphs_per_s": ok / makespan, "edges_per_s": edges / makespan,
            "p50_ms": round(1e3 * serve.percentile(lat, 50), 3),
            "p99_ms": round(1e3 * serve.percentile(lat, 99), 3),
            "max_ms": round(1e3 * max(lat), 3) if lat else None,
            "batches": stats.get("batches", 0),
            "batched_requests": stats.get("batched_requests", 0),
            "single_requests": stats.get("single", 0), "rejected": stats.get("rejected", 0)}


def _time(fn, reps: int = 3) -> float:
    """Median milliseconds of fn() (enqueues work on the current stream), HIP events."""
    import torch
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[len(ts) // 2]


def split_section(dev, parts=(1, 3, 5, 8), workload="rmat23"):
    """Graphs beyond device memory: the headline graph counted through tc_split_prepare (host:
    checks, pre-filter, partition into K parts, edges bucketed by block into pinned memory) and
    tc_split_count (device: every subgraph's blocks copied in on a second stream while the
    previous one is counted, signed sum), per K: the host pass, the device time from the first
    copy to the total (median of 3, HIP events), the device workspace against the one-graph
    path's, and the total against the stored oracle total."""
    import torch
    from paper_1503_00576_amd import api
    edges, n = make_graph(workload, dev)
    m = int(edges.shape[0])
    host = edges.cpu().numpy()
    del edges
    torch.cuda.empty_cache()
    g = (golden("workloads.json") or {}).get(GOLDEN_KEYS[workload])
    want = g["total"] if g else None
    whole = api.workspace_size(n, m)
    out = {"workload": WORKLOADS[workload]["label"], "n": n, "m": m,
           "one_graph_workspace_bytes": whole, "parts": {}}
    for K in parts:
        t0 = time.perf_counter()
        sp = api.Split(host, n, parts=K, device_budget=0)
        prep_s = time.perf_counter() - t0
        ws = torch.empty(max(sp.info["device_bytes"], 256), dtype=torch.uint8, device=dev)
        total = int(sp.count_async(dev, workspace=ws).check().total.item())
        ts = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            r = sp.count_async(dev, workspace=ws)
            b.record()
            torch.cuda.synchronize()
            r.check()
            ts.append(a.elapsed_time(b))
        ms = sorted(ts)[1]
        out["parts"][str(K)] = {
            "subgraphs": sp.info["subgraphs"], "host_prepare_s": round(prep_s, 2),
            "device_ms": round(ms, 2), "intersections_per_s": m / (ms * 1e-3),
            "device_workspace_bytes": sp.info["device_bytes"],
            "workspace_vs_one_graph": round(sp.info["device_bytes"] / whole, 3),
            "max_subgraph_edges": sp.info["max_sub_m"],
            "golden_match": (total == want) if want is not None else None}
        log(f"split K={K}: {sp.info['subgraphs']} subgraphs, {ms:.1f} ms on the device, "
            f"host pass {prep_s:.1f} s, total {'ok' if total == want else total}")
        del ws, sp
        torch.cuda.empty_cache()
    return out


def ablation_section(dev, workloads=("rmat20", "rmat23")):
    """The paper's own counting design (Section 3.3: one thread per oriented edge, two-pointer
    merge) and its Section 3.4 optimisations on this GPU, beside the shipped kernels: every
    yardstick count is checked against the stored oracle total."""
    import torch
    from paper_1503_00576_amd import ablation as ab
    from paper_1503_00576_amd import api
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    out = {}
    for wl in workloads:
        edges, n = make_graph(wl, dev)
        m = int(edges.shape[0])
        g = (golden("workloads.json") or {}).get(GOLDEN_KEYS[wl])
        want = g["total"] if g else None
        prep = api.Prepared(edges, n)
        shipped_total = prep.count()
        res = api.Result(torch.empty(1, dtype=torch.int64, device=dev),
                         torch.empty(1, dtype=torch.int32, device=dev))
        shipped_ms = _time(lambda: prep.count_async(out=res))
        pre_ms = _time(lambda: api.Prepared(edges, n, workspace=prep.workspace), reps=3)
        em = ab.EdgeMerge(prep)
        em.zip()
        rows = {}
        variants = [("final loop, SoA, const restrict, 64 x 8/CU", 0, 64, 8),
                    ("two reads per step (preliminary loop)", ab.TWO_READS, 64, 8),
                    ("array of (u, v) structures (not unzipped)", ab.AOS, 64, 8),
                    ("plain pointers (no const restrict)", ab.PLAIN_PTRS, 64, 8),
                    ("half waves (32 of 64 lanes work)", ab.HALF_WAVE, 64, 16),
                    ("256 threads x 2/CU", 0, 256, 2), ("256 threads x 8/CU", 0, 256, 8),
                    ("1024 threads x 1/CU", 0, 1024, 1), ("128 threads x 16/CU", 0, 128, 16)]
        for name, flags, threads, per_cu in variants:
            blocks = per_cu * cus
            tot = em.count(flags, threads, blocks)
            ms = _time(lambda: em.run_async(flags, threads, blocks), reps=2)
            rows[name] = {"ms": round(ms, 3), "match": tot == want if want else None,
                          "vs_shipped": round(ms / shipped_ms, 2)}
            log(f"ablation {wl}: {name}: {ms:.2f} ms")
        # edge sorts of the oriented keys (u, v ranks) in a shuffled order
        a = prep.arrays()
        b = a["id_bits"]
        perm = torch.randperm(m, device=dev, generator=torch.Generator(device=dev).manual_seed(0))
        u0 = a["src"][perm].contiguous()
        v0 = a["col"][perm].contiguous()
        del perm
        sorts = {}
        pairs = torch.empty(2 * m, dtype=torch.int32, device=dev)
        pv = pairs.view(m, 2)

        def fill_pairs():
            pv[:, 0].copy_(u0)
            pv[:, 1].copy_(v0)
        fill_pairs()
        temp = ab.sort_async(ab.SORT_PAIRS_COMPARE, b, pairs)
        ts = []
        for _ in range(2):
            fill_pairs()
            torch.cuda.synchronize()
            ts.append(_time(lambda: ab.sort_async(ab.SORT_PAIRS_COMPARE, b, pairs, temp=temp),
                            reps=1))
        sorts["pairs, comparison merge sort (library)"] = round(min(ts), 3)
        del pairs, pv, temp
        ua, va = torch.empty_like(u0), torch.empty_like(v0)
        ua2, va2 = torch.empty_like(u0), torch.empty_like(v0)
        ua.copy_(u0)
        va.copy_(v0)
        temp = ab.sort_async(ab.SORT_PAIRS_RADIX, b, ua, va, ua2, va2)
        ts = []
        for _ in range(3):
            ua.copy_(u0)
            va.copy_(v0)
            torch.cuda.synchronize()
            ts.append(_time(lambda: ab.sort_async(ab.SORT_PAIRS_RADIX, b, ua, va, ua2, va2, temp),
                            reps=1))
        sorts["pairs, two radix passes over (key, value) arrays (library)"] = round(sorted(ts)[1], 3)
        del ua, va, ua2, va2, temp
        keys = (u0.to(torch.int64) << b) | v0.to(torch.int64)
        work, out_k = torch.empty_like(keys), torch.empty_like(keys)
        temp = ab.sort_async(ab.SORT_PACKED_RADIX, b, keys, None, out_k)
        sorts["packed 64-bit keys, radix (library)"] = round(
            _time(lambda: ab.sort_async(ab.SORT_PACKED_RADIX, b, keys, None, out_k, temp=temp)), 3)
        ts = []
        for _ in range(3):
            work.copy_(keys)
            torch.cuda.synchronize()
            ts.append(_time(lambda: api.sort_u64(work, 2 * b), reps=1))
        sorts["packed 64-bit keys, libtc radix sort (tc_sort_u64)"] = round(sorted(ts)[1], 3)
        del keys, work, out_k, temp, u0, v0, a
        out[wl] = {"n": n, "m": m, "triangles_shipped": shipped_total,
                   "shipped_count_ms": round(shipped_ms, 3),
                   "shipped_preprocess_ms": round(pre_ms, 3),
                   "golden_match": (shipped_total == want) if want else None,
                   "edge_merge": rows, "edge_sort_ms": sorts}
        del em, prep, edges
        torch.cuda.empty_cache()
    # random-gather rate (lines per second) by table size and element width
    gather = {}
    sink = torch.empty(1, dtype=torch.int64, device=dev)
    count = 1 << 27
    for mb in (0.03125, 2, 4, 8, 32, 256, 2048):
        table = torch.ones(int(mb * (1 << 20)) // 4, dtype=torch.int32, device=dev)
        row = {}
        for eb in (4, 8, 16):
            ms = _time(lambda: ab.gather_async(table, eb, count, 7, sink))
            row[f"{eb}B"] = round(count / (ms * 1e-3) / 1e9, 1)
        gather[f"{mb:g}MB"] = row
        del table
    out["gather_G_per_s"] = gather
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat23", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="count with the library's default options instead of tuning them")
    ap.add_argument("--options", default=None,
                    help="JSON dict of tc_options fields to count with (no tuning)")
    ap.add_argument("--no-pcie", action="store_true",
                    help="skip the PCIe-inclusive runs (profiling: one counting launch per step)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched measurement (4096 small graphs)")
    ap.add_argument("--batched-only", action="store_true")
    ap.add_argument("--batched-graphs", type=int, default=4096,
                    help="graphs in the batched measurement (profiling runs use fewer)")
    ap.add_argument("--no-loop", action="store_true",
                    help="batched: skip the per-graph tc_count comparison loop")
    ap.add_argument("--serve", action="store_true",
                    help="only run the serving trace (Poisson arrivals of mixed R-MAT graphs)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving trace (profiling runs)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--ablation", action="store_true",
                    help="only run the yardstick: the paper's thread-per-edge merge and its "
                         "Section 3.4 variants at R-MAT scales 20 and 23, edge sorts, and the "
                         "random-gather rate of the chip")
    ap.add_argument("--split", action="store_true",
                    help="only run the graphs-beyond-device-memory path on the headline graph "
                         "(host partition into K parts, subgraphs streamed to the device)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three plain 1 GiB device-to-device copies (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the counting path is single-GPU); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1503_00576_amd import api

    dev = torch.device("cuda:0")
    torch.cuda.init()
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    if args.serve:
        print(json.dumps({"serve": serve_section(dev, args.serve_seconds, args.serve_rate)}),
              flush=True)
        return
    if args.ablation:
        print(json.dumps({"ablation": ablation_section(dev)}), flush=True)
        return
    if args.split:
        print(json.dumps({"split": split_section(dev)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_section(dev, args.steps, args.batched_graphs,
                                                     not args.no_loop)}), flush=True)
        return
    log(f"generating {WORKLOADS[args.workload]['label']}")
    t0 = time.perf_counter()
    edges, n = make_graph(args.workload, dev)
    torch.cuda.synchronize()
    m = int(edges.shape[0])
    log(f"n={n} m={m} generated in {time.perf_counter() - t0:.1f} s")

    # the counting-phase options: given, or picked by the autotuner on this graph
    if args.options:
        opts = json.loads(args.options)
        tuning = {"source": "given", "options": opts}
    elif args.no_tune:
        opts, tuning = None, {"source": "library defaults", "options": api.default_options()}
    else:
        from paper_1503_00576_amd import autotune
        log("tuning the counting-phase options")
        opts, timings = autotune.tune_single(edges, n)
        tuning = {"source": "autotune.tune_single on this graph", "options": opts,
                  "timings_ms": [[t, round(ms, 3)] for t, ms in timings]}
        torch.cuda.empty_cache()
        log(f"tuned: {opts}")
    op = api._opts(opts)
    ws = api.alloc_workspace(n, m, False, dev, opts)
    out = api.Result(torch.empty(1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int32, device=dev))
    L = api._native.lib()
    stream = torch.cuda.current_stream(dev)
    sp = api._stream(dev)
    wsz = ws.numel()

    def step():
        api._raise(L.tc_preprocess(api._ptr(edges), n, m, 0, op, api._ptr(ws), wsz, sp, None),
                   "tc_preprocess")
        api._raise(L.tc_count_prepared(n, m, 0, op, api._ptr(ws), wsz, sp, api._ptr(out.total),
                                       None, api._ptr(out.status)), "tc_count_prepared")

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    total = None
    if args.warmup > 0:
        out.check()
        total = int(out.total.item())

    # per step: start, end of preprocessing (= start of counting), end of counting, all on the
    # stream the library enqueues on
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        api._raise(L.tc_preprocess(api._ptr(edges), n, m, 0, op, api._ptr(ws), wsz, sp, None),
                   "tc_preprocess")
        ev[i][1].record(stream)
        api._raise(L.tc_count_prepared(n, m, 0, op, api._ptr(ws), wsz, sp, api._ptr(out.total),
                                       None, api._ptr(out.status)), "tc_count_prepared")
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out.check()
    if total is None:
        total = int(out.total.item())
    assert int(out.total.item()) == total, "count changed between runs"
    ms_per_step = elapsed * 1e3 / args.steps
    count_ms = sum(b.elapsed_time(c) for _, b, c in ev) / args.steps
    pre_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / args.steps
    step_ev = sorted(a.elapsed_time(c) for a, _, c in ev)
    step_mean = sum(step_ev) / len(step_ev)
    step_stats = {"mean": round(step_mean, 4), "median": round(step_ev[len(step_ev) // 2], 4),
                  "sd": round((sum((x - step_mean) ** 2 for x in step_ev) / len(step_ev)) ** 0.5, 4),
                  "min": round(step_ev[0], 4), "max": round(step_ev[-1], 4),
                  "source": "HIP events around each step on the library's stream"}
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, counting kernel {count_ms:.3f} ms")

    # graph statistics for the roofline: wedges of the oriented graph W = sum_u C(d+(u), 2)
    # (one membership test each in the middle-vertex formulation), and the elements the
    # kernel actually streams (panels merge the tests of 32 middle vertices)
    prep = api.Prepared(edges, n, options=opts)
    arrs = prep.arrays()
    dplus = (arrs["row_ptr"][1:] - arrs["row_ptr"][:-1]).to(torch.int64)
    wedges = int((dplus * (dplus - 1) // 2).sum().item())
    full_opts = dict(api.default_options(), **(opts or {}))
    p0 = n - min(full_opts["panel_ranks"], n)
    hbase = min(max(n - full_opts["high_ranks"], 0), p0)
    streamed, segments, streamed_low = streamed_elements(arrs["row_ptr"], arrs["col"], p0, hbase)
    del arrs, prep, dplus
    torch.cuda.empty_cache()
    g = (golden("workloads.json") or {}).get(GOLDEN_KEYS[args.workload])
    golden_ok = None if g is None else (g["total"] == total)

    # Roofline of the counting kernel.  achieved / frac: the DRAM-side bytes of one launch
    # (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated, committed under
    # profiles/) over the launch time measured here with HIP events; null when the committed
    # counters were taken on other sources.  algorithmic: 4 B per element the kernel streams
    # + 12 B per segment (its range and panel mask) + the node array and out-lists once.
    ctr = load_counters("k_count", args.workload)
    if ctr and json.loads(ctr.get("options", "{}")) != {k: full_opts[k] for k in
                                                        json.loads(ctr.get("options", "{}"))}:
        ctr = None  # taken with other counting-phase options than the ones timed here
    t_s = count_ms * 1e-3
    alg_bytes = (4.0 * streamed_low + 2.0 * (streamed - streamed_low) + 12.0 * segments +
                 4.0 * (n + 1) + 4.0 * m)
    alg_gbs = alg_bytes / t_s / 1e9
    traffic = ctr["hbm_bytes_per_launch"] if ctr else None
    if traffic:
        achieved, basis = traffic / t_s / 1e9, "counter bytes (FETCH_SIZE, WRITE_SIZE) / kernel time"
    else:
        achieved, basis = alg_gbs, ("algorithmic bytes / kernel time (no counters for these "
                                    "sources and options)")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "basis": basis, "kernel": "k_count<false>", "kernel_ms": round(count_ms, 4),
                "l2_hit_rate": (round(ctr["l2_hit_rate"], 4)
                                if ctr and "l2_hit_rate" in ctr else None),
                "algorithmic": {"bytes": alg_bytes, "gbs": round(alg_gbs, 1),
                                "frac": round(alg_gbs / HBM_PEAK_GBS, 4),
                                "streamed_elements": streamed,
                                "streamed_below_hbase": streamed_low, "segments": segments,
                                "unit": "2 B per streamed element (4 B below the 16-bit "
                                        "region) + 12 B per segment + 4 B per CSR entry and "
                                        "row offset"},
                "logical_wvtx": {"bytes": 4.0 * wedges, "gbs": round(4.0 * wedges / t_s / 1e9, 1),
                                 "note": "4 B per wedge of the oriented graph (one membership "
                                         "test each without panels); context, not a bandwidth"}}

    # per-vertex counts (T(x) for every vertex, for clustering coefficients): the counting
    # phase with per-vertex output on the prepared graph, HIP events around each launch
    pv_out = torch.empty(n, dtype=torch.int64, device=dev)
    pv_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(3)]
    for a, b in pv_ev:
        a.record(stream)
        api._raise(L.tc_count_prepared(n, m, 0, op, api._ptr(ws), wsz, sp, api._ptr(out.total),
                                       api._ptr(pv_out), api._ptr(out.status)),
                   "tc_count_prepared")
        b.record(stream)
    torch.cuda.synchronize()
    out.check()
    pv_sum = int(pv_out.sum().item())
    assert int(out.total.item()) == total and pv_sum == 3 * total, "per-vertex counts"
    pv_ms = sorted(a.elapsed_time(b) for a, b in pv_ev)[1]
    pv_golden = None if g is None or "per_vertex_sha256" not in g else \
        (pv_digest(pv_out) == g["per_vertex_sha256"])
    # the one-shot call (preprocessing without panels + per-vertex counting)
    for a, b in pv_ev:
        a.record(stream)
        api._raise(L.tc_count_per_vertex(api._ptr(edges), n, m, 0, op, api._ptr(ws), wsz, sp,
                                         api._ptr(out.total), api._ptr(pv_out),
                                         api._ptr(out.status)), "tc_count_per_vertex")
        b.record(stream)
    torch.cuda.synchronize()
    out.check()
    assert int(out.total.item()) == total and int(pv_out.sum().item()) == 3 * total
    pv1_ms = sorted(a.elapsed_time(b) for a, b in pv_ev)[1]
    per_vertex = {"count_ms": round(pv_ms, 4), "one_shot_ms": round(pv1_ms, 4),
                  "sum_equals_3T": pv_sum == 3 * total, "golden_match": pv_golden,
                  "note": "count_ms: counting phase with per-vertex output on the prepared "
                          "graph (tc_count_prepared with d_per_vertex); one_shot_ms: "
                          "tc_count_per_vertex, preprocessing included; medians of 3"}
    del pv_out
    log(f"per-vertex counting: {pv_ms:.3f} ms on the prepared graph, {pv1_ms:.3f} ms one-shot")

    pcie_inclusive = None
    if not args.no_pcie:
        pcie_inclusive = pcie_section(edges, n, m, total, ws, out, L, sp, op)
        log(f"PCIe-inclusive step: {pcie_inclusive['ms']:.3f} ms")

    res = {
        "metric": "oriented-edge intersections/s",
        "value": m / (ms_per_step * 1e-3),
        "unit": "intersections/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32/uint64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload]["label"], "n": n, "m": m,
                   "triangles": total, "golden_match": golden_ok, "wedges": wedges,
                   "parallelism": "single GPU"},
        "tuning": tuning,
        "count_kernel_intersections_per_s": m / (count_ms * 1e-3),
        "stages_ms": {"preprocess": round(pre_ms, 4), "count": round(count_ms, 4)},
        "step_ms": step_stats,
        "pcie_inclusive": pcie_inclusive,
        "per_vertex": per_vertex,
        "triangles_per_s": total / (ms_per_step * 1e-3),
        "roofline": roofline,
        "cpu_baseline": None,
        "batched": None,
        "serve": None,
    }
    del ws
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched: 4096 graphs ...")
        res["batched"] = batched_section(dev, args.steps)
        log("batched done")
    if not args.no_serve:
        log(f"serving: {args.serve_seconds:.0f} s of Poisson arrivals at {args.serve_rate:.0f}/s")
        res["serve"] = serve_section(dev, args.serve_seconds, args.serve_rate)
        log("serving done")
    res["golden_match"] = {"headline_total": golden_ok,
                           "headline_per_vertex": per_vertex["golden_match"],
                           "batched": (res["batched"] or {}).get("golden_match"),
                           "serve": (res["serve"] or {}).get("golden_match")}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample) ...")
        res["cpu_baseline"] = cpu_baseline(dev)
        log("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
