"""Autotuners for the work distribution of the counting kernels.

Batched plans (tune_batched): "chunk_e", the number of consecutive forward edges in one work
item of the edge-per-lane path, "items_k", the number of out-neighbours of one larger vertex
handled by one work item, and "light_max", the forward degree up to which a vertex takes the
edge-per-lane path.  The tuner captures one plan per candidate and replays it on the caller's
batch.

Single graphs (tune_single): the options of tc_options that shape the counting phase --
"panel_ranks" (how many top ranks are counted as panels of 32 middle vertices),
"wave_item_edges" and "block_item_edges" (in-edges per work item of the per-wave and the
per-workgroup queue).  The tuner times the whole step (tc_preprocess + tc_count_prepared) on
the caller's graph for every candidate, in one workspace large enough for all of them.

Both keep the fastest candidate (for single graphs the library defaults when they come within
TIE of it) and can cache the choice in a JSON file, keyed by the device
and a size class of the input (sizes by powers of two, and the share of the work in the
heaviest rows, which decides how much the panel region and the heavy path matter)."""
from __future__ import annotations

import json
import os

import torch

from . import api

# batched plan
CHUNK_E = (256, 512, 1024, 1536)
ITEMS_K = (64, 256, 1024)
LIGHT_MAX = (64, 128, 256)

# single graph
PANEL_RANKS = (0, 8192, 16384, 32736)
WAVE_ITEM_EDGES = (256, 512, 1024)
BLOCK_ITEM_EDGES = (4096, 16384, 65536)
TIE = 0.005  # relative margin within which the library defaults are kept


def _device_key(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def _bucket(x: float) -> int:
    """Size class: the power of two of x (0 for x < 1)."""
    return int(x).bit_length()


def _batch_key(device, b: api.Batch) -> str:
    """Device, batch sizes, and the degree profile: the share of adjacency entries in rows of
    more than 256 entries (the heavy path's share), in tenths."""
    rp = b.row_ptr.to(torch.int64)
    # per-graph row offsets are local; lengths are differences inside each graph's block
    lens = rp[1:] - rp[:-1]
    heavy = int(lens[lens > 256].sum().item()) if b.adj_total else 0
    share = int(10 * heavy / max(b.adj_total, 1))
    shape = f"G{_bucket(b.G)}-N{_bucket(b.n_total)}-A{_bucket(b.adj_total)}-H{share}"
    return f"{_device_key(device)}|batched|{shape}"


def _load(cache):
    if cache and os.path.exists(cache):
        with open(cache) as f:
            return json.load(f)
    return {}


def _store(cache, key, best, timings):
    if not cache:
        return
    saved = _load(cache)
    saved[key] = {"best": best, "timings": timings}
    with open(cache, "w") as f:
        json.dump(saved, f, indent=1)


def time_plan(plan: api.BatchPlan, b: api.Batch, reps: int = 3) -> float:
    """Median milliseconds of one replay."""
    plan.run_async(b)
    torch.cuda.synchronize(plan.device)
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        plan.run_async(b)
        e.record()
        torch.cuda.synchronize(plan.device)
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2]


def tune_batched(b: api.Batch, reps: int = 3, cache: str | None = None,
                 candidates=None) -> tuple[dict, list]:
    """Returns (best tuning dict, [(tuning, ms), ...])."""
    device = b.vtx_off.device
    key = _batch_key(device, b)
    saved = _load(cache)
    if key in saved:
        return saved[key]["best"], saved[key]["timings"]
    cands = candidates or [{"chunk_e": c, "items_k": k, "light_max": lm}
                           for c in CHUNK_E for k in ITEMS_K for lm in LIGHT_MAX]
    timings = []
    for t in cands:
        plan = api.BatchPlan(b.G, b.n_total, b.adj_total, t, device=device)
        timings.append((t, time_plan(plan, b, reps)))
        plan.close()
    best = min(timings, key=lambda x: x[1])[0]
    _store(cache, key, best, timings)
    return best, timings


def _single_key(device, edges: torch.Tensor, n: int) -> str:
    m = int(edges.shape[0])
    return f"{_device_key(device)}|single|n{_bucket(n)}-m{_bucket(m)}-d{_bucket(2 * m / max(n, 1))}"


def time_step(edges: torch.Tensor, n: int, options: dict, workspace: torch.Tensor,
              reps: int = 2) -> float:
    """Median milliseconds of tc_preprocess + tc_count_prepared with these options."""
    dev = edges.device
    out = api.Result(torch.empty(1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int32, device=dev))
    api.Prepared(edges, n, workspace=workspace, options=options).count_async(out=out)
    torch.cuda.synchronize(dev)
    out.check()
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        api.Prepared(edges, n, workspace=workspace, options=options).count_async(out=out)
        e.record()
        torch.cuda.synchronize(dev)
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2]


def tune_single(edges: torch.Tensor, n: int, reps: int = 2, cache: str | None = None,
                candidates=None) -> tuple[dict, list]:
    """Returns (best options dict, [(options, ms), ...]) for counting this graph's totals."""
    device = edges.device
    key = _single_key(device, edges, n)
    saved = _load(cache)
    if key in saved:
        return saved[key]["best"], saved[key]["timings"]
    m = int(edges.shape[0])
    cands = candidates or [{"panel_ranks": min(p, n), "wave_item_edges": a, "block_item_edges": b}
                           for p in PANEL_RANKS for a in WAVE_ITEM_EDGES
                           for b in BLOCK_ITEM_EDGES]
    uniq = []
    for c in cands:
        if c not in uniq:
            uniq.append(c)
    need = max(api.workspace_size(n, m, options=c) for c in uniq)
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    timings = [(c, time_step(edges, n, c, ws, reps)) for c in uniq]
    del ws
    best = _prefer_defaults(timings)
    _store(cache, key, best, timings)
    return best, timings


def _prefer_defaults(timings, tie: float = TIE) -> dict:
    """The fastest candidate, or the library defaults when they are within `tie` of it (the
    candidates near the top often differ by less than the run-to-run spread)."""
    best, best_ms = min(timings, key=lambda x: x[1])
    defaults = api.default_options()
    for c, ms in timings:
        if all(defaults.get(k) == v for k, v in c.items()) and ms <= best_ms * (1.0 + tie):
            return c
    return best
