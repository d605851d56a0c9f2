"""Autotuner for the batched counting plan.

The tunables are the work distribution of the batched counting kernel -- "chunk_e", the number
of consecutive forward edges in one work item of the edge-per-lane path (vertices with at most
256 forward neighbours), "items_k", the number of out-neighbours of one larger vertex handled
by one work item -- and "wgs_per_cu", the persistent grid's workgroups per compute unit.  The
tuner captures one plan per candidate, replays it on the caller's batch, keeps the fastest,
and can cache the choice in a JSON file keyed by device and batch shape."""
from __future__ import annotations

import json
import os

import torch

from . import api

CHUNK_E = (256, 512, 1024, 1536)
ITEMS_K = (64, 256, 1024)
WGS_PER_CU = (1,)  # one 1024-thread workgroup per CU is all the LDS holds


def _key(device, b: api.Batch) -> str:
    p = torch.cuda.get_device_properties(device)
    shape = f"G{b.G}-N{b.n_total.bit_length()}-A{b.adj_total.bit_length()}"
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}|{shape}"


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
    key = _key(device, b)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            saved = json.load(f)
        if key in saved:
            return saved[key]["best"], saved[key]["timings"]
    cands = candidates or [{"chunk_e": c, "items_k": k, "wgs_per_cu": w}
                           for c in CHUNK_E for k in ITEMS_K for w in WGS_PER_CU]
    timings = []
    for t in cands:
        plan = api.BatchPlan(b.G, b.n_total, b.adj_total, t, device=device)
        timings.append((t, time_plan(plan, b, reps)))
        plan.close()
    best = min(timings, key=lambda x: x[1])[0]
    if cache:
        saved = {}
        if os.path.exists(cache):
            with open(cache) as f:
                saved = json.load(f)
        saved[key] = {"best": best, "timings": timings}
        with open(cache, "w") as f:
            json.dump(saved, f, indent=1)
    return best, timings
