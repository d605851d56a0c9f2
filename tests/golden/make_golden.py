"""Writes the stored expected values: the oracle's exact results for the seeded synthetic
workloads, with the sha256 of the generated edge bytes so a consumer can confirm it
regenerated the same graph.  Only oracle/ computes the values; synth only makes the inputs.

  python tests/golden/make_golden.py            # ER(1000, 0.02), R-MAT scales 16 and 20
  python tests/golden/make_golden.py --c3       # also R-MAT scale 23, edgefactor 24 (slow)
  python tests/golden/make_golden.py --batch    # the 4096-graph BA/WS batch -> batch4096.json
  python tests/golden/make_golden.py --pool     # the serving request pool -> serve_pool.json
  python tests/golden/make_golden.py --only-new # with --batch / --pool: skip workloads.json

Per-vertex arrays are stored as the sha256 of their little-endian uint64 bytes (vertex-id
order), plus a sample of values and the sum.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import hashlib  # noqa: E402

import oracle  # noqa: E402
from paper_1503_00576_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "workloads.json")
BATCH_PATH = os.path.join(HERE, "batch4096.json")
POOL_PATH = os.path.join(HERE, "serve_pool.json")


def pv_digest(pv: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(pv, dtype="<u8").tobytes()).hexdigest()


def entry(name, e, n, per_vertex_sample=True):
    t = time.time()
    tot, pv = oracle.count(e, n, per_vertex=True)
    dt = time.time() - t
    rec = {"n": n, "m": int(e.shape[0]), "sha256": synth.edges_sha256(e), "total": tot,
           "oracle_seconds": round(dt, 3), "per_vertex_sha256": pv_digest(pv)}
    if per_vertex_sample:
        q = np.unique(np.linspace(0, n - 1, 257).astype(np.int64))
        rec["per_vertex_sample"] = {str(int(v)): int(pv[v]) for v in q}
        rec["per_vertex_sum"] = int(pv.sum())
        rec["per_vertex_max"] = int(pv.max()) if n else 0
    print(name, {k: v for k, v in rec.items() if k != "per_vertex_sample"}, flush=True)
    return rec


def batch_entry(spec: synth.BatchSpec) -> dict:
    """Per-graph totals and the digest of the concatenated per-vertex counts (union order)."""
    t = time.time()
    graphs = synth.batch_graphs(spec)
    h = hashlib.sha256()
    for e, n in graphs:
        h.update(np.int64(n).tobytes())
        h.update(np.ascontiguousarray(e.numpy()).tobytes())
    gen = time.time() - t
    totals, pvs = [], []
    t = time.time()
    for e, n in graphs:
        tot, pv = oracle.count(e, n, per_vertex=True)
        totals.append(tot)
        pvs.append(pv)
    dt = time.time() - t
    pv = np.concatenate(pvs)
    rec = {"graphs": spec.graphs, "seed": spec.seed,
           "n_total": int(sum(n for _, n in graphs)),
           "edges": int(sum(int(e.shape[0]) for e, _ in graphs)),
           "inputs_sha256": h.hexdigest(), "totals": totals, "total": int(sum(totals)),
           "per_vertex_sha256": pv_digest(pv), "per_vertex_sum": int(pv.sum()),
           "oracle_seconds": round(dt, 3), "generate_seconds": round(gen, 3)}
    print("batch", {k: v for k, v in rec.items() if k != "totals"}, flush=True)
    return rec


def pool_entry() -> dict:
    out = {}
    for sc, k in synth.SERVE_POOL.items():
        out[str(sc)] = []
        for i in range(k):
            e, n = synth.serve_pool_graph(sc, i)
            t = time.time()
            tot = oracle.count(e, n)
            dt = time.time() - t
            out[str(sc)].append({"seed": synth.serve_pool_seed(sc, i), "n": n,
                                 "m": int(e.shape[0]), "sha256": synth.edges_sha256(e),
                                 "total": tot, "oracle_seconds": round(dt, 3)})
            print("pool", sc, i, out[str(sc)][-1], flush=True)
            del e
    return out


def main():
    if "--only-new" not in sys.argv:
        out = json.load(open(PATH)) if os.path.exists(PATH) else {}
        e, n = synth.er_1000()
        out["er_1000_p0.02_s0"] = entry("er", e, n)
        for scale, ef in [(16, 16), (20, 16)]:
            e, n = synth.rmat_graph(scale, ef, seed=0)
            out[f"rmat_s{scale}_ef{ef}_s0"] = entry(f"rmat{scale}", e, n)
            del e
        if "--c3" in sys.argv:
            e, n = synth.rmat_graph(23, 24, seed=0)
            out["rmat_s23_ef24_s0"] = entry("rmat23", e, n)
            del e
        with open(PATH, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
    if "--batch" in sys.argv:
        rec = batch_entry(synth.BatchSpec(graphs=4096, seed=0))
        with open(BATCH_PATH, "w") as f:
            json.dump(rec, f, indent=0)
    if "--pool" in sys.argv:
        rec = pool_entry()
        with open(POOL_PATH, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
