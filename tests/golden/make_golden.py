"""Writes workloads.json: the oracle's exact results for the seeded synthetic workloads,
with the sha256 of the generated edge bytes so a consumer can confirm it regenerated the
same graph.  Only oracle/ computes the values.

  python tests/golden/make_golden.py            # ER(1000, 0.02) and R-MAT scales 16, 20
  python tests/golden/make_golden.py --c3       # also R-MAT scale 23, edgefactor 24 (slow)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1503_00576_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "workloads.json")


def entry(name, e, n, per_vertex_sample=True):
    t = time.time()
    tot, pv = oracle.count(e, n, per_vertex=True)
    dt = time.time() - t
    rec = {"n": n, "m": int(e.shape[0]), "sha256": synth.edges_sha256(e), "total": tot,
           "oracle_seconds": round(dt, 3)}
    if per_vertex_sample:
        q = np.unique(np.linspace(0, n - 1, 257).astype(np.int64))
        rec["per_vertex_sample"] = {str(int(v)): int(pv[v]) for v in q}
        rec["per_vertex_sum"] = int(pv.sum())
        rec["per_vertex_max"] = int(pv.max()) if n else 0
    print(name, {k: v for k, v in rec.items() if k != "per_vertex_sample"}, flush=True)
    return rec


def main():
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
    with open(PATH, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
