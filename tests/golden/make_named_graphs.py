"""Writes named_graphs.json: small graphs whose triangle counts are known facts of
geometry or of the literature (not computed by any code of this repository).

  octahedron     8  -- the regular octahedron has 8 triangular faces and no other triangles
  icosahedron   20  -- 20 triangular faces, each vertex on 5 of them
  dodecahedron   0  -- pentagonal faces, girth 5
  petersen       0  -- girth 5
  karate        45  -- Zachary's karate-club network (34 members, 78 ties)
  tutte          0  -- cubic, girth 4 graph of Tutte's counterexample
Edges are taken from networkx's constructors; run:  python tests/golden/make_named_graphs.py
"""
import json
import os

import networkx as nx

FACTS = {
    "octahedron": (nx.octahedral_graph, 8, {"per_vertex_all": 4}),
    "icosahedron": (nx.icosahedral_graph, 20, {"per_vertex_all": 5}),
    "dodecahedron": (nx.dodecahedral_graph, 0, {}),
    "petersen": (nx.petersen_graph, 0, {}),
    "karate": (nx.karate_club_graph, 45, {}),
    "tutte": (nx.tutte_graph, 0, {}),
}

out = {}
for name, (ctor, total, extra) in FACTS.items():
    g = ctor()
    nodes = sorted(g.nodes())
    idx = {v: i for i, v in enumerate(nodes)}
    edges = sorted((min(idx[a], idx[b]), max(idx[a], idx[b])) for a, b in g.edges())
    out[name] = {"n": len(nodes), "edges": edges, "total": total, **extra}

here = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(here, "named_graphs.json"), "w") as f:
    json.dump(out, f, indent=0)
print({k: (v["n"], len(v["edges"]), v["total"]) for k, v in out.items()})
