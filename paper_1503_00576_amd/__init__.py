"""Exact triangle counting on AMD Instinct MI355X (gfx950): the forward algorithm of
A. Polak, "Counting Triangles in Large Graphs on GPU" (arXiv 1503.00576), as hand-written HIP
kernels behind a C ABI (libtc.so, include/tc.h).

The library is loaded on first use; importing the package (e.g. for ``synth``) does not need
it.  ``api`` holds the binding; ``synth`` the seeded synthetic inputs."""
from .api import (Batch, BatchPlan, BatchResult, EDGES_BOTH, batched_workspace_size, count_batched, EDGES_ONCE, Result, TCError, alloc_workspace, clustering, count,  # noqa: F401
                  count_async, count_per_vertex, layout, Prepared, preprocess, sort_u64, transitivity,
                  workspace_size)
