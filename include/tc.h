/*
 * tc.h -- exact triangle counting on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of libtc.so.  The library implements the *forward* algorithm of A. Polak,
 * "Counting Triangles in Large Graphs on GPU" (IPDPS Workshops 2016, arXiv 1503.00576):
 * Section 2.2 (order vertices consistently with degree, keep every edge only in its forward
 * direction, sort the adjacency lists, sum the sizes of the lists' pairwise intersections
 * over all remaining edges), with the preprocessing steps of Section 3.2 (degrees, sort of
 * packed 64-bit edge keys, node array = CSR row offsets, removal of backward edges, unzipping
 * into a structure of arrays) and the counting phase of Section 3.3.
 *
 * Conventions for every entry point below
 *   - Pointers named d_* are device pointers (hipMalloc'ed or torch CUDA tensors) on the
 *     current HIP device; the caller owns all of them.  The library never allocates device
 *     memory: it works inside the caller's workspace d_ws of at least tc_workspace_size()
 *     bytes, 256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls only enqueue work;
 *     they never synchronise.  Outputs are overwritten, not accumulated.
 *   - Errors that the host can see (null pointers, sizes out of range, short workspace) are
 *     returned before anything is enqueued.  Errors in the data (an id outside [0, n), a
 *     self-loop, a repeated edge, a missing mirror entry, an unsorted batched row) are found
 *     on the device and written to *d_status (a tc_status value; the first error found wins;
 *     0 when the input is valid).  After a data error the counts are unspecified, but no
 *     kernel reads or writes outside the caller's buffers.
 *   - Vertex ids are int32 in [0, n); n < 2^31 and the number of edge entries m < 2^32.
 *     Counts are exact uint64.
 *   - Tuning: the environment variable TC_ROW_BLOCK_BYTES (unset = one block) splits the
 *     counting phase's in-edge lists into up to 8 row blocks of at most that many bytes of
 *     neighbour ids, worked through one after another.  TC_PANEL_RANKS (unset = the
 *     largest value the counting kernel supports, 32736; 0 = off) sets how many of the
 *     highest ranks of the order of Section 2.2 are counted as panels of 32 consecutive
 *     middle vertices (tc_count_per_vertex prepares without panels, whose lists per-vertex
 *     counts would have to split again).  TC_HUB_RANKS (unset = 0 = off; at most 65536) sets how many of the
 *     highest ranks are hubs, whose triangles (those whose lowest vertex is a hub) are
 *     counted as a masked int8 matrix product on the matrix cores (two hubs x hubs byte
 *     matrices in the workspace).  They change tc_workspace_size and must not change between
 *     a tc_preprocess and the calls that use its workspace.  TC_DEGREE_PARTITION=0 (for
 *     tests) computes degrees with one atomic per endpoint and orients the edges in input
 *     order, the path that graphs of more than 2^27 vertices or 2^32 endpoints take; it
 *     changes tc_workspace_size like the others.  TC_WAVE_BITMAP_SPAN (for tests; unset =
 *     65504, the largest rank span a wave's LDS bitmap holds) lowers the span below which a
 *     middle vertex's out-list is tested as a bitmap rather than a sorted list.
 *     TC_SORT_ONESWEEP=1 switches the radix passes of sorts of at least 2^20 keys to the
 *     single-sweep variant (decoupled look-back instead of a histogram pass and a scan).
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tc_status {
    TC_OK = 0,
    TC_E_ARG = 1,        /* bad argument: null pointer, negative size, bad flags */
    TC_E_RANGE = 2,      /* a vertex id outside [0, n) */
    TC_E_SELF_LOOP = 3,  /* an entry (u, u) */
    TC_E_DUP_EDGE = 4,   /* an undirected edge listed more often than the format allows */
    TC_E_ASYMMETRIC = 5, /* TC_EDGES_BOTH: m odd, or not exactly m/2 forward entries;
                            batched: entries not closed under mirroring (an exact count
                            test plus a sum of 64-bit pair hashes, which misses with
                            probability about 2^-64) */
    TC_E_UNSORTED = 6,   /* batched input: a CSR row not strictly ascending */
    TC_E_WORKSPACE = 7,  /* d_ws smaller than tc_workspace_size() or misaligned */
    TC_E_TOO_LARGE = 8,  /* n >= 2^31 or m >= 2^32 */
    TC_E_HIP = 9         /* a HIP runtime call (launch) failed */
} tc_status;

/* Edge-array multiplicity (Section 3.1 reading).
 * TC_EDGES_ONCE: every undirected edge appears once, as (u, v) or (v, u), any order.
 * TC_EDGES_BOTH: the paper's format -- every undirected edge appears twice, once in each
 *                direction, any order; m must be even. */
#define TC_EDGES_ONCE 0u
#define TC_EDGES_BOTH 1u

/* Human-readable name of a status code (static storage). */
const char *tc_strerror(int status);

/* Bytes of device workspace tc_count / tc_count_per_vertex / tc_preprocess need for a graph
 * of n vertices and m edge-array entries in the given format.  Pure host arithmetic; returns
 * 0 when the arguments are invalid. */
size_t tc_workspace_size(int64_t n, int64_t m, uint32_t flags);

/* Triangle count of an edge array (Sections 2.2, 3.2, 3.3).
 *   d_edges : int32[2*m], entry i is the pair (d_edges[2i], d_edges[2i+1])
 *   n       : number of vertices (ids in [0, n); isolated vertices allowed); n = 0 needs m = 0
 *   m       : number of entries in d_edges
 *   flags   : TC_EDGES_ONCE or TC_EDGES_BOTH
 *   d_total : uint64[1], receives the number of triangles
 *   d_status: int32[1] or NULL, receives the data-error status (see above) */
int tc_count(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags, void *d_ws,
             size_t ws_bytes, void *stream, uint64_t *d_total, int32_t *d_status);

/* As tc_count, and also the number of triangles containing each vertex (the quantity behind
 * the clustering coefficient of the paper's introduction):
 *   d_per_vertex: uint64[n]; sum over v equals 3 * (*d_total). */
int tc_count_per_vertex(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                        void *d_ws, size_t ws_bytes, void *stream, uint64_t *d_total,
                        uint64_t *d_per_vertex, int32_t *d_status);

/* Where the preprocessing results live inside the workspace (byte offsets from d_ws), so that
 * callers can inspect the intermediate arrays after tc_preprocess:
 *   deg      uint32[n]    vertex degrees
 *   perm     uint32[n]    perm[r] = the vertex of rank r in the order (degree, id)
 *   rank     uint32[n]    rank[v] = position of v in that order (inverse of perm)
 *   row_ptr  uint32[n+1]  node array of the oriented graph, rows indexed by rank
 *   col      uint32[m_fwd] forward neighbours by rank, every row strictly ascending
 *   m_fwd    number of oriented edges (m for TC_EDGES_ONCE, m/2 for TC_EDGES_BOTH) */
typedef struct tc_layout {
    size_t deg, perm, rank, row_ptr, col;
    int64_t m_fwd;
    int32_t id_bits; /* b = bits per packed vertex id in the sort keys */
} tc_layout;

int tc_workspace_layout(int64_t n, int64_t m, uint32_t flags, tc_layout *out);

/* Run the preprocessing phase of tc_count (degrees, order, orientation, key sort, node
 * array) and build the counting phase's work lists, leaving everything in the workspace at
 * the offsets of tc_workspace_layout.  A graph preprocessed once can be counted any number
 * of times with tc_count_prepared while its workspace stays resident. */
int tc_preprocess(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags, void *d_ws,
                  size_t ws_bytes, void *stream, int32_t *d_status);

/* Counting phase only (Section 3.3), on a workspace filled by tc_preprocess with the same
 * (n, m, flags) and enqueued after it (same stream, or synchronised).  d_per_vertex may be
 * NULL (total only).  A data error found by the preprocessing is reported again here. */
int tc_count_prepared(int64_t n, int64_t m, uint32_t flags, void *d_ws, size_t ws_bytes,
                      void *stream, uint64_t *d_total, uint64_t *d_per_vertex,
                      int32_t *d_status);

/* Stable ascending LSD radix sort of uint64 keys on their low `bits` bits (1..64); the
 * library's sort of packed edge keys (Section 3.2, step 3), exposed for testing.
 *   d_keys : uint64[count], sorted in place
 *   d_tmp  : uint64[count] scratch
 *   d_ws   : at least tc_sort_workspace_size(count) bytes */
size_t tc_sort_workspace_size(int64_t count);
int tc_sort_u64(uint64_t *d_keys, uint64_t *d_tmp, int64_t count, int32_t bits, void *d_ws,
                size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- batched counting
 *
 * Many independent graphs counted by one launch sequence.  Input: the graphs' symmetric
 * adjacency lists (every undirected edge in both rows, rows strictly ascending; the
 * adjacency-list format of Section 3.1), concatenated:
 *   d_vtx_off: int64[G+1], d_vtx_off[0] = 0; graph g has n_g = d_vtx_off[g+1] - d_vtx_off[g]
 *              vertices, numbered d_vtx_off[g] .. d_vtx_off[g+1]-1 in the union
 *   d_adj_off: int64[G+1], d_adj_off[0] = 0; graph g's adjacency entries are
 *              d_col[d_adj_off[g] .. d_adj_off[g+1])
 *   d_row_ptr: int32[n_total + G]; graph g's n_g + 1 row offsets (0 .. its entry count) are at
 *              d_row_ptr[d_vtx_off[g] + g ..]
 *   d_col    : int32[adj_total], local vertex ids 0 .. n_g - 1
 * Output: d_totals uint64[G] (triangles per graph), d_per_vertex uint64[n_total] (per vertex of
 * the union, nullable), d_status int32[G] (per-graph data error, nullable: range, self-loop,
 * duplicate or unsorted row, missing mirror entry, inconsistent offsets).
 * Method: degree = row length; a stable per-row filter keeps the neighbours later in the
 * order of Section 2.2, so the oriented rows stay sorted without any sort; the counting kernel
 * computes Section 2.2's intersections grouped by u: for a vertex u with more than 256 forward
 * neighbours it stages N+(u) in LDS and streams the lists N+(v) of u's out-neighbours; the
 * other edges are taken in chunks of consecutive forward edges, one edge u -> v per lane,
 * with the chunk's short lists N+(u) staged in LDS and N+(v) streamed through them.
 *
 * A plan binds a workspace of tc_batched_workspace_size(g_cap, n_cap, adj_cap) bytes and
 * captures the whole launch sequence once per mode (with / without per-vertex counts) into a
 * hipGraph on its first run; later runs only write a small argument block and replay the
 * graph, for any batch within the capacities.  tuning_json (nullable) may set "chunk_e"
 * (forward edges per chunk, 64 .. 1536, default 1024), "items_k" (out-neighbours of a large
 * vertex per work item, >= 16, default 256) and "wgs_per_cu" (workgroups per compute unit,
 * at least 1; values above what the counting kernel's LDS allows, currently 1, are clamped).
 * Runs of one plan must not overlap (they share the workspace); the plan must outlive its
 * last run on the GPU.  flags must be 0. */
typedef struct tc_plan tc_plan;

size_t tc_batched_workspace_size(int32_t g_cap, int64_t n_cap, int64_t adj_cap);
int tc_batched_plan_create(int32_t g_cap, int64_t n_cap, int64_t adj_cap, uint32_t flags,
                           const char *tuning_json, void *d_ws, size_t ws_bytes,
                           tc_plan **out);
int tc_batched_plan_run(tc_plan *plan, int32_t G, const int64_t *d_vtx_off,
                        const int64_t *d_adj_off, const int32_t *d_row_ptr, const int32_t *d_col,
                        int64_t n_total, int64_t adj_total, void *stream, uint64_t *d_totals,
                        uint64_t *d_per_vertex, int32_t *d_status);
void tc_batched_plan_destroy(tc_plan *plan);

/* One-shot form: the same launch sequence enqueued directly (no graph capture). */
int tc_count_batched(int32_t G, const int64_t *d_vtx_off, const int64_t *d_adj_off,
                     const int32_t *d_row_ptr, const int32_t *d_col, int64_t n_total,
                     int64_t adj_total, void *d_ws, size_t ws_bytes, void *stream,
                     uint64_t *d_totals, uint64_t *d_per_vertex, int32_t *d_status);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
