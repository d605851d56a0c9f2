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
 *   - Tuning and test options of the single-graph path are explicit arguments (tc_options
 *     below; NULL means the defaults).  The library reads no environment variables.
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
    TC_E_HIP = 9,        /* a HIP runtime call (launch) failed */
    TC_E_MISMATCH = 10,  /* tc_count_prepared on a workspace that tc_preprocess did not fill
                            for the same (n, m, flags, options) */
    TC_E_SCRATCH = 11    /* tc_count_noalloc: the graph's workspace exceeds the static
                            scratch (TC_NOALLOC_SCRATCH_BYTES) */
} tc_status;

/* Edge-array multiplicity (Section 3.1 reading).
 * TC_EDGES_ONCE: every undirected edge appears once, as (u, v) or (v, u), any order.
 * TC_EDGES_BOTH: the paper's format -- every undirected edge appears twice, once in each
 *                direction, any order; m must be even. */
#define TC_EDGES_ONCE 0u
#define TC_EDGES_BOTH 1u

/* Human-readable name of a status code (static storage). */
const char *tc_strerror(int status);

/* Options of the single-graph path (tc_workspace_size, tc_workspace_layout, tc_preprocess,
 * tc_count, tc_count_per_vertex, tc_count_prepared).  Fill with tc_options_init() and change
 * fields; a NULL pointer means the defaults.  Every field takes part in the workspace layout
 * or in the work lists built by the preprocessing, so tc_workspace_size, tc_preprocess and
 * every tc_count_prepared on one workspace must get equal options: tc_preprocess records a
 * fingerprint of (n, m, flags, options) in the workspace, and tc_count_prepared with other
 * values reports TC_E_MISMATCH through d_status (on the device, before any counting kernel
 * runs).  Values are checked by every entry point (TC_E_ARG when out of range).
 *
 * Counting-phase structure (the intersections of Section 3.3 grouped by the middle vertex v
 * of each triangle u < v < w: N+(v) staged in LDS, the in-neighbours' lists streamed):
 *   panel_ranks       the top ranks of the order of Section 2.2 counted as panels of 32
 *                     consecutive middle vertices; 0..32736, default 32736 (the largest the
 *                     counting kernel's LDS table holds); 0 = no panels.
 *   hub_ranks         the top ranks whose triangles (lowest vertex a hub) are counted as a
 *                     masked int8 matrix product on the matrix cores; 0..65536, default 0 (off).
 *   row_blocks        the in-edge lists split into this many contiguous CSR row blocks,
 *                     counted one after another; 1..8, default 1.
 *   wave_item_edges   in-edges per work item of the per-wave queue; 16..65536, default 512.
 *   block_item_edges  in-edges per work item of the per-workgroup queue; 16..1048576,
 *                     default 65536.
 * Per-item structure of N+(v) (the defaults are the largest values the LDS holds; lower values
 * send items to the other forms, which the tests use to reach every form on small graphs):
 *   wave_bitmap_span  a wave item tests membership in an LDS bitmap when the rank span of
 *                     N+(v) is below this; 0..65504, default 65504.
 *   wave_list_max     otherwise a sorted LDS list when N+(v) has at most this many entries
 *                     (per-vertex counts: at most half of it); 0..2048, default 2048; a list
 *                     that fits neither goes to the per-workgroup queue.
 *   block_bitmap_span a workgroup item uses an LDS bitmap below this span; 0..1048544,
 *                     default 1048544 (totals only).
 *   block_list_max    otherwise a sorted LDS list of at most this many entries (per-vertex:
 *                     at most half), else the list is searched in global memory; 0..32768,
 *                     default 32768.
 * Preprocessing:
 *   degree_partition  1 (default): degrees by a bucket partition of the endpoints and LDS
 *                     counting, edges also placed in cells of id ranges for the orientation;
 *                     0: one atomic per endpoint and orientation in input order (the path that
 *                     graphs beyond the partition's limits, 2^27 vertices or 2^32 endpoints,
 *                     take anyway).
 *   sort_onesweep     0 (default): every radix pass is a histogram pass, a scan and a scatter;
 *                     1: the sort of the oriented edges, when it has at least 2^20 keys,
 *                     uses single-sweep passes (decoupled look-back), except for the last
 *                     pass of the source-only sort, which unzips the keys.
 *   high_ranks        the node array's entries among the top high_ranks ranks are also kept
 *                     as 16-bit offsets, and total counts stream them at two bytes instead of
 *                     four (on R-MAT graphs nearly all streamed entries are such ranks); the
 *                     region is widened to take in the whole panel region.  1..65536, default
 *                     65536; 0: no 16-bit region (panels and totals read 32-bit ranks only).
 *                     The region is also dropped when its padded copy of the node array would
 *                     need 2^32 or more entries.
 *   row_sort          1 (default): the oriented edges are sorted by source only and every
 *                     adjacency list is then sorted in place (per thread, per wave or per
 *                     workgroup by its length), with the duplicate check; graphs of 2^29 or
 *                     more oriented edges, whose lists may exceed the workgroup form's 32768
 *                     entries, take the full sort anyway.  0: the oriented edges are sorted by
 *                     (source, target). */
typedef struct tc_options {
    uint32_t size; /* sizeof(tc_options); set by tc_options_init */
    uint32_t panel_ranks;
    uint32_t hub_ranks;
    uint32_t row_blocks;
    uint32_t wave_item_edges;
    uint32_t block_item_edges;
    uint32_t wave_bitmap_span;
    uint32_t wave_list_max;
    uint32_t block_bitmap_span;
    uint32_t block_list_max;
    uint32_t degree_partition;
    uint32_t sort_onesweep;
    uint32_t high_ranks;
    uint32_t row_sort;
} tc_options;

/* Fills *opts with the defaults.  Returns TC_E_ARG for a NULL pointer. */
int tc_options_init(tc_options *opts);

/* Bytes of device workspace tc_count / tc_count_per_vertex / tc_preprocess need for a graph
 * of n vertices and m edge-array entries in the given format.  Pure host arithmetic; returns
 * 0 when the arguments are invalid. */
size_t tc_workspace_size(int64_t n, int64_t m, uint32_t flags, const tc_options *opts);

/* Triangle count of an edge array (Sections 2.2, 3.2, 3.3).
 *   d_edges : int32[2*m], entry i is the pair (d_edges[2i], d_edges[2i+1])
 *   n       : number of vertices (ids in [0, n); isolated vertices allowed); n = 0 needs m = 0
 *   m       : number of entries in d_edges
 *   flags   : TC_EDGES_ONCE or TC_EDGES_BOTH
 *   d_total : uint64[1], receives the number of triangles
 *   d_status: int32[1] or NULL, receives the data-error status (see above) */
int tc_count(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
             const tc_options *opts, void *d_ws, size_t ws_bytes, void *stream,
             uint64_t *d_total, int32_t *d_status);

/* As tc_count, and also the number of triangles containing each vertex (the quantity behind
 * the clustering coefficient of the paper's introduction):
 *   d_per_vertex: uint64[n]; sum over v equals 3 * (*d_total). */
int tc_count_per_vertex(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                        const tc_options *opts, void *d_ws, size_t ws_bytes, void *stream,
                        uint64_t *d_total, uint64_t *d_per_vertex, int32_t *d_status);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tc_count with the workspace in a static
 * device array of TC_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  Nothing is allocated, by the library or anything it calls; the
 * caller passes only the edges and the outputs, with the arguments and results of tc_count.
 * Graphs whose tc_workspace_size(n, m, flags, opts) exceeds TC_NOALLOC_SCRATCH_BYTES
 * (64 MiB: about 10^6 edges) are rejected with TC_E_SCRATCH before anything is enqueued.
 * The array's address on the current device is looked up once per device on the first call
 * (TC_E_HIP if that fails).  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (each call clears what it needs): calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race and give unspecified
 * results; calls on one stream are ordered and safe. */
#define TC_NOALLOC_SCRATCH_BYTES (64u << 20)
int tc_count_noalloc(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                     const tc_options *opts, void *stream, uint64_t *d_total,
                     int32_t *d_status);

/* Where the preprocessing results live inside the workspace (byte offsets from d_ws), so that
 * callers can inspect the intermediate arrays after tc_preprocess:
 *   deg      uint32[n]    vertex degrees
 *   perm     uint32[n]    perm[r] = the vertex of rank r in the order (degree, id)
 *   rank     uint32[n]    rank[v] = position of v in that order (inverse of perm)
 *   row_ptr  uint32[n+1]  node array of the oriented graph, rows indexed by rank
 *   col      uint32[m_fwd] forward neighbours by rank, every row strictly ascending, followed
 *            by at least 16 entries of padding
 *   src      uint32[m_fwd] the row (source rank) of every entry of col
 *   m_fwd    number of oriented edges (m for TC_EDGES_ONCE, m/2 for TC_EDGES_BOTH) */
typedef struct tc_layout {
    size_t deg, perm, rank, row_ptr, col;
    int64_t m_fwd;
    int32_t id_bits; /* b = bits per packed vertex id in the sort keys */
    size_t src;
} tc_layout;

int tc_workspace_layout(int64_t n, int64_t m, uint32_t flags, const tc_options *opts,
                        tc_layout *out);

/* Run the preprocessing phase of tc_count (degrees, order, orientation, key sort, node
 * array) and build the counting phase's work lists, leaving everything in the workspace at
 * the offsets of tc_workspace_layout.  A graph preprocessed once can be counted any number
 * of times with tc_count_prepared while its workspace stays resident. */
int tc_preprocess(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                  const tc_options *opts, void *d_ws, size_t ws_bytes, void *stream,
                  int32_t *d_status);

/* Counting phase only (Section 3.3), on a workspace filled by tc_preprocess with the same
 * (n, m, flags, options) and enqueued after it (same stream, or synchronised); other values
 * give TC_E_MISMATCH in d_status.  d_per_vertex may be NULL (total only).  A data error found
 * by the preprocessing is reported again here.  Calls on one workspace must not overlap on
 * the device (they share its work-queue counters): enqueue them on one stream. */
int tc_count_prepared(int64_t n, int64_t m, uint32_t flags, const tc_options *opts,
                      void *d_ws, size_t ws_bytes, void *stream, uint64_t *d_total,
                      uint64_t *d_per_vertex, int32_t *d_status);

/* Stable ascending LSD radix sort of uint64 keys on their low `bits` bits (1..64); the
 * library's sort of packed edge keys (Section 3.2, step 3), exposed for testing.
 *   d_keys : uint64[count], sorted in place
 *   d_tmp  : uint64[count] scratch
 *   d_ws   : at least tc_sort_workspace_size(count) bytes */
size_t tc_sort_workspace_size(int64_t count);
int tc_sort_u64(uint64_t *d_keys, uint64_t *d_tmp, int64_t count, int32_t bits, void *d_ws,
                size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- graphs beyond the GPU
 *
 * Two extensions for graphs whose working set does not fit in device memory.
 *
 * The host pre-pass of Section 3.4 ("CPU preprocessing for very large graphs"): for
 * two-direction input (TC_EDGES_BOTH) the host computes the degrees and drops the backward
 * entries, so that only half of the array ever reaches the device.
 *
 * Subgraph splitting (the direction Section 6 proposes for graphs that do not fit the GPU),
 * as an exact partition scheme.  The vertices are cut into K parts by a hash of their ids;
 * E_xy (x <= y) are the edges between parts x and y.  The subgraphs G_abc = E_ab + E_ac + E_bc
 * (a < b < c), G_ac = E_aa + E_ac + E_cc (a < c) and E_aa are ordinary graphs counted one after
 * another by tc_count (tc_count_per_vertex) on the device, and
 *     T = sum T(G_abc) + sum T(G_ac) - (K - 2) * sum T(E_aa)      (K >= 2; K = 1: T(E_00)),
 * the same identity holding vertex by vertex.  A subgraph holds about 6m/K^2 edges, so the
 * device working set shrinks about K^2/6 times; the edges cross the host-device link about
 * K + 2 times in all.
 *
 * Usage: tc_split_prepare (host only: checks, pre-filter, partition, edges bucketed by block
 * into the host workspace), then tc_split_count (device).  The host workspace must stay
 * unchanged and alive until the device work of tc_split_count has finished; it should be
 * pinned (hipHostMalloc) for the copies to overlap the counting. */
#define TC_SPLIT_MAX_PARTS 64u

typedef struct tc_split_info {
    uint32_t parts;       /* K */
    uint32_t subgraphs;   /* subgraphs with at least one edge (the ones counted) */
    int64_t m_kept;       /* undirected edges kept: m, or m/2 for TC_EDGES_BOTH */
    int64_t max_sub_n;    /* largest subgraph: vertices */
    int64_t max_sub_m;    /*                   edges */
    size_t device_bytes;  /* device workspace tc_split_count needs */
    size_t host_bytes;    /* host workspace in use */
} tc_split_info;

/* Host workspace bytes for a graph of n vertices and m entries (enough for any K). */
size_t tc_split_host_workspace_size(int64_t n, int64_t m, uint32_t flags);

/* Host pass over the edge array:
 *   h_edges      : int32[2*m] in host memory, the format of tc_count (flags as there)
 *   parts        : K in 1..TC_SPLIT_MAX_PARTS, or 0 = the smallest K (never 2, which splits
 *                  nothing) whose device workspace is at most device_budget bytes
 *   opts         : the options the subgraphs will be counted with (they size the workspace)
 *   h_ws         : at least tc_split_host_workspace_size(n, m, flags) bytes, 64-byte aligned
 *   info         : nullable; receives K, the subgraph count and the device bytes needed
 * Data errors are found here, on the host, and returned directly: TC_E_RANGE, TC_E_SELF_LOOP,
 * TC_E_ASYMMETRIC (two-direction input whose forward entries are not exactly half).  A
 * repeated edge lands in one block and is reported by the device count (TC_E_DUP_EDGE).
 * TC_E_TOO_LARGE: no K fits the budget (or a subgraph exceeds tc_count's limits).
 * Multi-threaded; touches no GPU. */
int tc_split_prepare(const int32_t *h_edges, int64_t n, int64_t m, uint32_t flags,
                     uint32_t parts, size_t device_budget, const tc_options *opts, void *h_ws,
                     size_t h_ws_bytes, tc_split_info *info);

/* Triangle count (and per-vertex counts) of the graph prepared in h_ws, on the device.
 *   d_ws        : at least info.device_bytes, 256-byte aligned
 *   stream      : the counting stream; copy_stream: nullable, a second stream for the
 *                 host-to-device copies of the next subgraph while one is counted (the call
 *                 makes `stream` wait for it at the end)
 *   d_total     : uint64[1]; d_per_vertex: uint64[n] or NULL; d_status: int32[1] or NULL
 *                 (the first data error of any subgraph's count)
 *   opts        : the options given to tc_split_prepare (TC_E_WORKSPACE when they need more)
 * Only enqueues work. */
int tc_split_count(const void *h_ws, const tc_options *opts, void *d_ws, size_t d_ws_bytes,
                   void *stream, void *copy_stream, uint64_t *d_total, uint64_t *d_per_vertex,
                   int32_t *d_status);

/* Inspection of a prepared split (host only, for tests and tools). */
typedef struct tc_split_subgraph_info {
    int64_t n, m;       /* local vertices (the parts' vertices) and edges */
    int64_t coef;       /* +1, or -(K - 2) for a one-part subgraph E_aa */
    uint32_t nparts;    /* 1..3 */
    uint32_t parts[3];  /* ascending */
} tc_split_subgraph_info;

int tc_split_subgraph(const void *h_ws, uint32_t index, tc_split_subgraph_info *out);
/* The subgraph's edge array with local ids (h_out: int32[2*m], nullable) and the global id of
 * every local vertex (h_vertex: int32[n], nullable), exactly as tc_split_count counts it. */
int tc_split_subgraph_edges(const void *h_ws, uint32_t index, int32_t *h_out,
                            int32_t *h_vertex);

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
 * vertex per work item, >= 16, default 256), "light_max" (vertices with at most this many
 * forward neighbours take the edge-per-lane path, 0 .. 256, default 256), "bitmap_span" and
 * "list_max" (a large vertex's N+(u) is an LDS bitmap when its id span is below bitmap_span,
 * 0 .. 65504, default 65504, else a sorted LDS list when it has at most list_max entries,
 * 0 .. 2048, default 2048 (per-vertex: at most 1024), else it is searched in global memory;
 * lower values exist for tests that reach every form on small graphs) and "wgs_per_cu"
 * (workgroups per compute unit, at least 1; values above what the counting kernel's LDS
 * allows, currently 1, are clamped).  Values out of range are clamped.
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

/* Packs G small graphs given as edge arrays (Section 3.1's input, every undirected edge once,
 * either orientation, local ids) into the batched input format above, on the device: one
 * radix sort of two keys per edge (row id in the union, neighbour's local id) orders every
 * row of every graph, and the row boundaries give the offsets.  Serving uses it to turn the
 * edge arrays of the small requests it batches into one tc_count_batched input.
 *   d_vtx_off : int64[G+1], vertex offsets as in tc_count_batched (graph g has n_g vertices)
 *   d_edge_off: int64[G+1], graph g's edges are entries d_edge_off[g] .. d_edge_off[g+1]-1
 *   d_edges   : int32[2*m_total], (u, v) pairs of local ids in [0, n_g)
 * Outputs (overwritten): d_adj_off int64[G+1], d_row_ptr int32[n_total+G], d_col
 * int32[2*m_total] (the first d_adj_off[G] entries used), d_status int32[G]: per graph
 * TC_E_RANGE (an id outside [0, n_g)) or TC_E_SELF_LOOP, in which case only that graph's
 * valid entries are packed, or TC_E_ARG for every graph when the offsets are not prefix sums
 * from 0 to n_total and m_total.  Duplicate edges are packed as they are (tc_count_batched
 * reports them).  Limits: 2*m_total < 2^31 and n_total + G < 2^31 (TC_E_TOO_LARGE).  The
 * workspace holds the sort: tc_batched_pack_workspace_size(G, n_total, m_total) bytes,
 * 256-byte aligned.  Nothing is allocated; the call only enqueues work on `stream`. */
size_t tc_batched_pack_workspace_size(int32_t G, int64_t n_total, int64_t m_total);
int tc_batched_pack(int32_t G, const int64_t *d_vtx_off, const int64_t *d_edge_off,
                    const int32_t *d_edges, int64_t n_total, int64_t m_total, void *d_ws,
                    size_t ws_bytes, void *stream, int64_t *d_adj_off, int32_t *d_row_ptr,
                    int32_t *d_col, int32_t *d_status);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
