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
 *     neighbour ids, worked through one after another; it changes tc_workspace_size and must
 *     not change between a tc_preprocess and the calls that use its workspace.
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
    TC_E_ASYMMETRIC = 5, /* TC_EDGES_BOTH: m odd, or not exactly m/2 forward entries */
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

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
