/*
 * tc_ablation.h -- yardstick kernels for measuring the paper's own GPU design on gfx950.
 *
 * C ABI of libtc_ablation.so, a separate library that the counting path never calls: it
 * exists so that the design choices of A. Polak, "Counting Triangles in Large Graphs on GPU"
 * (arXiv 1503.00576), Section 3.3 (one thread per edge, two-pointer merge of both adjacency
 * lists) and the optimisations of Section 3.4, can be timed on this chip beside libtc's own
 * kernels.  Conventions as in tc.h: d_* are device pointers owned by the caller, `stream` is a
 * hipStream_t, calls only enqueue work, host-visible errors are returned (tc_status values)
 * before anything is enqueued, nothing is allocated.
 */
#ifndef TC_ABLATION_H
#define TC_ABLATION_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Variants of the thread-per-edge merge (flags, combinable):
 *   TCA_TWO_READS   Section 3.4 "Avoiding Unnecessary Reads": the preliminary loop, which loads
 *                   both current list elements in every step (default: the final loop, one new
 *                   element per step except on a match)
 *   TCA_AOS         Section 3.4 "Unzipping Edges": the edges are read as (u, v) pairs from one
 *                   array of structures (d_pairs) instead of two arrays (d_src, d_dst)
 *   TCA_PLAIN_PTRS  Section 3.4 "Read-Only Data Cache": the lists are read through plain
 *                   pointers instead of const __restrict__ ones
 *   TCA_HALF_WAVE   Section 3.4 "Reducing Warp Size": only the lower 32 lanes of every wave
 *                   work (twice the threads for the same work) */
#define TCA_TWO_READS 1u
#define TCA_AOS 2u
#define TCA_PLAIN_PTRS 4u
#define TCA_HALF_WAVE 8u

/* Triangle count by Section 3.3's counting phase: thread t takes the oriented edges
 * t, t + T, t + 2T, ... (T = threads of the grid) and adds the size of the intersection of the
 * sorted lists N+(u) and N+(v) of each, found by a two-pointer merge; per-thread counts are
 * summed into *d_total (uint64, overwritten).  Input: an oriented CSR with every row strictly
 * ascending (libtc's tc_preprocess output: row_ptr, col, src at tc_workspace_layout's offsets).
 *   d_row_ptr uint32[n+1]; d_col uint32[mf + 16] (16 entries of padding: the final loop reads
 *   one element past a list's end); d_src / d_dst uint32[mf] (edge u -> v; d_dst may be d_col);
 *   d_pairs uint32[2 mf] (u, v) pairs, used with TCA_AOS (tca_zip_edges makes it).
 *   threads_per_block in {64, 128, 256, 512, 1024}; blocks >= 1. */
int tca_edge_merge(const uint32_t *d_row_ptr, const uint32_t *d_col, const uint32_t *d_src,
                   const uint32_t *d_dst, const uint32_t *d_pairs, int64_t mf, uint32_t flags,
                   int32_t threads_per_block, int32_t blocks, uint64_t *d_total, void *stream);

/* d_pairs[2e] = d_src[e], d_pairs[2e+1] = d_dst[e] (the array-of-structures edge form). */
int tca_zip_edges(const uint32_t *d_src, const uint32_t *d_dst, int64_t mf, uint32_t *d_pairs,
                  void *stream);

/* Sorts of edges for Section 3.4 "Sorting Edges as 64-bit Integers", all with the ROCm
 * library's device sorts (as the paper used its platform's library sort), ascending by (u, v):
 *   TCA_SORT_PAIRS_COMPARE  d_a: uint32[2 count] (u, v) pairs, comparison merge sort with a
 *                           lexicographic comparator, in place
 *   TCA_SORT_PAIRS_RADIX    d_a: u[count], d_b: v[count]; radix sort by v carrying u, then a
 *                           stable radix sort by u carrying v, on `bits` bits each; results
 *                           back in d_a, d_b (d_a_alt, d_b_alt: scratch of the same sizes)
 *   TCA_SORT_PACKED_RADIX   d_a: uint64[count] keys (u << bits | v), radix sort on 2 bits bits
 *                           into d_a_alt
 * d_temp: tca_sort_temp_bytes(method, count, bits) bytes. */
#define TCA_SORT_PAIRS_COMPARE 0
#define TCA_SORT_PAIRS_RADIX 1
#define TCA_SORT_PACKED_RADIX 2
size_t tca_sort_temp_bytes(int32_t method, int64_t count, int32_t bits);
int tca_sort(int32_t method, int64_t count, int32_t bits, void *d_a, void *d_b, void *d_a_alt,
             void *d_b_alt, void *d_temp, size_t temp_bytes, void *stream);

/* Random-gather rate of the memory system (the ceiling of a kernel bound by random line
 * reads): `count` reads of elem_bytes (4, 8 or 16) at pseudo-random element positions of a
 * table of table_bytes, summed into *d_sink (overwritten) so that no read is dropped. */
int tca_gather(const void *d_table, int64_t table_bytes, int32_t elem_bytes, int64_t count,
               uint32_t seed, uint64_t *d_sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TC_ABLATION_H */
