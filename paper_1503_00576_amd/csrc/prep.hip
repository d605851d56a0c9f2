// Preprocessing phase (Section 3.2) on the device, in "rank space".
//
//   k_part_*     degrees of the vertices (bucket partition + LDS counting) and the input
//                checks of Section 3.1; in the one-direction format the same pass places
//                the edges in cells of id ranges for k_orient_cells
//   k_vkeys      packs (degree, id) so that a stable sort yields the total order of Section 2.2
//                (degree first, ties by id); the position of a vertex in that order is its rank
//                (the sort's last pass writes perm[r] = vertex of rank r, rank[v] = r)
//   k_orient*    every edge becomes a packed key (rank s << b) | rank t with s < t, i.e. the
//                edge kept only in its forward direction (Section 3.2, steps 5-6); in the
//                paper's two-direction format backward entries are dropped
//   k_row_*      with the keys sorted by source only (the sort's last pass unzips them into
//                the neighbour and source arrays, step 7): row boundaries for the node array
//                (steps 4/8: row_ptr[x] = first key whose source is >= x), every row sorted
//                in place with the duplicate check
//   k_csr        the same from keys sorted by (source, target): unzip, boundaries, duplicates
//   k_csc_*      for every vertex v the list of in-edges u -> v with a non-empty suffix of
//                N+(u) after v (the elements that can close a triangle through v), stored
//                as a [begin, end) range;
//                built by a radix sort of (list << 32 | e) keys, so no atomics are needed;
//                from rank p0 on, one list per panel of consecutive middle vertices, with the
//                mask of u's panel vertices per entry
//   k_items_*    work items of the counting kernels (see count.hip)
//
// Working with ranks instead of ids makes the order test a plain comparison, groups the
// high-degree vertices (whose lists are read most often) into one contiguous region, and
// keeps each out-list inside a short range of ranks, which the counting kernels exploit.
#include "internal.h"

namespace tc {

// ---------------------------------------------------------------- degrees
// Degrees are a histogram of the 2m endpoints over n vertices.  Scattered atomics into an
// n-entry array miss the caches on every increment, so the endpoints are first partitioned by
// their high id bits into at most 256 buckets (bucket = x >> sh, a range of 2^sh ids), then
// every bucket is counted in LDS.  The first pass also checks the input (Section 3.1).
constexpr int kPartThreads = 256;
constexpr int kPartEdges = 16;                               // edges per thread
constexpr uint32_t kPartTile = kPartThreads * kPartEdges;    // 4096 edges per tile
constexpr uint32_t kPartWindow = 32768;                      // LDS counters per workgroup
constexpr uint32_t kPartLoads = 4;                           // 16-byte loads in flight per thread

// 16-byte loads and stores with a non-temporal hint (streams touched once)
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 load_nt_u4(const uint4 *p) {
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_nt_u4(uint4 *p, uint4 x) {
    const u32x4_t v = {x.x, x.y, x.z, x.w};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t *>(p));
}

// an edge of the input stream, read once per pass: non-temporal hint
__device__ __forceinline__ int2 load_edge_nt(const int2 *edges, uint64_t i) {
    const uint64_t w = __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(edges) + i);
    return make_int2((int)(uint32_t)w, (int)(uint32_t)(w >> 32));
}

__device__ __forceinline__ bool endpoint_ok(int2 e, uint32_t n) {
    return (uint32_t)e.x < n && (uint32_t)e.y < n && e.x != e.y;
}

// Cells for the orientation's rank lookups (one-direction format): edge (a, b) goes to cell
// (a >> cs) * 16 + (b >> cs), a pair of id ranges of 2^cs ids each, so that the lookups of
// a run of edges of one cell touch two short stretches of the rank array.
__device__ __forceinline__ uint32_t edge_cell(int2 e, int cs) {
    return (((uint32_t)e.x >> cs) << 4) | ((uint32_t)e.y >> cs);
}

// hist: digit-major table of per-tile counts, digits 0..255 the endpoint buckets and, when
// cs >= 0, digits 256..511 the edge cells
__global__ __launch_bounds__(kPartThreads) void k_part_hist(
    const int2 *__restrict__ edges, uint64_t m, uint32_t n, uint32_t both, int sh, int cs,
    uint32_t *__restrict__ hist, uint32_t tiles, int32_t *__restrict__ status) {
    __shared__ uint32_t h[256], hc[256];
    const uint32_t t = threadIdx.x;
    h[t] = 0;
    hc[t] = 0;
    __syncthreads();
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    const uint64_t base = (uint64_t)tile * kPartTile;
    int2 ed[kPartEdges];
#pragma unroll
    for (int r = 0; r < kPartEdges; ++r) {
        uint64_t i = base + (uint64_t)r * kPartThreads + t;
        ed[r] = i < m ? load_edge_nt(edges, i) : make_int2(-1, -1);
    }
#pragma unroll
    for (int r = 0; r < kPartEdges; ++r) {
        uint64_t i = base + (uint64_t)r * kPartThreads + t;
        if (i >= m) continue;
        const int2 e = ed[r];
        if (!endpoint_ok(e, n)) {
            set_status(status, ((uint32_t)e.x >= n || (uint32_t)e.y >= n) ? TC_E_RANGE
                                                                          : TC_E_SELF_LOOP);
            continue;
        }
        atomicAdd(&h[(uint32_t)e.x >> sh], 1u);
        if (!both) atomicAdd(&h[(uint32_t)e.y >> sh], 1u);
        if (cs >= 0) atomicAdd(&hc[edge_cell(e, cs)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)t * tiles + tile] = h[t];
    if (cs >= 0) hist[(uint64_t)(256 + t) * tiles + tile] = hc[t];
}

// Endpoints of one tile placed bucket by bucket in LDS, then written as contiguous runs of
// their offsets inside the bucket (type P: 16 bits when a bucket holds at most 2^16 ids); with
// cs >= 0 the tile's edges then go through the same LDS buffer to their cells' runs (any
// order inside a run).
template <class P>
__global__ __launch_bounds__(kPartThreads) void k_part_scatter(
    const int2 *__restrict__ edges, uint64_t m, uint32_t n, uint32_t both, int sh, int cs,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ offs, uint32_t tiles,
    P *__restrict__ parts, int2 *__restrict__ cells) {
    __shared__ __align__(16) uint32_t s_stage[2 * kPartTile];  // endpoints, then edges (int2)
    __shared__ uint32_t s_fill[256], s_glob[256], s_wsum[kPartThreads / kWave];
    const uint32_t t = threadIdx.x, w = t / kWave;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    const uint32_t c = hist[(uint64_t)t * tiles + tile];
    const uint32_t incl = wave_incl_scan(c);
    if (lane_id() == kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < w; ++k) before += s_wsum[k];
    const uint32_t loc = before + incl - c;
    s_fill[t] = loc;
    s_glob[t] = offs[(uint64_t)t * tiles + tile] - loc;
    __syncthreads();
    const uint64_t base = (uint64_t)tile * kPartTile;
    int2 ed[kPartEdges];
#pragma unroll
    for (int r = 0; r < kPartEdges; ++r) {
        uint64_t i = base + (uint64_t)r * kPartThreads + t;
        ed[r] = i < m ? load_edge_nt(edges, i) : make_int2(-1, -1);
    }
#pragma unroll
    for (int r = 0; r < kPartEdges; ++r) {
        const int2 e = ed[r];
        if (!endpoint_ok(e, n)) continue;  // also the padding beyond m
        s_stage[atomicAdd(&s_fill[(uint32_t)e.x >> sh], 1u)] = (uint32_t)e.x;
        if (!both) s_stage[atomicAdd(&s_fill[(uint32_t)e.y >> sh], 1u)] = (uint32_t)e.y;
    }
    __syncthreads();
    const uint32_t total = s_fill[255];  // end of the last bucket = endpoints in this tile
    const uint32_t omask = (uint32_t)((1ull << sh) - 1);
    for (uint32_t j = t; j < total; j += kPartThreads) {
        const uint32_t x = s_stage[j];
        parts[s_glob[x >> sh] + j] = (P)(x & omask);
    }
    if (cs < 0) return;
    // cells: the same placement with the cell digits (entries 256.. of the tables; their
    // global positions start after all endpoints, at entry 256 * tiles of the scan)
    const uint32_t cc = hist[(uint64_t)(256 + t) * tiles + tile];
    const uint32_t cincl = wave_incl_scan(cc);
    __syncthreads();  // every read of s_stage, s_fill, s_glob and s_wsum above is done
    if (lane_id() == kWave - 1) s_wsum[w] = cincl;
    __syncthreads();
    uint32_t cbefore = 0;
    for (uint32_t k = 0; k < w; ++k) cbefore += s_wsum[k];
    const uint32_t cloc = cbefore + cincl - cc;
    s_fill[t] = cloc;
    s_glob[t] = offs[(uint64_t)(256 + t) * tiles + tile] - offs[(uint64_t)256 * tiles] - cloc;
    __syncthreads();
    int2 *s_edges = reinterpret_cast<int2 *>(s_stage);
#pragma unroll
    for (int r = 0; r < kPartEdges; ++r) {
        const int2 e = ed[r];
        if (!endpoint_ok(e, n)) continue;
        s_edges[atomicAdd(&s_fill[edge_cell(e, cs)], 1u)] = e;
    }
    __syncthreads();
    const uint32_t ctotal = s_fill[255];  // edges of this tile that are valid
    for (uint32_t j = t; j < ctotal; j += kPartThreads) {
        const int2 e = s_edges[j];
        cells[s_glob[edge_cell(e, cs)] + j] = e;
    }
}

// Workgroup (bucket, slice): counts its slice of the bucket's endpoints (offsets inside the
// bucket) in LDS, window by window of kPartWindow ids, and adds the counts to deg (zeroed
// beforehand).
template <class P>
__global__ __launch_bounds__(1024) void k_part_count(const P *__restrict__ parts,
                                                     const uint32_t *__restrict__ offs,
                                                     uint32_t tiles, int sh, uint32_t n,
                                                     uint32_t slices,
                                                     uint32_t *__restrict__ deg,
                                                     const int32_t *__restrict__ status) {
    if (*status) return;
    __shared__ uint32_t cntr[kPartWindow];
    const uint32_t t = threadIdx.x, bucket = blockIdx.x / slices, g = blockIdx.x % slices;
    const uint32_t beg = offs[(uint64_t)bucket * tiles];
    const uint32_t end = offs[(uint64_t)(bucket + 1) * tiles];  // entry 256 * tiles = total
    const uint64_t len = end - beg;
    const uint32_t s0 = beg + (uint32_t)(len * g / slices);
    const uint32_t s1 = beg + (uint32_t)(len * (g + 1) / slices);
    const uint64_t id0 = (uint64_t)bucket << sh;
    if (id0 >= n) return;
    const uint64_t ids = ((1ull << sh) < n - id0) ? (1ull << sh) : (n - id0);
    for (uint64_t w0 = 0; w0 < ids; w0 += kPartWindow) {
        const uint32_t wn = (uint32_t)((ids - w0) < kPartWindow ? (ids - w0) : kPartWindow);
        for (uint32_t i = t; i < wn; i += blockDim.x) cntr[i] = 0;
        __syncthreads();
        const uint32_t lo = (uint32_t)w0;  // window start, as an offset inside the bucket
        // the slice's 16-byte aligned body as uint4 loads (kPer endpoints each), kPartLoads of
        // them in flight per thread before their LDS increments; the unaligned ends one
        // endpoint per thread
        constexpr uint32_t kPer = 16 / sizeof(P);
        const uint32_t q0 = (s0 + kPer - 1) / kPer, q1 = s1 / kPer;  // body: [kPer q0, kPer q1)
        const uint32_t e0 = q0 < q1 ? kPer * q0 : s1, e1 = q0 < q1 ? kPer * q1 : s1;
        if (t < e0 - s0) {
            const uint32_t x = (uint32_t)parts[s0 + t] - lo;
            if (x < wn) atomicAdd(&cntr[x], 1u);
        }
        if (t < s1 - e1) {
            const uint32_t x = (uint32_t)parts[e1 + t] - lo;
            if (x < wn) atomicAdd(&cntr[x], 1u);
        }
        const uint4 *__restrict__ parts4 = reinterpret_cast<const uint4 *>(parts);
        const uint32_t stride = blockDim.x * kPartLoads;
        for (uint32_t j0 = q0 + t; j0 < q1; j0 += stride) {
            uint4 x[kPartLoads];
#pragma unroll
            for (uint32_t k = 0; k < kPartLoads; ++k) {
                const uint32_t j = j0 + k * blockDim.x;
                x[k] = j < q1 ? load_nt_u4(parts4 + j) : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (uint32_t k = 0; k < kPartLoads; ++k) {
                if (j0 + k * blockDim.x >= q1) continue;
                const uint32_t wd[4] = {x[k].x, x[k].y, x[k].z, x[k].w};
#pragma unroll
                for (uint32_t q = 0; q < 4; ++q) {
                    if (sizeof(P) == 2) {  // two offsets per word
                        const uint32_t a = (wd[q] & 0xFFFFu) - lo, b = (wd[q] >> 16) - lo;
                        if (a < wn) atomicAdd(&cntr[a], 1u);
                        if (b < wn) atomicAdd(&cntr[b], 1u);
                    } else {
                        const uint32_t a = wd[q] - lo;
                        if (a < wn) atomicAdd(&cntr[a], 1u);
                    }
                }
            }
        }
        __syncthreads();
        for (uint32_t i = t; i < wn; i += blockDim.x) {
            const uint32_t c = cntr[i];
            if (c) atomicAdd(&deg[id0 + lo + i], c);
        }
        __syncthreads();
    }
}

template __global__ void k_part_scatter<uint16_t>(const int2 *, uint64_t, uint32_t, uint32_t, int,
                                                  int, const uint32_t *, const uint32_t *,
                                                  uint32_t, uint16_t *, int2 *);
template __global__ void k_part_scatter<uint32_t>(const int2 *, uint64_t, uint32_t, uint32_t, int,
                                                  int, const uint32_t *, const uint32_t *,
                                                  uint32_t, uint32_t *, int2 *);
template __global__ void k_part_count<uint16_t>(const uint16_t *, const uint32_t *, uint32_t, int,
                                                uint32_t, uint32_t, uint32_t *, const int32_t *);
template __global__ void k_part_count<uint32_t>(const uint32_t *, const uint32_t *, uint32_t, int,
                                                uint32_t, uint32_t, uint32_t *, const int32_t *);

// Fallback for inputs whose endpoint count does not fit the partition's 32-bit offsets, or
// whose buckets would need too many LDS windows: one atomic increment per endpoint.
__global__ void k_degree_atomic(const int2 *__restrict__ edges, uint64_t m, uint32_t n,
                                uint32_t both, uint32_t *__restrict__ deg,
                                int32_t *__restrict__ status) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) {
        const int2 e = edges[i];
        if (!endpoint_ok(e, n)) {
            set_status(status, ((uint32_t)e.x >= n || (uint32_t)e.y >= n) ? TC_E_RANGE
                                                                          : TC_E_SELF_LOOP);
            continue;
        }
        atomicAdd(&deg[e.x], 1u);
        if (!both) atomicAdd(&deg[e.y], 1u);
    }
}

// vkeys[x] = (degree << b) | x, whose stable sort on the degree bits yields the total order
// of Section 2.2 (degree first, ties by id)
__global__ void k_vkeys(const uint32_t *__restrict__ deg, uint32_t n, int b,
                        uint64_t *__restrict__ vkeys) {
    uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t lim = (1ull << b) - 1;
    uint64_t d = deg[x];
    if (d > lim) d = lim;  // only possible for invalid input, which is reported elsewhere
    vkeys[x] = (d << b) | x;
}

__global__ void k_orient(const int2 *__restrict__ edges, uint64_t m, uint32_t both,
                         const uint32_t *__restrict__ rank, int b, uint64_t *__restrict__ keys,
                         uint32_t *__restrict__ counter, const int32_t *__restrict__ status) {
    if (*status) return;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (!both) {
        for (; i < m; i += stride) {
            const int2 e = edges[i];
            const uint32_t ru = rank[e.x], rv = rank[e.y];
            keys[i] = ((uint64_t)min(ru, rv) << b) | max(ru, rv);
        }
        return;
    }
    // two-direction format: keep the forward entries, compacted per wave; a uniform trip
    // count so that every lane takes part in the wave-wide ballots
    const uint64_t rounds = (m + stride - 1) / stride;
    for (uint64_t r = 0; r < rounds; ++r, i += stride) {
        bool in = i < m;
        uint32_t ru = 0, rv = 0;
        if (in) {
            int2 e = edges[i];
            ru = rank[e.x];
            rv = rank[e.y];
        }
        bool keep = in && ru < rv;
        uint64_t mask = __ballot(keep);
        if (mask == 0) continue;
        uint32_t leader = (uint32_t)__ffsll((long long)mask) - 1;
        uint32_t base = 0;
        if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
        base = wave_bcast(base, (int)leader);
        if (keep) keys[base + lanes_below(mask)] = ((uint64_t)ru << b) | rv;
    }
}

// One-direction format, edges in cell order: the workgroups of one XCD (workgroup b runs on
// XCD b % 8) sweep that XCD's eighth of the array together, so the rank lookups of the
// edges in flight on an XCD fall into one or two cells, whose two rank stretches stay in
// that XCD's L2.  Each thread has two edges in flight (a step apart).  The grid is a multiple
// of 8; ids are checked again, since the cell array holds only the valid edges (an invalid
// one has already set the status).
__global__ void k_orient_cells(const int2 *__restrict__ cells, uint64_t m, uint32_t n,
                               const uint32_t *__restrict__ rank, int b,
                               uint64_t *__restrict__ keys, const int32_t *__restrict__ status) {
    if (*status) return;
    const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds, per = gridDim.x / kXcds;
    const uint64_t lo = m * x / kXcds, hi = m * (x + 1) / kXcds;
    const uint64_t step = (uint64_t)per * blockDim.x;
    // the edge stream is read and the keys written with non-temporal hints, so that they do
    // not push the two rank stretches out of the XCD's L2
    const uint64_t *cw = reinterpret_cast<const uint64_t *>(cells);
    for (uint64_t i0 = lo + (uint64_t)j * blockDim.x + threadIdx.x; i0 < hi; i0 += 2 * step) {
        const uint64_t i1 = i0 + step;
        const uint64_t w0 = __builtin_nontemporal_load(cw + i0);
        const uint64_t w1 = i1 < hi ? __builtin_nontemporal_load(cw + i1) : 0ull;
        const int2 e0 = make_int2((int)(uint32_t)w0, (int)(uint32_t)(w0 >> 32));
        const int2 e1 = make_int2((int)(uint32_t)w1, (int)(uint32_t)(w1 >> 32));
        const bool ok0 = (uint32_t)e0.x < n && (uint32_t)e0.y < n;
        const bool ok1 = i1 < hi && (uint32_t)e1.x < n && (uint32_t)e1.y < n;
        uint32_t r0u = 0, r0v = 0, r1u = 0, r1v = 0;
        if (ok0) {
            r0u = rank[e0.x];
            r0v = rank[e0.y];
        }
        if (ok1) {
            r1u = rank[e1.x];
            r1v = rank[e1.y];
        }
        const uint64_t k0 = ((uint64_t)min(r0u, r0v) << b) | max(r0u, r0v);
        const uint64_t k1 = ((uint64_t)min(r1u, r1v) << b) | max(r1u, r1v);
        if (ok0) __builtin_nontemporal_store(k0, keys + i0);
        if (ok1) __builtin_nontemporal_store(k1, keys + i1);
    }
}

// two-direction format: exactly half of the entries must be forward
__global__ void k_both_check(const uint32_t *__restrict__ counter, uint32_t expect,
                             int32_t *__restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *counter != expect)
        set_status(status, TC_E_ASYMMETRIC);
}

constexpr uint32_t kCsrKeys = 4;
constexpr uint32_t kRowChunk = 4096;  // CSR positions per workgroup of k_row_sort

// Unzip the sorted keys into the neighbour array (Section 3.2, step 7) and mark where every
// non-empty row starts and ends; row lengths and their prefix sum give the node array.
// hrow[u] receives the position of the first entry >= hbase of row u (left untouched, all
// ones from the caller's fill, when the row has none).  (Keys sorted by (source, target): the
// path of graphs too large for the row sort, or with it switched off.)
__global__ void k_csr(const uint64_t *__restrict__ keys, uint32_t mf, uint32_t n, int b,
                      uint32_t hbase, uint32_t *__restrict__ col, uint32_t *__restrict__ src,
                      uint32_t *__restrict__ rs, uint32_t *__restrict__ re,
                      uint32_t *__restrict__ hrow, int32_t *__restrict__ status) {
    if (*status) return;
    // kCsrKeys keys a block apart per thread, all loaded before any is used
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x * kCsrKeys + threadIdx.x;
    uint64_t k[kCsrKeys], kp[kCsrKeys], kn[kCsrKeys];
#pragma unroll
    for (uint32_t t = 0; t < kCsrKeys; ++t) {
        const uint64_t i = i0 + (uint64_t)t * blockDim.x;
        k[t] = i < mf ? keys[i] : 0ull;
        kp[t] = (i < mf && i > 0) ? keys[i - 1] : ~0ull;
        kn[t] = i + 1 < mf ? keys[i + 1] : ~0ull;
    }
#pragma unroll
    for (uint32_t t = 0; t < kCsrKeys; ++t) {
        const uint64_t i = i0 + (uint64_t)t * blockDim.x;
        if (i >= mf) continue;
        const uint32_t s = (uint32_t)(k[t] >> b);
        const uint32_t c = (uint32_t)(k[t] & ((1ull << b) - 1));
        col[i] = c;
        src[i] = s;
        if (s >= n) continue;  // only for invalid input, reported elsewhere
        const bool row_start = i == 0 || (uint32_t)(kp[t] >> b) != s;
        if (row_start) rs[s] = (uint32_t)i;
        if (c >= hbase && (row_start || (uint32_t)(kp[t] & ((1ull << b) - 1)) < hbase))
            hrow[s] = (uint32_t)i;
        if (i > 0 && kp[t] == k[t]) set_status(status, TC_E_DUP_EDGE);
        if (i == mf - 1 || (uint32_t)(kn[t] >> b) != s) re[s] = (uint32_t)(i + 1);
    }
}

// With the keys sorted by source only and unzipped by the sort's last pass (col, src): where
// every non-empty row starts and ends, and rchunk[c] = the first row starting at or after
// position c * kRowChunk (the chunks of k_row_sort, which sorts the rows, checks them for
// duplicates and records hrow).
__global__ void k_row_bounds(const uint32_t *__restrict__ src, uint32_t mf, uint32_t n,
                             uint32_t *__restrict__ rs, uint32_t *__restrict__ re,
                             uint32_t *__restrict__ rchunk, const int32_t *__restrict__ status) {
    if (*status) return;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x * kCsrKeys + threadIdx.x;
    uint32_t x[kCsrKeys], xp[kCsrKeys], xn[kCsrKeys];
#pragma unroll
    for (uint32_t t = 0; t < kCsrKeys; ++t) {
        const uint64_t i = i0 + (uint64_t)t * blockDim.x;
        x[t] = i < mf ? __builtin_nontemporal_load(src + i) : 0u;
        xp[t] = (i < mf && i > 0) ? src[i - 1] : ~0u;
        xn[t] = i + 1 < mf ? src[i + 1] : ~0u;
    }
#pragma unroll
    for (uint32_t t = 0; t < kCsrKeys; ++t) {
        const uint64_t i = i0 + (uint64_t)t * blockDim.x;
        const uint32_t s = x[t];
        if (i >= mf || s >= n) continue;  // (s >= n only for invalid input, reported elsewhere)
        const bool row_start = i == 0 || xp[t] != s;
        if (row_start) rs[s] = (uint32_t)i;
        if ((i & (kRowChunk - 1)) == 0) rchunk[i / kRowChunk] = row_start ? s : s + 1;
        if (i == mf - 1 || xn[t] != s) re[s] = (uint32_t)(i + 1);
    }
}

// ---------------------------------------------------------------- rows sorted in place
//
// With the edge keys sorted by source only (three radix passes instead of six), every row of
// col holds its targets in input order; these kernels sort each row ascending, then check it
// for duplicates and record hrow (as k_csr does for fully sorted keys).  A workgroup takes
// the rows starting in one chunk of kRowChunk positions: rows of at most kRowWave entries by
// groups of lanes sized to the row (a bitonic network over the group's registers, 16 entries
// per lane, the smaller strides in registers and the others across the group's lanes; a
// short row takes one lane, so that small rows do not pay for a whole wave's network),
// longer rows are listed for k_row_sort_long (a wave's registers, or a bitonic network in a
// workgroup's LDS).  Rows of a simple graph hold fewer than sqrt(2 m) entries (Section 2.2),
// below kRowLong for the graphs this path is used on; a longer row means repeated edges and
// is reported as TC_E_DUP_EDGE.
constexpr uint32_t kRowWave = 1024;
constexpr uint32_t kRowWaveLong = 2048;  // listed rows up to this length: one wave each
constexpr uint32_t kRowLong = 32768;

__device__ __forceinline__ void cswap(uint32_t &a, uint32_t &b) {
    const uint32_t lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

// duplicates and the first entry >= hbase of a sorted row, from a lane's view of consecutive
// positions: entries v[0..k) at positions p .. p + k - 1 of the row, the entry before them
// (prev, valid when p > 0)
__device__ __forceinline__ void row_checks(const uint32_t *v, uint32_t k, uint32_t p,
                                           uint32_t prev, uint32_t rb, uint32_t hbase,
                                           uint32_t *__restrict__ hrow, uint32_t r,
                                           int32_t *__restrict__ status) {
    for (uint32_t j = 0; j < k; ++j) {
        const uint32_t before = j ? v[j - 1] : prev;
        const bool has_before = j > 0 || p > 0;
        if (has_before && before == v[j]) set_status(status, TC_E_DUP_EDGE);
        if (v[j] >= hbase && (!has_before || before < hbase)) hrow[r] = rb + p + j;
    }
}

// x of lane (lane ^ ls) for ls a power of two below 64 (a constant once the networks are
// unrolled): DPP moves inside rows of 16 lanes (quad permutations; a half-row or row mirror
// followed by a second mirror gives xor 4 and xor 8), a swizzle across the 32-lane halves'
// rows for 16, a permute through the LDS crossbar for 32.
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, uint32_t ls) {
    switch (ls) {
    case 1:  // quad_perm [1, 0, 3, 2]
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
    case 2:  // quad_perm [2, 3, 0, 1]
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
    case 4: {  // row_half_mirror (lane ^ 7), then quad_perm [3, 2, 1, 0] (lane ^ 3)
        const int y = __builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, y, 0x1B, 0xF, 0xF, false);
    }
    case 8: {  // row_mirror (lane ^ 15), then row_half_mirror (lane ^ 7)
        const int y = __builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, y, 0x141, 0xF, 0xF, false);
    }
    case 16:  // swizzle, bit mode: and 0x1f, or 0, xor 0x10
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);
    default:
        return (uint32_t)__shfl_xor((int)x, (int)ls, kWave);
    }
}

// A row of at most G E entries, sorted by an aligned group of G lanes (G a power of two up to
// 64; every lane of the wave takes part, each group with its own row, len 0 for none): a
// bitonic network on P = G E entries, the group's lane g holding positions g E .. g E + E - 1.
// Strides below E compare registers of one lane, the others exchange with lane g ^ (stride /
// E), which stays inside the group.
template <uint32_t E, uint32_t G>
__device__ __forceinline__ void sort_row_group(uint32_t *__restrict__ col, uint32_t rb,
                                               uint32_t len, uint32_t g, uint32_t hbase,
                                               uint32_t *__restrict__ hrow, uint32_t r,
                                               int32_t *__restrict__ status) {
    constexpr uint32_t P = G * E;
    uint32_t v[E];
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
        const uint32_t i = g * E + j;
        v[j] = i < len ? col[rb + i] : ~0u;
    }
#pragma unroll
    for (uint32_t k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (uint32_t st = k >> 1; st; st >>= 1) {
            if (st >= E) {  // across lanes: partner lane ^ (st / E), same slot
                const uint32_t ls = st / E;
#pragma unroll
                for (uint32_t j = 0; j < E; ++j) {
                    const uint32_t i = g * E + j;
                    // (32 entries per lane: the permutes through the crossbar measured faster)
                    const uint32_t y = E <= 16 ? lane_xor(v[j], ls)
                                               : (uint32_t)__shfl_xor((int)v[j], (int)ls, kWave);
                    const bool lower = (i & st) == 0, asc = (i & k) == 0;
                    v[j] = (lower == asc) ? min(v[j], y) : max(v[j], y);
                }
            } else {  // inside the lane
#pragma unroll
                for (uint32_t j = 0; j < E; ++j) {
                    const uint32_t q = j ^ st;
                    if (q > j) {
                        const uint32_t i = g * E + j;
                        if ((i & k) == 0) cswap(v[j], v[q]);
                        else cswap(v[q], v[j]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
        const uint32_t i = g * E + j;
        if (i < len) col[rb + i] = v[j];
    }
    // the entry before this lane's: the previous lane's last (used only when g > 0)
    const uint32_t prev = G > 1 ? (uint32_t)__shfl_up((int)v[E - 1], 1, kWave) : 0u;
    const uint32_t p = g * E;
    const uint32_t k = p < len ? min(E, len - p) : 0u;
    row_checks(v, k, p, prev, rb, hbase, hrow, r, status);
}

// Rows of the chunk's class C (G = 2^C lanes of kRowLane entries per row), 64 / G rows per
// wave at a time.
constexpr uint32_t kRowLane = 16;  // entries per lane in k_row_sort
constexpr uint32_t kRowClasses = 7;  // G = 1 .. 64
template <uint32_t C>
__device__ __forceinline__ void sort_row_class(uint32_t *__restrict__ col,
                                               const uint32_t *__restrict__ row_ptr,
                                               const uint32_t *list, uint32_t off, uint32_t cnt,
                                               uint32_t hbase, uint32_t *__restrict__ hrow,
                                               int32_t *__restrict__ status) {
    constexpr uint32_t G = 1u << C, per = kWave / G;
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave, waves = blockDim.x / kWave;
    for (uint32_t base = w * per; base < cnt; base += waves * per) {
        const uint32_t q = base + lane / G;
        uint32_t r = 0, rb = 0, len = 0;
        if (q < cnt) {
            r = list[off + q];
            rb = row_ptr[r];
            len = row_ptr[r + 1] - rb;
        }
        sort_row_group<kRowLane, G>(col, rb, len, lane % G, hbase, hrow, r, status);
    }
}

// Rows starting in chunk c (rows rchunk[c] .. rchunk[c + 1] - 1), listed in LDS by class:
// the non-empty rows of at most kRowWave entries by G = the smallest power of two with
// G kRowLane >= length (C = log2 G), each class sorted by groups of G lanes; longer rows go
// to the list for k_row_sort_long.  At most kRowChunk non-empty rows start in a chunk.
__device__ __forceinline__ uint32_t row_class(uint32_t len) {  // len >= 1
    if (len > kRowWave) return kRowClasses;
    return len <= kRowLane ? 0u : 32u - (uint32_t)__builtin_clz(len - 1) - 4u;
}
__global__ __launch_bounds__(256) void k_row_sort(uint32_t *__restrict__ col,
                                                  const uint32_t *__restrict__ row_ptr,
                                                  const uint32_t *__restrict__ rchunk,
                                                  uint32_t chunks, uint32_t n, uint32_t hbase,
                                                  uint32_t *__restrict__ hrow,
                                                  uint32_t *__restrict__ long_rows,
                                                  uint32_t *__restrict__ n_long,
                                                  int32_t *__restrict__ status) {
    if (*status) return;
    static_assert(kRowLane << (kRowClasses - 1) == kRowWave, "classes cover the wave rows");
    __shared__ uint32_t list[kRowChunk];
    __shared__ uint32_t ccount[kRowClasses], coff[kRowClasses], ccur[kRowClasses];
    const uint32_t c = blockIdx.x;
    const uint32_t r0 = rchunk[c], r1 = c + 1 < chunks ? rchunk[c + 1] : n;
    const uint32_t t = threadIdx.x;
    if (t < kRowClasses) ccount[t] = 0;
    __syncthreads();
    for (uint32_t r = r0 + t; r < r1; r += blockDim.x) {
        const uint32_t len = row_ptr[r + 1] - row_ptr[r];
        if (len == 0) continue;
        const uint32_t cls = row_class(len);
        if (cls < kRowClasses) atomicAdd(&ccount[cls], 1u);
        else long_rows[atomicAdd(n_long, 1u)] = r;
    }
    __syncthreads();
    if (t == 0) {
        uint32_t o = 0;
        for (uint32_t k = 0; k < kRowClasses; ++k) {
            coff[k] = ccur[k] = o;
            o += ccount[k];
        }
    }
    __syncthreads();
    for (uint32_t r = r0 + t; r < r1; r += blockDim.x) {
        const uint32_t len = row_ptr[r + 1] - row_ptr[r];
        if (len == 0) continue;
        const uint32_t cls = row_class(len);
        if (cls < kRowClasses) list[atomicAdd(&ccur[cls], 1u)] = r;
    }
    __syncthreads();
    sort_row_class<0>(col, row_ptr, list, coff[0], ccount[0], hbase, hrow, status);
    sort_row_class<1>(col, row_ptr, list, coff[1], ccount[1], hbase, hrow, status);
    sort_row_class<2>(col, row_ptr, list, coff[2], ccount[2], hbase, hrow, status);
    sort_row_class<3>(col, row_ptr, list, coff[3], ccount[3], hbase, hrow, status);
    sort_row_class<4>(col, row_ptr, list, coff[4], ccount[4], hbase, hrow, status);
    sort_row_class<5>(col, row_ptr, list, coff[5], ccount[5], hbase, hrow, status);
    sort_row_class<6>(col, row_ptr, list, coff[6], ccount[6], hbase, hrow, status);
}

// The listed long rows: those of at most kRowWaveLong entries one per wave (the register
// network with 32 entries per lane, kept out of k_row_sort so that its other rows run at a
// higher occupancy), longer ones one per workgroup of 1024 threads in a bitonic network in LDS
// on the row padded to a power of two (at most kRowLong entries).
__global__ __launch_bounds__(1024) void k_row_sort_long(uint32_t *__restrict__ col,
                                                        const uint32_t *__restrict__ row_ptr,
                                                        const uint32_t *__restrict__ long_rows,
                                                        const uint32_t *__restrict__ n_long,
                                                        uint32_t hbase,
                                                        uint32_t *__restrict__ hrow,
                                                        int32_t *__restrict__ status) {
    if (*status) return;
    __shared__ uint32_t a[kRowLong];
    const uint32_t t = threadIdx.x, nl = *n_long;
    const uint32_t waves = blockDim.x / kWave;
    for (uint32_t q = blockIdx.x * waves + t / kWave; q < nl; q += gridDim.x * waves) {
        const uint32_t r = long_rows[q];
        const uint32_t rb = row_ptr[r], len = row_ptr[r + 1] - rb;
        if (len <= kRowWaveLong)
            sort_row_group<32, kWave>(col, rb, len, lane_id(), hbase, hrow, r, status);
    }
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint32_t r = long_rows[q];
        const uint32_t rb = row_ptr[r], len = row_ptr[r + 1] - rb;
        if (len <= kRowWaveLong) continue;  // sorted above
        if (len > kRowLong) {  // only with repeated edges
            if (t == 0) set_status(status, TC_E_DUP_EDGE);
            continue;
        }
        uint32_t P = kRowWave;
        while (P < len) P <<= 1;
        __syncthreads();
        for (uint32_t i = t; i < P; i += blockDim.x) a[i] = i < len ? col[rb + i] : ~0u;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1)
            for (uint32_t st = k >> 1; st; st >>= 1) {
                for (uint32_t i = t; i < P; i += blockDim.x) {
                    const uint32_t q2 = i ^ st;
                    if (q2 > i) {
                        const uint32_t x = a[i], y = a[q2];
                        const bool asc = (i & k) == 0;
                        if ((x > y) == asc) {
                            a[i] = y;
                            a[q2] = x;
                        }
                    }
                }
                __syncthreads();
            }
        for (uint32_t i = t; i < len; i += blockDim.x) {
            const uint32_t x = a[i];
            col[rb + i] = x;
            const bool has_before = i > 0;
            const uint32_t before = has_before ? a[i - 1] : 0u;
            if (has_before && before == x) set_status(status, TC_E_DUP_EDGE);
            if (x >= hbase && (!has_before || before < hbase)) hrow[r] = rb + i;
        }
    }
}

uint32_t row_sort_chunk() { return kRowChunk; }
uint32_t row_sort_wave() { return kRowWave; }

// row length = end - start (both zero for empty rows); entry n is 0 so that the exclusive
// scan over n + 1 entries ends with row_ptr[n] = m_fwd
__global__ void k_rowlen(const uint32_t *__restrict__ rs, const uint32_t *__restrict__ re,
                         uint32_t n, uint32_t *__restrict__ len) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    len[r] = r < n ? re[r] - rs[r] : 0u;
}

// Room of every row's entries >= hbase in hcol: none for a row without such entries, else
// their number rounded up to a multiple of 8, plus `pad` zeros (the counting kernel's pieces,
// read from 8-aligned positions inside the row's part, never leave it).  Entry n is 0, so that
// the exclusive scan ends with the total.
__global__ void k_hlen(const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ hrow,
                       uint32_t n, uint32_t pad, uint32_t *__restrict__ hlen) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    uint32_t len = 0;
    if (r < n && hrow[r] != ~0u) len = ((row_ptr[r + 1] - hrow[r] + 7u) & ~7u) + pad;
    hlen[r] = len;
}

// Rank span of every out-list from rank v0 on (the panel region, whose spans k_panel_range
// combines): (min << 32) | max, or 0xFFFFFFFF00000000 (min > max) if empty.
__global__ void k_vrange(const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ col,
                         uint32_t v0, uint32_t n, uint64_t *__restrict__ vr) {
    uint32_t v = v0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint32_t r0 = row_ptr[v], r1 = row_ptr[v + 1];
    vr[v] = r1 > r0 ? ((uint64_t)col[r0] << 32) | col[r1 - 1] : 0xFFFFFFFF00000000ull;
}

// Rank span of the union of the out-lists of every panel (ranks p0 + i * kp .. + kp - 1), in
// the format of k_vrange.
__global__ void k_panel_range(const uint64_t *__restrict__ vr, uint32_t n, uint32_t p0,
                              uint32_t kp, uint32_t panels, uint64_t *__restrict__ pr) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= panels) return;
    const uint32_t P = p0 + i * kp, pe = min(P + kp, n);
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
    for (uint32_t v = P; v < pe; ++v) {
        const uint64_t r = vr[v];
        const uint32_t l = (uint32_t)(r >> 32), h = (uint32_t)r;
        if (l <= h) {
            lo = min(lo, l);
            hi = max(hi, h);
        }
    }
    pr[i] = ((uint64_t)lo << 32) | hi;
}

// In-edge u -> v (CSR position e) can close a triangle u < v < w only through an element w of
// N+(u) after v that also lies in N+(v), so only in-edges with a non-empty suffix are listed
// (k_items skips the lists of vertices with an empty N+(v)).  They are keyed by their list
// c = row block * (n + 1) + v (row blocks: contiguous CSR ranges, see the host code), the
// others by `lists` (sorted last); written as 32-bit list ids ckey[e], whose sort on the keys
// (ckey[e] << 32) | e groups every list in CSR order.  (A test of the suffix's rank range
// against that of N+(v) was dropped: on R-MAT graphs it rejected no in-edge and cost one
// random 8-byte lookup per edge.)  From rank p0 on, middle vertices form panels of kp
// consecutive ranks with one list per panel, keyed by its first rank P: only the first
// in-edge of each run of u's out-neighbours inside the panel is kept (it stands for the whole
// run), tested against the panel's span (a small table).  eu[e], the in-edge's record read by
// the counting kernels, = (end of u's row, mask of the run's panel vertices for a kept panel
// entry or, for any other kept entry, the col position where the suffix's entries >= hbase
// start, the hcol position where they start, u).  In-edges from hubs (u >= h0) are left out:
// their triangles are counted on the matrix cores.  Every entry >= hbase is also written to
// its row's part of hcol (hrow and hstart: k_csr, k_hlen and a scan).
// Each thread takes kCscEdges entries a block apart and issues every stage's loads for all of
// them before using any (the stages depend on each other: entry -> row -> row end).
constexpr uint32_t kCscEdges = 4;

__global__ void k_csc_keys(const uint32_t *__restrict__ col, const uint32_t *__restrict__ src,
                           const uint32_t *__restrict__ row_ptr,
                           const uint32_t *__restrict__ hrow,
                           const uint32_t *__restrict__ hstart, uint32_t hbase,
                           const uint64_t *__restrict__ pr, uint32_t mf, uint32_t n,
                           uint32_t nblk, uint32_t p0, uint32_t kp, uint32_t h0,
                           uint32_t *__restrict__ ckey, uint4 *__restrict__ eu,
                           uint16_t *__restrict__ hcol, const int32_t *__restrict__ status) {
    if (*status) return;
    // kp is a power of two; row blocks are rare (nblk > 1 only when asked for)
    const uint32_t kp_shift = __builtin_ctz(kp);
    const uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x * kCscEdges + threadIdx.x;
    uint32_t u[kCscEdges], v[kCscEdges], prv[kCscEdges], nxt[kCscEdges];
#pragma unroll
    for (uint32_t k = 0; k < kCscEdges; ++k) {
        const uint64_t e = e0 + (uint64_t)k * blockDim.x;
        const bool in = e < mf;
        u[k] = in ? __builtin_nontemporal_load(src + e) : 0u;
        v[k] = in ? col[e] : 0u;
        prv[k] = (in && e > 0) ? col[e - 1] : 0u;
        nxt[k] = (in && e + 1 < mf) ? col[e + 1] : 0u;
    }
    uint32_t rb[kCscEdges], re[kCscEdges], hr[kCscEdges], hs[kCscEdges];
#pragma unroll
    for (uint32_t k = 0; k < kCscEdges; ++k) {
        const bool in = e0 + (uint64_t)k * blockDim.x < mf;
        rb[k] = in ? row_ptr[u[k]] : 0u;
        re[k] = in ? row_ptr[u[k] + 1] : 0u;
        hr[k] = in ? hrow[u[k]] : 0u;
        hs[k] = in ? hstart[u[k]] : 0u;
    }
    uint32_t last[kCscEdges];
    uint64_t r[kCscEdges];
#pragma unroll
    for (uint32_t k = 0; k < kCscEdges; ++k) {
        const uint64_t e = e0 + (uint64_t)k * blockDim.x;
        const bool pan = e + 1 < re[k] && u[k] < h0 && v[k] >= p0;
        last[k] = pan ? col[re[k] - 1] : 0u;
        r[k] = pan ? pr[(v[k] - p0) >> kp_shift] : 0xFFFFFFFF00000000ull;
    }
#pragma unroll
    for (uint32_t k = 0; k < kCscEdges; ++k) {
        const uint64_t e = e0 + (uint64_t)k * blockDim.x;
        if (e >= mf) continue;
        const uint32_t end_u = re[k];
        // the row's entries >= hbase in hcol (hr[k] <= e: the row is ascending)
        if (v[k] >= hbase) hcol[hs[k] + ((uint32_t)e - hr[k])] = (uint16_t)(v[k] - hbase);
        uint64_t c = (uint64_t)nblk * (n + 1);
        uint32_t mask = 1u, hpos = hs[k];
        if (e + 1 < end_u && u[k] < h0) {  // triangles whose lowest vertex is a hub: hub.hip
            uint32_t list = v[k];
            bool keep = true, run_start = false;
            if (v[k] >= p0) {
                list = p0 + (((v[k] - p0) >> kp_shift) << kp_shift);
                run_start = e == rb[k] || prv[k] < list;
                const uint32_t lo = (uint32_t)(r[k] >> 32), hi = (uint32_t)r[k];
                keep = run_start && lo <= hi && nxt[k] <= hi && last[k] >= lo;
            }
            if (keep) {
                const uint64_t blk = nblk == 1 ? 0 : (e * nblk) / mf;
                c = blk * (n + 1) + list;
                // where the suffix's entries >= hbase start, in col (outside the panels, in
                // place of the mask) and in hcol; a panel suffix is high throughout
                const uint32_t hb = v[k] >= hbase ? (uint32_t)e + 1u : min(hr[k], end_u);
                if (v[k] < p0) mask = hb;
                if (hb < end_u) hpos = hs[k] + (hb - hr[k]);
                if (run_start) {  // the run's mask: u's consecutive entries inside the panel
                    mask = 1u << (v[k] - list);
                    for (uint64_t x = e + 1; x < end_u; x += 4) {  // four loads at a time
                        uint32_t w[4];
#pragma unroll
                        for (uint32_t i = 0; i < 4; ++i) w[i] = x + i < end_u ? col[x + i] : ~0u;
                        bool out = false;
#pragma unroll
                        for (uint32_t i = 0; i < 4; ++i) {
                            out = out || w[i] >= list + kp;
                            if (!out) mask |= 1u << (w[i] - list);
                        }
                        if (out) break;
                    }
                }
            }
        }
        ckey[e] = (uint32_t)c;  // list ids are below 2^32 (the host bounds the row blocks)
        store_nt_u4(eu + e, make_uint4(end_u, mask, hpos, u[k]));
    }
}

// The lists themselves: list c occupies sorted positions [rs[c], re[c]) (useful in-edges
// only, *kept of them; rs and re zeroed beforehand), found from the sorted list ids; entry j
// names its in-edge by cbeg[j] = e + 1, the start of the suffix (written by the sort's last
// pass); the counting kernels read the in-edge's record (k_csc_keys) from there.
// kCscFinalKeys ids a block apart per thread, all loaded before any is used.
constexpr uint32_t kCscFinalKeys = 4;
__global__ void k_csc_final(const uint32_t *__restrict__ list, uint32_t mf,
                            const uint32_t *__restrict__ kept, uint64_t lists,
                            uint32_t *__restrict__ rs, uint32_t *__restrict__ re,
                            const int32_t *__restrict__ status) {
    if (*status) return;
    mf = min(mf, *kept);
    const uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x * kCscFinalKeys + threadIdx.x;
    uint32_t k[kCscFinalKeys], kp[kCscFinalKeys], kn[kCscFinalKeys];
#pragma unroll
    for (uint32_t t = 0; t < kCscFinalKeys; ++t) {
        const uint64_t j = j0 + (uint64_t)t * blockDim.x;
        k[t] = j < mf ? __builtin_nontemporal_load(list + j) : ~0u;
        kp[t] = (j < mf && j > 0) ? list[j - 1] : ~0u;
        kn[t] = j + 1 < mf ? list[j + 1] : ~0u;
    }
#pragma unroll
    for (uint32_t t = 0; t < kCscFinalKeys; ++t) {
        const uint64_t j = j0 + (uint64_t)t * blockDim.x;
        const uint32_t c = k[t];
        if (j >= mf || c >= lists) continue;
        if (j == 0 || kp[t] != c) rs[c] = (uint32_t)j;
        if (j == mf - 1 || kn[t] != c) re[c] = (uint32_t)j + 1;
    }
}

// Work items of the counting kernel.  A vertex's in-edges are cut into chunks; the chunks go
// to the per-wave queue when the vertex's out-list fits one wave's LDS slice (as a bitmap over
// its rank span or as a sorted list; for per-vertex counts as a list with counters),
// otherwise to the per-workgroup queue.  Both classifications are prepared, so a prepared
// graph can be counted either way.  Panel lists (first rank >= p0) always go to the
// per-workgroup queue.
__global__ void k_items(const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ col,
                        const uint32_t *__restrict__ cnt, uint32_t n, uint32_t nblk, uint32_t p0,
                        uint32_t wave_span, uint32_t wave_list, uint32_t wave_list_pv,
                        uint32_t ka, uint32_t kb,
                        uint32_t *__restrict__ ia, uint32_t *__restrict__ ib,
                        uint32_t *__restrict__ ia_pv, uint32_t *__restrict__ ib_pv,
                        const int32_t *__restrict__ status) {
    if (*status) return;
    const uint64_t total = (uint64_t)nblk * (n + 1);
    uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > total) return;
    uint32_t a = 0, b = 0, apv = 0, bpv = 0;
    const uint32_t v = c < total ? (uint32_t)(c % (n + 1)) : n;
    if (v < n && cnt[c] > 0 && v >= p0) {
        b = bpv = (cnt[c] + kb - 1) / kb;
    } else if (v < n && cnt[c] > 0 && row_ptr[v + 1] > row_ptr[v]) {  // N+(v) non-empty
        const uint32_t r0 = row_ptr[v], d = row_ptr[v + 1] - r0;
        const uint32_t span = col[r0 + d - 1] - col[r0];
        const uint32_t na = (cnt[c] + ka - 1) / ka, nb = (cnt[c] + kb - 1) / kb;
        if (span < wave_span || d <= wave_list) a = na; else b = nb;
        if (d <= wave_list_pv) apv = na; else bpv = nb;
    }
    ia[c] = a;
    ib[c] = b;
    ia_pv[c] = apv;
    ib_pv[c] = bpv;
}

__global__ void k_item_fill(const uint32_t *__restrict__ items, const uint32_t *__restrict__ off,
                            uint64_t total, uint32_t *__restrict__ item_c,
                            const int32_t *__restrict__ status) {
    if (*status) return;
    uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    uint32_t k = items[c], o = off[c];
    for (uint32_t j = 0; j < k; ++j) item_c[o + j] = (uint32_t)c;
}

// per-vertex counts back from rank space to vertex ids
__global__ void k_pv_out(const unsigned long long *__restrict__ t_rank,
                         const uint32_t *__restrict__ perm, uint32_t n,
                         unsigned long long *__restrict__ out) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[perm[r]] = t_rank[r];
}

__global__ void k_zero_u64(unsigned long long *__restrict__ p, uint64_t count) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = 0ull;
}

}  // namespace tc
