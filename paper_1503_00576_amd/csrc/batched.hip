// Batched counting: many small graphs in one launch sequence, captured once in a hipGraph.
//
// Input: the graphs' symmetric adjacency lists (the format Section 3.1 contrasts with the
// edge array), concatenated.  Graph g has n_g = vtx_off[g+1] - vtx_off[g] vertices and its
// own CSR: row_ptr entries [vtx_off[g] + g, vtx_off[g+1] + g] (local offsets 0..len_g) and
// col entries [adj_off[g], adj_off[g+1]) (local ids, rows strictly ascending).  In the disjoint
// union, vertex x of graph g has id vtx_off[g] + x.
//
// Preprocessing needs no sort: the degree of a vertex is its row length, and keeping in every
// row only the neighbours that come later in the order of Section 2.2 ((degree, id)
// ascending) is a stable filter, so the oriented rows stay sorted by id.  The counting kernel
// (k_count_u) then stages N+(u) and streams N+(v) for the out-neighbours v.
//
// Every kernel reads the sizes and the caller's pointers from an argument block at the start
// of the workspace and runs over the plan's capacities, so one captured graph serves every
// batch that fits the plan.
#include <stdlib.h>
#include <string.h>

#include "internal.h"

namespace tc {

struct BatchArgs {
    const int64_t *vtx_off;
    const int64_t *adj_off;
    const int32_t *row_ptr;
    const int32_t *col;
    unsigned long long *totals;
    unsigned long long *per_vertex;
    int32_t *status;  // per graph, may be null
    uint32_t G, N, kitem;
    uint32_t A;      // adjacency entries in total
    uint32_t chunk;  // forward edges per light chunk
};

__device__ __forceinline__ void graph_error(const BatchArgs &a, uint32_t g, int32_t code,
                                            int32_t *gstat) {
    atomicCAS(&gstat[g], 0, code);
}

// graph of union vertex x: the last g with vtx_off[g] <= x
__device__ __forceinline__ uint32_t graph_of(const int64_t *vtx_off, uint32_t G, uint32_t x) {
    uint32_t lo = 0, len = G;
    while (len > 1) {
        const uint32_t half = len >> 1;
        if (vtx_off[lo + half] <= (int64_t)x) lo += half;
        len -= half;
    }
    return lo;
}

__global__ void k_b_set_args(BatchArgs *dst, BatchArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = a;
}

// zero the outputs and the internal status / queues
__global__ void k_b_clear(const BatchArgs *__restrict__ args, int32_t *__restrict__ gstat,
                          unsigned long long *__restrict__ ghash,
                          uint32_t *__restrict__ queue, uint32_t cap) {
    const BatchArgs a = *args;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) queue[i] = 0;
    for (uint32_t x = i; x < cap; x += gridDim.x * blockDim.x) {
        if (x < a.G) {
            a.totals[x] = 0;
            gstat[x] = 0;
            ghash[x] = 0;
        }
        if (a.per_vertex && x < a.N) a.per_vertex[x] = 0;
    }
}

// Pair hash for the symmetry check: the 64-bit finalizer of MurmurHash3 (fmix64) applied to
// (x << 32 | y).
__device__ __forceinline__ uint64_t pair_hash(uint32_t x, uint32_t y) {
    uint64_t k = ((uint64_t)x << 32) | y;
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Per-vertex work over the input rows is done wave by wave: the wave takes 64 consecutive
// vertices (lane k: vertex xb + k), whose rows are consecutive in the input, and walks their
// entries 64 at a time, so that loads and stores are coalesced whatever the row lengths.
// Entry idx of the walk belongs to the last lane k whose exclusive prefix off[k] <= idx.
struct RowWalk {
    uint32_t off[kWave + 1];  // exclusive prefix of the row lengths; off[64] = all entries
    uint32_t ebeg[kWave];     // position of the row in the input's col
    uint32_t len[kWave];      // row length (0 for rows that failed their checks)
    uint32_t local[kWave];    // local vertex id
    uint32_t rpb[kWave];      // index of the graph's row offsets in row_ptr
    uint32_t ng[kWave];       // vertices of the graph
    uint32_t g[kWave];        // graph
    uint32_t acc[kWave];      // per-row count of forward entries (counted), or the row's next
                              // output position (written)
    uint32_t fend[kWave];     // end of the row's forward entries in the output (written)
};

__device__ __forceinline__ uint32_t walk_owner(const RowWalk &rw, uint32_t idx) {
    uint32_t k = 0;
#pragma unroll
    for (uint32_t step = 32; step; step >>= 1)
        if (rw.off[k + step] <= idx) k += step;
    return k;
}

// lanes a .. b (inclusive) of a wave
__device__ __forceinline__ uint64_t lane_range(uint32_t a, uint32_t b) {
    return ((2ull << b) - 1ull) & ~((1ull << a) - 1ull);
}

// Loads the wave's 64 rows into `rw` (lane = vertex x) from already validated per-vertex
// values; returns the number of entries.
__device__ __forceinline__ uint32_t walk_begin(RowWalk &rw, uint32_t d, uint32_t ebeg,
                                               uint32_t local, uint32_t rpb, uint32_t ng,
                                               uint32_t g) {
    const uint32_t lane = lane_id();
    const uint32_t incl = wave_incl_scan(d);
    const uint32_t total = wave_bcast(incl, kWave - 1);
    rw.off[lane] = incl - d;
    if (lane == 0) rw.off[kWave] = total;
    rw.ebeg[lane] = ebeg;
    rw.len[lane] = d;
    rw.local[lane] = local;
    rw.rpb[lane] = rpb;
    rw.ng[lane] = ng;
    rw.g[lane] = g;
    rw.acc[lane] = 0;
    wave_lds_sync();
    return total;
}

// One step of the walk: the entry of this lane (if any) with its owner k, its index j in the
// row, its value y (local id), whether it is a forward entry of an in-range id (the same
// test in both kernels: the degree of y is its row length in the input), the previous entry
// of the row (-1 at the row start), and the lanes of the owner's row in this step
// [first, last].
struct WalkEntry {
    bool valid, ok, fwd;
    uint32_t k, j, first, last;
    int32_t y, prev;
};

// kWalkSteps consecutive steps of the walk at once: every load of all of them (entries,
// previous entries, the row offsets behind the degree test) is issued before any is used,
// so a wave waits once per kWalkSteps steps instead of once per step.  Addresses of lanes
// past the end or with an out-of-range id are clamped onto valid ones and their values
// ignored.
constexpr int kWalkSteps = 4;
constexpr int kFillSteps = 8;  // the forward fill's walk needs fewer registers per step

// The argument block's pointers are generic; the walk reads through global-address-space
// views so that its loads are global loads (waited for apart from the LDS traffic).
typedef const __attribute__((address_space(1))) int32_t *gptr_i32;

__device__ __forceinline__ void walk_entries(const RowWalk &rw, uint32_t base, uint32_t total,
                                             const int32_t *col_p, const int32_t *row_ptr_p,
                                             WalkEntry (&en)[kWalkSteps]) {
    const gptr_i32 col = (gptr_i32)col_p, row_ptr = (gptr_i32)row_ptr_p;
    const uint32_t lane = lane_id();
    int32_t r0[kWalkSteps], r1[kWalkSteps];
#pragma unroll
    for (int u = 0; u < kWalkSteps; ++u) {
        const uint32_t idx = base + (uint32_t)u * kWave + lane;
        en[u].valid = idx < total;
        const uint32_t k = walk_owner(rw, en[u].valid ? idx : total - 1);
        en[u].k = k;
        en[u].j = (en[u].valid ? idx : total - 1) - rw.off[k];
        const uint32_t at = rw.ebeg[k] + en[u].j;
        en[u].y = col[at];
        en[u].prev = col[at - (en[u].j > 0 ? 1u : 0u)];
    }
#pragma unroll
    for (int u = 0; u < kWalkSteps; ++u) {
        const uint32_t k = en[u].k, lk = rw.local[k];
        const int32_t y = en[u].y;
        if (en[u].j == 0) en[u].prev = -1;
        en[u].ok = en[u].valid && y >= 0 && (uint32_t)y < rw.ng[k] && (uint32_t)y != lk;
        const uint32_t at = rw.rpb[k] + (en[u].ok ? (uint32_t)y : 0u);
        r0[u] = row_ptr[at];
        r1[u] = row_ptr[at + 1];
    }
#pragma unroll
    for (int u = 0; u < kWalkSteps; ++u) {
        const uint32_t k = en[u].k, lk = rw.local[k];
        const int64_t dy = (int64_t)r1[u] - r0[u], dx = rw.len[k];
        en[u].fwd = en[u].ok && (dy > dx || (dy == dx && (uint32_t)en[u].y > lk));
        const uint32_t sb = base + (uint32_t)u * kWave;
        const uint32_t rb = rw.off[k], re = rw.off[k] + rw.len[k];
        en[u].first = (rb > sb ? rb : sb) - sb;
        en[u].last = (re < sb + kWave ? re : sb + kWave) - 1 - sb;
    }
}

// The steps of k_b_ffill's walk: the entries and their forward flags from k_b_setup (no degree
// lookups); fills valid, fwd, k, first, last and y.
__device__ __forceinline__ void walk_entries_flagged(const RowWalk &rw, uint32_t base,
                                                     uint32_t total, const int32_t *col_p,
                                                     const uint8_t *__restrict__ fflag,
                                                     WalkEntry (&en)[kFillSteps]) {
    const gptr_i32 col = (gptr_i32)col_p;
    const uint32_t lane = lane_id();
    uint32_t f[kFillSteps];
#pragma unroll
    for (int u = 0; u < kFillSteps; ++u) {
        const uint32_t idx = base + (uint32_t)u * kWave + lane;
        en[u].valid = idx < total;
        const uint32_t k = walk_owner(rw, en[u].valid ? idx : total - 1);
        en[u].k = k;
        en[u].j = (en[u].valid ? idx : total - 1) - rw.off[k];
        const uint32_t at = rw.ebeg[k] + en[u].j;
        en[u].y = col[at];
        f[u] = fflag[at];
    }
#pragma unroll
    for (int u = 0; u < kFillSteps; ++u) {
        const uint32_t k = en[u].k;
        en[u].fwd = en[u].valid && f[u] != 0u;
        const uint32_t sb = base + (uint32_t)u * kWave;
        const uint32_t rb = rw.off[k], re = rw.off[k] + rw.len[k];
        en[u].first = (rb > sb ? rb : sb) - sb;
        en[u].last = (re < sb + kWave ? re : sb + kWave) - 1 - sb;
    }
}

// Per vertex: graph id, degree (row length), forward out-degree (entries ncap.. stay zero for
// the scan), checks of its row (offsets in range, ids in range, no self-loop, strictly
// ascending), and its share of the graph's symmetry sum: sum over the row's entries (x, y) of
// pair_hash(x, y) - pair_hash(y, x), which is zero over a graph whose rows are symmetric.
// Graph ids are non-decreasing across a wave, so the shares are added per run of equal ids.
__global__ __launch_bounds__(256) void k_b_setup(const BatchArgs *__restrict__ args,
                                                 uint32_t ncap, uint32_t *__restrict__ gid,
                                                 uint32_t *__restrict__ deg,
                                                 uint32_t *__restrict__ fdeg,
                                                 uint8_t *__restrict__ fflag,
                                                 unsigned long long *__restrict__ ghash,
                                                 int32_t *__restrict__ gstat) {
    __shared__ RowWalk s_rw[4];
    const BatchArgs a = *args;
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    RowWalk &rw = s_rw[w];
    const uint32_t x = (blockIdx.x * 4 + w) * kWave + lane;
    uint32_t g = 0xFFFFFFFFu, d = 0, ebeg = 0, local = 0, rpb = 0, ng = 0;
    if (x < a.N) {
        g = graph_of(a.vtx_off, a.G, x);
        gid[x] = g;
        const int64_t v0 = a.vtx_off[g], n_g = a.vtx_off[g + 1] - v0;
        const int64_t a0 = a.adj_off[g], alen = a.adj_off[g + 1] - a0;
        const int64_t lx = (int64_t)x - v0;
        // offsets arrays must be prefix sums: check what this vertex relies on (the whole
        // vertex range of its graph, whose row offsets the forward test reads)
        if (v0 < 0 || lx < 0 || lx >= n_g || v0 + n_g > (int64_t)a.N || a0 < 0 || alen < 0 ||
            a0 + alen > (int64_t)a.A) {
            graph_error(a, g, TC_E_ARG, gstat);
        } else {
            const int32_t *rp = a.row_ptr + v0 + g;
            const int64_t r0 = rp[lx], r1 = rp[lx + 1];
            if (r0 < 0 || r1 < r0 || r1 > alen) {
                graph_error(a, g, TC_E_ARG, gstat);
            } else {
                d = (uint32_t)(r1 - r0);
                ebeg = (uint32_t)(a0 + r0);
                local = (uint32_t)lx;
                rpb = (uint32_t)(v0 + g);
                ng = (uint32_t)n_g;
            }
        }
    }
    const uint32_t total = walk_begin(rw, d, ebeg, local, rpb, ng, g);
    // this lane's symmetry shares, for graph hg (the graphs of a lane's entries never
    // decrease; a change flushes the sum)
    uint32_t hg = 0xFFFFFFFFu;
    uint64_t hsum = 0;
    for (uint32_t base = 0; base < total; base += kWalkSteps * kWave) {
        WalkEntry ens[kWalkSteps];
        walk_entries(rw, base, total, a.col, a.row_ptr, ens);
#pragma unroll
        for (int u = 0; u < kWalkSteps; ++u) {
            const WalkEntry &en = ens[u];
            if (en.valid) {
                const uint32_t gk = rw.g[en.k], lk = rw.local[en.k];
                if (!en.ok) {
                    graph_error(a, gk,
                                (en.y < 0 || (uint32_t)en.y >= rw.ng[en.k]) ? TC_E_RANGE
                                                                            : TC_E_SELF_LOOP,
                                gstat);
                } else {
                    if (en.j > 0 && en.y <= en.prev)
                        graph_error(a, gk, en.y == en.prev ? TC_E_DUP_EDGE : TC_E_UNSORTED,
                                    gstat);
                    if (gk != hg) {
                        if (hsum) atomicAdd(&ghash[hg], (unsigned long long)hsum);
                        hg = gk;
                        hsum = 0;
                    }
                    hsum += pair_hash(lk, (uint32_t)en.y) - pair_hash((uint32_t)en.y, lk);
                }
            }
            if (en.valid) fflag[rw.ebeg[en.k] + en.j] = en.fwd ? 1u : 0u;
            const uint64_t F = __ballot(en.valid && en.fwd);
            // forward entries per row in this step, added by the row's last lane in the step
            if (en.valid && lane == en.last)
                rw.acc[en.k] += (uint32_t)__popcll(F & lane_range(en.first, lane));
            wave_lds_sync();
        }
    }
    if (x < ncap) deg[x] = d;
    if (x <= ncap) fdeg[x] = rw.acc[lane];
    // the lanes' last sums: one atomic when they all belong to one graph (the usual case)
    const uint32_t hg0 = wave_bcast(hg, 0);
    if (__ballot(hsum != 0 && hg != hg0) == 0) {
        const uint64_t hs = wave_sum_u64(hsum);
        if (lane == 0 && hs) atomicAdd(&ghash[hg0], (unsigned long long)hs);
    } else if (hsum) {
        atomicAdd(&ghash[hg], (unsigned long long)hsum);
    }
}

// the forward rows (union ids, input order kept) with the row of every entry
__global__ __launch_bounds__(256) void k_b_ffill(const BatchArgs *__restrict__ args,
                                                 const uint32_t *__restrict__ gid,
                                                 const uint32_t *__restrict__ deg,
                                                 const uint32_t *__restrict__ frp,
                                                 const uint8_t *__restrict__ fflag,
                                                 uint32_t *__restrict__ fcol,
                                                 uint32_t *__restrict__ fsrc) {
    __shared__ RowWalk s_rw[4];
    const BatchArgs a = *args;
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    RowWalk &rw = s_rw[w];
    const uint32_t x = (blockIdx.x * 4 + w) * kWave + lane;
    uint32_t g = 0xFFFFFFFFu, d = 0, ebeg = 0, local = 0, rpb = 0, ng = 0;
    if (x < a.N && deg[x] > 0) {  // rows that passed k_b_setup's checks
        g = gid[x];
        const int64_t v0 = a.vtx_off[g];
        const int32_t *rp = a.row_ptr + v0 + g;
        local = (uint32_t)((int64_t)x - v0);
        d = deg[x];
        ebeg = (uint32_t)(a.adj_off[g] + rp[local]);
        rpb = (uint32_t)(v0 + g);
        ng = (uint32_t)(a.vtx_off[g + 1] - v0);
    }
    const uint32_t total = walk_begin(rw, d, ebeg, local, rpb, ng, g);
    rw.acc[lane] = x < a.N ? frp[x] : 0u;
    rw.fend[lane] = x < a.N ? frp[x + 1] : 0u;
    wave_lds_sync();
    for (uint32_t base = 0; base < total; base += kFillSteps * kWave) {
        WalkEntry ens[kFillSteps];
        walk_entries_flagged(rw, base, total, a.col, fflag, ens);
#pragma unroll
        for (int u = 0; u < kFillSteps; ++u) {
            const WalkEntry &en = ens[u];
            const uint64_t F = __ballot(en.valid && en.fwd);
            if (en.valid && en.fwd) {
                const uint32_t xk = x - lane + en.k;
                const uint32_t pos = rw.acc[en.k] + (uint32_t)__popcll(
                                                        F & lane_range(en.first, lane) &
                                                        ~(1ull << lane));
                if (pos < rw.fend[en.k]) {  // always true: k_b_setup counted the same entries
                    fsrc[pos] = xk;
                    fcol[pos] = rw.rpb[en.k] - rw.g[en.k] + (uint32_t)en.y;
                }
            }
            wave_lds_sync();  // every lane has read acc before the row's last lane adds to it
            if (en.valid && lane == en.last)
                rw.acc[en.k] += (uint32_t)__popcll(F & lane_range(en.first, lane));
            wave_lds_sync();
        }
    }
}

// work items: heavy rows (more than `light_max` forward neighbours) in chunks of kitem; the
// light rows are counted in chunks of consecutive forward edges: light[0] = forward edges,
// light[1] = chunks
__global__ void k_b_items(const BatchArgs *__restrict__ args, uint32_t ncap,
                          const uint32_t *__restrict__ fdeg, const uint32_t *__restrict__ frp,
                          uint32_t light_max, uint32_t *__restrict__ items,
                          uint32_t *__restrict__ light) {
    const BatchArgs a = *args;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x > ncap) return;
    const uint32_t d = (x < a.N) ? fdeg[x] : 0u;
    items[x] = d > light_max ? (d + a.kitem - 1) / a.kitem : 0u;
    if (x == ncap) {
        const uint32_t mf = frp[ncap];
        light[0] = mf;
        light[1] = (mf + a.chunk - 1) / a.chunk;
    }
}

__global__ void k_b_item_fill(const uint32_t *__restrict__ items,
                              const uint32_t *__restrict__ off, uint32_t ncap,
                              uint32_t *__restrict__ item_u) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ncap) return;
    const uint32_t k = items[x], o = off[x];
    for (uint32_t j = 0; j < k; ++j) item_u[o + j] = x;
}

// per-graph checks that need the whole graph, and the per-graph status out (the caller's
// array, when given).  Offsets: the graph's vertex and adjacency ranges must lie inside the
// batch (k_b_setup checked them only for graphs that have vertices).  Symmetry: the entries
// must number twice the forward entries, and the graph's symmetry sum must be zero (a set of
// entries that is not closed under mirroring passes this with probability about 2^-64).
__global__ void k_b_finish(const BatchArgs *__restrict__ args, const uint32_t *__restrict__ frp,
                           const unsigned long long *__restrict__ ghash,
                           int32_t *__restrict__ gstat) {
    const BatchArgs a = *args;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.G) return;
    int32_t st = gstat[g];
    if (st == 0) {
        const int64_t v0 = a.vtx_off[g], v1 = a.vtx_off[g + 1];
        const int64_t a0 = a.adj_off[g], a1 = a.adj_off[g + 1];
        if (v0 < 0 || v1 < v0 || v1 > (int64_t)a.N || a0 < 0 || a1 < a0 || a1 > (int64_t)a.A)
            st = TC_E_ARG;
        else if (2 * (int64_t)(frp[v1] - frp[v0]) != a1 - a0 || ghash[g] != 0)
            st = TC_E_ASYMMETRIC;
        gstat[g] = st;
    }
    if (a.status) a.status[g] = st;
}

// ------------------------------------------------------------------ workspace + plan

struct BatchLayout {
    size_t args, ctl, gstat, ghash, gid, deg, fdeg, frp, fcol, fsrc, fflag, items, ioff, item_u,
        scan, total;
};

constexpr uint32_t kMinItemEdges = 16;

static BatchLayout batch_layout(uint32_t gcap, uint32_t ncap, uint64_t acap) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1), 256);
        return at;
    };
    const uint64_t n1 = (uint64_t)ncap + 1;
    L.args = take(sizeof(BatchArgs));
    L.ctl = take(64 * 4);
    L.gstat = take((size_t)gcap * 4);
    L.ghash = take((size_t)gcap * 8);
    L.gid = take((size_t)ncap * 4);
    L.deg = take((size_t)ncap * 4);
    L.fdeg = take(n1 * 4);
    L.frp = take(n1 * 4);
    L.fcol = take((size_t)acap * 4 + count_col_pad_bytes());
    L.fsrc = take((size_t)acap * 4);
    L.fflag = take((size_t)acap);  // one byte per input entry: forward (k_b_setup)
    L.items = take(n1 * 4);
    L.ioff = take(n1 * 4);
    L.item_u = take(((size_t)acap / kMinItemEdges + n1 + 1) * 4);
    L.scan = take(scan_scratch_words(n1) * 4);
    L.total = off;
    return L;
}

}  // namespace tc

using namespace tc;

struct tc_plan {
    uint32_t gcap, ncap;
    uint64_t acap;
    uint32_t kitem, chunk, wgs_per_cu;
    uint32_t light_max;  // forward-degree threshold of the edge-per-lane path
    uint32_t wave_bits;  // heavy items: bitmap below this id span
    uint32_t wave_list;  // heavy items: sorted LDS list of at most this many entries
    void *ws;
    size_t ws_bytes;
    BatchLayout L;
    hipGraph_t graph[2];
    hipGraphExec_t exec[2];
};

static uint32_t parse_tuning(const char *json, const char *key, uint32_t dflt) {
    if (!json) return dflt;
    const char *p = strstr(json, key);
    if (!p) return dflt;
    p = strchr(p + strlen(key), ':');
    if (!p) return dflt;
    long v = strtol(p + 1, nullptr, 10);
    return v > 0 ? (uint32_t)v : dflt;
}

// as parse_tuning, but 0 is a value (negative values give the default)
static uint32_t parse_tuning_or_zero(const char *json, const char *key, uint32_t dflt) {
    if (!json) return dflt;
    const char *p = strstr(json, key);
    if (!p) return dflt;
    p = strchr(p + strlen(key), ':');
    if (!p) return dflt;
    long v = strtol(p + 1, nullptr, 10);
    return v >= 0 ? (uint32_t)(v > 0x7FFFFFFFl ? 0x7FFFFFFFl : v) : dflt;
}

// enqueue the whole sequence (this is what gets captured)
static int batch_enqueue(tc_plan *p, bool pv, hipStream_t s) {
    const BatchLayout &L = p->L;
    char *ws = (char *)p->ws;
    const BatchArgs *args = (const BatchArgs *)(ws + L.args);
    uint32_t *ctl = (uint32_t *)(ws + L.ctl);
    int32_t *gstat = (int32_t *)(ws + L.gstat);
    unsigned long long *ghash = (unsigned long long *)(ws + L.ghash);
    uint32_t *gid = (uint32_t *)(ws + L.gid), *deg = (uint32_t *)(ws + L.deg);
    uint32_t *fdeg = (uint32_t *)(ws + L.fdeg), *frp = (uint32_t *)(ws + L.frp);
    uint32_t *fcol = (uint32_t *)(ws + L.fcol), *items = (uint32_t *)(ws + L.items);
    uint32_t *fsrc = (uint32_t *)(ws + L.fsrc);
    uint32_t *ioff = (uint32_t *)(ws + L.ioff), *item_u = (uint32_t *)(ws + L.item_u);
    uint32_t *scan = (uint32_t *)(ws + L.scan);
    const uint32_t ncap = p->ncap, n1 = ncap + 1;
    const uint32_t cap = ncap > p->gcap ? ncap : p->gcap;
    auto grid = [](uint64_t n) { return dim3((uint32_t)((n + 255) / 256)); };
    hipLaunchKernelGGL(k_b_clear, dim3(1024), dim3(256), 0, s, args, gstat, ghash, ctl, cap);
    // one wave per 64 vertices, four waves per workgroup
    auto vgrid = [](uint64_t n) { return dim3((uint32_t)((n + 255) / 256)); };
    uint8_t *fflag = (uint8_t *)(ws + L.fflag);
    hipLaunchKernelGGL(k_b_setup, vgrid(n1), dim3(256), 0, s, args, ncap, gid, deg, fdeg, fflag,
                       ghash, gstat);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    if (scan_exclusive_u32(fdeg, frp, n1, scan, s) != hipSuccess) return TC_E_HIP;
    hipLaunchKernelGGL(k_b_ffill, vgrid(ncap), dim3(256), 0, s, args, gid, deg, frp, fflag, fcol,
                       fsrc);
    // ctl: [0] heavy-item queue, [1] light-chunk queue, [2] forward edges, [3] light chunks
    hipLaunchKernelGGL(k_b_items, grid(n1), dim3(256), 0, s, args, ncap, fdeg, frp,
                       p->light_max, items, ctl + 2);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    if (scan_exclusive_u32(items, ioff, n1, scan, s) != hipSuccess) return TC_E_HIP;
    hipLaunchKernelGGL(k_b_item_fill, grid(ncap), dim3(256), 0, s, items, ioff, ncap, item_u);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    BatchKernelArgs ka;
    ka.frp = frp;
    ka.fcol = fcol;
    ka.fsrc = fsrc;
    ka.gid = gid;
    ka.item_u = item_u;
    ka.item_off = ioff;
    ka.n_items = ioff + ncap;
    ka.kitem = &args->kitem;
    ka.chunk = &args->chunk;
    ka.light = ctl + 2;
    ka.queue = ctl;
    ka.totals_pp = &args->totals;
    ka.tpv_pp = &args->per_vertex;
    ka.light_max = p->light_max;
    ka.wave_bits = p->wave_bits;
    ka.wave_list = pv ? (p->wave_list < count_wave_list(true) ? p->wave_list
                                                              : count_wave_list(true))
                      : p->wave_list;
    if (launch_count_u(ka, pv, device_cu_count() * p->wgs_per_cu, s) != hipSuccess)
        return TC_E_HIP;
    hipLaunchKernelGGL(k_b_finish, grid(p->gcap), dim3(256), 0, s, args, frp, ghash, gstat);
    return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

static int batch_capture(tc_plan *p, bool pv) {
    const int k = pv ? 1 : 0;
    if (p->exec[k]) return TC_OK;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return TC_E_HIP;
    int st = TC_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return TC_E_HIP;
    }
    st = batch_enqueue(p, pv, cs);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) st = TC_E_HIP;
    (void)hipStreamDestroy(cs);
    if (st != TC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return TC_E_HIP;
    }
    p->graph[k] = g;
    p->exec[k] = ex;
    return TC_OK;
}

static int plan_set_args(tc_plan *p, int32_t G, const int64_t *d_vtx_off,
                         const int64_t *d_adj_off, const int32_t *d_row_ptr,
                         const int32_t *d_col, int64_t n_total, int64_t adj_total,
                         hipStream_t s, uint64_t *d_totals, uint64_t *d_per_vertex,
                         int32_t *d_status) {
    if (G <= 0 || !d_vtx_off || !d_adj_off || !d_row_ptr || !d_totals) return TC_E_ARG;
    if ((uint32_t)G > p->gcap || n_total < 0 || (uint64_t)n_total > p->ncap || adj_total < 0 ||
        (uint64_t)adj_total > p->acap)
        return TC_E_TOO_LARGE;
    if (adj_total > 0 && !d_col) return TC_E_ARG;
    BatchArgs a;
    a.vtx_off = d_vtx_off;
    a.adj_off = d_adj_off;
    a.row_ptr = d_row_ptr;
    a.col = d_col;
    a.totals = (unsigned long long *)d_totals;
    a.per_vertex = (unsigned long long *)d_per_vertex;
    a.status = d_status;
    a.G = (uint32_t)G;
    a.N = (uint32_t)n_total;
    a.kitem = p->kitem;
    a.A = (uint32_t)adj_total;
    a.chunk = p->chunk;
    hipLaunchKernelGGL(k_b_set_args, dim3(1), dim3(64), 0, s,
                       (BatchArgs *)((char *)p->ws + p->L.args), a);
    return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

extern "C" {

size_t tc_batched_workspace_size(int32_t g_cap, int64_t n_cap, int64_t adj_cap) {
    if (g_cap <= 0 || n_cap < 0 || adj_cap < 0 || n_cap >= (1ll << 31) ||
        adj_cap >= (1ll << 32))
        return 0;
    return batch_layout((uint32_t)g_cap, (uint32_t)n_cap, (uint64_t)adj_cap).total;
}

int tc_batched_plan_create(int32_t g_cap, int64_t n_cap, int64_t adj_cap, uint32_t flags,
                           const char *tuning_json, void *d_ws, size_t ws_bytes,
                           tc_plan **out) {
    if (!out) return TC_E_ARG;
    *out = nullptr;
    if (g_cap <= 0 || n_cap < 0 || adj_cap < 0 || flags != 0) return TC_E_ARG;
    if (n_cap >= (1ll << 31) || adj_cap >= (1ll << 32)) return TC_E_TOO_LARGE;
    const BatchLayout L = batch_layout((uint32_t)g_cap, (uint32_t)n_cap, (uint64_t)adj_cap);
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < L.total) return TC_E_WORKSPACE;
    tc_plan *p = (tc_plan *)calloc(1, sizeof(tc_plan));
    if (!p) return TC_E_ARG;
    p->gcap = (uint32_t)g_cap;
    p->ncap = (uint32_t)n_cap;
    p->acap = (uint64_t)adj_cap;
    p->kitem = parse_tuning(tuning_json, "\"items_k\"", 256);
    if (p->kitem < kMinItemEdges) p->kitem = kMinItemEdges;
    p->chunk = parse_tuning(tuning_json, "\"chunk_e\"", 1024);
    if (p->chunk < 64) p->chunk = 64;
    if (p->chunk > count_light_chunk_max()) p->chunk = count_light_chunk_max();
    p->wgs_per_cu = parse_tuning(tuning_json, "\"wgs_per_cu\"", count_wgs_per_cu());
    if (p->wgs_per_cu > count_wgs_per_cu()) p->wgs_per_cu = count_wgs_per_cu();  // LDS limit
    // the light/heavy threshold and the heavy items' LDS forms: the defaults are the largest
    // values the LDS holds; lower values are accepted (tuning, and tests that reach every
    // form on small graphs)
    p->light_max = parse_tuning_or_zero(tuning_json, "\"light_max\"", count_light_max());
    if (p->light_max > count_light_max()) p->light_max = count_light_max();
    p->wave_bits = parse_tuning_or_zero(tuning_json, "\"bitmap_span\"", count_wave_span());
    if (p->wave_bits > count_wave_span()) p->wave_bits = count_wave_span();
    p->wave_list = parse_tuning_or_zero(tuning_json, "\"list_max\"", count_wave_list(false));
    if (p->wave_list > count_wave_list(false)) p->wave_list = count_wave_list(false);
    p->ws = d_ws;
    p->ws_bytes = ws_bytes;
    p->L = L;
    *out = p;
    return TC_OK;
}

int tc_batched_plan_run(tc_plan *p, int32_t G, const int64_t *d_vtx_off,
                        const int64_t *d_adj_off, const int32_t *d_row_ptr, const int32_t *d_col,
                        int64_t n_total, int64_t adj_total, void *stream, uint64_t *d_totals,
                        uint64_t *d_per_vertex, int32_t *d_status) {
    if (!p) return TC_E_ARG;
    const bool pv = d_per_vertex != nullptr;
    int st = batch_capture(p, pv);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    st = plan_set_args(p, G, d_vtx_off, d_adj_off, d_row_ptr, d_col, n_total, adj_total, s,
                       d_totals, d_per_vertex, d_status);
    if (st) return st;
    if (hipGraphLaunch(p->exec[pv ? 1 : 0], s) != hipSuccess) return TC_E_HIP;
    return TC_OK;
}

void tc_batched_plan_destroy(tc_plan *p) {
    if (!p) return;
    for (int k = 0; k < 2; ++k) {
        if (p->exec[k]) (void)hipGraphExecDestroy(p->exec[k]);
        if (p->graph[k]) (void)hipGraphDestroy(p->graph[k]);
    }
    free(p);
}

int tc_count_batched(int32_t G, const int64_t *d_vtx_off, const int64_t *d_adj_off,
                     const int32_t *d_row_ptr, const int32_t *d_col, int64_t n_total,
                     int64_t adj_total, void *d_ws, size_t ws_bytes, void *stream,
                     uint64_t *d_totals, uint64_t *d_per_vertex, int32_t *d_status) {
    tc_plan *p = nullptr;
    int st = tc_batched_plan_create(G, n_total, adj_total, 0, nullptr, d_ws, ws_bytes, &p);
    if (st) return st;
    st = plan_set_args(p, G, d_vtx_off, d_adj_off, d_row_ptr, d_col, n_total, adj_total,
                       (hipStream_t)stream, d_totals, d_per_vertex, d_status);
    if (st == TC_OK) st = batch_enqueue(p, d_per_vertex != nullptr, (hipStream_t)stream);
    tc_batched_plan_destroy(p);
    return st;
}

}  // extern "C"
