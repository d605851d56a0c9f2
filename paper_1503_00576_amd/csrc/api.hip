// C ABI of libtc.so: argument checks, workspace layout and the launch sequence of the
// preprocessing and counting phases.  Everything is enqueued on the caller's stream; the
// library never allocates device memory and never synchronises.
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "internal.h"

namespace tc {

// kernels of prep.hip
__global__ void k_part_hist(const int2 *, uint64_t, uint32_t, uint32_t, int, int, uint32_t *,
                            uint32_t, int32_t *);
template <class P>
__global__ void k_part_scatter(const int2 *, uint64_t, uint32_t, uint32_t, int, int,
                               const uint32_t *, const uint32_t *, uint32_t, P *, int2 *);
template <class P>
__global__ void k_part_count(const P *, const uint32_t *, uint32_t, int, uint32_t, uint32_t,
                             uint32_t *, const int32_t *);
__global__ void k_degree_atomic(const int2 *, uint64_t, uint32_t, uint32_t, uint32_t *,
                                int32_t *);
__global__ void k_vkeys(const uint32_t *, uint32_t, int, uint64_t *);
__global__ void k_orient(const int2 *, uint64_t, uint32_t, const uint32_t *, int, uint64_t *,
                         uint32_t *, const int32_t *);
__global__ void k_orient_cells(const int2 *, uint64_t, uint32_t, const uint32_t *, int,
                               uint64_t *, const int32_t *);
__global__ void k_both_check(const uint32_t *, uint32_t, int32_t *);
__global__ void k_csr(const uint64_t *, uint32_t, uint32_t, int, uint32_t, uint32_t *,
                      uint32_t *, uint32_t *, uint32_t *, uint32_t *, int32_t *);
__global__ void k_row_bounds(const uint32_t *, uint32_t, uint32_t, uint32_t *, uint32_t *,
                             uint32_t *, const int32_t *);
__global__ void k_row_sort(uint32_t *, const uint32_t *, const uint32_t *, uint32_t, uint32_t,
                           uint32_t, uint32_t *, uint32_t *, uint32_t *, int32_t *);
__global__ void k_row_sort_long(uint32_t *, const uint32_t *, const uint32_t *,
                                const uint32_t *, uint32_t, uint32_t *, int32_t *);
__global__ void k_hlen(const uint32_t *, const uint32_t *, uint32_t, uint32_t, uint32_t *);
__global__ void k_rowlen(const uint32_t *, const uint32_t *, uint32_t, uint32_t *);
__global__ void k_vrange(const uint32_t *, const uint32_t *, uint32_t, uint32_t, uint64_t *);
__global__ void k_panel_range(const uint64_t *, uint32_t, uint32_t, uint32_t, uint32_t,
                              uint64_t *);
__global__ void k_csc_keys(const uint32_t *, const uint32_t *, const uint32_t *,
                           const uint32_t *, const uint32_t *, uint32_t, const uint64_t *,
                           uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t,
                           uint32_t *, uint4 *, uint16_t *, const int32_t *);
__global__ void k_csc_final(const uint32_t *, uint32_t, const uint32_t *, uint64_t, uint32_t *,
                            uint32_t *, const int32_t *);
__global__ void k_items(const uint32_t *, const uint32_t *, const uint32_t *, uint32_t, uint32_t,
                        uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t *,
                        uint32_t *,
                        uint32_t *, uint32_t *, const int32_t *);
__global__ void k_item_fill(const uint32_t *, const uint32_t *, uint64_t, uint32_t *,
                            const int32_t *);
__global__ void k_pv_out(const unsigned long long *, const uint32_t *, uint32_t,
                         unsigned long long *);
__global__ void k_zero_u64(unsigned long long *, uint64_t);

__global__ void k_copy_status(const int32_t *__restrict__ src, int32_t *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

int device_cu_count() {
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

// ------------------------------------------------------------------ workspace layout

struct Layout {
    size_t ctl, part_hist, part_offs, part_scan, deg, perm, rank, keys_a, keys_b, sort_scratch,
        rs, re, rowlen, row_ptr, col, hcol, hrow, hstart, src, vrange, prange, eu, lrs, lre, cnt,
        cptr, cbeg, items[4], off[4], item_v[4], scan_scratch, tpv, hub_a, hub_at, rchunk,
        long_rows, total_bytes;
    uint32_t part_tiles;  // 0: degrees by atomics (inputs too large for the partition)
    int part_shift;
    int cell_shift;       // >= 0: edges also partitioned into cells for the orientation
    uint32_t n, m, mf, kcap, id_bits, nblk;
    uint32_t p0, panels;  // panel region: ranks [p0, n) in panels of count_panel() ranks
    uint32_t h0, hp;      // hubs: ranks [h0, n), matrices hp x hp (hp = 0: no hubs)
    uint32_t hbase;       // ranks >= hbase are also held as 16-bit offsets (hcol); n: none
    uint64_t hcap;        // hcol entries
    uint64_t lists;       // in-edge lists: nblk * (n + 1)
    tc_options opt;       // resolved options
    uint32_t finger;      // fingerprint of (n, m, flags, options, panels), never 0
};

// item spaces: [0] wave / [1] workgroup items for total counts, [2] / [3] for per-vertex counts
// ctl words: status of the preprocessing, forward-entry counter (two-direction format), the
// two item queues, the fingerprint of the prepared layout, status of the current count
enum {
    kCtlStatus = 0, kCtlBoth = 1, kCtlQueueA = 2, kCtlQueueB = 3, kCtlFinger = 4, kCtlRun = 5,
    kCtlQueueC = 6, kCtlLongRows = 7, kCtlKept = 8, kCtlWords = 64
};
// start of a preprocessing: clear the control words and record the layout's fingerprint
__global__ void k_ctl_init(uint32_t *__restrict__ ctl, uint32_t finger) {
    const uint32_t t = threadIdx.x;
    ctl[t] = t == kCtlFinger ? finger : 0u;  // 64 threads, one word each
}

// start of a count on a prepared workspace: its status is the preprocessing's, or a mismatch
// when the workspace was prepared for another layout; the item queues restart
__global__ void k_ctl_check(uint32_t *__restrict__ ctl, uint32_t finger) {
    if (threadIdx.x != 0) return;
    int32_t st = (int32_t)ctl[kCtlStatus];
    if (st == 0 && ctl[kCtlFinger] != finger) st = TC_E_MISMATCH;
    ctl[kCtlRun] = (uint32_t)st;
    ctl[kCtlQueueA] = 0;
    ctl[kCtlQueueB] = 0;
    ctl[kCtlQueueC] = 0;
}

constexpr uint32_t kPartTileEdges = 4096;  // edges per tile of the degree partition
// workgroups of the orientation over cell-ordered edges (a multiple of the 8 XCDs; 2 per CU
// measured faster than 4 or 8: fewer edges in flight per XCD keep its lookups inside fewer
// cells)
constexpr uint32_t kOrientGrid = 512;
constexpr uint32_t kCscPerThread = 4;  // in-edge keys per thread (prep.hip, kCscEdges)
// the per-row sort (prep.hip) is used when every row of a simple graph fits its long-row
// kernel: m_fwd < 2^29, so that d+ < sqrt(2 m_fwd) <= 2^15
constexpr uint32_t kRowSortMaxEdges = 1u << 29;
constexpr uint32_t kMaxRowBlocks = 8;
constexpr uint32_t kMaxHubRanks = 1u << 16;  // two matrices of at most 4 GiB each
// the top ranks, whose entries of the node array are also stored as 16-bit offsets: on R-MAT
// graphs nearly every element the counting kernel streams (98% at scale 23) is one of them
constexpr uint32_t kHighRanks = 1u << 16;

static void default_options(tc_options &o) {
    memset(&o, 0, sizeof(o));
    o.size = sizeof(tc_options);
    o.panel_ranks = count_panel_ranks();
    o.hub_ranks = 0;  // off: at R-MAT scale 23 (1.9e8 edges) 16384 hubs take the sparse kernel
                      // from 20.95 to 19.59 ms but add 3.9 ms of matrix products
    o.row_blocks = 1;  // blocking at the memory-side cache size measured slower on R-MAT 23
    o.wave_item_edges = count_item_edges_wave();
    o.block_item_edges = count_item_edges_block();
    o.wave_bitmap_span = count_wave_span();
    o.wave_list_max = count_wave_list(false);
    o.block_bitmap_span = count_block_span();
    o.block_list_max = count_block_list(false);
    o.degree_partition = 1;
    o.sort_onesweep = 0;
    o.high_ranks = kHighRanks;
    o.row_sort = 1;
}

// the caller's options (NULL: defaults), checked against the limits the kernels are built for
static bool resolve_options(const tc_options *in, tc_options &o) {
    default_options(o);
    if (!in) return true;
    if (in->size != sizeof(tc_options)) return false;
    o = *in;
    return o.panel_ranks <= count_panel_ranks() && o.hub_ranks <= kMaxHubRanks &&
           o.row_blocks >= 1 && o.row_blocks <= kMaxRowBlocks && o.wave_item_edges >= 16 &&
           o.wave_item_edges <= (1u << 16) && o.block_item_edges >= 16 &&
           o.block_item_edges <= (1u << 20) && o.wave_bitmap_span <= count_wave_span() &&
           o.wave_list_max <= count_wave_list(false) &&
           o.block_bitmap_span <= count_block_span() &&
           o.block_list_max <= count_block_list(false) && o.degree_partition <= 1 &&
           o.sort_onesweep <= 1 && o.high_ranks <= kHighRanks && o.row_sort <= 1;
}

// FNV-1a over 32-bit words
static uint32_t fnv_words(const uint32_t *w, size_t k) {
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < k; ++i)
        for (int b = 0; b < 4; ++b) {
            h ^= (w[i] >> (8 * b)) & 0xFFu;
            h *= 16777619u;
        }
    return h;
}

static int id_bits_for(uint32_t n) {
    int b = 1;
    while (b < 31 && (1ull << b) < n) ++b;
    return b;
}

// bits needed to hold values in [0, x)
static int id_bits_for64(uint64_t x) {
    int b = 1;
    while (b < 63 && (1ull << b) < x) ++b;
    return b;
}

static bool make_layout(int64_t n, int64_t m, uint32_t flags, const tc_options *opts,
                        Layout &L) {
    if (n < 0 || m < 0 || n >= (1ll << 31) || m >= (1ll << 32)) return false;
    if (flags & ~TC_EDGES_BOTH) return false;
    if (!resolve_options(opts, L.opt)) return false;
    const tc_options &o = L.opt;
    L.n = (uint32_t)n;
    L.m = (uint32_t)m;
    L.mf = (flags & TC_EDGES_BOTH) ? (uint32_t)(m / 2) : (uint32_t)m;
    L.kcap = L.m > L.n ? L.m : L.n;
    L.id_bits = (uint32_t)id_bits_for(L.n);
    // row blocks: at most what 32-bit list ids (block * (n + 1) + v) allow
    L.nblk = o.row_blocks;
    while (L.nblk > 1 && (uint64_t)L.nblk * ((uint64_t)n + 1) >= (1ull << 32)) --L.nblk;
    const uint32_t pr = o.panel_ranks < L.n ? o.panel_ranks : L.n;
    L.p0 = L.n - pr;
    {
        const uint32_t h = o.hub_ranks < L.n ? o.hub_ranks : L.n;
        L.h0 = L.n - h;
        L.hp = (h + 63u) & ~63u;
    }
    L.panels = ceil_div(L.n - L.p0, count_panel());
    // The 16-bit region holds the panel region (whose streamed entries are all panel ranks or
    // higher) and spans at most 2^16 ranks (panel regions are smaller).  Its rows' parts in
    // hcol take at most 7 + count_hcol_pad() padding entries each; 32-bit positions must
    // address them all, or there is no region (as for high_ranks = 0).
    {
        const uint64_t rows = (uint64_t)n < L.mf ? (uint64_t)n : L.mf;
        L.hcap = ((uint64_t)L.mf + (7 + count_hcol_pad()) * rows + 64 + 7) & ~7ull;
        if (o.high_ranks == 0 || L.hcap >= (1ull << 32)) {
            L.hbase = L.n;
            L.hcap = 64;
        } else {
            L.hbase = L.n > o.high_ranks ? L.n - o.high_ranks : 0u;
            L.hbase = L.hbase < L.p0 ? L.hbase : L.p0;
        }
    }
    const uint64_t n1 = (uint64_t)n + 1;
    L.lists = (uint64_t)L.nblk * n1;
    const uint64_t l1 = L.lists + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1), 256);
        return at;
    };
    L.ctl = take(kCtlWords * 4);
    // degree partition: buckets of 2^part_shift ids, at most 256 of them
    {
        const uint64_t endpoints = (flags & TC_EDGES_BOTH) ? (uint64_t)m : 2ull * (uint64_t)m;
        const int db = L.id_bits < 8 ? (int)L.id_bits : 8;
        L.part_shift = (int)L.id_bits - db;
        // degree_partition = 0 forces the atomic path (the one that inputs of more than 2^27
        // vertices or 2^32 endpoints take)
        const bool part_on = o.degree_partition != 0;
        L.part_tiles = (part_on && endpoints < (1ull << 32) && L.part_shift <= 19)
                           ? ceil_div((uint64_t)m > 0 ? (uint64_t)m : 1, kPartTileEdges)
                           : 0u;
        // one-direction format: the edges are also partitioned into 16 x 16 cells of id ranges
        L.cell_shift = (L.part_tiles && !(flags & TC_EDGES_BOTH))
                           ? (L.id_bits > 4 ? (int)L.id_bits - 4 : 0)
                           : -1;
        const uint64_t hp = (L.cell_shift >= 0 ? 512ull : 256ull) *
                                (L.part_tiles ? L.part_tiles : 1) + 1;
        L.part_hist = take(hp * 4);
        L.part_offs = take(hp * 4);
        L.part_scan = take(scan_scratch_words(hp) * 4);
    }
    L.deg = take((size_t)n * 4);
    L.perm = take((size_t)n * 4);
    L.rank = take((size_t)n * 4);
    L.keys_a = take((size_t)L.kcap * 8);
    L.keys_b = take((size_t)L.kcap * 8);
    L.sort_scratch = take(sort_scratch_bytes(L.kcap));  // edge, vertex and in-edge sorts
    L.rs = take(n1 * 4);
    L.re = take(n1 * 4);
    L.rowlen = take(n1 * 4);
    L.row_ptr = take(n1 * 4);
    L.col = take((size_t)L.mf * 4 + count_col_pad_bytes());  // piece reads may pass the end
    L.hcol = take((size_t)L.hcap * 2);
    L.hrow = take((size_t)n * 4);
    L.hstart = take(n1 * 4);
    L.src = take((size_t)L.mf * 4);
    // rows sorted in place after a sort by source only: chunk table and the long rows' list
    L.rchunk = take(((size_t)L.mf / row_sort_chunk() + 2) * 4);
    L.long_rows = take(((size_t)L.mf / (row_sort_wave() + 1) + 2) * 4);
    L.vrange = take((size_t)n * 8);
    L.prange = take((size_t)L.panels * 8);
    L.eu = take((size_t)L.mf * 16);  // also the cell-ordered edges (8 bytes per entry)
    L.lrs = take(l1 * 4);
    L.lre = take(l1 * 4);
    L.cnt = take(l1 * 4);
    L.cptr = take(l1 * 4);
    L.cbeg = take((size_t)L.mf * 4);
    for (int k = 0; k < 4; ++k) {
        const uint32_t per = (k & 1) ? o.block_item_edges : o.wave_item_edges;
        L.items[k] = take(l1 * 4);
        L.off[k] = take(l1 * 4);
        L.item_v[k] = take(((size_t)L.mf / per + l1 + 1) * 4);
    }
    L.scan_scratch = take(scan_scratch_words(l1 > n1 ? l1 : n1) * 4);
    L.tpv = take((size_t)n * 8);
    L.hub_a = take((size_t)L.hp * L.hp);
    L.hub_at = take((size_t)L.hp * L.hp);
    L.total_bytes = off;
    {
        uint32_t w[8 + sizeof(tc_options) / 4];
        w[0] = L.n;
        w[1] = L.m;
        w[2] = flags;
        w[3] = L.p0;
        w[4] = L.h0;
        w[5] = L.nblk;
        w[6] = L.part_tiles;
        w[7] = (uint32_t)L.cell_shift;
        memcpy(w + 8, &o, sizeof(tc_options));
        L.finger = fnv_words(w, sizeof(w) / 4) | 1u;
    }
    return true;
}

template <class T>
static T *at(void *ws, size_t off) {
    return (T *)((char *)ws + off);
}

static inline uint32_t grid_for(uint64_t items, uint32_t threads, uint32_t cap = 0x7FFFFFFFu) {
    uint64_t g = (items + threads - 1) / threads;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

#define TC_LAUNCH_CHECK()                    \
    do {                                     \
        if (hipGetLastError() != hipSuccess) \
            return TC_E_HIP;                 \
    } while (0)

#define TC_HIP(x)                \
    do {                         \
        if ((x) != hipSuccess)   \
            return TC_E_HIP;     \
    } while (0)

static int check_args(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                      const tc_options *opts, void *d_ws, size_t ws_bytes, Layout &L) {
    if (n < 0 || m < 0 || (flags & ~TC_EDGES_BOTH)) return TC_E_ARG;
    if (n >= (1ll << 31) || m >= (1ll << 32)) return TC_E_TOO_LARGE;
    if (n == 0 && m > 0) return TC_E_ARG;
    if (m > 0 && (!d_edges || ((uintptr_t)d_edges & 7))) return TC_E_ARG;
    if ((flags & TC_EDGES_BOTH) && (m & 1)) return TC_E_ASYMMETRIC;
    if (!make_layout(n, m, flags, opts, L)) return TC_E_ARG;
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < L.total_bytes) return TC_E_WORKSPACE;
    return TC_OK;
}

// Preprocessing (Section 3.2) plus the counting kernel's work lists: degrees, order,
// orientation, key sort, node array, in-edge lists, work items.
static int run_preprocess(const int32_t *d_edges, uint32_t flags, void *ws, const Layout &L,
                          hipStream_t s) {
    const uint32_t n = L.n, m = L.m, mf = L.mf, n1 = L.n + 1;
    const int b = (int)L.id_bits;
    uint32_t *ctl = at<uint32_t>(ws, L.ctl);
    int32_t *status = (int32_t *)ctl + kCtlStatus;
    uint32_t *deg = at<uint32_t>(ws, L.deg);
    uint32_t *perm = at<uint32_t>(ws, L.perm);
    uint32_t *rank = at<uint32_t>(ws, L.rank);
    uint64_t *ka = at<uint64_t>(ws, L.keys_a), *kb = at<uint64_t>(ws, L.keys_b);
    void *sort_scr = at<void>(ws, L.sort_scratch);
    uint32_t *row_ptr = at<uint32_t>(ws, L.row_ptr);
    uint32_t *col = at<uint32_t>(ws, L.col);
    uint32_t *src = at<uint32_t>(ws, L.src);
    const int2 *edges = (const int2 *)d_edges;
    const bool both = flags & TC_EDGES_BOTH;

    uint32_t *scan_scr = at<uint32_t>(ws, L.scan_scratch);
    // cell-ordered edges for the orientation: the in-edge payload buffer, unused until later
    int2 *cells = L.cell_shift >= 0 ? at<int2>(ws, L.eu) : nullptr;
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, L.finger);
    TC_LAUNCH_CHECK();
    const bool onesweep = L.opt.sort_onesweep != 0;
    const bool row_sort = L.opt.row_sort && L.mf < kRowSortMaxEdges;
    TC_HIP(fill_u32(deg, 0u, n, s));
    if (m > 0 && L.part_tiles) {
        const uint32_t tiles = L.part_tiles;
        const uint64_t hp = (L.cell_shift >= 0 ? 512ull : 256ull) * tiles;
        uint32_t *ph = at<uint32_t>(ws, L.part_hist), *po = at<uint32_t>(ws, L.part_offs);
        // the endpoints' offsets inside their buckets, 2 bytes each when a bucket holds at most
        // 2^16 ids, else 4 (either fits the 8-byte key buffer)
        const bool narrow = L.part_shift <= 16;
        TC_HIP(fill_u32(ph + hp, 0u, 1, s));
        hipLaunchKernelGGL(k_part_hist, dim3(tiles), dim3(256), 0, s, edges, (uint64_t)m, n,
                           (uint32_t)both, L.part_shift, L.cell_shift, ph, tiles, status);
        TC_LAUNCH_CHECK();
        TC_HIP(scan_exclusive_u32(ph, po, hp + 1, at<uint32_t>(ws, L.part_scan), s));
        if (narrow)
            hipLaunchKernelGGL((k_part_scatter<uint16_t>), dim3(tiles), dim3(256), 0, s, edges,
                               (uint64_t)m, n, (uint32_t)both, L.part_shift, L.cell_shift, ph,
                               po, tiles, (uint16_t *)kb, cells);
        else
            hipLaunchKernelGGL((k_part_scatter<uint32_t>), dim3(tiles), dim3(256), 0, s, edges,
                               (uint64_t)m, n, (uint32_t)both, L.part_shift, L.cell_shift, ph,
                               po, tiles, (uint32_t *)kb, cells);
        TC_LAUNCH_CHECK();
        const uint32_t buckets = 1u << (L.id_bits - L.part_shift);
        const uint32_t slices = buckets >= 512 ? 1u : 512u / buckets;
        if (narrow)
            hipLaunchKernelGGL((k_part_count<uint16_t>), dim3(buckets * slices), dim3(1024), 0, s,
                               (const uint16_t *)kb, po, tiles, L.part_shift, n, slices, deg,
                               status);
        else
            hipLaunchKernelGGL((k_part_count<uint32_t>), dim3(buckets * slices), dim3(1024), 0, s,
                               (const uint32_t *)kb, po, tiles, L.part_shift, n, slices, deg,
                               status);
        TC_LAUNCH_CHECK();
    } else if (m > 0) {
        hipLaunchKernelGGL(k_degree_atomic, dim3(grid_for(m, 256, 8192)), dim3(256), 0, s, edges,
                           (uint64_t)m, n, (uint32_t)both, deg, status);
        TC_LAUNCH_CHECK();
    }
    // the order of Section 2.2 as ranks: stable sort of (degree << b | id) on the degree bits
    if (n > 0) {
        hipLaunchKernelGGL(k_vkeys, dim3(grid_for(n, 256)), dim3(256), 0, s, deg, n, b, ka);
        TC_LAUNCH_CHECK();
        // the last pass writes perm and rank
        TC_HIP(sort_ranks(ka, kb, n, b, 2 * b, b, perm, rank, sort_scr, nullptr, s));
    }
    uint64_t *sorted = ka;
    if (m > 0) {
        if (cells) {
            hipLaunchKernelGGL(k_orient_cells, dim3(kOrientGrid), dim3(256), 0, s, cells,
                               (uint64_t)m, n, rank, b, ka, status);
        } else {
            hipLaunchKernelGGL(k_orient, dim3(grid_for(m, 256, 8192)), dim3(256), 0, s, edges,
                               (uint64_t)m, (uint32_t)both, rank, b, ka, ctl + kCtlBoth, status);
        }
        TC_LAUNCH_CHECK();
        if (both) {
            hipLaunchKernelGGL(k_both_check, dim3(1), dim3(64), 0, s, ctl + kCtlBoth, mf, status);
            TC_LAUNCH_CHECK();
        }
        if (row_sort)  // by source only, unzipped by the last pass (rows sorted by k_row_sort)
            TC_HIP(sort_unzip(ka, kb, mf, b, 2 * b, b, col, src, sort_scr, status, s, onesweep));
        else
            TC_HIP(sort_u64(ka, kb, mf, 0, 2 * b, sort_scr, status, s, &sorted, onesweep));
    }
    if (mf == 0) {
        TC_HIP(fill_u32(row_ptr, 0u, n1, s));
        return TC_OK;
    }
    // node array: row boundaries -> row lengths -> exclusive scan
    uint32_t *rs = at<uint32_t>(ws, L.rs), *re = at<uint32_t>(ws, L.re);
    uint32_t *rowlen = at<uint32_t>(ws, L.rowlen);
    TC_HIP(fill_u32(rs, 0u, n1, s));
    TC_HIP(fill_u32(re, 0u, n1, s));
    uint32_t *hrow = at<uint32_t>(ws, L.hrow);
    TC_HIP(fill_u32(hrow, ~0u, n, s));
    uint32_t *rchunk = at<uint32_t>(ws, L.rchunk);
    // 4 entries per thread (prep.hip, kCsrKeys)
    if (row_sort)
        hipLaunchKernelGGL(k_row_bounds, dim3(grid_for(mf, 256 * 4)), dim3(256), 0, s, src, mf,
                           n, rs, re, rchunk, status);
    else
        hipLaunchKernelGGL(k_csr, dim3(grid_for(mf, 256 * 4)), dim3(256), 0, s, sorted, mf, n,
                           b, L.hbase, col, src, rs, re, hrow, status);
    TC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rowlen, dim3(grid_for(n1, 256)), dim3(256), 0, s, rs, re, n, rowlen);
    TC_LAUNCH_CHECK();
    TC_HIP(scan_exclusive_u32(rowlen, row_ptr, n1, scan_scr, s));
    if (row_sort) {  // every row sorted in place, with the duplicate check and hrow
        const uint32_t chunks = ceil_div(mf, row_sort_chunk());
        uint32_t *long_rows = at<uint32_t>(ws, L.long_rows);
        hipLaunchKernelGGL(k_row_sort, dim3(chunks), dim3(256), 0, s, col, row_ptr, rchunk,
                           chunks, n, L.hbase, hrow, long_rows, ctl + kCtlLongRows, status);
        TC_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_row_sort_long, dim3(device_cu_count()), dim3(1024), 0, s, col,
                           row_ptr, long_rows, ctl + kCtlLongRows, L.hbase, hrow, status);
        TC_LAUNCH_CHECK();
    }
    // every row's part of hcol (row lengths are no longer needed: their array takes the parts'
    // sizes); hcol starts as zeros, the parts' padding
    uint32_t *hstart = at<uint32_t>(ws, L.hstart);
    uint16_t *hcol = at<uint16_t>(ws, L.hcol);
    hipLaunchKernelGGL(k_hlen, dim3(grid_for(n1, 256)), dim3(256), 0, s, row_ptr, hrow, n,
                       count_hcol_pad(), rowlen);
    TC_LAUNCH_CHECK();
    TC_HIP(scan_exclusive_u32(rowlen, hstart, n1, scan_scr, s));
    TC_HIP(fill_u32((uint32_t *)hcol, 0u, L.hcap / 2, s));
    // the hub matrices
    if (L.hp) {
        uint8_t *ha = at<uint8_t>(ws, L.hub_a), *hat = at<uint8_t>(ws, L.hub_at);
        TC_HIP(fill_u32((uint32_t *)ha, 0u, (uint64_t)L.hp * L.hp / 4, s));
        TC_HIP(fill_u32((uint32_t *)hat, 0u, (uint64_t)L.hp * L.hp / 4, s));
        TC_HIP(launch_hub_fill(src, col, row_ptr, mf, L.h0, L.hp, ha, hat, status, s));
    }
    // in-edge lists (grouped by list c = row block * (n + 1) + v) and the counting kernel's
    // work items
    const uint64_t l1 = L.lists + 1;
    uint32_t *lrs = at<uint32_t>(ws, L.lrs), *lre = at<uint32_t>(ws, L.lre);
    uint32_t *cnt = at<uint32_t>(ws, L.cnt), *cptr = at<uint32_t>(ws, L.cptr);
    uint64_t *vr = at<uint64_t>(ws, L.vrange);
    uint32_t *items[4], *offs[4], *iv[4];
    for (int k = 0; k < 4; ++k) {
        items[k] = at<uint32_t>(ws, L.items[k]);
        offs[k] = at<uint32_t>(ws, L.off[k]);
        iv[k] = at<uint32_t>(ws, L.item_v[k]);
    }
    if (L.panels) {  // spans of the panel region's out-lists
        hipLaunchKernelGGL(k_vrange, dim3(grid_for(n - L.p0, 256)), dim3(256), 0, s, row_ptr, col,
                           L.p0, n, vr);
        TC_LAUNCH_CHECK();
    }
    // the in-edge keys: 32-bit list ids in the buffer of the sorted edge keys (no longer
    // needed), sorted into 64-bit (list, position) keys in the other buffer
    uint64_t *ck = (sorted == ka) ? kb : ka;
    uint64_t *ck2 = (sorted == ka) ? ka : kb;
    uint32_t *cid = (uint32_t *)ck2;
    uint4 *eu = at<uint4>(ws, L.eu);
    uint64_t *pr = at<uint64_t>(ws, L.prange);
    if (L.panels) {
        hipLaunchKernelGGL(k_panel_range, dim3(grid_for(L.panels, 256)), dim3(256), 0, s, vr, n,
                           L.p0, count_panel(), L.panels, pr);
        TC_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_csc_keys, dim3(grid_for(mf, 256 * kCscPerThread)), dim3(256), 0, s, col,
                       src, row_ptr, hrow, hstart, L.hbase, pr, mf, n, L.nblk, L.p0,
                       count_panel(), L.h0, cid, eu, hcol, status);
    TC_LAUNCH_CHECK();
    // sorted into (list id, cbeg) pairs: the list ids land in ck or ck2 (as 32-bit words);
    // the in-edges of no list are dropped by the first pass (ctl[kCtlKept] of them remain)
    uint32_t *clist = nullptr;
    TC_HIP(sort_lists(cid, (uint32_t)L.lists, mf, id_bits_for64(l1), ck, ck2,
                      at<uint32_t>(ws, L.cbeg), ctl + kCtlKept, sort_scr, status, s, &clist));
    TC_HIP(fill_u32(lrs, 0u, l1, s));
    TC_HIP(fill_u32(lre, 0u, l1, s));
    hipLaunchKernelGGL(k_csc_final, dim3(grid_for(mf, 256 * 4)), dim3(256), 0, s, clist, mf,
                       ctl + kCtlKept, L.lists, lrs, lre,
                       status);  // 4 ids per thread (prep.hip, kCscFinalKeys)
    TC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rowlen, dim3(grid_for(l1, 256)), dim3(256), 0, s, lrs, lre,
                       (uint32_t)L.lists, cnt);
    TC_LAUNCH_CHECK();
    TC_HIP(scan_exclusive_u32(cnt, cptr, l1, scan_scr, s));
    const tc_options &o = L.opt;
    const uint32_t wl_pv = o.wave_list_max < count_wave_list(true) ? o.wave_list_max
                                                                     : count_wave_list(true);
    hipLaunchKernelGGL(k_items, dim3(grid_for(l1, 256)), dim3(256), 0, s, row_ptr, col, cnt, n,
                       L.nblk, L.p0, o.wave_bitmap_span, o.wave_list_max, wl_pv,
                       o.wave_item_edges, o.block_item_edges, items[0], items[1], items[2],
                       items[3], status);
    TC_LAUNCH_CHECK();
    for (int k = 0; k < 4; ++k) TC_HIP(scan_exclusive_u32(items[k], offs[k], l1, scan_scr, s));
    for (int k = 0; k < 4; ++k) {
        hipLaunchKernelGGL(k_item_fill, dim3(grid_for(L.lists, 256)), dim3(256), 0, s, items[k],
                           offs[k], L.lists, iv[k], status);
        TC_LAUNCH_CHECK();
    }
    return TC_OK;
}

// Counting phase on a prepared workspace.
static int run_count_prepared(void *ws, const Layout &L, hipStream_t s, uint64_t *d_total,
                              uint64_t *d_pv) {
    const bool pv = d_pv != nullptr;
    const uint32_t n = L.n;
    uint32_t *ctl = at<uint32_t>(ws, L.ctl);
    // this count's status: the preprocessing's, or a mismatch of the prepared layout (the
    // check also resets the item queues)
    int32_t *status = (int32_t *)ctl + kCtlRun;
    hipLaunchKernelGGL(k_ctl_check, dim3(1), dim3(64), 0, s, ctl, L.finger);
    TC_LAUNCH_CHECK();
    unsigned long long *total = (unsigned long long *)d_total;
    unsigned long long *tpv = at<unsigned long long>(ws, L.tpv);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)1);
    TC_LAUNCH_CHECK();
    if (pv && n > 0) {
        hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, tpv,
                           (uint64_t)n);
        TC_LAUNCH_CHECK();
    }
    if (L.mf > 0) {
        const int a0 = pv ? 2 : 0, b0 = pv ? 3 : 1;
        CountArgs a;
        a.row_ptr = at<uint32_t>(ws, L.row_ptr);
        a.col = at<uint32_t>(ws, L.col);
        a.hcol = at<uint16_t>(ws, L.hcol);
        a.hrow = at<uint32_t>(ws, L.hrow);
        a.hbase = L.hbase;
        a.cptr = at<uint32_t>(ws, L.cptr);
        a.cbeg = at<uint32_t>(ws, L.cbeg);
        a.er = at<uint4>(ws, L.eu);
        a.item_v_a = at<uint32_t>(ws, L.item_v[a0]);
        a.item_off_a = at<uint32_t>(ws, L.off[a0]);
        a.n_items_a = a.item_off_a + L.lists;
        a.item_v_b = at<uint32_t>(ws, L.item_v[b0]);
        a.item_off_b = at<uint32_t>(ws, L.off[b0]);
        a.n_items_b = a.item_off_b + L.lists;
        a.queue_a = ctl + kCtlQueueA;
        a.queue_b = ctl + kCtlQueueB;
        a.queue_c = ctl + kCtlQueueC;
        a.total = total;
        a.tpv = tpv;
        a.n1 = n + 1;
        a.p0 = L.p0;
        const tc_options &o = L.opt;
        a.wave_bits = o.wave_bitmap_span;
        a.block_bits = o.block_bitmap_span;
        a.block_list = o.block_list_max < count_block_list(pv) ? o.block_list_max
                                                                : count_block_list(pv);
        a.kitem_a = o.wave_item_edges;
        a.kitem_b = o.block_item_edges;
        a.status = status;
        TC_HIP(launch_count(a, pv, s));
        TC_HIP(launch_hub_count(at<uint8_t>(ws, L.hub_a), at<uint8_t>(ws, L.hub_at), L.hp, L.h0,
                                total, tpv, pv, status, s));
    }
    if (pv && n > 0) {
        hipLaunchKernelGGL(k_pv_out, dim3(grid_for(n, 256)), dim3(256), 0, s, tpv,
                           at<uint32_t>(ws, L.perm), n, (unsigned long long *)d_pv);
        TC_LAUNCH_CHECK();
    }
    return TC_OK;
}

static int copy_status(void *ws, const Layout &L, int32_t *d_status, hipStream_t s,
                       int word) {
    if (!d_status) return TC_OK;
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, at<int32_t>(ws, L.ctl) + word,
                       d_status);
    TC_LAUNCH_CHECK();
    return TC_OK;
}

// Preprocessing and counting in one call.
static int run_count(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                     const tc_options *opts, void *ws, size_t ws_bytes, hipStream_t s,
                     uint64_t *d_total, uint64_t *d_pv, int32_t *d_status) {
    Layout L;
    int st = check_args(d_edges, n, m, flags, opts, ws, ws_bytes, L);
    if (st) return st;
    if (!d_total) return TC_E_ARG;
    st = run_preprocess(d_edges, flags, ws, L, s);
    if (st) return st;
    st = run_count_prepared(ws, L, s, d_total, L.n > 0 ? d_pv : nullptr);
    if (st) return st;
    return copy_status(ws, L, d_status, s, kCtlRun);
}

// ------------------------------------------------------------------ static scratch

// The workspace of tc_count_noalloc: a file-scope device array that every GPU the library
// runs on holds until the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): each device's own address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is the workspace
// pointer the kernels get.
constexpr size_t kScratchBytes = TC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// this device's address of `scratch` (nullptr on a HIP error)
static void *scratch_on_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace tc

using namespace tc;

extern "C" {

const char *tc_strerror(int status) {
    switch (status) {
        case TC_OK: return "ok";
        case TC_E_ARG: return "invalid argument";
        case TC_E_RANGE: return "vertex id out of range";
        case TC_E_SELF_LOOP: return "self-loop";
        case TC_E_DUP_EDGE: return "duplicate edge";
        case TC_E_ASYMMETRIC: return "two-direction edge array without matching mirror entries";
        case TC_E_UNSORTED: return "adjacency row not strictly ascending";
        case TC_E_WORKSPACE: return "workspace too small or misaligned";
        case TC_E_TOO_LARGE: return "graph too large for 32-bit indices";
        case TC_E_HIP: return "HIP runtime error";
        case TC_E_MISMATCH: return "workspace prepared for another graph size or other options";
        case TC_E_SCRATCH:
            return "graph needs more workspace than tc_count_noalloc's static scratch "
                   "(TC_NOALLOC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}

int tc_options_init(tc_options *opts) {
    if (!opts) return TC_E_ARG;
    default_options(*opts);
    return TC_OK;
}

size_t tc_workspace_size(int64_t n, int64_t m, uint32_t flags, const tc_options *opts) {
    Layout L;
    if (!make_layout(n, m, flags, opts, L)) return 0;
    return L.total_bytes;
}

int tc_workspace_layout(int64_t n, int64_t m, uint32_t flags, const tc_options *opts,
                        tc_layout *out) {
    Layout L;
    if (!out) return TC_E_ARG;
    if (!make_layout(n, m, flags, opts, L)) return TC_E_ARG;
    out->deg = L.deg;
    out->perm = L.perm;
    out->rank = L.rank;
    out->row_ptr = L.row_ptr;
    out->col = L.col;
    out->src = L.src;
    out->m_fwd = L.mf;
    out->id_bits = (int32_t)L.id_bits;
    return TC_OK;
}

int tc_count(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
             const tc_options *opts, void *d_ws, size_t ws_bytes, void *stream,
             uint64_t *d_total, int32_t *d_status) {
    return run_count(d_edges, n, m, flags, opts, d_ws, ws_bytes, (hipStream_t)stream, d_total,
                     nullptr, d_status);
}

int tc_count_per_vertex(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                        const tc_options *opts, void *d_ws, size_t ws_bytes, void *stream,
                        uint64_t *d_total, uint64_t *d_per_vertex, int32_t *d_status) {
    if (!d_per_vertex && n > 0) return TC_E_ARG;
    return run_count(d_edges, n, m, flags, opts, d_ws, ws_bytes, (hipStream_t)stream, d_total,
                     d_per_vertex, d_status);
}

int tc_preprocess(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                  const tc_options *opts, void *d_ws, size_t ws_bytes, void *stream,
                  int32_t *d_status) {
    Layout L;
    int st = check_args(d_edges, n, m, flags, opts, d_ws, ws_bytes, L);
    if (st) return st;
    st = run_preprocess(d_edges, flags, d_ws, L, (hipStream_t)stream);
    if (st) return st;
    return copy_status(d_ws, L, d_status, (hipStream_t)stream, kCtlStatus);
}

int tc_count_noalloc(const int32_t *d_edges, int64_t n, int64_t m, uint32_t flags,
                     const tc_options *opts, void *stream, uint64_t *d_total,
                     int32_t *d_status) {
    Layout L;
    if (n < 0 || m < 0 || (flags & ~TC_EDGES_BOTH)) return TC_E_ARG;
    if (n >= (1ll << 31) || m >= (1ll << 32)) return TC_E_TOO_LARGE;
    if (!make_layout(n, m, flags, opts, L)) return TC_E_ARG;
    if (L.total_bytes > kScratchBytes) return TC_E_SCRATCH;
    void *ws = scratch_on_current_device();
    if (!ws) return TC_E_HIP;
    return run_count(d_edges, n, m, flags, opts, ws, kScratchBytes, (hipStream_t)stream, d_total,
                     nullptr, d_status);
}

int tc_count_prepared(int64_t n, int64_t m, uint32_t flags, const tc_options *opts,
                      void *d_ws, size_t ws_bytes, void *stream, uint64_t *d_total,
                      uint64_t *d_per_vertex, int32_t *d_status) {
    Layout L;
    if (n < 0 || m < 0 || (flags & ~TC_EDGES_BOTH)) return TC_E_ARG;
    if (n >= (1ll << 31) || m >= (1ll << 32)) return TC_E_TOO_LARGE;
    if (!make_layout(n, m, flags, opts, L) || !d_total) return TC_E_ARG;
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < L.total_bytes) return TC_E_WORKSPACE;
    int st = run_count_prepared(d_ws, L, (hipStream_t)stream, d_total,
                                L.n > 0 ? d_per_vertex : nullptr);
    if (st) return st;
    return copy_status(d_ws, L, d_status, (hipStream_t)stream, kCtlRun);
}

size_t tc_sort_workspace_size(int64_t count) {
    if (count < 0 || count >= (1ll << 32)) return 0;
    return sort_scratch_bytes((uint64_t)count);
}

int tc_sort_u64(uint64_t *d_keys, uint64_t *d_tmp, int64_t count, int32_t bits, void *d_ws,
                size_t ws_bytes, void *stream) {
    if (count < 0 || bits < 1 || bits > 64) return TC_E_ARG;
    if (count >= (1ll << 32)) return TC_E_TOO_LARGE;
    if (count > 0 && (!d_keys || !d_tmp)) return TC_E_ARG;
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < sort_scratch_bytes((uint64_t)count))
        return TC_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    uint64_t *res = nullptr;
    TC_HIP(sort_u64(d_keys, d_tmp, (uint32_t)count, 0, bits, d_ws, nullptr, s, &res));
    if (res != d_keys)
        TC_HIP(hipMemcpyAsync(d_keys, res, (size_t)count * 8, hipMemcpyDeviceToDevice, s));
    return TC_OK;
}

}  // extern "C"
