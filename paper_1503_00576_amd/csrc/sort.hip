// Device-wide exclusive scan and stable LSD radix sort of uint64 keys.
//
// The sort replaces the library sort of packed 64-bit edge keys in the preprocessing phase
// (Section 3.2, step 3, and the note on sorting edges as 64-bit integers): keys are ordered
// on a bit range [lo_bit, hi_bit) with 8-bit digits, least significant digit first; every
// pass is an upsweep (per-tile digit histograms), an exclusive scan of the digit-major
// histogram table, and a stable scatter in which every wave ranks its own contiguous part of
// the tile with ballots, the tile is ordered by digit in LDS, and every digit's run is
// written out contiguously.
//
// Single-sweep variant (large sorts that report errors through a status word): one upfront
// kernel counts the digits of every pass over all keys; each pass is then one kernel whose
// tiles take consecutive ids in launch order, publish their digit counts, and add up their
// predecessors' published counts (decoupled look-back) instead of reading a scanned table,
// which saves the upsweep's read of every key and the scan per pass.  A tile only waits on
// tiles that started before it and publish before they wait themselves, so the waits end;
// every wait is also bounded and reports TC_E_HIP if the bound is ever reached.
#include "internal.h"

namespace tc {

// ======================================================================= fill

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, uint64_t count) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

hipError_t fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

// ======================================================================= scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

__device__ __forceinline__ uint32_t pad_idx(uint32_t i) { return i + (i >> 5); }

// Block-level exclusive scan of one 4096-element tile.
//   mode 0: write only the tile total to sums[blockIdx.x]
//   mode 1: write the exclusive scan, offset by carry[blockIdx.x] (if carry != nullptr)
__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out,
                                                            uint64_t N, int mode,
                                                            uint32_t *__restrict__ sums,
                                                            const uint32_t *__restrict__ carry) {
    __shared__ uint32_t s[kScanTile + kScanTile / 32];
    __shared__ uint32_t s_wave[kScanThreads / kWave];
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint32_t i = j * kScanThreads + t;
        s[pad_idx(i)] = (base + i < N) ? in[base + i] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems];
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = run;
        run += s[pad_idx(t * kScanItems + j)];
    }
    uint32_t incl = wave_incl_scan(run);
    const uint32_t w = t / kWave;
    if (lane_id() == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    uint32_t wave_off = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        if ((uint32_t)k < w) wave_off += s_wave[k];
        total += s_wave[k];
    }
    if (mode == 0) {
        if (t == 0) sums[blockIdx.x] = total;
        return;
    }
    uint32_t off = (incl - run) + wave_off + (carry ? carry[blockIdx.x] : 0u);
    // all reads of s above happened before the barrier below
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s[pad_idx(t * kScanItems + j)] = v[j] + off;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint32_t i = j * kScanThreads + t;
        if (base + i < N) out[base + i] = s[pad_idx(i)];
    }
}

size_t scan_scratch_words(uint64_t N) {
    uint64_t nb = (N + kScanTile - 1) / kScanTile;
    uint64_t words = nb + 1;
    if (nb > 1) words += scan_scratch_words(nb);
    return (size_t)align_up(words, 64);
}

hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint64_t N, uint32_t *scratch,
                              hipStream_t s) {
    if (N == 0) return hipSuccess;
    uint32_t nb = ceil_div(N, kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kScanThreads), 0, s, in, out, N, 1,
                           (uint32_t *)nullptr, (const uint32_t *)nullptr);
        return hipGetLastError();
    }
    uint32_t *sums = scratch;
    uint32_t *rest = scratch + align_up((size_t)nb + 1, 64);
    hipLaunchKernelGGL(k_scan_tile, dim3(nb), dim3(kScanThreads), 0, s, in, out, N, 0, sums,
                       (const uint32_t *)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive_u32(sums, sums, nb, rest, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_tile, dim3(nb), dim3(kScanThreads), 0, s, in, out, N, 1,
                       (uint32_t *)nullptr, (const uint32_t *)sums);
    return hipGetLastError();
}

// ======================================================================= radix sort

// A tile is 8192 keys for 512 threads; wave w owns the contiguous keys [1024 w, 1024 (w + 1))
// of the tile as 16 rows of 64, so that a wave ranks its keys with counters of its own and
// the tile needs no barrier per row: the stable order of the tile is wave by wave, row by
// row, lane by lane.
constexpr int kSortThreads = 512;
constexpr int kSortItems = 16;
constexpr int kSortWaves = kSortThreads / kWave;     // 8
constexpr int kSortTile = kSortThreads * kSortItems;  // 8192 keys per tile

// Lanes holding the same 8-bit digit as the calling lane: returns the mask of such (valid)
// lanes.  Per bit: m = all ones where the lane's bit is set, the ballot of that bit, and
// peers &= ~(ballot ^ m) on both halves.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint32_t m = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
        const uint64_t bb = __ballot(m != 0u);
        lo &= ~((uint32_t)bb ^ m);
        hi &= ~((uint32_t)(bb >> 32) ^ m);
    }
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t tile_key_index(uint64_t base, uint32_t w, int r) {
    return base + (uint64_t)w * (kSortItems * kWave) + (uint64_t)r * kWave + lane_id();
}

// Where a pass reads its keys: 64-bit keys, or (for the first pass of a sort of keys
// (value << 32) | position) 32-bit values whose key is formed with the value's own index, so
// that the producer writes and the first pass reads 4 bytes per key instead of 8.
// keep(key): whether the pass takes the key (the others are dropped, and the output holds
// only the kept keys, in order).
struct Keys64 {  // (read once per pass, with a non-temporal hint: no reuse within a pass)
    const uint64_t *p;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const {
        return __builtin_nontemporal_load(p + i);
    }
    __device__ __forceinline__ bool keep(uint64_t) const { return true; }
};
struct KeysHiIndex {  // drops the keys whose value is `drop`
    const uint32_t *p;
    uint32_t drop;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const {
        return ((uint64_t)__builtin_nontemporal_load(p + i) << 32) | (uint32_t)i;
    }
    __device__ __forceinline__ bool keep(uint64_t key) const {
        return (uint32_t)(key >> 32) != drop;
    }
};

// Where a pass writes its keys: 64-bit keys, or split for the last pass of the in-edge list
// sort into the list id (high half) and the list entry cbeg = position + 1 (low half + 1).
struct Out64 {
    uint64_t *p;
    __device__ __forceinline__ void operator()(uint64_t pos, uint64_t key) const { p[pos] = key; }
};
// ... or unzipped, for the last pass of the edge sort: target (low b bits) and source.
struct OutColSrc {
    uint32_t *col, *src;
    uint64_t tmask;
    int b;
    __device__ __forceinline__ void operator()(uint64_t pos, uint64_t key) const {
        col[pos] = (uint32_t)(key & tmask);
        src[pos] = (uint32_t)(key >> b);
    }
};
// ... or, for the last pass of the vertex order: perm[r] = the vertex (low b bits) of the key
// at position r, rank[vertex] = r.
struct OutPermRank {
    uint32_t *perm, *rank;
    uint64_t mask;
    __device__ __forceinline__ void operator()(uint64_t pos, uint64_t key) const {
        const uint32_t x = (uint32_t)(key & mask);
        perm[pos] = x;
        rank[x] = (uint32_t)pos;
    }
};
struct OutListBeg {
    uint32_t *list, *beg;
    __device__ __forceinline__ void operator()(uint64_t pos, uint64_t key) const {
        list[pos] = (uint32_t)(key >> 32);
        beg[pos] = (uint32_t)key + 1u;
    }
};

// Loads the calling wave's 16 rows of the tile (all loads in flight before any use) and
// returns the lane's mask of rows whose key takes part (below count, and kept);
// kFull: the whole tile lies below count.
template <bool kFull, class Src>
__device__ __forceinline__ uint32_t load_tile_keys(const Src in, uint32_t count, uint64_t base,
                                                   uint32_t w, uint64_t (&keys)[kSortItems]) {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t idx = tile_key_index(base, w, r);
        keys[r] = (kFull || idx < count) ? in(idx) : 0ull;
    }
    uint32_t vmask = 0;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t idx = tile_key_index(base, w, r);
        if ((kFull || idx < count) && in.keep(keys[r])) vmask |= 1u << r;
    }
    return vmask;
}

// Per-wave digit counts of the wave's rows into cnt[256] (the wave's own row of counters,
// zero on entry), and each key's rank among the wave's earlier keys of the same digit.
__device__ __forceinline__ void wave_rank_rows(const uint64_t (&keys)[kSortItems], uint32_t vmask,
                                               int shift, uint32_t mask, uint32_t *cnt,
                                               uint32_t (&ranks)[kSortItems]) {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool valid = (vmask >> r) & 1u;
        const uint32_t d = (uint32_t)(keys[r] >> shift) & mask;
        const uint64_t peers = match_digit(d, valid);
        const uint32_t below = lanes_below(peers);
        const uint32_t prev = valid ? cnt[d] : 0u;
        ranks[r] = prev + below;
        if (valid && below == 0) cnt[d] = prev + (uint32_t)__popcll(peers);
        wave_lds_sync();  // this row's counter updates before the next row's reads
    }
}

// Shared state of one tile's stable placement in digit order.
struct SortTileLds {
    uint64_t stage[kSortTile];
    uint32_t wcnt[kSortWaves][256];  // per-wave digit counts, then per-wave digit offsets
    uint32_t loc[256];               // tile-local start of each digit
    uint32_t glob[256];              // global start minus local start of each digit
    uint32_t dsum[4];                // per-wave sums of the digit scan (digits by 4 waves)
    uint32_t gsum[4];                // the same for the global digit counts (single sweep)
    uint32_t total;                  // keys of the tile that take part
};

// Block part of the placement (all threads, after the waves' counts are in wcnt): turns wcnt
// into per-wave digit offsets, fills loc, and returns the tile's count of digit t (t < 256).
__device__ __forceinline__ uint32_t tile_digit_offsets(SortTileLds &L) {
    const uint32_t t = threadIdx.x;
    __syncthreads();
    uint32_t c = 0;
    if (t < 256) {
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            const uint32_t x = L.wcnt[k][t];
            L.wcnt[k][t] = c;
            c += x;
        }
    }
    const uint32_t incl = wave_incl_scan(t < 256 ? c : 0u);
    if (t < 256 && lane_id() == kWave - 1) L.dsum[t / kWave] = incl;
    __syncthreads();
    if (t < 256) {
        uint32_t before = 0;
        for (uint32_t k = 0; k < t / kWave; ++k) before += L.dsum[k];
        L.loc[t] = before + incl - c;
        if (t == 255) L.total = before + incl;
    }
    return c;
}

// Places the wave's keys in L.stage (after tile_digit_offsets and a barrier).
__device__ __forceinline__ void stage_keys(SortTileLds &L, const uint64_t (&keys)[kSortItems],
                                           const uint32_t (&ranks)[kSortItems], uint32_t vmask,
                                           uint32_t w, int shift, uint32_t mask) {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if ((vmask >> r) & 1u) {
            const uint32_t d = (uint32_t)(keys[r] >> shift) & mask;
            L.stage[L.loc[d] + L.wcnt[w][d] + ranks[r]] = keys[r];
        }
    }
}

// Writes the staged tile (L.total keys): consecutive threads write consecutive positions of
// one digit's run (L.glob[d] + j is the output position of staged key j of digit d).
template <class Dst>
__device__ __forceinline__ void write_staged(const SortTileLds &L, const Dst out, uint32_t count,
                                             int shift, uint32_t mask, int32_t *status) {
    const uint32_t ntile = L.total;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t j = (uint32_t)i * kSortThreads + threadIdx.x;
        if (j < ntile) {
            const uint64_t key = L.stage[j];
            const uint32_t d = (uint32_t)(key >> shift) & mask;
            const uint32_t pos = L.glob[d] + j;
            if (!status) {
                out(pos, key);
            } else if (pos < count) {  // holds whenever the prefixes are right
                out(pos, key);
            } else {
                set_status(status, TC_E_HIP);
            }
        }
    }
}

template <bool kFull, class Src>
__device__ __forceinline__ void hist_tile(const Src in, uint32_t count, int shift,
                                          uint32_t mask, uint32_t *__restrict__ hist,
                                          uint32_t tiles, uint32_t tile,
                                          uint32_t (&h)[kSortWaves][256]) {
    const uint32_t t = threadIdx.x, w = t / kWave;
    const uint64_t base = (uint64_t)tile * kSortTile;
    uint64_t keys[kSortItems];
    const uint32_t vmask = load_tile_keys<kFull>(in, count, base, w, keys);
    for (uint32_t k = lane_id(); k < 256; k += kWave) h[w][k] = 0;
    wave_lds_sync();
    // counts only (no ranks): the keys of a row that share the first lane's digit are added
    // with one LDS atomic, the others one atomic each, into the wave's own counters (skewed
    // keys -- hub ranks, long runs of equal digits after the first pass -- would otherwise
    // serialise many atomics on one counter)
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool valid = (vmask >> r) & 1u;
        const uint32_t d = (uint32_t)(keys[r] >> shift) & mask;
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
        const uint64_t same = __ballot(valid && d == d0);
        if (lane_id() == 0 && same) atomicAdd(&h[w][d0], (uint32_t)__popcll(same));
        if (valid && d != d0) atomicAdd(&h[w][d], 1u);
    }
    __syncthreads();
    if (t < 256) {
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) sum += h[k][t];
        hist[(uint64_t)t * tiles + tile] = sum;
    }
}

// dcount (nullable): the number of keys, read from the device (a bound set by an earlier pass
// that dropped keys; count is then the capacity the grid was sized for)
template <class Src>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const Src in, uint32_t count,
                                                             const uint32_t *__restrict__ dcount,
                                                             int shift, uint32_t nbits,
                                                             uint32_t *__restrict__ hist,
                                                             uint32_t tiles,
                                                             const int32_t *__restrict__ status) {
    if (status && *status) return;
    if (dcount) count = min(count, *dcount);
    __shared__ uint32_t h[kSortWaves][256];
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    const uint32_t mask = (1u << nbits) - 1u;
    if ((uint64_t)(tile + 1) * kSortTile <= count)
        hist_tile<true>(in, count, shift, mask, hist, tiles, tile, h);
    else
        hist_tile<false>(in, count, shift, mask, hist, tiles, tile, h);
}

// Stable scatter of one tile: the keys are ranked and placed in LDS in digit order (a
// tile-local counting sort), then written out digit run by digit run.
//   offs: exclusive scan of the digit-major table of per-tile digit counts
template <bool kFull, class Src, class Dst>
__device__ __forceinline__ void scatter_tile(const Src in, const Dst out, uint32_t count,
                                             int shift, uint32_t mask,
                                             const uint32_t *__restrict__ offs, uint32_t tiles,
                                             uint32_t tile, SortTileLds &L) {
    const uint32_t t = threadIdx.x, w = t / kWave;
    const uint64_t base = (uint64_t)tile * kSortTile;
    uint64_t keys[kSortItems];
    const uint32_t vmask = load_tile_keys<kFull>(in, count, base, w, keys);
    for (uint32_t k = lane_id(); k < 256; k += kWave) L.wcnt[w][k] = 0;
    wave_lds_sync();
    uint32_t ranks[kSortItems];
    wave_rank_rows(keys, vmask, shift, mask, L.wcnt[w], ranks);
    tile_digit_offsets(L);
    if (t < 256) L.glob[t] = offs[(uint64_t)t * tiles + tile] - L.loc[t];
    __syncthreads();
    stage_keys(L, keys, ranks, vmask, w, shift, mask);
    __syncthreads();
    write_staged(L, out, count, shift, mask, nullptr);
}

template <class Src, class Dst>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const Src in, const Dst out, uint32_t count, const uint32_t *__restrict__ dcount, int shift,
    uint32_t nbits, const uint32_t *__restrict__ offs, uint32_t tiles,
    const int32_t *__restrict__ status) {
    if (status && *status) return;
    if (dcount) count = min(count, *dcount);
    __shared__ SortTileLds L;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    if ((uint64_t)tile * kSortTile >= count) return;  // past the keys (a device count)
    const uint32_t mask = (1u << nbits) - 1u;
    if ((uint64_t)(tile + 1) * kSortTile <= count)
        scatter_tile<true>(in, out, count, shift, mask, offs, tiles, tile, L);
    else
        scatter_tile<false>(in, out, count, shift, mask, offs, tiles, tile, L);
}

// ---------------------------------------------------------------- single-sweep variant

constexpr uint32_t kLbAgg = 1u << 30;       // published: this tile's own count
constexpr uint32_t kLbIncl = 2u << 30;      // published: inclusive prefix up to this tile
constexpr uint32_t kLbValue = (1u << 30) - 1u;
constexpr uint32_t kLbMaxPolls = 1u << 20;  // bound on the polls of one look-back
constexpr uint32_t kLbWindow = 16;          // predecessors' flags read per round trip
constexpr int kMaxPasses = 8;

// digit counts of every pass over all keys: ghist[p * 256 + d]
__global__ __launch_bounds__(256) void k_radix_digits(
    const uint64_t *__restrict__ in, uint32_t count, int lo_bit, int passes, int hi_bit,
    uint32_t *__restrict__ ghist, const int32_t *__restrict__ status) {
    if (*status) return;
    __shared__ uint32_t h[kMaxPasses][256];
    const uint32_t t = threadIdx.x;
    for (int p = 0; p < kMaxPasses; ++p) h[p][t] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + t; i < count; i += stride) {
        const uint64_t k = in[i];
        for (int p = 0; p < passes; ++p) {
            const int sh = lo_bit + 8 * p;
            const uint32_t nb = (hi_bit - sh) < 8 ? (uint32_t)(hi_bit - sh) : 8u;
            atomicAdd(&h[p][(uint32_t)(k >> sh) & ((1u << nb) - 1u)], 1u);
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        if (h[p][t]) atomicAdd(&ghist[p * 256 + t], h[p][t]);
}

// One pass: tile ids in launch order; flags[tile * 256 + d] = kLbAgg | count, then
// kLbIncl | inclusive prefix, of digit d.
template <bool kFull>
__device__ __forceinline__ void onesweep_tile(const uint64_t *__restrict__ in,
                                              uint64_t *__restrict__ out, uint32_t count,
                                              int shift, uint32_t mask,
                                              const uint32_t *__restrict__ ghist,
                                              uint32_t *__restrict__ flags, uint32_t tile,
                                              int32_t *__restrict__ status, SortTileLds &L) {
    const uint32_t t = threadIdx.x, w = t / kWave;
    const uint64_t base = (uint64_t)tile * kSortTile;
    uint64_t keys[kSortItems];
    const uint32_t vmask = load_tile_keys<kFull>(Keys64{in}, count, base, w, keys);
    for (uint32_t k = lane_id(); k < 256; k += kWave) L.wcnt[w][k] = 0;
    wave_lds_sync();
    uint32_t ranks[kSortItems];
    wave_rank_rows(keys, vmask, shift, mask, L.wcnt[w], ranks);
    const uint32_t c = tile_digit_offsets(L);
    if (t < 256)
        __hip_atomic_store(&flags[(uint64_t)tile * 256 + t], (tile == 0 ? kLbIncl : kLbAgg) | c,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the global start of every digit
    const uint32_t gc = t < 256 ? ghist[t] : 0u;
    const uint32_t gincl = wave_incl_scan(gc);
    if (t < 256 && lane_id() == kWave - 1) L.gsum[w] = gincl;
    __syncthreads();
    stage_keys(L, keys, ranks, vmask, w, shift, mask);
    if (t < 256) {
        uint32_t gbefore = 0;
        for (uint32_t k = 0; k < w; ++k) gbefore += L.gsum[k];
        const uint32_t gstart = gbefore + gincl - gc;
        // look-back: keys of digit t in the tiles before this one.  The flags of kLbWindow
        // predecessors are read together (one memory round trip instead of one per tile) and
        // taken nearest first until an inclusive prefix; an unpublished flag is waited for
        uint32_t excl = 0;
        if (tile > 0) {
            uint32_t j = tile - 1, polls = 0;
            bool done = false;
            while (!done) {
                uint32_t f[kLbWindow];
#pragma unroll
                for (uint32_t i = 0; i < kLbWindow; ++i)
                    f[i] = i <= j ? __hip_atomic_load(&flags[(uint64_t)(j - i) * 256 + t],
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : kLbIncl;  // never reached: tile 0 is inclusive
                uint32_t taken = 0;
                bool wait = false;
#pragma unroll
                for (uint32_t i = 0; i < kLbWindow; ++i) {
                    if (done || wait) continue;
                    if ((f[i] & ~kLbValue) == 0) {
                        wait = true;
                        continue;
                    }
                    excl += f[i] & kLbValue;
                    ++taken;
                    if (f[i] & kLbIncl) done = true;
                }
                if (done) break;
                j -= taken;  // tile 0 publishes an inclusive prefix, so j never passes it
                if (wait) {
                    if (++polls >= kLbMaxPolls) {
                        set_status(status, TC_E_HIP);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __hip_atomic_store(&flags[(uint64_t)tile * 256 + t], kLbIncl | (excl + c),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        L.glob[t] = gstart + excl - L.loc[t];
    }
    __syncthreads();
    write_staged(L, Out64{out}, count, shift, mask, status);
}

__global__ __launch_bounds__(kSortThreads) void k_radix_onesweep(
    const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint32_t count, int shift,
    uint32_t nbits, const uint32_t *__restrict__ ghist, uint32_t *__restrict__ flags,
    uint32_t *__restrict__ tile_counter, int32_t *__restrict__ status) {
    __shared__ SortTileLds L;
    __shared__ uint32_t s_tile;
    __shared__ int s_stop;
    if (threadIdx.x == 0) {
        s_tile = atomicAdd(tile_counter, 1u);
        s_stop = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __syncthreads();
    // after an error (earlier kernels, or a look-back bound reached in this one) tiles stop
    // before publishing; their successors' bounded waits end too
    if (s_stop) return;
    const uint32_t tile = s_tile;
    const uint32_t mask = (1u << nbits) - 1u;
    if ((uint64_t)(tile + 1) * kSortTile <= count)
        onesweep_tile<true>(in, out, count, shift, mask, ghist, flags, tile, status, L);
    else
        onesweep_tile<false>(in, out, count, shift, mask, ghist, flags, tile, status, L);
}

size_t sort_scratch_bytes(uint64_t count) {
    uint64_t tiles = (count + kSortTile - 1) / kSortTile;
    if (tiles == 0) tiles = 1;
    uint64_t hist = 256 * tiles;
    return 2 * align_up(hist * 4, 256) + align_up(scan_scratch_words(hist) * 4, 256);
}

// the number of keys a pass wrote: the end of the last digit run of the last tile
__global__ void k_sort_total(const uint32_t *__restrict__ hist, const uint32_t *__restrict__ offs,
                             uint64_t last, uint32_t *__restrict__ total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *total = offs[last] + hist[last];
}

// One stable two-kernel pass on the digit at `shift` (at most 8 bits, below hi_bit) from the
// keys `in` yields to dst.  dcount (nullable): the number of keys on the device (count: the
// capacity); total (nullable): receives the number of keys written (the kept ones).
template <class Src, class Dst>
static hipError_t radix_pass(const Src in, const Dst dst, uint32_t count, int shift, int hi_bit,
                             void *scratch, int32_t *status, hipStream_t s,
                             const uint32_t *dcount = nullptr, uint32_t *total = nullptr) {
    const uint32_t tiles = ceil_div(count, kSortTile);
    const uint64_t hist_n = 256ull * tiles;
    uint32_t *hist = (uint32_t *)scratch;
    uint32_t *offs = (uint32_t *)((char *)scratch + align_up(hist_n * 4, 256));
    uint32_t *scan_scratch = (uint32_t *)((char *)scratch + 2 * align_up(hist_n * 4, 256));
    const uint32_t nbits = (uint32_t)((hi_bit - shift) < 8 ? (hi_bit - shift) : 8);
    hipLaunchKernelGGL(k_radix_hist<Src>, dim3(tiles), dim3(kSortThreads), 0, s, in, count,
                       dcount, shift, nbits, hist, tiles, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive_u32(hist, offs, hist_n, scan_scratch, s);
    if (e != hipSuccess) return e;
    if (total) {
        hipLaunchKernelGGL(k_sort_total, dim3(1), dim3(64), 0, s, hist, offs, hist_n - 1, total);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_radix_scatter<Src, Dst>), dim3(tiles), dim3(kSortThreads), 0, s, in,
                       dst, count, dcount, shift, nbits, offs, tiles, status);
    return hipGetLastError();
}

hipError_t sort_u64(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                    void *scratch, int32_t *status, hipStream_t s, uint64_t **result,
                    bool onesweep) {
    *result = keys;
    if (count <= 1 || hi_bit <= lo_bit) return hipSuccess;
    uint32_t tiles = ceil_div(count, kSortTile);
    uint64_t hist_n = 256ull * tiles;
    uint32_t *hist = (uint32_t *)scratch;
    uint32_t *offs = (uint32_t *)((char *)scratch + align_up(hist_n * 4, 256));
    uint64_t *src = keys, *dst = tmp;
    const int passes = (hi_bit - lo_bit + 7) / 8;
    if (status && onesweep && count >= (1u << 20) && count <= kLbValue &&
        hist_n >= (uint64_t)kMaxPasses * 256 + kMaxPasses) {
        // flags: the first table; digit counts and tile counters: the second
        uint32_t *flags = hist, *ghist = offs, *counters = offs + kMaxPasses * 256;
        hipError_t e = fill_u32(ghist, 0u, kMaxPasses * 256 + kMaxPasses, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_digits, dim3(2048), dim3(256), 0, s, keys, count,
                           lo_bit, passes, hi_bit, ghist, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int p = 0; p < passes; ++p) {
            const int shift = lo_bit + 8 * p;
            const uint32_t nbits = (uint32_t)((hi_bit - shift) < 8 ? (hi_bit - shift) : 8);
            if ((e = fill_u32(flags, 0u, hist_n, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_radix_onesweep, dim3(tiles), dim3(kSortThreads), 0, s, src, dst,
                               count, shift, nbits, ghist + p * 256, flags, counters + p,
                               status);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            uint64_t *x = src;
            src = dst;
            dst = x;
        }
        *result = src;
        return hipSuccess;
    }
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        hipError_t e =
            radix_pass(Keys64{src}, Out64{dst}, count, shift, hi_bit, scratch, status, s);
        if (e != hipSuccess) return e;
        uint64_t *x = src;
        src = dst;
        dst = x;
    }
    *result = src;
    return hipSuccess;
}

hipError_t sort_unzip(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                      int b, uint32_t *col, uint32_t *src, void *scratch, int32_t *status,
                      hipStream_t s, bool onesweep) {
    if (count == 0) return hipSuccess;
    const int passes = hi_bit > lo_bit ? (hi_bit - lo_bit + 7) / 8 : 1;
    const int last = hi_bit > lo_bit ? lo_bit + 8 * (passes - 1) : hi_bit;
    uint64_t *mid = keys;
    hipError_t e = sort_u64(keys, tmp, count, lo_bit, last, scratch, status, s, &mid, onesweep);
    if (e != hipSuccess) return e;
    return radix_pass(Keys64{mid}, OutColSrc{col, src, (1ull << b) - 1, b}, count, last, hi_bit,
                      scratch, status, s);
}

hipError_t sort_ranks(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                      int b, uint32_t *perm, uint32_t *rank, void *scratch, int32_t *status,
                      hipStream_t s) {
    if (count == 0) return hipSuccess;
    const int passes = hi_bit > lo_bit ? (hi_bit - lo_bit + 7) / 8 : 1;
    const int last = hi_bit > lo_bit ? lo_bit + 8 * (passes - 1) : hi_bit;
    uint64_t *mid = keys;
    hipError_t e = sort_u64(keys, tmp, count, lo_bit, last, scratch, status, s, &mid);
    if (e != hipSuccess) return e;
    return radix_pass(Keys64{mid}, OutPermRank{perm, rank, (1ull << b) - 1}, count, last, hi_bit,
                      scratch, status, s);
}

hipError_t sort_lists(const uint32_t *cid, uint32_t drop, uint32_t count, int bits,
                      uint64_t *a, uint64_t *b, uint32_t *cbeg, uint32_t *kept, void *scratch,
                      int32_t *status, hipStream_t s, uint32_t **list) {
    *list = (uint32_t *)a;
    if (count == 0) return fill_u32(kept, 0u, 1, s);
    const int hi_bit = 32 + (bits > 0 ? bits : 0);
    const int passes = bits > 0 ? (bits + 7) / 8 : 1;
    const KeysHiIndex first{cid, drop};
    if (passes == 1)  // one pass from the ids to the split output
        return radix_pass(first, OutListBeg{*list, cbeg}, count, 32, hi_bit, scratch, status, s,
                          nullptr, kept);
    hipError_t e =
        radix_pass(first, Out64{a}, count, 32, hi_bit, scratch, status, s, nullptr, kept);
    if (e != hipSuccess) return e;
    uint64_t *src = a, *dst = b;
    for (int p = 1; p < passes - 1; ++p) {  // the middle passes, on the kept keys
        e = radix_pass(Keys64{src}, Out64{dst}, count, 32 + 8 * p, hi_bit, scratch, status, s,
                       kept);
        if (e != hipSuccess) return e;
        uint64_t *x = src;
        src = dst;
        dst = x;
    }
    *list = (uint32_t *)dst;  // the buffer the last pass does not read
    return radix_pass(Keys64{src}, OutListBeg{*list, cbeg}, count, 32 + 8 * (passes - 1), hi_bit,
                      scratch, status, s, kept);
}

}  // namespace tc
