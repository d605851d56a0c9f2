// Device-wide exclusive scan and stable LSD radix sort of uint64 keys.
//
// The sort replaces the library sort of packed 64-bit edge keys in the preprocessing phase
// (Section 3.2, step 3, and the note on sorting edges as 64-bit integers): keys are ordered
// on a bit range [lo_bit, hi_bit) with 8-bit digits, least significant digit first; every
// pass is an upsweep (per-tile digit histograms), an exclusive scan of the digit-major
// histogram table, and a stable scatter in which a wave ranks equal digits with ballots,
// the tile is ordered by digit in LDS, and every digit's run is written out contiguously.
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

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per tile
constexpr int kSortWaves = kSortThreads / kWave;

// Lanes holding the same digit: returns the mask of such (valid) lanes.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint32_t nbits, bool valid) {
    uint64_t peers = __ballot(valid);
    for (uint32_t b = 0; b < nbits; ++b) {
        uint64_t bb = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *__restrict__ in,
                                                             uint32_t count, int shift,
                                                             uint32_t nbits,
                                                             uint32_t *__restrict__ hist,
                                                             uint32_t tiles,
                                                             const int32_t *__restrict__ status) {
    if (status && *status) return;
    __shared__ uint32_t h[kSortWaves][256];
    const uint32_t t = threadIdx.x, w = t / kWave;
    for (int k = 0; k < kSortWaves; ++k) h[k][t] = 0;
    __syncthreads();
    const uint32_t mask = (1u << nbits) - 1u;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    const uint64_t base = (uint64_t)tile * kSortTile;
    uint32_t dg[kSortItems];  // all loads in flight before any ranking
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        uint64_t idx = base + (uint64_t)r * kSortThreads + t;
        dg[r] = idx < count ? (uint32_t)(in[idx] >> shift) & mask : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        bool valid = dg[r] != 0xFFFFFFFFu;
        uint32_t d = valid ? dg[r] : 0u;
        uint64_t peers = match_digit(d, nbits, valid);
        if (valid && lanes_below(peers) == 0) h[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t sum = 0;
    for (int k = 0; k < kSortWaves; ++k) sum += h[k][t];
    hist[(uint64_t)t * tiles + tile] = sum;
}

// Stable scatter of one 4096-key tile: the keys are first ranked and placed in LDS in digit
// order (tile-local counting sort), then written out so that consecutive threads write
// consecutive positions of one digit's run.
//   hist: raw per-tile digit counts (digit-major), offs: their exclusive scan
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint32_t count, int shift,
    uint32_t nbits, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ offs,
    uint32_t tiles, const int32_t *__restrict__ status) {
    if (status && *status) return;
    __shared__ uint64_t s_stage[kSortTile];
    __shared__ uint32_t s_loc[256];   // next local position per digit
    __shared__ uint32_t s_glob[256];  // global start minus local start per digit
    __shared__ uint32_t s_wcnt[kSortWaves][256];
    __shared__ uint32_t s_wsum[kSortWaves];
    const uint32_t t = threadIdx.x, w = t / kWave;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    // tile-local exclusive offsets of the digits
    const uint32_t c = hist[(uint64_t)t * tiles + tile];
    const uint32_t incl = wave_incl_scan(c);
    if (lane_id() == kWave - 1) s_wsum[w] = incl;
    for (int k = 0; k < kSortWaves; ++k) s_wcnt[k][t] = 0;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < w; ++k) before += s_wsum[k];
    const uint32_t loc = before + incl - c;
    s_loc[t] = loc;
    s_glob[t] = offs[(uint64_t)t * tiles + tile] - loc;
    __syncthreads();
    const uint32_t mask = (1u << nbits) - 1u;
    const uint64_t base = (uint64_t)tile * kSortTile;
    uint64_t keys[kSortItems];  // all loads in flight before any ranking
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        uint64_t idx = base + (uint64_t)r * kSortThreads + t;
        keys[r] = idx < count ? in[idx] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        uint64_t idx = base + (uint64_t)r * kSortThreads + t;
        bool valid = idx < count;
        uint64_t key = keys[r];
        uint32_t d = (uint32_t)(key >> shift) & mask;
        uint64_t peers = match_digit(d, nbits, valid);
        uint32_t rank = lanes_below(peers);
        if (valid && rank == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = s_loc[d] + rank;
            for (uint32_t k = 0; k < w; ++k) pos += s_wcnt[k][d];
            s_stage[pos] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < kSortWaves; ++k) {
            add += s_wcnt[k][t];
            s_wcnt[k][t] = 0;
        }
        s_loc[t] += add;
        __syncthreads();
    }
    const uint64_t rest = count - base;
    const uint32_t ntile = rest < (uint64_t)kSortTile ? (uint32_t)rest : (uint32_t)kSortTile;
    for (uint32_t j = t; j < ntile; j += kSortThreads) {
        const uint64_t key = s_stage[j];
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        out[s_glob[d] + j] = key;
    }
}

// ---------------------------------------------------------------- single-sweep variant

constexpr uint32_t kLbAgg = 1u << 30;       // published: this tile's own count
constexpr uint32_t kLbIncl = 2u << 30;      // published: inclusive prefix up to this tile
constexpr uint32_t kLbValue = (1u << 30) - 1u;
constexpr uint32_t kLbMaxPolls = 1u << 20;  // bound on the polls of one look-back
constexpr int kMaxPasses = 8;

// digit counts of every pass over all keys: ghist[p * 256 + d]
__global__ __launch_bounds__(kSortThreads) void k_radix_digits(
    const uint64_t *__restrict__ in, uint32_t count, int lo_bit, int passes, int hi_bit,
    uint32_t *__restrict__ ghist, const int32_t *__restrict__ status) {
    if (*status) return;
    __shared__ uint32_t h[kMaxPasses][256];
    const uint32_t t = threadIdx.x;
    for (int p = 0; p < kMaxPasses; ++p) h[p][t] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kSortThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kSortThreads + t; i < count; i += stride) {
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
__global__ __launch_bounds__(kSortThreads) void k_radix_onesweep(
    const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint32_t count, int shift,
    uint32_t nbits, const uint32_t *__restrict__ ghist, uint32_t *__restrict__ flags,
    uint32_t *__restrict__ tile_counter, int32_t *__restrict__ status) {
    __shared__ uint64_t s_stage[kSortTile];
    __shared__ uint32_t s_loc[256], s_glob[256];
    __shared__ uint32_t s_wcnt[kSortWaves][256];
    __shared__ uint32_t s_wsum[kSortWaves], s_gsum[kSortWaves];
    __shared__ uint32_t s_tile;
    __shared__ int s_stop;
    const uint32_t t = threadIdx.x, w = t / kWave;
    if (t == 0) {
        s_tile = atomicAdd(tile_counter, 1u);
        s_stop = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    for (int k = 0; k < kSortWaves; ++k) s_wcnt[k][t] = 0;
    __syncthreads();
    // after an error (earlier kernels, or a look-back bound reached in this one) tiles stop
    // before publishing; their successors' bounded waits end too
    if (s_stop) return;
    const uint32_t tile = s_tile;
    const uint32_t mask = (1u << nbits) - 1u;
    const uint64_t base = (uint64_t)tile * kSortTile;
    uint64_t keys[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t idx = base + (uint64_t)r * kSortThreads + t;
        keys[r] = idx < count ? in[idx] : 0ull;
    }
    // this tile's digit counts
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool valid = base + (uint64_t)r * kSortThreads + t < count;
        const uint32_t d = (uint32_t)(keys[r] >> shift) & mask;
        const uint64_t peers = match_digit(d, nbits, valid);
        if (valid && lanes_below(peers) == 0) s_wcnt[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t c = 0;
    for (int k = 0; k < kSortWaves; ++k) {
        c += s_wcnt[k][t];
        s_wcnt[k][t] = 0;
    }
    __hip_atomic_store(&flags[(uint64_t)tile * 256 + t], (tile == 0 ? kLbIncl : kLbAgg) | c,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // tile-local exclusive offsets of the digits, and the global digit starts
    const uint32_t gc = ghist[t];
    const uint32_t incl = wave_incl_scan(c), gincl = wave_incl_scan(gc);
    if (lane_id() == kWave - 1) {
        s_wsum[w] = incl;
        s_gsum[w] = gincl;
    }
    __syncthreads();
    uint32_t before = 0, gbefore = 0;
    for (uint32_t k = 0; k < w; ++k) {
        before += s_wsum[k];
        gbefore += s_gsum[k];
    }
    const uint32_t loc = before + incl - c;
    const uint32_t gstart = gbefore + gincl - gc;
    s_loc[t] = loc;
    __syncthreads();
    // stable placement of the tile in digit order (as in k_radix_scatter)
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool valid = base + (uint64_t)r * kSortThreads + t < count;
        const uint64_t key = keys[r];
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        const uint64_t peers = match_digit(d, nbits, valid);
        const uint32_t rank = lanes_below(peers);
        if (valid && rank == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = s_loc[d] + rank;
            for (uint32_t k = 0; k < w; ++k) pos += s_wcnt[k][d];
            s_stage[pos] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < kSortWaves; ++k) {
            add += s_wcnt[k][t];
            s_wcnt[k][t] = 0;
        }
        s_loc[t] += add;
        __syncthreads();
    }
    // look-back: keys of digit t in the tiles before this one
    uint32_t excl = 0;
    if (tile > 0) {
        uint32_t j = tile - 1, polls = 0;
        for (;;) {
            const uint32_t f = __hip_atomic_load(&flags[(uint64_t)j * 256 + t],
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((f & ~kLbValue) == 0) {
                if (++polls >= kLbMaxPolls) {
                    set_status(status, TC_E_HIP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += f & kLbValue;
            if (f & kLbIncl) break;
            --j;  // tile 0 publishes an inclusive prefix, so j never passes it
        }
        __hip_atomic_store(&flags[(uint64_t)tile * 256 + t], kLbIncl | (excl + c),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_glob[t] = gstart + excl - loc;
    __syncthreads();
    const uint64_t rest = count - base;
    const uint32_t ntile = rest < (uint64_t)kSortTile ? (uint32_t)rest : (uint32_t)kSortTile;
    for (uint32_t j = t; j < ntile; j += kSortThreads) {
        const uint64_t key = s_stage[j];
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        const uint32_t pos = s_glob[d] + j;
        if (pos < count)  // holds whenever the prefixes are right; never write outside `out`
            out[pos] = key;
        else
            set_status(status, TC_E_HIP);
    }
}

static bool onesweep_enabled() {  // TC_SORT_ONESWEEP=1 switches the variant on
    const char *env = getenv("TC_SORT_ONESWEEP");
    return env && env[0] == '1';
}

size_t sort_scratch_bytes(uint64_t count) {
    uint64_t tiles = (count + kSortTile - 1) / kSortTile;
    if (tiles == 0) tiles = 1;
    uint64_t hist = 256 * tiles;
    return 2 * align_up(hist * 4, 256) + align_up(scan_scratch_words(hist) * 4, 256);
}

hipError_t sort_u64(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                    void *scratch, int32_t *status, hipStream_t s, uint64_t **result) {
    *result = keys;
    if (count <= 1 || hi_bit <= lo_bit) return hipSuccess;
    uint32_t tiles = ceil_div(count, kSortTile);
    uint64_t hist_n = 256ull * tiles;
    uint32_t *hist = (uint32_t *)scratch;
    uint32_t *offs = (uint32_t *)((char *)scratch + align_up(hist_n * 4, 256));
    uint32_t *scan_scratch = (uint32_t *)((char *)scratch + 2 * align_up(hist_n * 4, 256));
    uint64_t *src = keys, *dst = tmp;
    const int passes = (hi_bit - lo_bit + 7) / 8;
    if (status && onesweep_enabled() && count >= (1u << 20) && count <= kLbValue &&
        hist_n >= (uint64_t)kMaxPasses * 256 + kMaxPasses) {
        // flags: the first table; digit counts and tile counters: the second
        uint32_t *flags = hist, *ghist = offs, *counters = offs + kMaxPasses * 256;
        hipError_t e = fill_u32(ghist, 0u, kMaxPasses * 256 + kMaxPasses, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_digits, dim3(2048), dim3(kSortThreads), 0, s, keys, count,
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
        uint32_t nbits = (uint32_t)((hi_bit - shift) < 8 ? (hi_bit - shift) : 8);
        hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(kSortThreads), 0, s, src, count,
                           shift, nbits, hist, tiles, status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_exclusive_u32(hist, offs, hist_n, scan_scratch, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(kSortThreads), 0, s, src, dst,
                           count, shift, nbits, hist, offs, tiles, status);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *x = src;
        src = dst;
        dst = x;
    }
    *result = src;
    return hipSuccess;
}

}  // namespace tc
