// Internal declarations shared by the HIP translation units of libtc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tc.h"

namespace tc {

constexpr int kWave = 64;

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` at lanes below the calling lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders this wave's LDS accesses before the ones that follow (all lanes of a wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_bcast(uint32_t x, int src) {
    return (uint32_t)__shfl((int)x, src, kWave);
}

// x of lane src (a per-lane index; all lanes active)
__device__ __forceinline__ uint32_t wave_bcast_from(uint32_t x, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)x);
}

// inclusive prefix sum over the 64 lanes (inactive lanes must hold 0 and be active)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
        if (l >= (uint32_t)d) x += y;
    }
    return x;
}

// inclusive prefix maximum over the 64 lanes (all lanes active): row shifts by 1, 2, 4, 8
// inside each 16-lane row (lanes shifted in from outside read 0), then the last lane of rows
// 0 and 2 into rows 1 and 3, and lane 31 into rows 2 and 3
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_max_step(uint32_t v) {
    return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, false));
}
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    v = dpp_max_step<0x111, 0xf>(v);  // row_shr:1
    v = dpp_max_step<0x112, 0xf>(v);  // row_shr:2
    v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
    v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8
    v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15
    v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, d, kWave);
        uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), d, kWave);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

__device__ __forceinline__ void set_status(int32_t *st, int32_t code) {
    atomicCAS(st, 0, code);
}

// ---------------------------------------------------------------- host helpers

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its own L2.  Tiled
// kernels whose neighbouring tiles share cache lines (per-tile tables stored tile-minor) map
// workgroup b of nb to tile xcd_tile(b, nb), so that every XCD works through one contiguous
// range of tiles.  A bijection of [0, nb).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
    const uint32_t x = b % kXcds, i = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// exclusive scan of uint32 (in may equal out); scratch: scan_scratch_words(N) words
size_t scan_scratch_words(uint64_t N);
hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint64_t N, uint32_t *scratch,
                              hipStream_t s);

// radix sort: result lands in *result (== keys or tmp); scratch: sort_scratch_bytes(count);
// onesweep: single-sweep passes for sorts of at least 2^20 keys (needs a status word)
size_t sort_scratch_bytes(uint64_t count);
hipError_t sort_u64(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                    void *scratch, int32_t *status, hipStream_t s, uint64_t **result,
                    bool onesweep = false);
// keys sorted (stably) on bits lo_bit .. hi_bit and written unzipped: col[i] = low b bits,
// src[i] = the bits above (keys and tmp are clobbered); same scratch as sort_u64
hipError_t sort_unzip(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                      int b, uint32_t *col, uint32_t *src, void *scratch, int32_t *status,
                      hipStream_t s, bool onesweep = false);
// the vertex order: keys (degree << b) | id sorted (stably) on bits lo_bit .. hi_bit, the last
// pass writing perm[r] = id of position r and rank[id] = r (keys and tmp are clobbered)
hipError_t sort_ranks(uint64_t *keys, uint64_t *tmp, uint32_t count, int lo_bit, int hi_bit,
                      int b, uint32_t *perm, uint32_t *rank, void *scratch, int32_t *status,
                      hipStream_t s);
// The in-edge lists: the keys (cid[i] << 32) | i with cid[i] != drop sorted (stably) on their
// bits 32 .. 32 + bits, written split: *list (list ids, in a or b, whichever the last pass
// does not read) and cbeg (position + 1), *kept of them (a device word).  The first pass
// reads the 32-bit ids and drops the others, the middle ones ping-pong between a and b on the
// kept keys (cid may alias b, not a); two-kernel passes; same scratch as sort_u64.
hipError_t sort_lists(const uint32_t *cid, uint32_t drop, uint32_t count, int bits,
                      uint64_t *a, uint64_t *b, uint32_t *cbeg, uint32_t *kept, void *scratch,
                      int32_t *status, hipStream_t s, uint32_t **list);

hipError_t fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s);

int device_cu_count();

// counting kernels (count.hip)
struct CountArgs {
    // in-edge lists: entry j of list c (cptr[c] <= j < cptr[c + 1]) is the in-edge at CSR
    // position cbeg[j] - 1, whose record er[cbeg[j] - 1] = (end of its row, panel mask or where
    // the suffix's entries >= hbase start in col, where they start in hcol, its row)
    const uint32_t *row_ptr, *col, *cptr, *cbeg;
    const uint4 *er;
    // every row's entries >= rank hbase as 16-bit offsets from hbase, each row's part 8-aligned
    // and followed by zeros (count_hcol_pad()); totals stream every in-edge suffix's entries
    // >= hbase from here
    const uint16_t *hcol;
    const uint32_t *hrow;  // first position >= hbase of every row, all ones for none
    uint32_t hbase;        // n: no high region
    const uint32_t *item_v_a, *item_off_a, *n_items_a;
    const uint32_t *item_v_b, *item_off_b, *n_items_b;
    uint32_t *queue_a, *queue_b;
    uint32_t *queue_c;  // per-vertex counts: the panels of k_count_panel_pv
    unsigned long long *total, *tpv;
    uint32_t n1;
    uint32_t p0;          // first rank of the panel region (n: no panels)
    uint32_t wave_bits;   // wave items use a bitmap below this rank span
    uint32_t block_bits;  // workgroup items use a bitmap below this rank span (totals)
    uint32_t block_list;  // ... else an LDS list of at most this many entries (<= kBlockList)
    uint32_t kitem_a;     // in-edges per wave item
    uint32_t kitem_b;     // in-edges per workgroup item
    const int32_t *status;
};
hipError_t launch_count(const CountArgs &a, bool per_vertex, hipStream_t s);
// LDS limits of the counting kernels' per-item structures (the defaults of the options)
uint32_t count_wave_span();         // wave bitmap: rank span below this
uint32_t count_wave_list(bool per_vertex);   // wave sorted list: entries
uint32_t count_block_span();        // workgroup bitmap: rank span below this
uint32_t count_block_list(bool per_vertex);  // workgroup sorted list: entries
uint32_t count_item_edges_wave();   // default in-edges per wave item
uint32_t count_item_edges_block();  // default in-edges per workgroup item
// bytes of padding `col` needs after its last element: a lane's aligned piece reads may run
// up to one piece past the end of a list
uint32_t count_col_pad_bytes();
// the per-row sort after a sort of the edge keys by source only: CSR positions per chunk
// (k_row_sort's workgroups), and the longest row one wave sorts (longer rows are listed)
uint32_t row_sort_chunk();
uint32_t row_sort_wave();
// zeros after every row's part of hcol beyond its rounding to 8 entries (a piece of the
// unmasked probes read from an 8-aligned position inside the part never leaves it)
uint32_t count_hcol_pad();
// middle-vertex panels: consecutive ranks per panel, and the largest rank region the
// counting kernel can handle as panels (its mask table must fit the workgroup's LDS)
uint32_t count_panel();
uint32_t count_wgs_per_cu();  // resident workgroups per CU of the counting kernels
uint32_t count_panel_ranks();
// hub triangles on the matrix cores (hub.hip): A / At are hp x hp int8, hubs = ranks h0 ..
hipError_t launch_hub_fill(const uint32_t *src, const uint32_t *col, const uint32_t *row_ptr,
                           uint32_t mf, uint32_t h0, uint32_t hp, uint8_t *A, uint8_t *At,
                           const int32_t *status, hipStream_t s);
hipError_t launch_hub_count(const uint8_t *A, const uint8_t *At, uint32_t hp, uint32_t h0,
                            unsigned long long *total, unsigned long long *tpv, bool per_vertex,
                            const int32_t *status, hipStream_t s);
struct BatchKernelArgs {
    const uint32_t *frp, *fcol, *fsrc, *gid;
    const uint32_t *item_u, *item_off, *n_items;  // heavy items
    const uint32_t *kitem, *chunk;                // sizes (device)
    const uint32_t *light;                        // [0] forward edges, [1] light chunks
    uint32_t *queue;                              // [0] heavy items, [1] light chunks
    unsigned long long *const *totals_pp;
    unsigned long long *const *tpv_pp;
    uint32_t light_max;   // rows with at most this many forward entries are light (<= 256)
    uint32_t wave_bits;   // heavy items use a bitmap below this id span (<= kWaveBits)
    uint32_t wave_list;   // ... else a sorted LDS list of at most this many entries
};
hipError_t launch_count_u(const BatchKernelArgs &a, bool per_vertex, uint32_t grid,
                          hipStream_t s);
// batched kernel: rows with at most count_light_max() forward entries are counted edge by
// edge in chunks of at most count_light_chunk_max() forward edges
uint32_t count_light_max();
uint32_t count_light_chunk_max();

}  // namespace tc
