// Yardstick kernels (libtc_ablation.so): the paper's own counting design of Section 3.3 and
// the variants of its Section 3.4 optimisations, for timing beside libtc's kernels on gfx950.
// Nothing in the counting path calls this library.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "../../include/tc.h"
#include "../../include/tc_ablation.h"

namespace tca {

constexpr int kWave = 64;

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, d, kWave);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), d, kWave);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

__global__ void k_zero(unsigned long long *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// |N+(u) n N+(v)| by a two-pointer merge of the two sorted lists [i, ie) and [j, je) of col.
// kTwoReads: both current elements loaded in every step; otherwise only the list that moves
// loads its next element (which may be one past the list's end: col is padded).
template <bool kTwoReads, class ColPtr>
__device__ __forceinline__ uint32_t merge_count(ColPtr col, uint32_t i, uint32_t ie, uint32_t j,
                                                uint32_t je) {
    uint32_t c = 0;
    if (kTwoReads) {
        while (i < ie && j < je) {
            const uint32_t x = col[i], y = col[j];
            c += x == y ? 1u : 0u;
            i += x <= y ? 1u : 0u;
            j += y <= x ? 1u : 0u;
        }
    } else {
        uint32_t x = col[i], y = col[j];
        while (i < ie && j < je) {
            const bool step_i = x <= y, step_j = y <= x;
            c += (step_i && step_j) ? 1u : 0u;
            if (step_i) x = col[++i];
            if (step_j) y = col[++j];
        }
    }
    return c;
}

// One thread per oriented edge (grid-stride), Section 3.3.  kHalf: lanes 32..63 of every wave
// stay idle and the active threads are numbered over the lower halves.
template <bool kTwoReads, bool kAoS, bool kHalf, class ColPtr, class IdxPtr>
__device__ __forceinline__ void edge_merge(ColPtr row_ptr, ColPtr col, IdxPtr src, IdxPtr dst,
                                           const uint2 *pairs, uint32_t mf,
                                           unsigned long long *total) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    uint64_t first = gt, step = nthreads;
    bool active = true;
    if (kHalf) {
        active = lane < kWave / 2;
        first = (gt / kWave) * (kWave / 2) + lane;
        step = nthreads / 2;
    }
    uint64_t cnt = 0;
    if (active) {
        for (uint64_t e = first; e < mf; e += step) {
            uint32_t u, v;
            if (kAoS) {
                const uint2 p = pairs[e];
                u = p.x;
                v = p.y;
            } else {
                u = src[e];
                v = dst[e];
            }
            cnt += merge_count<kTwoReads>(col, row_ptr[u], row_ptr[u + 1], row_ptr[v],
                                          row_ptr[v + 1]);
        }
    }
    cnt = wave_sum_u64(cnt);
    if (lane == 0 && cnt) atomicAdd(total, (unsigned long long)cnt);
}

template <bool kTwoReads, bool kAoS, bool kHalf>
__global__ void k_merge_restrict(const uint32_t *__restrict__ row_ptr,
                                 const uint32_t *__restrict__ col,
                                 const uint32_t *__restrict__ src,
                                 const uint32_t *__restrict__ dst,
                                 const uint2 *__restrict__ pairs, uint32_t mf,
                                 unsigned long long *__restrict__ total) {
    edge_merge<kTwoReads, kAoS, kHalf>(row_ptr, col, src, dst, pairs, mf, total);
}

template <bool kTwoReads, bool kAoS, bool kHalf>
__global__ void k_merge_plain(uint32_t *row_ptr, uint32_t *col, uint32_t *src, uint32_t *dst,
                              uint2 *pairs, uint32_t mf, unsigned long long *total) {
    edge_merge<kTwoReads, kAoS, kHalf>(row_ptr, col, src, dst, pairs, mf, total);
}

template <bool kTwoReads, bool kAoS, bool kHalf>
static void launch_merge(bool plain, dim3 grid, dim3 block, hipStream_t s, const uint32_t *rp,
                         const uint32_t *col, const uint32_t *src, const uint32_t *dst,
                         const uint2 *pairs, uint32_t mf, unsigned long long *total) {
    if (plain)
        hipLaunchKernelGGL((k_merge_plain<kTwoReads, kAoS, kHalf>), grid, block, 0, s,
                           const_cast<uint32_t *>(rp), const_cast<uint32_t *>(col),
                           const_cast<uint32_t *>(src), const_cast<uint32_t *>(dst),
                           const_cast<uint2 *>(pairs), mf, total);
    else
        hipLaunchKernelGGL((k_merge_restrict<kTwoReads, kAoS, kHalf>), grid, block, 0, s, rp,
                           col, src, dst, pairs, mf, total);
}

__global__ void k_zip(const uint32_t *__restrict__ src, const uint32_t *__restrict__ dst,
                      uint64_t mf, uint2 *__restrict__ pairs) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mf; e += stride)
        pairs[e] = make_uint2(src[e], dst[e]);
}

// 32-bit finaliser of MurmurHash3 (fmix32), for pseudo-random positions
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

template <int kWords>
__global__ void k_gather(const uint32_t *__restrict__ table, uint64_t elems, uint64_t count,
                         uint32_t seed, unsigned long long *__restrict__ sink) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint32_t h = fmix32((uint32_t)i ^ fmix32((uint32_t)(i >> 32) ^ seed));
        const uint64_t at = ((uint64_t)h * elems) >> 32;  // < elems (elems < 2^32)
        if (kWords == 4) {
            const uint4 x = reinterpret_cast<const uint4 *>(table)[at];
            acc += x.x ^ x.y ^ x.z ^ x.w;
        } else if (kWords == 2) {
            const uint2 x = reinterpret_cast<const uint2 *>(table)[at];
            acc += x.x ^ x.y;
        } else {
            acc += table[at];
        }
    }
    const uint64_t s = wave_sum_u64(acc);
    if (threadIdx.x % kWave == 0) atomicAdd(sink, (unsigned long long)s);
}

struct PairLess {
    __device__ bool operator()(const uint2 &a, const uint2 &b) const {
        return a.x < b.x || (a.x == b.x && a.y < b.y);
    }
};

}  // namespace tca

using namespace tca;

extern "C" {

int tca_edge_merge(const uint32_t *d_row_ptr, const uint32_t *d_col, const uint32_t *d_src,
                   const uint32_t *d_dst, const uint32_t *d_pairs, int64_t mf, uint32_t flags,
                   int32_t threads_per_block, int32_t blocks, uint64_t *d_total, void *stream) {
    if (mf < 0 || mf >= (1ll << 32) || !d_total || blocks < 1 ||
        (flags & ~(TCA_TWO_READS | TCA_AOS | TCA_PLAIN_PTRS | TCA_HALF_WAVE)))
        return TC_E_ARG;
    if (threads_per_block != 64 && threads_per_block != 128 && threads_per_block != 256 &&
        threads_per_block != 512 && threads_per_block != 1024)
        return TC_E_ARG;
    if (mf > 0 && (!d_row_ptr || !d_col || ((flags & TCA_AOS) ? !d_pairs : (!d_src || !d_dst))))
        return TC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *total = (unsigned long long *)d_total;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, total);
    if (mf == 0) return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
    const dim3 grid((uint32_t)blocks), block((uint32_t)threads_per_block);
    const bool two = flags & TCA_TWO_READS, aos = flags & TCA_AOS, plain = flags & TCA_PLAIN_PTRS,
               half = flags & TCA_HALF_WAVE;
    const uint2 *pairs = (const uint2 *)d_pairs;
    const uint32_t m = (uint32_t)mf;
#define TCA_MERGE(T, A, H) \
    launch_merge<T, A, H>(plain, grid, block, s, d_row_ptr, d_col, d_src, d_dst, pairs, m, total)
    if (two) {
        if (aos) { if (half) TCA_MERGE(true, true, true); else TCA_MERGE(true, true, false); }
        else { if (half) TCA_MERGE(true, false, true); else TCA_MERGE(true, false, false); }
    } else {
        if (aos) { if (half) TCA_MERGE(false, true, true); else TCA_MERGE(false, true, false); }
        else { if (half) TCA_MERGE(false, false, true); else TCA_MERGE(false, false, false); }
    }
#undef TCA_MERGE
    return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

int tca_zip_edges(const uint32_t *d_src, const uint32_t *d_dst, int64_t mf, uint32_t *d_pairs,
                  void *stream) {
    if (mf < 0 || (mf > 0 && (!d_src || !d_dst || !d_pairs))) return TC_E_ARG;
    if (mf == 0) return TC_OK;
    uint64_t g = ((uint64_t)mf + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_zip, dim3((uint32_t)g), dim3(256), 0, (hipStream_t)stream, d_src, d_dst,
                       (uint64_t)mf, (uint2 *)d_pairs);
    return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

static int sort_impl(int32_t method, uint32_t count, int32_t bits, void *a, void *b,
                     void *a_alt, void *b_alt, void *temp, size_t &temp_bytes, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (method == TCA_SORT_PAIRS_COMPARE) {
        e = hipcub::DeviceMergeSort::SortKeys(temp, temp_bytes, (uint2 *)a, count, PairLess(),
                                              s);
    } else if (method == TCA_SORT_PAIRS_RADIX) {
        uint32_t *u = (uint32_t *)a, *v = (uint32_t *)b, *u2 = (uint32_t *)a_alt,
                 *v2 = (uint32_t *)b_alt;
        if (!temp) {  // size query: the larger of the two passes (they are the same)
            return hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, v, v2, u, u2, count, 0,
                                                      bits, s) == hipSuccess ? TC_OK : TC_E_HIP;
        }
        e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, v, v2, u, u2, count, 0, bits,
                                               s);
        if (e == hipSuccess)
            e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, u2, u, v2, v, count, 0, bits,
                                                   s);
    } else if (method == TCA_SORT_PACKED_RADIX) {
        e = hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, (const uint64_t *)a,
                                              (uint64_t *)a_alt, count, 0, 2 * bits, s);
    } else {
        return TC_E_ARG;
    }
    return e == hipSuccess ? TC_OK : TC_E_HIP;
}

size_t tca_sort_temp_bytes(int32_t method, int64_t count, int32_t bits) {
    if (count < 0 || count >= (1ll << 31) || bits < 1 || bits > 32) return 0;
    size_t bytes = 0;
    if (sort_impl(method, (uint32_t)count, bits, nullptr, nullptr, nullptr, nullptr, nullptr,
                  bytes, nullptr) != TC_OK)
        return 0;
    return bytes > 0 ? bytes : 1;
}

int tca_sort(int32_t method, int64_t count, int32_t bits, void *d_a, void *d_b, void *d_a_alt,
             void *d_b_alt, void *d_temp, size_t temp_bytes, void *stream) {
    if (count < 0 || count >= (1ll << 31) || bits < 1 || bits > 32) return TC_E_ARG;
    if (method < 0 || method > 2) return TC_E_ARG;
    if (count == 0) return TC_OK;
    if (!d_a || !d_temp) return TC_E_ARG;
    if (method == TCA_SORT_PAIRS_RADIX && (!d_b || !d_a_alt || !d_b_alt)) return TC_E_ARG;
    if (method == TCA_SORT_PACKED_RADIX && !d_a_alt) return TC_E_ARG;
    if (temp_bytes < tca_sort_temp_bytes(method, count, bits)) return TC_E_WORKSPACE;
    size_t tb = temp_bytes;
    return sort_impl(method, (uint32_t)count, bits, d_a, d_b, d_a_alt, d_b_alt, d_temp, tb,
                     (hipStream_t)stream);
}

int tca_gather(const void *d_table, int64_t table_bytes, int32_t elem_bytes, int64_t count,
               uint32_t seed, uint64_t *d_sink, void *stream) {
    if (!d_table || !d_sink || count < 0 || (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16))
        return TC_E_ARG;
    const int64_t elems = table_bytes / elem_bytes;
    if (elems < 1 || elems >= (1ll << 32) || ((uintptr_t)d_table & 15)) return TC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *sink = (unsigned long long *)d_sink;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, sink);
    const dim3 grid(8192), block(256);
    const uint32_t *t = (const uint32_t *)d_table;
    if (elem_bytes == 16)
        hipLaunchKernelGGL(k_gather<4>, grid, block, 0, s, t, (uint64_t)elems, (uint64_t)count,
                           seed, sink);
    else if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather<2>, grid, block, 0, s, t, (uint64_t)elems, (uint64_t)count,
                           seed, sink);
    else
        hipLaunchKernelGGL(k_gather<1>, grid, block, 0, s, t, (uint64_t)elems, (uint64_t)count,
                           seed, sink);
    return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

}  // extern "C"
