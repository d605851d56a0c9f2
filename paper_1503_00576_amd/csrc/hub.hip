// Triangles among the hubs on the matrix cores.
//
// The hubs are the h highest ranks of the order of Section 2.2 (the highest degrees); every
// out-neighbour of a hub is a hub.  Their oriented adjacency, re-indexed from 0, is an upper
// triangular 0/1 matrix A (A[u][w] = 1 iff u -> w, so u < w), and the triangles u < v < w with
// all three vertices hubs number
//     T_H = sum over u, w of A[u][w] * (A A)[u][w],
// since (A A)[u][w] counts the v with u -> v -> w.  A triangle whose lowest vertex is a hub is
// a hub triangle, so the middle-vertex kernel skips every in-edge that starts at a hub and the
// two parts add up to the total.  The product is a dense int8 contraction: it runs on
// 32x32x32 int8 MFMA tiles, only over the block upper triangle (tiles u-block <= w-block, and
// for each only the v-blocks that can be nonzero), with the mask and the sum fused in.
//
// Per-vertex counts: T(u) and T(w) are the row and column sums of A o (A A); the middle vertex
// gets T(v) = sum over u of A[u][v] * (A A^T)[u][v] (column sums of A o (A A^T)).
//
// Layout: A and At = A^T, int8, row-major, hp x hp (hp = h rounded up to 64, zero padded).
// MFMA operand layout (32x32x32 i8): lane l supplies row l % 32 of the A operand and column
// l % 32 of the B operand, 16 consecutive k per lane half (l / 32); result register r of lane
// l is element (8 (r / 4) + 4 (l / 32) + r % 4, l % 32).
#include "internal.h"

namespace tc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// A[u - h0][w - h0] = At[w - h0][u - h0] = 1 for every CSR entry of the hub rows (the last rows
// of the CSR, from row_ptr[h0] on); both matrices zeroed beforehand
__global__ void k_hub_fill(const uint32_t *__restrict__ src, const uint32_t *__restrict__ col,
                           const uint32_t *__restrict__ row_ptr, uint32_t mf, uint32_t h0,
                           uint32_t hp, uint8_t *__restrict__ A, uint8_t *__restrict__ At,
                           const int32_t *__restrict__ status) {
    if (*status) return;
    const uint32_t e0 = row_ptr[h0];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mf; e += stride) {
        const uint32_t u = src[e] - h0, w = col[e] - h0;
        A[(uint64_t)u * hp + w] = 1;
        At[(uint64_t)w * hp + u] = 1;
    }
}

__device__ __forceinline__ v4i load16(const uint8_t *p) { return *(const v4i *)p; }

// tile t of the block upper triangle of nb x nb 64-blocks, row-major over (bi, bk), bi <= bk
__device__ __forceinline__ void tile_of(uint32_t t, uint32_t nb, uint32_t &bi, uint32_t &bk) {
    // rows of the triangle have nb, nb - 1, ... tiles; find bi by a short search
    uint32_t lo = 0, hi = nb;  // bi in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        const uint64_t before = (uint64_t)mid * nb - (uint64_t)mid * (mid - 1) / 2;
        if (before <= t) lo = mid; else hi = mid;
    }
    bi = lo;
    bk = bi + (uint32_t)(t - ((uint64_t)bi * nb - (uint64_t)bi * (bi - 1) / 2));
}

// One wave per 64 x 64 output tile (2 x 2 MFMA tiles of 32 x 32).
template <bool PV>
__global__ __launch_bounds__(256) void k_hub_count(const uint8_t *__restrict__ A,
                                                   const uint8_t *__restrict__ At, uint32_t hp,
                                                   uint32_t h0, unsigned long long *__restrict__ total,
                                                   unsigned long long *__restrict__ tpv,
                                                   const int32_t *__restrict__ status) {
    if (*status) return;
    const uint32_t lane = lane_id(), half = lane / 32, l32 = lane % 32;
    const uint32_t nb = hp / 64, tiles = nb * (nb + 1) / 2;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t waves = gridDim.x * blockDim.x / kWave;
    uint64_t sum = 0;
    for (uint32_t t = wave; t < tiles; t += waves) {
        uint32_t bi, bk;
        tile_of(t, nb, bi, bk);
        const uint32_t i0 = bi * 64, k0 = bk * 64;
        v16i acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = v16i{};
        // (A A)[u][w] = sum over v of A[u][v] A[v][w]: v in [i0, k0 + 64)
        for (uint32_t kv = i0; kv < k0 + 64; kv += 32) {
            const uint32_t kk = kv + 16 * half;
            const v4i a0 = load16(A + (uint64_t)(i0 + l32) * hp + kk);
            const v4i a1 = load16(A + (uint64_t)(i0 + 32 + l32) * hp + kk);
            const v4i b0 = load16(At + (uint64_t)(k0 + l32) * hp + kk);
            const v4i b1 = load16(At + (uint64_t)(k0 + 32 + l32) * hp + kk);
            acc[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc[1][1], 0, 0, 0);
        }
        // mask by A[u][w] = At[w][u]: for one lane, the rows 4 (r / 4) .. + 3 are consecutive
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
#pragma unroll
            for (int tk = 0; tk < 2; ++tk) {
                const uint32_t w = k0 + 32 * tk + l32;
                uint32_t colsum = 0;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const uint32_t ub = i0 + 32 * ti + 8 * g + 4 * half;
                    const uint32_t m4 = *(const uint32_t *)(At + (uint64_t)w * hp + ub);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t v = (uint32_t)acc[ti][tk][4 * g + q] * ((m4 >> (8 * q)) & 1u);
                        colsum += v;
                        if (PV) {  // row sum over the 32 columns of this half's lanes
                            uint32_t rs = v;
#pragma unroll
                            for (int o = 16; o >= 1; o >>= 1)
                                rs += (uint32_t)__shfl_xor((int)rs, o, kWave);
                            if (l32 == 0 && rs)
                                atomicAdd(&tpv[h0 + ub + q], (unsigned long long)rs);
                        }
                    }
                }
                sum += colsum;
                if (PV) {
                    const uint32_t cs = colsum + (uint32_t)__shfl_xor((int)colsum, 32, kWave);
                    if (half == 0 && cs) atomicAdd(&tpv[h0 + w], (unsigned long long)cs);
                }
            }
        }
        if (PV) {  // middle vertices: (A A^T)[u][v] = sum over w > v of A[u][w] A[v][w]
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = v16i{};
            for (uint32_t kw = k0; kw < hp; kw += 32) {
                const uint32_t kk = kw + 16 * half;
                const v4i a0 = load16(A + (uint64_t)(i0 + l32) * hp + kk);
                const v4i a1 = load16(A + (uint64_t)(i0 + 32 + l32) * hp + kk);
                const v4i b0 = load16(A + (uint64_t)(k0 + l32) * hp + kk);
                const v4i b1 = load16(A + (uint64_t)(k0 + 32 + l32) * hp + kk);
                acc[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc[1][1], 0, 0, 0);
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti) {
#pragma unroll
                for (int tk = 0; tk < 2; ++tk) {
                    const uint32_t v = k0 + 32 * tk + l32;
                    uint32_t colsum = 0;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const uint32_t ub = i0 + 32 * ti + 8 * g + 4 * half;
                        const uint32_t m4 = *(const uint32_t *)(At + (uint64_t)v * hp + ub);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            colsum += (uint32_t)acc[ti][tk][4 * g + q] * ((m4 >> (8 * q)) & 1u);
                    }
                    const uint32_t cs = colsum + (uint32_t)__shfl_xor((int)colsum, 32, kWave);
                    if (half == 0 && cs) atomicAdd(&tpv[h0 + v], (unsigned long long)cs);
                }
            }
        }
    }
    sum = wave_sum_u64(sum);
    if (lane == 0 && sum) atomicAdd(total, (unsigned long long)sum);
}

hipError_t launch_hub_fill(const uint32_t *src, const uint32_t *col, const uint32_t *row_ptr,
                           uint32_t mf, uint32_t h0, uint32_t hp, uint8_t *A, uint8_t *At,
                           const int32_t *status, hipStream_t s) {
    if (hp == 0 || mf == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hub_fill, dim3(4096), dim3(256), 0, s, src, col, row_ptr, mf, h0, hp, A,
                       At, status);
    return hipGetLastError();
}

hipError_t launch_hub_count(const uint8_t *A, const uint8_t *At, uint32_t hp, uint32_t h0,
                            unsigned long long *total, unsigned long long *tpv, bool per_vertex,
                            const int32_t *status, hipStream_t s) {
    if (hp == 0) return hipSuccess;
    const uint32_t nb = hp / 64, tiles = nb * (nb + 1) / 2;
    uint32_t blocks = (tiles + 3) / 4;  // four waves per workgroup, one tile per wave and round
    const uint32_t cap = (uint32_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (per_vertex)
        hipLaunchKernelGGL(k_hub_count<true>, dim3(blocks), dim3(256), 0, s, A, At, hp, h0, total,
                           tpv, status);
    else
        hipLaunchKernelGGL(k_hub_count<false>, dim3(blocks), dim3(256), 0, s, A, At, hp, h0,
                           total, tpv, status);
    return hipGetLastError();
}

}  // namespace tc
