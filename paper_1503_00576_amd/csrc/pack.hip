// Packing many small edge arrays into the batched input format (symmetric CSR per graph, rows
// ascending), on the device.
//
// Every valid entry (u, v) of graph g becomes two keys (U << b) | v and (V << b) | u, with
// U = vtx_off[g] + u the union id of the row and v the local id of the neighbour; one radix
// sort of the keys on 2b bits orders every row of every graph at once (rows of one graph
// are consecutive in the union, and inside a row the local ids order the neighbours as the
// union ids would).  Row boundaries of the sorted keys give the row lengths, whose exclusive
// scan gives the union row offsets; the per-graph local offsets are differences of those.
// An entry with an id outside [0, n_g) or a self-loop marks its graph's status and becomes a
// key with all 2b bits set, which sorts after every valid key, so the other graphs are
// unaffected; duplicates are left in place for the batched count to report.
#include "internal.h"

namespace tc {

__global__ void k_rowlen(const uint32_t *, const uint32_t *, uint32_t, uint32_t *);  // prep.hip

constexpr uint32_t kPackThreads = 256;

// last g in [0, G) with off[g] <= x (off non-decreasing on valid input; any input gives a g
// in range)
__device__ __forceinline__ uint32_t last_le(const int64_t *__restrict__ off, uint32_t G,
                                            int64_t x) {
    uint32_t lo = 0, len = G;
    while (len > 1) {
        const uint32_t half = len >> 1;
        if (off[lo + half] <= x) lo += half;
        len -= half;
    }
    return lo;
}

// The offsets must be prefix sums over the batch (non-decreasing, from 0 to N and to M);
// otherwise graph ranges may overlap, so any violation marks every graph of the batch.
// Pass 1 clears the statuses and raises *bad on a violation; pass 2 marks the graphs.
__global__ void k_pk_graphs(const int64_t *__restrict__ vtx_off,
                            const int64_t *__restrict__ edge_off, uint32_t G, uint64_t N,
                            uint64_t M, int32_t *__restrict__ status, uint32_t *__restrict__ bad) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int64_t v0 = vtx_off[g], v1 = vtx_off[g + 1], e0 = edge_off[g], e1 = edge_off[g + 1];
    const bool ok = v0 >= 0 && v1 >= v0 && (uint64_t)v1 <= N && e0 >= 0 && e1 >= e0 &&
                    (uint64_t)e1 <= M && (g > 0 || (v0 == 0 && e0 == 0)) &&
                    (g + 1 < G || ((uint64_t)v1 == N && (uint64_t)e1 == M));
    status[g] = 0;
    if (!ok) atomicOr(bad, 1u);
}

__global__ void k_pk_mark(uint32_t G, const uint32_t *__restrict__ bad,
                          int32_t *__restrict__ status) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G && *bad) status[g] = TC_E_ARG;
}

// two keys per entry (see the file comment); 2 * M keys in all
__global__ void k_pk_keys(const int2 *__restrict__ edges, uint64_t M,
                          const int64_t *__restrict__ vtx_off,
                          const int64_t *__restrict__ edge_off, uint32_t G, int b,
                          uint64_t *__restrict__ keys, int32_t *__restrict__ status) {
    const uint64_t sentinel = (b >= 32) ? ~0ull : ((1ull << (2 * b)) - 1ull);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += stride) {
        const uint32_t g = last_le(edge_off, G, (int64_t)i);
        const int64_t v0 = vtx_off[g], ng = vtx_off[g + 1] - v0;
        const int2 e = edges[i];
        uint64_t k0 = sentinel, k1 = sentinel;
        if (status[g] == TC_E_ARG) {
            // offsets inconsistent: the graph is reported, none of its entries is used
        } else if (e.x < 0 || e.y < 0 || (int64_t)e.x >= ng || (int64_t)e.y >= ng) {
            atomicCAS(&status[g], 0, TC_E_RANGE);
        } else if (e.x == e.y) {
            atomicCAS(&status[g], 0, TC_E_SELF_LOOP);
        } else {
            const uint64_t U = (uint64_t)(v0 + e.x), V = (uint64_t)(v0 + e.y);
            k0 = (U << b) | (uint32_t)e.y;
            k1 = (V << b) | (uint32_t)e.x;
        }
        keys[2 * i] = k0;
        keys[2 * i + 1] = k1;
    }
}

// sorted keys -> local neighbour ids, and the start / end of every non-empty union row
// (rs, re zeroed beforehand); sentinel keys (at the end) are skipped
__global__ void k_pk_rows(const uint64_t *__restrict__ keys, uint32_t K, uint64_t N, int b,
                          int32_t *__restrict__ col, uint32_t *__restrict__ rs,
                          uint32_t *__restrict__ re) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const uint64_t k = keys[j];
    const uint64_t U = k >> b;
    if (U >= N) return;  // a sentinel
    col[j] = (int32_t)(k & ((1ull << b) - 1ull));
    if (j == 0 || (keys[j - 1] >> b) != U) rs[U] = j;
    if (j + 1 == K || (keys[j + 1] >> b) != U) re[U] = j + 1;
}

// grp: union row offsets (N + 1 entries).  Per union vertex U of graph g: its local row offset
// at row_ptr[U + g]; per graph: adj_off[g] and the graph's closing offset at
// row_ptr[vtx_off[g + 1] + g].  Graphs with inconsistent offsets write nothing of theirs.
__global__ void k_pk_offsets(const uint32_t *__restrict__ grp,
                             const int64_t *__restrict__ vtx_off, uint32_t G, uint64_t N,
                             const int32_t *__restrict__ status, int64_t *__restrict__ adj_off,
                             int32_t *__restrict__ row_ptr) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) {
        // the graph whose vertex range [vtx_off[g], vtx_off[g + 1]) holds t (empty graphs
        // before it share its first offset)
        const uint32_t g = last_le(vtx_off, G, (int64_t)t);
        if (status[g] != TC_E_ARG && vtx_off[g] <= (int64_t)t && (int64_t)t < vtx_off[g + 1])
            row_ptr[t + g] = (int32_t)(grp[t] - grp[vtx_off[g]]);
    }
    if (t <= G) {
        const uint32_t g = (uint32_t)t;
        if (g == G) {
            adj_off[G] = grp[N];
        } else if (status[g] != TC_E_ARG) {
            const int64_t v0 = vtx_off[g], v1 = vtx_off[g + 1];
            adj_off[g] = grp[v0];
            row_ptr[v1 + g] = (int32_t)(grp[v1] - grp[v0]);
        } else {
            adj_off[g] = 0;
        }
    }
}

struct PackLayout {
    size_t ctl, keys_a, keys_b, sort_scratch, rs, re, rowlen, grp, scan, total;
};

static PackLayout pack_layout(uint64_t N, uint64_t M) {
    PackLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1), 256);
        return at;
    };
    const uint64_t K = 2 * M, n1 = N + 1;
    L.ctl = take(64 * 4);
    L.keys_a = take(K * 8);
    L.keys_b = take(K * 8);
    L.sort_scratch = take(sort_scratch_bytes(K));
    L.rs = take(n1 * 4);
    L.re = take(n1 * 4);
    L.rowlen = take(n1 * 4);
    L.grp = take(n1 * 4);
    L.scan = take(scan_scratch_words(n1) * 4);
    L.total = off;
    return L;
}

// int32 row offsets: 2 m_total < 2^31; union ids and row_ptr positions below 2^31
static bool pack_sizes_ok(int32_t G, int64_t n_total, int64_t m_total) {
    return G > 0 && n_total >= 0 && m_total >= 0 && n_total < (1ll << 31) &&
           2 * m_total < (1ll << 31) && n_total + G < (1ll << 31);
}

}  // namespace tc

using namespace tc;

extern "C" {

size_t tc_batched_pack_workspace_size(int32_t G, int64_t n_total, int64_t m_total) {
    if (!pack_sizes_ok(G, n_total, m_total)) return 0;
    return pack_layout((uint64_t)n_total, (uint64_t)m_total).total;
}

int tc_batched_pack(int32_t G, const int64_t *d_vtx_off, const int64_t *d_edge_off,
                    const int32_t *d_edges, int64_t n_total, int64_t m_total, void *d_ws,
                    size_t ws_bytes, void *stream, int64_t *d_adj_off, int32_t *d_row_ptr,
                    int32_t *d_col, int32_t *d_status) {
    if (G <= 0 || n_total < 0 || m_total < 0) return TC_E_ARG;
    if (!pack_sizes_ok(G, n_total, m_total)) return TC_E_TOO_LARGE;
    if (!d_vtx_off || !d_edge_off || !d_adj_off || !d_row_ptr || !d_status) return TC_E_ARG;
    if (m_total > 0 && (!d_edges || !d_col || ((uintptr_t)d_edges & 7))) return TC_E_ARG;
    const uint64_t N = (uint64_t)n_total, M = (uint64_t)m_total, K = 2 * M;
    const PackLayout L = pack_layout(N, M);
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < L.total) return TC_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    uint64_t *ka = (uint64_t *)(ws + L.keys_a), *kb = (uint64_t *)(ws + L.keys_b);
    uint32_t *rs = (uint32_t *)(ws + L.rs), *re = (uint32_t *)(ws + L.re);
    uint32_t *rowlen = (uint32_t *)(ws + L.rowlen), *grp = (uint32_t *)(ws + L.grp);
    int b = 1;  // bits of a union row id below the sentinel: 2^b - 1 >= N
    while (b < 31 && (1ull << b) - 1 < N) ++b;
    const uint32_t T = kPackThreads;
    auto blocks = [](uint64_t n, uint32_t per, uint64_t cap) {
        uint64_t g = (n + per - 1) / per;
        if (g == 0) g = 1;
        return (uint32_t)(g < cap ? g : cap);
    };
    uint32_t *bad = (uint32_t *)(ws + L.ctl);
    if (fill_u32(bad, 0u, 1, s) != hipSuccess) return TC_E_HIP;
    hipLaunchKernelGGL(k_pk_graphs, dim3(blocks(G, T, 1u << 30)), dim3(T), 0, s, d_vtx_off,
                       d_edge_off, (uint32_t)G, N, M, d_status, bad);
    hipLaunchKernelGGL(k_pk_mark, dim3(blocks(G, T, 1u << 30)), dim3(T), 0, s, (uint32_t)G,
                       bad, d_status);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    if (fill_u32(rs, 0u, N + 1, s) != hipSuccess || fill_u32(re, 0u, N + 1, s) != hipSuccess)
        return TC_E_HIP;
    uint64_t *sorted = ka;
    if (M > 0) {
        hipLaunchKernelGGL(k_pk_keys, dim3(blocks(M, T, 65536)), dim3(T), 0, s,
                           (const int2 *)d_edges, M, d_vtx_off, d_edge_off, (uint32_t)G, b, ka,
                           d_status);
        if (hipGetLastError() != hipSuccess) return TC_E_HIP;
        if (sort_u64(ka, kb, (uint32_t)K, 0, 2 * b, ws + L.sort_scratch, nullptr, s, &sorted) !=
            hipSuccess)
            return TC_E_HIP;
        hipLaunchKernelGGL(k_pk_rows, dim3(blocks(K, T, 1u << 30)), dim3(T), 0, s, sorted,
                           (uint32_t)K, N, b, d_col, rs, re);
        if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    }
    // row lengths (entry N is 0) and their exclusive scan: grp[N] = valid entries
    hipLaunchKernelGGL(k_rowlen, dim3(blocks(N + 1, T, 1u << 30)), dim3(T), 0, s, rs, re,
                       (uint32_t)N, rowlen);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    if (scan_exclusive_u32(rowlen, grp, N + 1, (uint32_t *)(ws + L.scan), s) != hipSuccess)
        return TC_E_HIP;
    const uint64_t work = N > (uint64_t)G + 1 ? N : (uint64_t)G + 1;
    hipLaunchKernelGGL(k_pk_offsets, dim3(blocks(work, T, 1u << 30)), dim3(T), 0, s, grp,
                       d_vtx_off, (uint32_t)G, N, d_status, d_adj_off, d_row_ptr);
    return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

}  // extern "C"
