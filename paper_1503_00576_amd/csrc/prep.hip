// Preprocessing phase (Section 3.2) on the device, in "rank space".
//
//   k_degree     degrees of the vertices and the input checks of Section 3.1
//   k_vkeys      packs (degree, id) so that a stable sort yields the total order of Section 2.2
//                (degree first, ties by id); the position of a vertex in that order is its rank
//   k_rank       perm[r] = vertex of rank r, rank[v] = r
//   k_orient     every edge becomes a packed key (rank s << b) | rank t with s < t, i.e. the
//                edge kept only in its forward direction (Section 3.2, steps 5-6); in the
//                paper's two-direction format backward entries are dropped
//   k_csr        node array (Section 3.2, step 4/8: row_ptr[x] = first key whose source is
//                >= x) and the unzipped neighbour array (step 7), duplicate check
//   k_csc_*      for every vertex v the list of in-edges u -> v that can close a triangle
//                through v: the suffix of N+(u) after v, stored as a [begin, end) range
//   k_items_*    work items of the counting kernels (see count.hip)
//
// Working with ranks instead of ids makes the order test a plain comparison, groups the
// high-degree vertices (whose lists are read most often) into one contiguous region, and
// keeps each out-list inside a short range of ranks, which the counting kernels exploit.
#include "internal.h"

namespace tc {

__global__ void k_degree(const int2 *__restrict__ edges, uint64_t m, uint32_t n, uint32_t both,
                         uint32_t *__restrict__ deg, int32_t *__restrict__ status) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) {
        int2 e = edges[i];
        if ((uint32_t)e.x >= n || (uint32_t)e.y >= n) {
            set_status(status, TC_E_RANGE);
            continue;
        }
        if (e.x == e.y) {
            set_status(status, TC_E_SELF_LOOP);
            continue;
        }
        atomicAdd(&deg[e.x], 1u);
        if (!both) atomicAdd(&deg[e.y], 1u);
    }
}

__global__ void k_vkeys(const uint32_t *__restrict__ deg, uint32_t n, int b,
                        uint64_t *__restrict__ vkeys) {
    uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t lim = (1ull << b) - 1;
    uint64_t d = deg[x];
    if (d > lim) d = lim;  // only possible for invalid input, which is reported elsewhere
    vkeys[x] = (d << b) | x;
}

__global__ void k_rank(const uint64_t *__restrict__ sorted, uint32_t n, int b,
                       uint32_t *__restrict__ perm, uint32_t *__restrict__ rank) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    uint32_t x = (uint32_t)(sorted[r] & ((1ull << b) - 1));
    perm[r] = x;
    rank[x] = r;
}

__global__ void k_orient(const int2 *__restrict__ edges, uint64_t m, uint32_t both,
                         const uint32_t *__restrict__ rank, int b, uint64_t *__restrict__ keys,
                         uint32_t *__restrict__ counter, const int32_t *__restrict__ status) {
    if (*status) return;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // uniform trip count so that every lane takes part in the wave-wide ballots
    const uint64_t rounds = (m + stride - 1) / stride;
    for (uint64_t r = 0; r < rounds; ++r, i += stride) {
        bool in = i < m;
        uint32_t ru = 0, rv = 0;
        if (in) {
            int2 e = edges[i];
            ru = rank[e.x];
            rv = rank[e.y];
        }
        if (!both) {
            if (in) {
                uint32_t s = ru < rv ? ru : rv, t = ru < rv ? rv : ru;
                keys[i] = ((uint64_t)s << b) | t;
            }
        } else {
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
}

// two-direction format: exactly half of the entries must be forward
__global__ void k_both_check(const uint32_t *__restrict__ counter, uint32_t expect,
                             int32_t *__restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *counter != expect)
        set_status(status, TC_E_ASYMMETRIC);
}

__global__ void k_csr(const uint64_t *__restrict__ keys, uint32_t mf, uint32_t n, int b,
                      uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ col,
                      int32_t *__restrict__ status) {
    if (*status) return;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mf) return;
    const uint64_t k = keys[i];
    const uint32_t s = (uint32_t)(k >> b);
    col[i] = (uint32_t)(k & ((1ull << b) - 1));
    int64_t prev = -1;
    if (i > 0) {
        uint64_t kp = keys[i - 1];
        prev = (int64_t)(kp >> b);
        if (kp == k) set_status(status, TC_E_DUP_EDGE);
    }
    const int64_t hi = s < n ? (int64_t)s : (int64_t)n - 1;
    for (int64_t r = prev + 1; r <= hi; ++r) row_ptr[r] = i;
    if (i == mf - 1)
        for (int64_t r = hi + 1; r <= (int64_t)n; ++r) row_ptr[r] = mf;
}

// In-edge u -> v (at CSR position e) can close a triangle u < v < w only through an element
// w of N+(u) after v that also lies in N+(v); the ranges of the two lists must overlap.
__device__ __forceinline__ bool useful_inedge(uint32_t e, uint32_t u, uint32_t v,
                                              const uint32_t *__restrict__ row_ptr,
                                              const uint32_t *__restrict__ col,
                                              uint32_t &end_u) {
    end_u = row_ptr[u + 1];
    if (e + 1 >= end_u) return false;
    uint32_t rv0 = row_ptr[v], rv1 = row_ptr[v + 1];
    if (rv1 == rv0) return false;
    return col[e + 1] <= col[rv1 - 1] && col[end_u - 1] >= col[rv0];
}

__global__ void k_csc_count(const uint64_t *__restrict__ keys, uint32_t mf, int b,
                            const uint32_t *__restrict__ row_ptr,
                            const uint32_t *__restrict__ col, uint32_t *__restrict__ cdeg,
                            const int32_t *__restrict__ status) {
    if (*status) return;
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mf) return;
    uint32_t u = (uint32_t)(keys[e] >> b), v = col[e], end_u;
    if (useful_inedge(e, u, v, row_ptr, col, end_u)) atomicAdd(&cdeg[v], 1u);
}

__global__ void k_csc_fill(const uint64_t *__restrict__ keys, uint32_t mf, int b,
                           const uint32_t *__restrict__ row_ptr,
                           const uint32_t *__restrict__ col, const uint32_t *__restrict__ cptr,
                           uint32_t *__restrict__ cfill, uint32_t *__restrict__ cbeg,
                           uint32_t *__restrict__ cend, uint32_t *__restrict__ cu,
                           const int32_t *__restrict__ status) {
    if (*status) return;
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mf) return;
    uint32_t u = (uint32_t)(keys[e] >> b), v = col[e], end_u;
    if (!useful_inedge(e, u, v, row_ptr, col, end_u)) return;
    uint32_t slot = cptr[v] + atomicAdd(&cfill[v], 1u);
    cbeg[slot] = e + 1;
    cend[slot] = end_u;
    cu[slot] = u;
}

// Work items of the counting kernel.  A vertex's in-edges are cut into chunks; the chunks go
// to the per-wave queue when the vertex's out-list fits one wave's LDS slice (as a bitmap over
// its rank span, or for per-vertex counts as a list with counters), otherwise to the
// per-workgroup queue.  Both classifications are prepared, so a prepared graph can be
// counted either way.
__global__ void k_items(const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ col,
                        const uint32_t *__restrict__ cdeg, uint32_t n, uint32_t wave_span,
                        uint32_t wave_list_pv, uint32_t ka, uint32_t kb,
                        uint32_t *__restrict__ ia, uint32_t *__restrict__ ib,
                        uint32_t *__restrict__ ia_pv, uint32_t *__restrict__ ib_pv,
                        const int32_t *__restrict__ status) {
    if (*status) return;
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    uint32_t a = 0, b = 0, apv = 0, bpv = 0;
    if (v < n && cdeg[v] > 0) {
        const uint32_t r0 = row_ptr[v], d = row_ptr[v + 1] - r0;
        const uint32_t span = col[r0 + d - 1] - col[r0];
        const uint32_t na = (cdeg[v] + ka - 1) / ka, nb = (cdeg[v] + kb - 1) / kb;
        if (span < wave_span) a = na; else b = nb;
        if (d <= wave_list_pv) apv = na; else bpv = nb;
    }
    ia[v] = a;
    ib[v] = b;
    ia_pv[v] = apv;
    ib_pv[v] = bpv;
}

__global__ void k_item_fill(const uint32_t *__restrict__ items, const uint32_t *__restrict__ off,
                            uint32_t n, uint32_t *__restrict__ item_v,
                            const int32_t *__restrict__ status) {
    if (*status) return;
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t k = items[v], o = off[v];
    for (uint32_t j = 0; j < k; ++j) item_v[o + j] = v;
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
