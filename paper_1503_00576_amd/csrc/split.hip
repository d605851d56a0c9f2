// Graphs beyond device memory: the host pre-pass of Section 3.4 ("CPU preprocessing for very
// large graphs": degrees and the removal of backward edges on the CPU, which halves the
// two-direction input) and the subgraph splitting that Section 6 proposes for graphs that do
// not fit the GPU at all, as an exact partition scheme.
//
// Splitting.  The vertices are cut into K parts by a hash of their ids.  Let E_xy (x <= y) be
// the edges with one end in part x and the other in part y.  Every triangle has a multiset
// of parts {x, y, z}; the subgraphs
//   G_abc = E_ab + E_ac + E_bc             (a < b < c)   hold exactly the triangles {a, b, c},
//   G_ac  = E_aa + E_ac + E_cc             (a < c)       those of {a,a,a}, {a,a,c}, {a,c,c},
//                                                        {c,c,c},
//   E_aa                                                 those of {a,a,a},
// so  T = sum T(G_abc) + sum T(G_ac) - (K - 2) sum T(E_aa)  for K >= 2 (each {a,a,a} triangle
// lies in the K - 1 subgraphs G_ac with c != a), and the same identity holds vertex by vertex
// for the per-vertex counts.  Each subgraph is an ordinary graph counted by tc_count on the
// device; the triangle count of a graph does not depend on the order used to orient it, so
// every subgraph is oriented by its own degrees.  A subgraph holds about 6m / K^2 edges (three
// blocks of 2m / K^2), so K parts shrink the device working set about K^2 / 6 times; the
// edges cross the host-device link about K + 2 times in all.
//
// The host pass (tc_split_prepare) checks every edge, applies the pre-filter of Section 3.4
// to two-direction input, and buckets the kept edges by block (x, y) into the caller's host
// workspace, as pairs of ids local to their parts.  tc_split_count streams the subgraphs'
// blocks to the device (on a copy stream while the previous subgraph is counted), relabels
// them to the subgraph's local ids, counts, and accumulates the signed results.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "internal.h"

namespace tc {

namespace {

constexpr uint64_t kSplitMagic = 0x3174696c70735f74ull;  // "t_split1"
constexpr uint32_t kMaxParts = TC_SPLIT_MAX_PARTS;

// MurmurHash3's 32-bit finaliser (Appleby): the vertex hash of the partition
inline uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
inline uint32_t part_of(int32_t x, uint32_t K) {
    return (uint32_t)(((uint64_t)fmix32((uint32_t)x) * K) >> 32);
}
// block (x, y), x <= y, in row-major order of the upper triangle
inline uint32_t block_id(uint32_t x, uint32_t y, uint32_t K) {
    return x * K - x * (x - 1) / 2 + (y - x);
}
inline uint32_t n_blocks(uint32_t K) { return K * (K + 1) / 2; }

struct Sub {
    uint32_t parts[3];   // ascending
    uint32_t np;         // parts used (1..3)
    uint32_t blocks[3];  // block ids
    uint32_t nb;         // blocks used (1..3)
    int64_t coef;        // +1, or -(K - 2) for E_aa
    int64_t n, m;        // local vertices and edges
};

// Host workspace: this header, then the arrays at the offsets it records (64-byte aligned).
struct Header {
    uint64_t magic;
    int64_t n, m_in, m_fwd;  // vertices, input entries, undirected edges kept
    uint32_t flags, K, nsub, pad;
    int64_t max_n, max_m;
    size_t dev_bytes, ws_bytes, host_bytes;  // device workspace in total / for tc_count
    size_t off_lid, off_vtx, off_deg, off_part, off_block, off_sub, off_edges;
};

inline size_t a64(size_t x) { return (x + 63) & ~(size_t)63; }

struct HostLayout {
    size_t lid, vtx, deg, part, block, sub, edges, total;
};
HostLayout host_layout(int64_t n, int64_t m_fwd, bool both) {
    const uint64_t K = kMaxParts;
    const uint64_t subs = K * (K - 1) * (K - 2) / 6 + K * (K - 1) / 2 + K;
    HostLayout h;
    size_t off = a64(sizeof(Header));
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = a64(off + bytes);
        return at;
    };
    h.lid = take((size_t)n * 4);
    h.vtx = take((size_t)n * 4);
    h.deg = take(both ? (size_t)n * 4 : 0);
    h.part = take((K + 1) * 8);
    h.block = take((K * (K + 1) / 2 + 1) * 8);
    h.sub = take(subs * sizeof(Sub));
    h.edges = take((size_t)m_fwd * 8);
    h.total = off;
    return h;
}

template <class T>
T *hat(void *ws, size_t off) {
    return (T *)((char *)ws + off);
}
template <class T>
const T *hat(const void *ws, size_t off) {
    return (const T *)((const char *)ws + off);
}

unsigned host_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 4;
    return t > 16 ? 16 : t;
}

// runs fn(thread, begin, end) over [0, count) in contiguous chunks, one per thread
template <class F>
void parallel_chunks(uint64_t count, unsigned T, F fn) {
    if (count < (1u << 16) || T <= 1) {
        fn(0u, (uint64_t)0, count);
        return;
    }
    std::vector<std::thread> th;
    const uint64_t per = (count + T - 1) / T;
    for (unsigned t = 0; t < T; ++t) {
        const uint64_t b = std::min(count, per * t), e = std::min(count, per * (t + 1));
        th.emplace_back(fn, t, b, e);
    }
    for (auto &x : th) x.join();
}

// the subproblems of K parts, with their local sizes
void build_subs(uint32_t K, const int64_t *psize, const int64_t *bcount, std::vector<Sub> &out) {
    out.clear();
    auto add = [&](std::initializer_list<uint32_t> parts,
                   std::initializer_list<std::pair<uint32_t, uint32_t>> blocks, int64_t coef) {
        Sub s{};
        s.np = 0;
        s.n = 0;
        for (uint32_t p : parts) {
            s.parts[s.np++] = p;
            s.n += psize[p];
        }
        s.nb = 0;
        s.m = 0;
        for (auto &b : blocks) {
            const uint32_t id = block_id(b.first, b.second, K);
            s.blocks[s.nb++] = id;
            s.m += bcount[id];
        }
        s.coef = coef;
        if (s.m > 0) out.push_back(s);  // no edges: no triangles, no per-vertex counts
    };
    if (K == 1) {
        add({0u}, {{0u, 0u}}, 1);
        return;
    }
    for (uint32_t a = 0; a < K; ++a)
        for (uint32_t b = a + 1; b < K; ++b)
            for (uint32_t c = b + 1; c < K; ++c) add({a, b, c}, {{a, b}, {a, c}, {b, c}}, 1);
    for (uint32_t a = 0; a < K; ++a)
        for (uint32_t c = a + 1; c < K; ++c) add({a, c}, {{a, a}, {a, c}, {c, c}}, 1);
    if (K > 2)
        for (uint32_t a = 0; a < K; ++a) add({a}, {{a, a}}, -(int64_t)(K - 2));
}

// device layout of tc_split_count: two edge buffers for the largest subgraph, tc_count's
// workspace for the largest of them, local per-vertex counts, the parts' vertex lists, and a
// few words
struct DevLayout {
    size_t ebuf[2], ws, pv, vtx, words, total;
};
DevLayout dev_layout(int64_t max_n, int64_t max_m, size_t ws_bytes, int64_t n) {
    DevLayout d;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1), 256);
        return at;
    };
    d.ebuf[0] = take((size_t)max_m * 8);
    d.ebuf[1] = take((size_t)max_m * 8);
    d.ws = take(ws_bytes);
    d.pv = take((size_t)max_n * 8);
    d.vtx = take((size_t)n * 4);
    d.words = take(64);
    d.total = off;
    return d;
}

// device bytes tc_split_count needs for these subproblems
struct DevNeed {
    size_t total, ws;
    int64_t max_n, max_m;
    bool ok;
};
DevNeed device_need(const std::vector<Sub> &subs, int64_t n, const tc_options *opts) {
    DevNeed d{0, 0, 0, 0, true};
    for (const Sub &s : subs) {
        d.max_n = std::max(d.max_n, s.n);
        d.max_m = std::max(d.max_m, s.m);
        if (s.n >= (1ll << 31) || s.m >= (1ll << 32)) {
            d.ok = false;
            continue;
        }
        const size_t w = tc_workspace_size(s.n, s.m, TC_EDGES_ONCE, opts);
        if (w == 0) d.ok = false;
        d.ws = std::max(d.ws, w);
    }
    d.total = dev_layout(d.max_n, d.max_m, d.ws, n).total;
    return d;
}

}  // namespace

// ------------------------------------------------------------------ device kernels

struct RelabelSeg {
    uint64_t end;        // entries [previous end, end) of the subgraph's edge buffer
    int32_t add_x, add_y;  // local id offsets of the block's two parts
};
struct Relabel3 {
    RelabelSeg seg[3];
    uint32_t nseg;
};

// part-local ids of the blocks' edges -> ids local to the subgraph
__global__ void k_split_relabel(int2 *__restrict__ e, Relabel3 r) {
    const uint64_t total = r.seg[r.nseg - 1].end;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t k = 0;
        while (k + 1 < r.nseg && i >= r.seg[k].end) ++k;
        int2 v = e[i];
        v.x += r.seg[k].add_x;
        v.y += r.seg[k].add_y;
        e[i] = v;
    }
}

__global__ void k_split_init(unsigned long long *__restrict__ total, int32_t *__restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (total) *total = 0;
        if (status) *status = 0;
    }
}

__global__ void k_split_zero(unsigned long long *__restrict__ p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// total += coef * subgraph total (mod 2^64: the signed sum is exact once all terms are in);
// the first nonzero subgraph status is kept
__global__ void k_split_fold(const unsigned long long *__restrict__ sub_total,
                             const int32_t *__restrict__ sub_status, long long coef,
                             unsigned long long *__restrict__ total,
                             int32_t *__restrict__ status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *total += (unsigned long long)coef * *sub_total;
    if (status && *status == 0 && *sub_status != 0) *status = *sub_status;
}

struct PartSeg {
    uint64_t end;         // local ids [previous end, end) belong to this part
    const int32_t *vtx;   // the part's vertices, by local id within the part
};
struct PartSeg3 {
    PartSeg seg[3];
    uint32_t nseg;
};

// per_vertex[global id] += coef * subgraph per-vertex count (each global id once per subgraph)
__global__ void k_split_pv(const unsigned long long *__restrict__ sub_pv, PartSeg3 p,
                           long long coef, unsigned long long *__restrict__ pv) {
    const uint64_t total = p.seg[p.nseg - 1].end;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t k = 0;
        while (k + 1 < p.nseg && i >= p.seg[k].end) ++k;
        const uint64_t base = k ? p.seg[k - 1].end : 0;
        const int32_t g = p.seg[k].vtx[i - base];
        pv[g] += (unsigned long long)coef * sub_pv[i];
    }
}

}  // namespace tc

using namespace tc;

extern "C" {

size_t tc_split_host_workspace_size(int64_t n, int64_t m, uint32_t flags) {
    if (n < 0 || m < 0 || n >= (1ll << 31) || (flags & ~TC_EDGES_BOTH)) return 0;
    const bool both = flags & TC_EDGES_BOTH;
    return host_layout(n, both ? m / 2 : m, both).total;
}

int tc_split_prepare(const int32_t *h_edges, int64_t n, int64_t m, uint32_t flags,
                     uint32_t parts, size_t device_budget, const tc_options *opts, void *h_ws,
                     size_t h_ws_bytes, tc_split_info *info) {
    if (n < 0 || m < 0 || (flags & ~TC_EDGES_BOTH) || parts > kMaxParts) return TC_E_ARG;
    if (n >= (1ll << 31)) return TC_E_TOO_LARGE;
    if (n == 0 && m > 0) return TC_E_ARG;
    if (m > 0 && !h_edges) return TC_E_ARG;
    if (!h_ws || ((uintptr_t)h_ws & 63)) return TC_E_ARG;
    const bool both = flags & TC_EDGES_BOTH;
    if (both && (m & 1)) return TC_E_ASYMMETRIC;
    const int64_t m_fwd = both ? m / 2 : m;
    const HostLayout hl = host_layout(n, m_fwd, both);
    if (h_ws_bytes < hl.total) return TC_E_WORKSPACE;
    if (tc_workspace_size(1, 1, TC_EDGES_ONCE, opts) == 0) return TC_E_ARG;  // bad options

    Header &H = *hat<Header>(h_ws, 0);
    memset(&H, 0, sizeof(H));
    H.n = n;
    H.m_in = m;
    H.m_fwd = m_fwd;
    H.flags = flags;
    H.off_lid = hl.lid;
    H.off_vtx = hl.vtx;
    H.off_deg = hl.deg;
    H.off_part = hl.part;
    H.off_block = hl.block;
    H.off_sub = hl.sub;
    H.off_edges = hl.edges;
    H.host_bytes = hl.total;
    const unsigned T = host_threads();
    const int2 *E = (const int2 *)h_edges;

    // 1. checks (ids in range, no self-loops) and, for two-direction input, the degrees:
    //    the entries with the vertex first (Section 3.2, step 2)
    std::atomic<int> err{0};
    uint32_t *deg = both ? hat<uint32_t>(h_ws, hl.deg) : nullptr;
    if (both) memset(deg, 0, (size_t)n * 4);
    parallel_chunks((uint64_t)m, T, [&](unsigned, uint64_t b, uint64_t e) {
        int local = 0;
        for (uint64_t i = b; i < e && !local; ++i) {
            const int2 x = E[i];
            if (x.x < 0 || x.x >= n || x.y < 0 || x.y >= n) local = TC_E_RANGE;
            else if (x.x == x.y) local = TC_E_SELF_LOOP;
            else if (both) __atomic_fetch_add(&deg[x.x], 1u, __ATOMIC_RELAXED);
        }
        if (local) {
            int z = 0;
            err.compare_exchange_strong(z, local);
        }
    });
    if (err.load()) return err.load();
    // the pre-filter of Section 3.4: an entry is kept iff it points forward in the order
    // (degree, id); a valid two-direction array keeps exactly half of its entries
    auto forward = [&](const int2 x) {
        const uint32_t du = deg[x.x], dv = deg[x.y];
        return du < dv || (du == dv && x.x < x.y);
    };
    if (both) {
        std::vector<uint64_t> kept(T, 0);
        parallel_chunks((uint64_t)m, T, [&](unsigned t, uint64_t b, uint64_t e) {
            uint64_t c = 0;
            for (uint64_t i = b; i < e; ++i) c += forward(E[i]) ? 1u : 0u;
            kept[t] = c;
        });
        uint64_t k = 0;
        for (uint64_t c : kept) k += c;
        if ((int64_t)k != m_fwd) return TC_E_ASYMMETRIC;
    }

    // 2. the number of parts: the caller's, or the smallest whose device footprint fits
    int64_t *psize = hat<int64_t>(h_ws, hl.part);     // part sizes, later offsets
    int64_t *bcount = hat<int64_t>(h_ws, hl.block);  // block sizes, later offsets
    std::vector<Sub> subs;
    auto size_parts = [&](uint32_t K, std::vector<std::vector<int64_t>> &tb) {
        std::fill(psize, psize + K + 1, 0);
        for (int64_t x = 0; x < n; ++x) ++psize[part_of((int32_t)x, K)];
        const uint32_t nb = n_blocks(K);
        tb.assign(T, std::vector<int64_t>(nb, 0));
        parallel_chunks((uint64_t)m, T, [&](unsigned t, uint64_t b, uint64_t e) {
            int64_t *c = tb[t].data();
            for (uint64_t i = b; i < e; ++i) {
                const int2 x = E[i];
                if (both && !forward(x)) continue;
                uint32_t pa = part_of(x.x, K), pb = part_of(x.y, K);
                if (pa > pb) std::swap(pa, pb);
                ++c[block_id(pa, pb, K)];
            }
        });
        std::fill(bcount, bcount + nb + 1, 0);
        for (unsigned t = 0; t < T; ++t)
            for (uint32_t i = 0; i < nb; ++i) bcount[i] += tb[t][i];
        build_subs(K, psize, bcount, subs);
    };
    std::vector<std::vector<int64_t>> tb;
    uint32_t K = parts;
    DevNeed need{};
    if (K) {
        size_parts(K, tb);
        need = device_need(subs, n, opts);
        if (!need.ok) return TC_E_TOO_LARGE;
    } else {
        bool found = false;
        for (K = 1; K <= kMaxParts; ++K) {
            if (K == 2) continue;  // G_01 is the whole graph: no smaller than one part
            size_parts(K, tb);
            need = device_need(subs, n, opts);
            if (need.ok && need.total <= device_budget) {
                found = true;
                break;
            }
        }
        if (!found) return TC_E_TOO_LARGE;
    }
    const uint32_t nb = n_blocks(K);

    // 3. local ids: the vertices of each part in id order
    int32_t *lid = hat<int32_t>(h_ws, hl.lid);
    int32_t *vtx = hat<int32_t>(h_ws, hl.vtx);
    {
        std::vector<int64_t> cur(K + 1, 0);
        int64_t acc = 0;
        for (uint32_t p = 0; p < K; ++p) {
            const int64_t sz = psize[p];
            psize[p] = acc;  // offsets from here on
            cur[p] = acc;
            acc += sz;
        }
        psize[K] = acc;
        for (int64_t x = 0; x < n; ++x) {
            const uint32_t p = part_of((int32_t)x, K);
            lid[x] = (int32_t)(cur[p] - psize[p]);
            vtx[cur[p]++] = (int32_t)x;
        }
    }
    // 4. the kept edges bucketed by block, as part-local id pairs (lower part first)
    {
        std::vector<int64_t> sizes(bcount, bcount + nb);
        int64_t acc = 0;
        for (uint32_t i = 0; i < nb; ++i) {
            bcount[i] = acc;
            acc += sizes[i];
        }
        bcount[nb] = acc;
        // per-thread write cursors: thread t writes its chunk's edges of block i after the
        // earlier threads' edges of that block
        for (uint32_t i = 0; i < nb; ++i) {
            int64_t c = bcount[i];
            for (unsigned t = 0; t < T; ++t) {
                const int64_t k = tb[t][i];
                tb[t][i] = c;
                c += k;
            }
        }
        int2 *out = hat<int2>(h_ws, hl.edges);
        parallel_chunks((uint64_t)m, T, [&](unsigned t, uint64_t b, uint64_t e) {
            int64_t *cur = tb[t].data();
            for (uint64_t i = b; i < e; ++i) {
                int2 x = E[i];
                if (both && !forward(x)) continue;
                uint32_t pa = part_of(x.x, K), pb = part_of(x.y, K);
                if (pa > pb) {
                    std::swap(pa, pb);
                    std::swap(x.x, x.y);
                }
                out[cur[block_id(pa, pb, K)]++] = make_int2(lid[x.x], lid[x.y]);
            }
        });
    }
    Sub *S = hat<Sub>(h_ws, hl.sub);
    std::copy(subs.begin(), subs.end(), S);
    H.K = K;
    H.nsub = (uint32_t)subs.size();
    H.max_n = need.max_n;
    H.max_m = need.max_m;
    H.ws_bytes = need.ws;
    H.dev_bytes = need.total;
    H.magic = kSplitMagic;
    if (info) {
        info->parts = K;
        info->subgraphs = H.nsub;
        info->m_kept = m_fwd;
        info->max_sub_n = need.max_n;
        info->max_sub_m = need.max_m;
        info->device_bytes = need.total;
        info->host_bytes = hl.total;
    }
    return TC_OK;
}

int tc_split_subgraph(const void *h_ws, uint32_t index, tc_split_subgraph_info *out) {
    if (!h_ws || !out) return TC_E_ARG;
    const Header &H = *hat<Header>(h_ws, 0);
    if (H.magic != kSplitMagic || index >= H.nsub) return TC_E_ARG;
    const Sub &s = hat<Sub>(h_ws, H.off_sub)[index];
    out->n = s.n;
    out->m = s.m;
    out->coef = s.coef;
    out->nparts = s.np;
    for (uint32_t i = 0; i < 3; ++i) out->parts[i] = i < s.np ? s.parts[i] : 0u;
    return TC_OK;
}

int tc_split_subgraph_edges(const void *h_ws, uint32_t index, int32_t *h_out,
                            int32_t *h_vertex) {
    if (!h_ws) return TC_E_ARG;
    const Header &H = *hat<Header>(h_ws, 0);
    if (H.magic != kSplitMagic || index >= H.nsub) return TC_E_ARG;
    const Sub &s = hat<Sub>(h_ws, H.off_sub)[index];
    const int64_t *poff = hat<int64_t>(h_ws, H.off_part);
    const int64_t *boff = hat<int64_t>(h_ws, H.off_block);
    const int2 *E = hat<int2>(h_ws, H.off_edges);
    const int32_t *vtx = hat<int32_t>(h_ws, H.off_vtx);
    const uint32_t K = H.K;
    auto base_of = [&](uint32_t p) {
        int64_t b = 0;
        for (uint32_t i = 0; i < s.np && s.parts[i] != p; ++i) b += poff[s.parts[i] + 1] - poff[s.parts[i]];
        return (int32_t)b;
    };
    if (h_out) {
        int64_t w = 0;
        for (uint32_t k = 0; k < s.nb; ++k) {
            // block id -> (x, y)
            uint32_t x = 0, id = s.blocks[k];
            while (id >= K - x) {
                id -= K - x;
                ++x;
            }
            const uint32_t y = x + id;
            const int32_t ax = base_of(x), ay = base_of(y);
            for (int64_t i = boff[s.blocks[k]]; i < boff[s.blocks[k] + 1]; ++i) {
                h_out[2 * w] = E[i].x + ax;
                h_out[2 * w + 1] = E[i].y + ay;
                ++w;
            }
        }
    }
    if (h_vertex) {
        int64_t w = 0;
        for (uint32_t i = 0; i < s.np; ++i)
            for (int64_t j = poff[s.parts[i]]; j < poff[s.parts[i] + 1]; ++j) h_vertex[w++] = vtx[j];
    }
    return TC_OK;
}

int tc_split_count(const void *h_ws, const tc_options *opts, void *d_ws, size_t d_ws_bytes,
                   void *stream, void *copy_stream, uint64_t *d_total, uint64_t *d_per_vertex,
                   int32_t *d_status) {
    if (!h_ws || !d_total) return TC_E_ARG;
    const Header &H = *hat<Header>(h_ws, 0);
    if (H.magic != kSplitMagic) return TC_E_ARG;
    if (!d_ws || ((uintptr_t)d_ws & 255) || d_ws_bytes < H.dev_bytes) return TC_E_WORKSPACE;
    const Sub *S = hat<Sub>(h_ws, H.off_sub);
    for (uint32_t i = 0; i < H.nsub; ++i) {  // options other than tc_split_prepare's
        const size_t w = tc_workspace_size(S[i].n, S[i].m, TC_EDGES_ONCE, opts);
        if (w == 0) return TC_E_ARG;
        if (w > H.ws_bytes) return TC_E_WORKSPACE;
    }
    const DevLayout D = dev_layout(H.max_n, H.max_m, H.ws_bytes, H.n);
    hipStream_t s = (hipStream_t)stream;
    hipStream_t cs = (hipStream_t)copy_stream;
    const bool overlap = cs && cs != s;
    const bool pv = d_per_vertex != nullptr && H.n > 0;
    char *base = (char *)d_ws;
    unsigned long long *words = (unsigned long long *)(base + D.words);
    unsigned long long *sub_total = words;
    int32_t *sub_status = (int32_t *)(words + 1);
    int32_t *d_vtx = (int32_t *)(base + D.vtx);
    unsigned long long *sub_pv = (unsigned long long *)(base + D.pv);
    const int64_t *poff = hat<int64_t>(h_ws, H.off_part);
    const int64_t *boff = hat<int64_t>(h_ws, H.off_block);
    const int2 *E = hat<int2>(h_ws, H.off_edges);
    const uint32_t K = H.K;

    hipLaunchKernelGGL(k_split_init, dim3(1), dim3(64), 0, s, (unsigned long long *)d_total,
                       d_status);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    if (pv) {
        hipLaunchKernelGGL(k_split_zero, dim3(std::min<uint64_t>(4096, (H.n + 255) / 256)),
                           dim3(256), 0, s, (unsigned long long *)d_per_vertex, (uint64_t)H.n);
        if (hipGetLastError() != hipSuccess) return TC_E_HIP;
        if (hipMemcpyAsync(d_vtx, hat<int32_t>(h_ws, H.off_vtx), (size_t)H.n * 4,
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return TC_E_HIP;
    }
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    int rc = TC_OK;
    if (overlap) {
        for (int i = 0; i < 2 && rc == TC_OK; ++i)
            if (hipEventCreateWithFlags(&ready[i], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&freed[i], hipEventDisableTiming) != hipSuccess)
                rc = TC_E_HIP;
        // the copy stream starts after everything the caller enqueued on `stream`
        if (rc == TC_OK && (hipEventRecord(freed[0], s) != hipSuccess ||
                            hipStreamWaitEvent(cs, freed[0], 0) != hipSuccess))
            rc = TC_E_HIP;
    }
    auto block_xy = [&](uint32_t id, uint32_t &x, uint32_t &y) {
        x = 0;
        while (id >= K - x) {
            id -= K - x;
            ++x;
        }
        y = x + id;
    };
    for (uint32_t i = 0; i < H.nsub && rc == TC_OK; ++i) {
        const Sub &sb = S[i];
        const int b = i & 1;
        int2 *ebuf = (int2 *)(base + D.ebuf[b]);
        hipStream_t qs = overlap ? cs : s;
        // the buffer was last read by subgraph i - 2's count
        if (overlap && i >= 2 && hipStreamWaitEvent(cs, freed[b], 0) != hipSuccess) {
            rc = TC_E_HIP;
            break;
        }
        Relabel3 r{};
        PartSeg3 ps{};
        int64_t at = 0;
        int64_t pbase[3];
        {
            int64_t acc = 0;
            for (uint32_t k = 0; k < sb.np; ++k) {
                pbase[k] = acc;
                const uint32_t p = sb.parts[k];
                acc += poff[p + 1] - poff[p];
                ps.seg[k].end = (uint64_t)acc;
                ps.seg[k].vtx = d_vtx + poff[p];
            }
            ps.nseg = sb.np;
        }
        auto local_base = [&](uint32_t p) {
            for (uint32_t k = 0; k < sb.np; ++k)
                if (sb.parts[k] == p) return (int32_t)pbase[k];
            return 0;
        };
        for (uint32_t k = 0; k < sb.nb; ++k) {
            const uint32_t id = sb.blocks[k];
            const int64_t cnt = boff[id + 1] - boff[id];
            if (cnt > 0 && hipMemcpyAsync(ebuf + at, E + boff[id], (size_t)cnt * 8,
                                          hipMemcpyHostToDevice, qs) != hipSuccess) {
                rc = TC_E_HIP;
                break;
            }
            at += cnt;
            uint32_t x, y;
            block_xy(id, x, y);
            r.seg[k].end = (uint64_t)at;
            r.seg[k].add_x = local_base(x);
            r.seg[k].add_y = local_base(y);
        }
        if (rc) break;
        r.nseg = sb.nb;
        if (overlap && (hipEventRecord(ready[b], cs) != hipSuccess ||
                        hipStreamWaitEvent(s, ready[b], 0) != hipSuccess)) {
            rc = TC_E_HIP;
            break;
        }
        const uint32_t grid = (uint32_t)std::min<uint64_t>(8192, ((uint64_t)sb.m + 255) / 256);
        hipLaunchKernelGGL(k_split_relabel, dim3(grid ? grid : 1), dim3(256), 0, s, ebuf, r);
        if (hipGetLastError() != hipSuccess) {
            rc = TC_E_HIP;
            break;
        }
        int st;
        if (pv)
            st = tc_count_per_vertex((const int32_t *)ebuf, sb.n, sb.m, TC_EDGES_ONCE, opts,
                                     base + D.ws, H.ws_bytes, s, (uint64_t *)sub_total,
                                     (uint64_t *)sub_pv, sub_status);
        else
            st = tc_count((const int32_t *)ebuf, sb.n, sb.m, TC_EDGES_ONCE, opts, base + D.ws,
                          H.ws_bytes, s, (uint64_t *)sub_total, sub_status);
        if (st) {
            rc = st;
            break;
        }
        if (overlap && hipEventRecord(freed[b], s) != hipSuccess) {
            rc = TC_E_HIP;
            break;
        }
        hipLaunchKernelGGL(k_split_fold, dim3(1), dim3(64), 0, s, sub_total, sub_status,
                           (long long)sb.coef, (unsigned long long *)d_total, d_status);
        if (hipGetLastError() != hipSuccess) {
            rc = TC_E_HIP;
            break;
        }
        if (pv) {
            const uint32_t g = (uint32_t)std::min<uint64_t>(4096, ((uint64_t)sb.n + 255) / 256);
            hipLaunchKernelGGL(k_split_pv, dim3(g ? g : 1), dim3(256), 0, s, sub_pv, ps,
                               (long long)sb.coef, (unsigned long long *)d_per_vertex);
            if (hipGetLastError() != hipSuccess) {
                rc = TC_E_HIP;
                break;
            }
        }
    }
    // `stream` ends after the copy stream's last work (nothing is left behind on it)
    if (overlap && rc == TC_OK && ready[0]) {
        if (hipEventRecord(ready[0], cs) != hipSuccess ||
            hipStreamWaitEvent(s, ready[0], 0) != hipSuccess)
            rc = TC_E_HIP;
    }
    for (int i = 0; i < 2; ++i) {
        if (ready[i]) (void)hipEventDestroy(ready[i]);
        if (freed[i]) (void)hipEventDestroy(freed[i]);
    }
    return rc;
}

}  // extern "C"
