// Counting phase (Section 2.2 and Section 3.3): the sum over oriented edges u -> v of
// |N+(u) n N+(v)|.
//
// Vertices are ranks in the order of Section 2.2, so every list N+(x) holds only ranks > x
// and is sorted ascending.  For an edge u -> v, every common element w of the two lists is
// > v, so |N+(u) n N+(v)| = |suffix of N+(u) after v  n  N+(v)|.  The kernel therefore groups
// the work by the middle vertex v: N+(v) is staged once in LDS and the suffixes of the lists
// of all in-neighbours u of v are streamed through it.  The number of membership tests is
// sum_u C(d+(u), 2) instead of the sum of the lengths of both lists per edge; each test is
// one LDS bit lookup when N+(v) fits a bitmap over its rank range.
//
// Work items are (v, a chunk of v's in-edges).  One persistent kernel pulls items from two
// device counters: first the "workgroup" items (out-lists whose rank span needs the
// workgroup's whole LDS bitmap, or a sorted list), cooperatively, then the "wave" items, each
// wave with its own slice of LDS.  Items run heaviest (highest-rank) vertices first.  Inside a
// wave every in-edge suffix is cut into pieces of kPiece consecutive elements and each lane
// runs whole pieces, so one load and one lookup per element are the per-element costs,
// whatever the spread of suffix lengths.
//
// Panels.  Most of the tests sit at the highest ranks (the highest degrees), where a list N+(u)
// holds several consecutive middle vertices and its suffix would be streamed once for each.
// The top ranks are therefore grouped into panels of kPanel consecutive middle vertices
// P .. P + kPanel - 1: a panel's table M in LDS holds, for every rank w, the kPanel-bit mask
// of the panel vertices whose out-list contains w, and a segment is a pair (u, panel) with
// the mask R(u) of the panel vertices in N+(u).  Its suffix after the first of them is
// streamed once and each element w adds popcount(M[w] & R(u)): every panel vertex v with
// v in N+(u) and w in N+(v) closes one triangle (w > v holds because w is in N+(v)).
//
// Per-vertex counts (T(x) = triangles through x) use sorted lists in LDS instead of bitmaps
// so that a hit's position indexes an LDS counter: T(w) for the third vertex is flushed once
// per item, T(u) once per in-edge, T(v) once per item and wave.
#include "internal.h"

namespace tc {

constexpr uint32_t kPiece = 16;
// pieces of the unmasked 16-bit probes (hcol rows carry the padding they need)
constexpr uint32_t kPieceHigh = 32;
constexpr int kThreads = 1024;
constexpr int kWgsPerCu = 1;  // workgroups per CU the LDS footprint allows
constexpr int kWaves = kThreads / kWave;
constexpr uint32_t kLdsWords = 32768;                 // 128 KiB per workgroup
constexpr uint32_t kSliceWords = kLdsWords / kWaves;  // 8 KiB per wave
constexpr uint32_t kWaveBits = kSliceWords * 32 - 32; // wave bitmap: span < 65504
constexpr uint32_t kWaveListPV = kSliceWords / 2;     // per-vertex: list + counters per wave
constexpr uint32_t kBlockBits = kLdsWords * 32 - 32;  // workgroup bitmap: span < 1048544
constexpr uint32_t kBlockList = kLdsWords;            // workgroup sorted list
constexpr uint32_t kBlockListPV = kLdsWords / 2;      // per-vertex: list + counters
constexpr uint32_t kItemEdgesWave = 512;     // default in-edges per wave item
constexpr uint32_t kItemEdgesBlock = 65536;  // default in-edges per workgroup item
constexpr uint32_t kPanel = 32;                       // one bit per panel vertex in a mask
constexpr uint32_t kPanelRanks = kLdsWords - 32;      // mask table: one word per rank
// per-vertex counts over a panel keep a third-vertex counter beside every mask word, so a
// panel's ranks are taken in windows of kPvWindow ranks, each with its table and counters in
// half of the workgroup's LDS (words 0 .. kPvWindow - 1, and word kPvWindow always zero)
constexpr uint32_t kPvPanelWords = kLdsWords / 2;
constexpr uint32_t kPvWindow = kPvPanelWords - 1;
// batched kernel: rows with at most kLightMax forward entries are counted edge by edge; a
// chunk of forward edges plus kLightMax entries on either side must fit one wave's slice
constexpr uint32_t kLightMax = 256;
constexpr uint32_t kLightChunkMax = kSliceWords - 2 * kLightMax;
// light segments' pieces: their lists are short (a few elements), so shorter pieces waste
// fewer lookups on masked positions
constexpr uint32_t kLightPiece = 8;

// ------------------------------------------------------------------ membership probes

// N+(v) as a bitmap over ranks [lo, lo + span].  Bit span + 1 is always zero and lies inside
// the LDS region (spans are kept below the region's bits minus 32), so an id outside the span
// is clamped onto it instead of branching: every lookup is one unconditional LDS read.
struct BitmapProbe {
    const uint32_t *bm;
    uint32_t lo, span;
    static constexpr bool kBranchFree = true;
    __device__ __forceinline__ uint32_t bit(uint32_t w) const {
        const uint32_t o = min(w - lo, span + 1u);
        return __builtin_amdgcn_ubfe(bm[__builtin_amdgcn_ubfe(o, 5u, 27u)], o, 1u);
    }
    __device__ __forceinline__ bool operator()(uint32_t w, uint32_t &) const { return bit(w); }
    static constexpr bool kMasked = false;
    static constexpr bool kList = false;
    // totals streamer (run_batch_t): both parts of a segment, positions tested
    static constexpr bool kLow = true;
    static constexpr bool kMaskHigh = true;
    static constexpr bool kPanel = false;
};

// Panel table M over ranks [lo, lo + span]: word w - lo holds the mask of the panel vertices
// whose out-list contains w.  Word span + 1 is always zero, so out-of-range ids clamp onto it.
struct PanelProbe {
    const uint32_t *m;
    uint32_t lo, span;
    static constexpr bool kBranchFree = true;
    static constexpr bool kMasked = true;
    static constexpr bool kList = false;
    __device__ __forceinline__ uint32_t count(uint32_t w, uint32_t r) const {
        return __popc(m[min(w - lo, span + 1u)] & r);
    }
};

// lower_bound with a lane-independent trip count (d is uniform)
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *list, uint32_t d,
                                                    uint32_t w) {
    uint32_t base = 0, len = d;
    while (len > 1) {
        uint32_t half = len >> 1;
        base = (list[base + half - 1] < w) ? base + half : base;
        len -= half;
    }
    return base + ((len == 1 && list[base] < w) ? 1u : 0u);
}

struct ListProbe {  // sorted list in LDS or in global memory (d >= 1)
    const uint32_t *list;
    uint32_t d;
    static constexpr bool kBranchFree = false;
    static constexpr bool kMasked = false;
    static constexpr bool kList = true;
    static constexpr bool kLow = true;
    static constexpr bool kMaskHigh = true;
    static constexpr bool kPanel = false;
    __device__ __forceinline__ bool operator()(uint32_t w, uint32_t &pos) const {
        pos = lower_bound_u32(list, d, w);
        return pos < d && list[pos] == w;
    }
};

// ------------------------------------------------------------------ per-batch streaming

struct WaveScratch {  // tag: the segment's owner (per-vertex counts) or its panel mask;
                     // the batched kernel's light segments keep their N+(u) in tag and aux
    uint32_t off[kWave], beg[kWave], first[kWave], end[kWave], cnt[kWave], tag[kWave],
        aux[kWave];
};

// Segment sources: segment e is a range [b, en) of `col` streamed through the staged list,
// and `owner` is the vertex credited with the segment's hits in per-vertex counts.  rec(e)
// fetches everything a streamer needs of segment e at once.
struct SegRec {
    uint32_t b, en;  // the range of col
    uint32_t y;      // panel mask, or where the entries >= hbase start in col
    uint32_t h;      // where the entries >= hbase start in hcol
    uint32_t owner;
};

// In-edge records: the in-edge u -> v at CSR position e (list entry j holds cbeg[j] = e + 1)
// has its record at er[e] = (end of u's row, panel mask of u's run in a panel list or else
// where the suffix's entries >= hbase start in col, where they start in hcol, u); reading
// it is one random 16-byte gather per segment.
struct InEdgeSegs {  // middle-vertex kernel: suffix of N+(u) after v, owner u
    const uint32_t *cbeg;
    const uint4 *er;
    __device__ __forceinline__ SegRec rec_from(uint32_t b) const {
        const uint4 x = er[b - 1];
        return SegRec{b, x.x, x.y, x.z, x.w};
    }
    __device__ __forceinline__ SegRec rec(uint32_t e) const { return rec_from(cbeg[e]); }
};

// Panel segment (u, panel): the suffix of N+(u) after u's first panel vertex, tagged with the
// mask R(u) of u's panel vertices; with a high region every entry after a panel vertex is a
// rank >= p0 >= hbase.
struct PanelSegs {
    const uint32_t *cbeg;
    const uint4 *er;
    __device__ __forceinline__ SegRec rec_from(uint32_t b) const {
        const uint4 x = er[b - 1];
        return SegRec{b, x.x, x.y, x.z, x.w};
    }
    __device__ __forceinline__ SegRec rec(uint32_t e) const { return rec_from(cbeg[e]); }
};

struct OutEdgeSegs {  // u-centric kernel: the whole list N+(v) of out-neighbour v, owner v
    const uint32_t *row_ptr, *col;
    __device__ __forceinline__ SegRec rec(uint32_t e) const {
        const uint32_t v = col[e];
        return SegRec{row_ptr[v], row_ptr[v + 1], 0u, 0u, v};
    }
};

// The calling wave streams segments [eb, min(eb + 64, e1)) of the current item through the
// probe and returns this lane's hits.  PV: per-vertex accumulation -- LDS counters `tcnt`
// indexed by the probe's position when `tcnt` is non-null, global atomics on `tpv` otherwise;
// every segment's hits go to its owner.
template <bool PV, class Probe, class Segs>
__device__ __forceinline__ uint32_t run_batch(uint32_t eb, uint32_t e1, const Segs &segs,
                                              const uint32_t *__restrict__ col, const Probe &probe,
                                              WaveScratch &ws, uint32_t *tcnt,
                                              unsigned long long *__restrict__ tpv) {
    const uint32_t lane = lane_id();
    const uint32_t e = eb + lane;
    const bool valid = e < e1;
    SegRec r{0u, 0u, 0u, 0u, 0u};
    if (valid) r = segs.rec(e);
    const uint32_t b = r.b, en = r.en;
    // pieces are kPiece-element windows starting at 4-element (16-byte) boundaries, so a lane
    // reads its piece with kPiece / 4 aligned 16-byte loads; elements outside [b, en) are masked
    const uint32_t a0 = b & ~3u;
    const uint32_t p = (valid && en > b) ? (en - a0 + kPiece - 1) / kPiece : 0u;
    const uint32_t incl = wave_incl_scan(p);
    const uint32_t Q = wave_bcast(incl, kWave - 1);
    ws.off[lane] = incl - p;
    ws.beg[lane] = a0;
    ws.first[lane] = b;
    ws.end[lane] = en;
    if (PV) {
        ws.cnt[lane] = 0;
        ws.tag[lane] = r.owner;
    } else if (Probe::kMasked) {
        ws.tag[lane] = r.y;
    }
    wave_lds_sync();
    uint32_t hits_total = 0;
    for (uint32_t q0 = 0; q0 < Q; q0 += kWave) {
        const uint32_t q = q0 + lane;
        if (q < Q) {
            // owner: the last in-edge whose first piece is <= q (zero-piece lanes share the
            // offset of the next lane and lose to it)
            uint32_t k = 0;
#pragma unroll
            for (uint32_t step = 32; step; step >>= 1)
                if (ws.off[k + step] <= q) k += step;
            const uint32_t start = ws.beg[k] + (q - ws.off[k]) * kPiece;
            const uint32_t first = ws.first[k], stop = ws.end[k];
            const uint4 *p4 = reinterpret_cast<const uint4 *>(col + start);
            uint32_t wv[kPiece];
#pragma unroll
            for (uint32_t j = 0; j < kPiece / 4; ++j) {
                const uint4 x = p4[j];
                wv[4 * j] = x.x;
                wv[4 * j + 1] = x.y;
                wv[4 * j + 2] = x.z;
                wv[4 * j + 3] = x.w;
            }
            uint32_t hits = 0;
            // element i of the piece belongs to the suffix iff start + i - first < stop - first
            const uint32_t rel0 = start - first, len = stop - first;
            if constexpr (!PV && Probe::kMasked) {
                // hits of element i: panel vertices of the owner whose lists hold it
                const uint32_t r = ws.tag[k];
                const uint32_t lo_i = first > start ? first - start : 0u;
                const uint32_t hi_i = min(stop - start, kPiece);
#pragma unroll
                for (uint32_t i = 0; i < kPiece; ++i) {
                    const uint32_t c = probe.count(wv[i], r);
                    hits += (i >= lo_i && i < hi_i) ? c : 0u;
                }
            } else if constexpr (Probe::kList) {
                // the piece's 16 lookups as binary searches in lockstep (the list length is
                // uniform), so that every step issues independent reads; position pos is the
                // first entry >= w, and w is in the list iff that entry equals w.  Per-vertex
                // counts credit the third vertex of every hit: an LDS counter by position, or
                // a global counter when the list is not in LDS.
                uint32_t base[kPiece];
#pragma unroll
                for (uint32_t i = 0; i < kPiece; ++i) base[i] = 0;
                for (uint32_t n_left = probe.d; n_left > 1;) {
                    const uint32_t half = n_left >> 1;
#pragma unroll
                    for (uint32_t i = 0; i < kPiece; ++i)
                        base[i] = probe.list[base[i] + half - 1] < wv[i] ? base[i] + half : base[i];
                    n_left -= half;
                }
                uint32_t packed = 0;
#pragma unroll
                for (uint32_t i = 0; i < kPiece; ++i) {
                    base[i] += probe.list[base[i]] < wv[i] ? 1u : 0u;
                    packed |= (probe.list[min(base[i], probe.d - 1u)] == wv[i] ? 1u : 0u) << i;
                }
                const uint32_t lo_i = first > start ? first - start : 0u;
                const uint32_t hi_i = min(stop - start, kPiece);
                const uint32_t hmask = hi_i >= 32u ? ~0u : ((1u << hi_i) - 1u);
                packed &= hmask & ~((1u << lo_i) - 1u);
                hits = __popc(packed);
                if (PV && packed) {
#pragma unroll
                    for (uint32_t i = 0; i < kPiece; ++i) {
                        if ((packed >> i) & 1u) {
                            if (tcnt) atomicAdd(&tcnt[base[i]], 1u);
                            else atomicAdd(&tpv[wv[i]], 1ull);
                        }
                    }
                }
            } else if constexpr (!PV && Probe::kBranchFree) {
                // the piece's valid elements are the contiguous range [lo_i, hi_i) of positions
                uint32_t packed = 0;
#pragma unroll
                for (uint32_t i = 0; i < kPiece; ++i) packed |= probe.bit(wv[i]) << i;
                const uint32_t lo_i = first > start ? first - start : 0u;
                const uint32_t hi_i = min(stop - start, kPiece);
                const uint32_t hmask = hi_i >= 32u ? ~0u : ((1u << hi_i) - 1u);
                const uint32_t mask = hmask & ~((1u << lo_i) - 1u);
                hits = __popc(packed & mask);
            } else {
#pragma unroll
                for (uint32_t i = 0; i < kPiece; ++i) {
                    if (rel0 + i < len) {
                        const uint32_t w = wv[i];
                        uint32_t pos;
                        if (probe(w, pos)) {
                            ++hits;
                            if (PV) {
                                if (tcnt) atomicAdd(&tcnt[pos], 1u);
                                else atomicAdd(&tpv[w], 1ull);
                            }
                        }
                    }
                }
            }
            hits_total += hits;
            if (PV && hits) atomicAdd(&ws.cnt[k], hits);
        }
    }
    wave_lds_sync();
    if (PV) {
        if (ws.cnt[lane]) atomicAdd(&tpv[ws.tag[lane]], (unsigned long long)ws.cnt[lane]);
        wave_lds_sync();
    }
    return hits_total;
}

// LDS access by byte address (32-bit LDS pointers)
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ uint32_t lds_word(uint32_t addr) {
    return *(const lds_u32 *)(uintptr_t)addr;
}
__device__ __forceinline__ uint32_t lds_addr(const uint32_t *p) {
    return (uint32_t)(uintptr_t)(const lds_u32 *)p;
}

// ------------------------------------------------------------------ totals streaming
//
// Total counts stream a segment in two parts: its entries below rank hbase from col (32-bit
// pieces of kPiece entries from 4-aligned positions), and its entries >= hbase from hcol as
// 16-bit offsets from hbase (pieces of kPiece, or kPieceHigh for unmasked probes, entries from
// 8-aligned positions).  In hcol every row's part starts at an 8-aligned position and is
// followed by zeros up to the next multiple of 8 and kPieceHigh - 8 more, so a piece never
// reaches another row.
//
// Masked probes test only the entries inside the segment.  Unmasked probes test every entry
// of a piece: the entries of u's row before the segment are ranks up to the middle vertex
// (or up to u's first panel vertex), and the padding zeros stand for rank hbase; the probes
// below are built so that none of these can hit.

// Bitmap over the whole high region: bit x for rank hbase + x (x < 2^16, the wave's LDS
// slice).  For middle vertices v >= hbase only: N+(v) lies in (v, n), so neither a rank <= v
// nor hbase is ever set.
struct HighBitmapProbe {
    uint32_t base;  // LDS byte address of the slice: a multiple of its 8 KiB
    static constexpr bool kLow = false;
    static constexpr bool kMaskHigh = false;
    static constexpr bool kPanel = false;
    // bits of the two entries of a packed pair of 16-bit entries: word x >> 5 is at byte
    // ((x >> 3) & 0x1ffc) | base, and the bit offset of v_bfe is the low 5 bits of its
    // operand, so the low entry needs no extraction
    __device__ __forceinline__ uint32_t bit_lo(uint32_t pr) const {
        return __builtin_amdgcn_ubfe(lds_word(((pr >> 3) & 0x1ffcu) | base), pr, 1u);
    }
    __device__ __forceinline__ uint32_t bit_hi(uint32_t pr) const {
        return __builtin_amdgcn_ubfe(lds_word(((pr >> 19) & 0x1ffcu) | base), pr >> 16, 1u);
    }
    __device__ __forceinline__ uint32_t bits2(uint32_t pr) const { return bit_lo(pr) + bit_hi(pr); }
};

// The entries >= hbase of N+(v) for a middle vertex below hbase (a rank span too wide for a
// bitmap) in a high-region bitmap (as HighBitmapProbe), for the 16-bit pieces only.  Masked:
// such a suffix's high part starts at its row's part of hcol, but the padding zeros (rank
// hbase) may be in N+(v).
struct HighMaskedProbe {
    HighBitmapProbe hi;
    static constexpr bool kLow = true;  // the segments have 32-bit parts (not streamed here)
    static constexpr bool kMaskHigh = true;
    static constexpr bool kPanel = false;
};

// Panel table over ranks [P, n) (as PanelProbe) read with 16-bit entries: rank hbase + x is
// word x - c (c = P - hbase), ranks below P saturate onto word 0 (rank P, in no out-list of
// the panel), and no entry exceeds word n - 1 - P.  An entry of u's row up to u's first panel
// vertex P + j only matches panel vertices below P + j, none of which is in u's mask.
struct PanelHighProbe {
    const uint32_t *m;
    uint32_t c;
    static constexpr bool kLow = false;
    static constexpr bool kMaskHigh = false;
    static constexpr bool kPanel = true;
    __device__ __forceinline__ uint32_t count(uint32_t x, uint32_t r) const {
        const uint32_t o = x > c ? x - c : 0u;
        return __popc(m[o] & r);
    }
};

// bit i set when position start + i of a piece lies in [first, stop) (start < stop)
__device__ __forceinline__ uint32_t piece_mask(uint32_t start, uint32_t first, uint32_t stop) {
    const uint32_t lo_i = first > start ? first - start : 0u;
    const uint32_t hi_i = min(stop - start, kPiece);
    const uint32_t hmask = hi_i >= 32u ? ~0u : ((1u << hi_i) - 1u);
    return hmask & ~((1u << lo_i) - 1u);
}

// hits of the entries wv[i] at positions start + i that lie in [first, stop)
template <class Probe>
__device__ __forceinline__ uint32_t masked_hits(const Probe &probe, const uint32_t (&wv)[kPiece],
                                                uint32_t start, uint32_t first, uint32_t stop) {
    const uint32_t mask = piece_mask(start, first, stop);
    uint32_t packed = 0;
    if constexpr (Probe::kList) {
        // the piece's lookups as binary searches in lockstep (the list length is uniform)
        uint32_t base[kPiece];
#pragma unroll
        for (uint32_t i = 0; i < kPiece; ++i) base[i] = 0;
        for (uint32_t n_left = probe.d; n_left > 1;) {
            const uint32_t half = n_left >> 1;
#pragma unroll
            for (uint32_t i = 0; i < kPiece; ++i)
                base[i] = probe.list[base[i] + half - 1] < wv[i] ? base[i] + half : base[i];
            n_left -= half;
        }
#pragma unroll
        for (uint32_t i = 0; i < kPiece; ++i) {
            base[i] += probe.list[base[i]] < wv[i] ? 1u : 0u;
            packed |= (probe.list[min(base[i], probe.d - 1u)] == wv[i] ? 1u : 0u) << i;
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kPiece; ++i) packed |= probe.bit(wv[i]) << i;
    }
    return __popc(packed & mask);
}

// Piece evaluations of the totals streamer.  Masked probes: a 32-bit piece (entries wv) and a
// 16-bit piece (packed pairs pr of offsets from hbase), positions start + i, counted inside
// [first, stop).  Unmasked probes: a 16-bit piece of kPieceHigh entries, all counted.
template <class Probe>
__device__ __forceinline__ uint32_t low_hits(const Probe &probe, const uint32_t (&wv)[kPiece],
                                             uint32_t start, uint32_t first, uint32_t stop) {
    return masked_hits(probe, wv, start, first, stop);
}
template <class Probe>
__device__ __forceinline__ uint32_t high_hits(const Probe &probe,
                                              const uint32_t (&pr)[kPiece / 2], uint32_t hbase,
                                              uint32_t start, uint32_t first, uint32_t stop) {
    uint32_t wv[kPiece];
#pragma unroll
    for (uint32_t i = 0; i < kPiece / 2; ++i) {
        wv[2 * i] = hbase + (pr[i] & 0xFFFFu);
        wv[2 * i + 1] = hbase + (pr[i] >> 16);
    }
    return masked_hits(probe, wv, start, first, stop);
}
__device__ __forceinline__ uint32_t high_hits(const HighMaskedProbe &probe,
                                              const uint32_t (&pr)[kPiece / 2], uint32_t,
                                              uint32_t start, uint32_t first, uint32_t stop) {
    uint32_t packed = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPiece / 2; ++i)
        packed |= (probe.hi.bit_lo(pr[i]) << (2 * i)) | (probe.hi.bit_hi(pr[i]) << (2 * i + 1));
    return __popc(packed & piece_mask(start, first, stop));
}
__device__ __forceinline__ uint32_t high_hits_u(const HighBitmapProbe &probe,
                                                const uint32_t (&pr)[kPieceHigh / 2], uint32_t) {
    uint32_t hits = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPieceHigh / 2; ++i) hits += probe.bits2(pr[i]);
    return hits;
}
__device__ __forceinline__ uint32_t high_hits_u(const PanelHighProbe &probe,
                                                const uint32_t (&pr)[kPieceHigh / 2], uint32_t r) {
    uint32_t hits = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPieceHigh / 2; ++i)
        hits += probe.count(pr[i] & 0xFFFFu, r) + probe.count(pr[i] >> 16, r);
    return hits;
}

// Owner of piece q0 + lane in a round of a piece sequence: every segment whose first piece
// (my_off, of this lane's segment, which has p pieces) falls in the round marks that lane in
// the wave's table (tagged with the round number, so older marks read as none), and the
// running maximum over the lanes carries the last mark forward; lanes before the round's
// first mark belong to carry, the previous round's last segment (plus one).  Returns the
// owner plus one (all lanes active).
__device__ __forceinline__ uint32_t round_owner(uint32_t *mark, uint32_t my_off, uint32_t p,
                                                uint32_t q0, uint32_t round, uint32_t &carry) {
    const uint32_t lane = lane_id();
    const uint32_t pos = my_off - q0;
    if (p && pos < kWave) mark[pos] = (round << 7) | (lane + 1u);
    wave_lds_sync();
    const uint32_t mv = mark[lane];
    const uint32_t m1 = wave_incl_max((mv >> 7) == round ? (mv & 127u) : 0u);
    const uint32_t owner1 = m1 ? m1 : carry;
    carry = (uint32_t)__builtin_amdgcn_readlane((int)owner1, kWave - 1);
    return owner1;
}

// The calling wave streams one batch of up to 64 segments (r: this lane's record, all zero
// for no segment) through the probe for total counts and returns this lane's hits.  A segment
// is the col range [b, en) whose entries from hb on are ranks >= hbase, found in hcol from
// position h; probes without kLow are only given segments with hb == b.  The batch's 32-bit
// pieces (of [b, hb)) run first, then its 16-bit pieces, each as its own sequence of rounds,
// so that a round holds pieces of one kind.
template <class Probe, int kParts = 3>
__device__ __forceinline__ uint32_t run_batch_t(const SegRec &r,
                                                const uint32_t *__restrict__ col,
                                                const uint16_t *__restrict__ hcol,
                                                uint32_t hbase, const Probe &probe,
                                                WaveScratch &ws) {
    const uint32_t lane = lane_id();
    // panel segments are high throughout; other segments switch to high entries at r.y
    const uint32_t b = r.b, en = r.en, h = r.h;
    const uint32_t hb = Probe::kPanel ? b : r.y;
    const uint32_t a0 = b & ~3u;
    const uint32_t pl = (Probe::kLow && hb > b) ? (hb - a0 + kPiece - 1) / kPiece : 0u;
    // unmasked probes read longer pieces (the per-piece search and setup is their overhead)
    constexpr uint32_t kPh = Probe::kMaskHigh ? kPiece : kPieceHigh;
    const uint32_t hl = en - hb;
    const uint32_t ph = hl ? (h + hl - (h & ~7u) + kPh - 1) / kPh : 0u;
    static_assert(kParts >= 1 && kParts <= 3, "kParts: 1 the 32-bit pieces, 2 the 16-bit ones");
    ws.off[lane] = 0u;  // the rounds' marker table
    ws.aux[lane] = h;
    if constexpr (Probe::kLow) {
        ws.beg[lane] = a0;
        ws.first[lane] = b;
        ws.end[lane] = hb;
    }
    if constexpr (Probe::kMaskHigh) ws.tag[lane] = h + hl;
    if constexpr (Probe::kPanel) ws.tag[lane] = r.y;
    uint32_t hits_total = 0, carry = 0, round = 0;
    if constexpr (Probe::kLow && (kParts & 1)) {  // the 32-bit pieces
        const uint32_t incl = wave_incl_scan(pl);
        const uint32_t Q = wave_bcast(incl, kWave - 1);
        const uint32_t my_off = incl - pl;
        wave_lds_sync();
        for (uint32_t q0 = 0; q0 < Q; q0 += kWave) {
            const uint32_t k = round_owner(ws.off, my_off, pl, q0, ++round, carry) - 1u;
            const uint32_t off_k = wave_bcast_from(my_off, k);
            const uint32_t q = q0 + lane;
            if (q < Q) {
                const uint32_t start = ws.beg[k] + (q - off_k) * kPiece;
                const uint4 *p4 = reinterpret_cast<const uint4 *>(col + start);
                uint32_t wv[kPiece];
#pragma unroll
                for (uint32_t i = 0; i < kPiece / 4; ++i) {
                    const uint4 x = p4[i];
                    wv[4 * i] = x.x;
                    wv[4 * i + 1] = x.y;
                    wv[4 * i + 2] = x.z;
                    wv[4 * i + 3] = x.w;
                }
                hits_total += low_hits(probe, wv, start, ws.first[k], ws.end[k]);
            }
        }
        carry = 0;
    }
    if constexpr ((kParts & 2) != 0) {  // the 16-bit pieces
        const uint32_t incl = wave_incl_scan(ph);
        const uint32_t Q = wave_bcast(incl, kWave - 1);
        const uint32_t my_off = incl - ph;
        wave_lds_sync();
        for (uint32_t q0 = 0; q0 < Q; q0 += kWave) {
            const uint32_t k = round_owner(ws.off, my_off, ph, q0, ++round, carry) - 1u;
            const uint32_t off_k = wave_bcast_from(my_off, k);
            const uint32_t q = q0 + lane;
            if (q < Q) {
                const uint32_t hs = ws.aux[k];
                const uint32_t start = (hs & ~7u) + (q - off_k) * kPh;
                const uint4 *p4 = reinterpret_cast<const uint4 *>(hcol + start);
                uint32_t pr[kPh / 2];
#pragma unroll
                for (uint32_t i = 0; i < kPh / 8; ++i) {
                    const uint4 x = p4[i];
                    pr[4 * i] = x.x;
                    pr[4 * i + 1] = x.y;
                    pr[4 * i + 2] = x.z;
                    pr[4 * i + 3] = x.w;
                }
                if constexpr (Probe::kMaskHigh)
                    hits_total += high_hits(probe, pr, hbase, start, hs, ws.tag[k]);
                else
                    hits_total += high_hits_u(probe, pr, ws.tag[k]);
            }
        }
    }
    wave_lds_sync();
    return hits_total;
}

// The calling wave streams the segments first, first + step, ... (its batches of 64: lanes
// take consecutive segments) of an item ending at e1 for total counts.  (Fetching the
// records a batch or two ahead measured no faster: the gathers' lines, not their latency,
// are the cost.)
template <int kParts = 3, class Probe, class Segs>
__device__ __forceinline__ uint32_t stream_t(uint32_t first, uint32_t e1, uint32_t step,
                                             const Segs &segs,
                                             const uint32_t *__restrict__ col,
                                             const uint16_t *__restrict__ hcol, uint32_t hbase,
                                             const Probe &probe, WaveScratch &ws) {
    const uint32_t lane = lane_id();
    uint32_t hits = 0;
    for (uint32_t eb = first; eb < e1; eb += step) {
        const SegRec r = eb + lane < e1 ? segs.rec(eb + lane) : SegRec{0u, 0u, 0u, 0u, 0u};
        hits += run_batch_t<Probe, kParts>(r, col, hcol, hbase, probe, ws);
    }
    return hits;
}

// Wave-private claims on a shared item counter: kClaim consecutive positions per atomic, so
// that the counter (one address that every XCD's waves update) sees few operations when items
// are small.  Items are sorted heaviest first, so a claim holds items of similar size.
template <uint32_t kClaim>
struct WaveQueue {
    uint32_t next = 0, end = 0;
    __device__ __forceinline__ bool pop(uint32_t *counter, uint32_t n_items, uint32_t &q) {
        if (next == end) {
            uint32_t c = 0;
            if (lane_id() == 0) c = atomicAdd(counter, kClaim);
            c = wave_bcast(c, 0);
            if (c >= n_items) return false;
            next = c;
            end = min(c + kClaim, n_items);
        }
        q = next++;
        return true;
    }
};
constexpr uint32_t kClaimWave = 8;     // middle-vertex kernel, wave items
constexpr uint32_t kClaimBatched = 64;  // batched kernel, heavy items
constexpr uint32_t kClaimLight = 4;     // batched kernel, light chunks

struct ItemRange {
    uint32_t v, e0, e1, r0, d;
};

// Item q of a queue covers in-edges [e0, e1) of list c = row block * (n + 1) + v.
__device__ __forceinline__ ItemRange item_range(uint32_t q, uint32_t kitem, uint32_t n1,
                                                const uint32_t *__restrict__ item_c,
                                                const uint32_t *__restrict__ item_off,
                                                const uint32_t *__restrict__ cptr,
                                                const uint32_t *__restrict__ row_ptr) {
    ItemRange it;
    const uint32_t c = item_c[q];
    it.v = c % n1;
    const uint32_t chunk = q - item_off[c];
    it.e0 = cptr[c] + chunk * kitem;
    it.e1 = min(it.e0 + kitem, cptr[c + 1]);
    it.r0 = row_ptr[it.v];
    it.d = row_ptr[it.v + 1] - it.r0;
    return it;
}

// ------------------------------------------------------------------ per-vertex panels
//
// Per-vertex counts over a panel P .. P+31 in one pass, with the panel table of the totals.
// Element w of segment (u, panel) closes one triangle u -> P+j -> w for every bit j of
// c = M[w] & R(u); each is credited three times:
//   the first vertex u: popcount(c), summed per segment (one atomic per segment);
//   the third vertex w: popcount(c) into an LDS counter beside M[w] (flushed once per item);
//   the middle vertex P+j: bit j of c, summed per lane in bit-sliced counters (bit j of
//   plane k is bit k of the count of panel vertex j), with a carry-save adder tree over the
//   16 elements of a piece, and flushed once per item.

// carry-save adder: (h, l) with 2h + l = l + b + c bitwise
__device__ __forceinline__ void csa(uint32_t &h, uint32_t &l, uint32_t b, uint32_t c) {
    const uint32_t u = l ^ b;
    h = (l & b) | (u & c);
    l = u ^ c;
}

// 32 counters (one per panel vertex) of one lane in bit slices: the count of vertex j is
// ones_j + 2 twos_j + 4 fours_j + 8 eights_j + 16 * (sum_k hi[k]_j 2^k)
struct MidCounters {
    // counts up to 4095 per lane between flushes: a flush every 255 pieces costs a few percent
    // of the pieces' work, and the largest panels reach it (the flush path runs in practice)
    static constexpr int kHi = 8;
    uint32_t ones, twos, fours, eights, hi[kHi];
    __device__ __forceinline__ void clear() {
        ones = twos = fours = eights = 0;
#pragma unroll
        for (int k = 0; k < kHi; ++k) hi[k] = 0;
    }
    // adds the 16 masks d[0..15] (Harley-Seal tree)
    __device__ __forceinline__ void add16(const uint32_t (&d)[16]) {
        uint32_t tA, tB, fA, fB, eA, eB, sx;
        csa(tA, ones, d[0], d[1]);
        csa(tB, ones, d[2], d[3]);
        csa(fA, twos, tA, tB);
        csa(tA, ones, d[4], d[5]);
        csa(tB, ones, d[6], d[7]);
        csa(fB, twos, tA, tB);
        csa(eA, fours, fA, fB);
        csa(tA, ones, d[8], d[9]);
        csa(tB, ones, d[10], d[11]);
        csa(fA, twos, tA, tB);
        csa(tA, ones, d[12], d[13]);
        csa(tB, ones, d[14], d[15]);
        csa(fB, twos, tA, tB);
        csa(eB, fours, fA, fB);
        csa(sx, eights, eA, eB);
        uint32_t carry = sx;
#pragma unroll
        for (int k = 0; k < kHi; ++k) {
            const uint32_t t = hi[k] & carry;
            hi[k] ^= carry;
            carry = t;
        }
    }
    __device__ __forceinline__ uint32_t count(uint32_t j) const {
        uint32_t h = 0;
#pragma unroll
        for (int k = kHi - 1; k >= 0; --k) h = (h << 1) | ((hi[k] >> j) & 1u);
        return ((ones >> j) & 1u) + 2u * ((twos >> j) & 1u) + 4u * ((fours >> j) & 1u) +
               8u * ((eights >> j) & 1u) + 16u * h;
    }
    // wave sums into the workgroup's 32 middle-vertex counters, then restart
    __device__ __forceinline__ void flush(unsigned long long *mid) {
#pragma unroll 1
        for (uint32_t j = 0; j < kPanel; ++j) {
            const uint64_t s = wave_sum_u64(count(j));
            if (lane_id() == 0 && s) atomicAdd(&mid[j], (unsigned long long)s);
        }
        clear();
    }
};
// pieces one lane may add between flushes (16 per piece per counter, kHi + 4 bits)
constexpr uint32_t kMidPieces = (1u << (MidCounters::kHi + 4)) / kPiece - 1;

// The calling wave streams panel segments [eb, min(eb + 64, e1)) of the current item through
// the mask table m (and third-vertex counters cnt3 at the same offsets) and returns this
// lane's hits; `pieces` is the wave's bound on the pieces any lane added to mc since its last
// flush.
__device__ __forceinline__ uint32_t run_panel_pv(uint32_t eb, uint32_t e1,
                                                 const PanelSegs &segs,
                                                 const uint32_t *__restrict__ col,
                                                 const uint32_t *m, uint32_t *cnt3, uint32_t lo,
                                                 uint32_t span, WaveScratch &ws,
                                                 MidCounters &mc, uint32_t &pieces,
                                                 unsigned long long *mid,
                                                 unsigned long long *__restrict__ tpv) {
    const uint32_t lane = lane_id();
    const uint32_t e = eb + lane;
    const bool valid = e < e1;
    SegRec r{0u, 0u, 0u, 0u, 0u};
    if (valid) r = segs.rec(e);
    const uint32_t b = r.b, en = r.en;
    const uint32_t a0 = b & ~3u;
    const uint32_t p = (valid && en > b) ? (en - a0 + kPiece - 1) / kPiece : 0u;
    const uint32_t incl = wave_incl_scan(p);
    const uint32_t Q = wave_bcast(incl, kWave - 1);
    ws.off[lane] = incl - p;
    ws.beg[lane] = a0;
    ws.first[lane] = b;
    ws.end[lane] = en;
    ws.cnt[lane] = 0;
    ws.tag[lane] = r.y;      // the panel mask R(u)
    ws.aux[lane] = r.owner;  // u
    wave_lds_sync();
    const uint32_t per_lane = (Q + kWave - 1) / kWave;
    if (pieces + per_lane > kMidPieces) {
        mc.flush(mid);
        pieces = 0;
    }
    pieces += per_lane;
    uint32_t hits_total = 0;
    for (uint32_t q0 = 0; q0 < Q; q0 += kWave) {
        const uint32_t q = q0 + lane;
        uint32_t c[kPiece];
#pragma unroll
        for (uint32_t i = 0; i < kPiece; ++i) c[i] = 0;
        if (q < Q) {
            uint32_t k = 0;
#pragma unroll
            for (uint32_t step = 32; step; step >>= 1)
                if (ws.off[k + step] <= q) k += step;
            const uint32_t start = ws.beg[k] + (q - ws.off[k]) * kPiece;
            const uint32_t first = ws.first[k], stop = ws.end[k];
            const uint4 *p4 = reinterpret_cast<const uint4 *>(col + start);
            uint32_t wv[kPiece];
#pragma unroll
            for (uint32_t j = 0; j < kPiece / 4; ++j) {
                const uint4 x = p4[j];
                wv[4 * j] = x.x;
                wv[4 * j + 1] = x.y;
                wv[4 * j + 2] = x.z;
                wv[4 * j + 3] = x.w;
            }
            const uint32_t r = ws.tag[k];
            const uint32_t lo_i = first > start ? first - start : 0u;
            const uint32_t hi_i = min(stop - start, kPiece);
            uint32_t hits = 0;
#pragma unroll
            for (uint32_t i = 0; i < kPiece; ++i) {
                // an id outside the table clamps onto word span + 1, which is always zero
                const uint32_t o = min(wv[i] - lo, span + 1u);
                const uint32_t ci = (i >= lo_i && i < hi_i) ? (m[o] & r) : 0u;
                c[i] = ci;
                const uint32_t h = __popc(ci);
                hits += h;
                if (h) atomicAdd(&cnt3[o], h);
            }
            hits_total += hits;
            if (hits) atomicAdd(&ws.cnt[k], hits);
        }
        mc.add16(c);
    }
    wave_lds_sync();
    if (ws.cnt[lane]) atomicAdd(&tpv[ws.aux[lane]], (unsigned long long)ws.cnt[lane]);
    wave_lds_sync();
    return hits_total;
}

// first position in hcol[b, e) (ascending) whose entry is >= x
__device__ __forceinline__ uint32_t hcol_lower_bound(const uint16_t *__restrict__ hcol,
                                                     uint32_t b, uint32_t e, uint32_t x) {
    while (b < e) {
        const uint32_t mid = b + ((e - b) >> 1);
        if (hcol[mid] < x) b = mid + 1;
        else e = mid;
    }
    return b;
}

// The same for panels in the high region: every suffix entry is read from hcol as a 16-bit
// offset from hbase, in unmasked pieces of kPieceHigh entries (entries of u's row up to its
// first panel vertex only match panel vertices below it, none of which is in its mask, and
// padding zeros, rank hbase, lie below the window; entries outside the window clamp onto the
// zero word), with the owners found as in the totals streamer.  The window's table covers
// offsets [c, c + wn) from hbase; with cut_lo / cut_hi the segment's entries below / above
// the window are found by a binary search and not streamed.
__device__ __forceinline__ uint32_t run_panel_pv_high(const SegRec &r,
                                                      const uint16_t *__restrict__ hcol,
                                                      const uint32_t *m, uint32_t *cnt3,
                                                      uint32_t c, uint32_t wn, bool cut_lo,
                                                      bool cut_hi, WaveScratch &ws,
                                                      MidCounters &mc, uint32_t &pieces,
                                                      unsigned long long *mid,
                                                      unsigned long long *__restrict__ tpv) {
    const uint32_t lane = lane_id();
    uint32_t h0 = r.h, h1 = r.h + (r.en - r.b);
    if (h1 > h0 && cut_lo) h0 = hcol_lower_bound(hcol, h0, h1, c);
    if (h1 > h0 && cut_hi) h1 = hcol_lower_bound(hcol, h0, h1, c + wn);
    const uint32_t hl = h1 > h0 ? h1 - h0 : 0u, h = h0;
    const uint32_t ph = hl ? (h + hl - (h & ~7u) + kPieceHigh - 1) / kPieceHigh : 0u;
    ws.off[lane] = 0u;  // the rounds' marker table
    ws.aux[lane] = h;
    ws.tag[lane] = r.y;      // the panel mask R(u)
    ws.beg[lane] = r.owner;  // u
    ws.cnt[lane] = 0u;
    const uint32_t incl = wave_incl_scan(ph);
    const uint32_t Q = wave_bcast(incl, kWave - 1);
    const uint32_t my_off = incl - ph;
    wave_lds_sync();
    // a piece adds kPieceHigh / kPiece groups of kPiece masks to the middle-vertex counters
    const uint32_t per_lane = (Q + kWave - 1) / kWave * (kPieceHigh / kPiece);
    if (pieces + per_lane > kMidPieces) {
        mc.flush(mid);
        pieces = 0;
    }
    pieces += per_lane;
    uint32_t hits_total = 0, carry = 0, round = 0;
    for (uint32_t q0 = 0; q0 < Q; q0 += kWave) {
        const uint32_t k = round_owner(ws.off, my_off, ph, q0, ++round, carry) - 1u;
        const uint32_t off_k = wave_bcast_from(my_off, k);
        const uint32_t q = q0 + lane;
        uint32_t cm[kPieceHigh];
#pragma unroll
        for (uint32_t i = 0; i < kPieceHigh; ++i) cm[i] = 0;
        if (q < Q) {
            const uint32_t start = (ws.aux[k] & ~7u) + (q - off_k) * kPieceHigh;
            const uint4 *p4 = reinterpret_cast<const uint4 *>(hcol + start);
            uint32_t pr[kPieceHigh / 2];
#pragma unroll
            for (uint32_t i = 0; i < kPieceHigh / 8; ++i) {
                const uint4 x = p4[i];
                pr[4 * i] = x.x;
                pr[4 * i + 1] = x.y;
                pr[4 * i + 2] = x.z;
                pr[4 * i + 3] = x.w;
            }
            const uint32_t rm = ws.tag[k];
            uint32_t hits = 0;
#pragma unroll
            for (uint32_t i = 0; i < kPieceHigh; ++i) {
                const uint32_t x = (i & 1u) ? (pr[i >> 1] >> 16) : (pr[i >> 1] & 0xFFFFu);
                const uint32_t o = min(x - c, wn);  // outside the window: the zero word
                const uint32_t ci = m[o] & rm;
                cm[i] = ci;
                const uint32_t hh = __popc(ci);
                hits += hh;
                if (hh) atomicAdd(&cnt3[o], hh);
            }
            hits_total += hits;
            if (hits) atomicAdd(&ws.cnt[k], hits);
        }
#pragma unroll
        for (uint32_t g = 0; g < kPieceHigh / kPiece; ++g) {
            uint32_t d[kPiece];
#pragma unroll
            for (uint32_t i = 0; i < kPiece; ++i) d[i] = cm[g * kPiece + i];
            mc.add16(d);
        }
    }
    wave_lds_sync();
    if (ws.cnt[lane]) atomicAdd(&tpv[ws.beg[lane]], (unsigned long long)ws.cnt[lane]);
    wave_lds_sync();
    return hits_total;
}

// Per-vertex counts of the panels: the workgroup items of the panel region, from their own
// queue counter (every other item is left to k_count<true>).  The ranks above P are taken in
// windows of kPvWindow: per window, the table and the third-vertex counters cover its ranks,
// every segment is streamed whole, and entries outside the window clamp onto the zero word
// (one window for panels within kPvWindow ranks of the top, two for the rest of a region of
// up to 32,736 ranks).
__global__ __launch_bounds__(kThreads) void k_count_panel_pv(
    const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ col,
    const uint32_t *__restrict__ cptr, const uint32_t *__restrict__ cbeg,
    const uint4 *__restrict__ er, const uint32_t *__restrict__ item_v_b,
    const uint32_t *__restrict__ item_off_b, const uint32_t *__restrict__ n_items_b_ptr,
    uint32_t *__restrict__ queue_c, unsigned long long *__restrict__ total,
    unsigned long long *__restrict__ tpv, uint32_t n1, uint32_t p0, uint32_t kitem_b,
    const uint16_t *__restrict__ hcol, uint32_t hbase, const int32_t *__restrict__ status) {
    __shared__ uint32_t s_mem[kLdsWords];
    __shared__ WaveScratch s_ws[kWaves];
    __shared__ unsigned long long s_mid[kPanel];
    __shared__ uint32_t s_item;
    if (*status) return;
    const uint32_t t = threadIdx.x, w = t / kWave, lane = lane_id();
    WaveScratch &ws = s_ws[w];
    const PanelSegs psegs{cbeg, er};
    uint32_t *m = s_mem, *cnt3 = s_mem + kPvPanelWords;
    for (uint32_t i = t; i < kLdsWords; i += kThreads) s_mem[i] = 0;
    if (t < kPanel) s_mid[t] = 0;
    uint64_t acc = 0;
    MidCounters mc;
    mc.clear();
    const uint32_t n_items_b = *n_items_b_ptr;
    for (;;) {
        __syncthreads();
        if (t == 0) s_item = atomicAdd(queue_c, 1u);
        __syncthreads();
        uint32_t q = s_item;
        if (q >= n_items_b) break;
        q = n_items_b - 1 - q;
        const ItemRange it = item_range(q, kitem_b, n1, item_v_b, item_off_b, cptr, row_ptr);
        if (it.v < p0) continue;  // left to k_count<true>
        const uint32_t P = it.v, np = min(kPanel, n1 - 1 - P);
        uint32_t cnt = 0, pieces = 0;
        // window of ranks [lo, lo + wn) above P (rank P itself is in no out-list of the panel)
        for (uint32_t lo = P; lo < n1 - 1; lo += kPvWindow) {
            const uint32_t wn = min(kPvWindow, n1 - 1 - lo);
            for (uint32_t j = w; j < np; j += kWaves)
                for (uint32_t i = row_ptr[P + j] + lane; i < row_ptr[P + j + 1]; i += kWave) {
                    const uint32_t o = col[i] - lo;
                    if (o < wn) atomicOr(&m[o], 1u << j);
                }
            __syncthreads();
            if (P >= hbase) {  // the suffixes are in hcol
                for (uint32_t eb = it.e0 + w * kWave; eb < it.e1; eb += kWaves * kWave) {
                    const SegRec r = eb + lane < it.e1 ? psegs.rec(eb + lane)
                                                       : SegRec{0u, 0u, 0u, 0u, 0u};
                    cnt += run_panel_pv_high(r, hcol, m, cnt3, lo - hbase, wn, lo > P,
                                             lo + wn < n1 - 1, ws, mc, pieces, s_mid, tpv);
                }
            } else {
                for (uint32_t eb = it.e0 + w * kWave; eb < it.e1; eb += kWaves * kWave)
                    cnt += run_panel_pv(eb, it.e1, psegs, col, m, cnt3, lo, wn - 1, ws, mc,
                                        pieces, s_mid, tpv);
            }
            __syncthreads();
            for (uint32_t j = w; j < np; j += kWaves)
                for (uint32_t i = row_ptr[P + j] + lane; i < row_ptr[P + j + 1]; i += kWave) {
                    const uint32_t o = col[i] - lo;
                    if (o < wn) m[o] = 0;
                }
            for (uint32_t i = t; i < wn; i += kThreads) {
                const uint32_t c3 = cnt3[i];
                if (c3) {
                    atomicAdd(&tpv[lo + i], (unsigned long long)c3);
                    cnt3[i] = 0;
                }
            }
            __syncthreads();
        }
        mc.flush(s_mid);
        acc += cnt;
        __syncthreads();
        if (t < np && s_mid[t]) {
            atomicAdd(&tpv[P + t], s_mid[t]);
            s_mid[t] = 0;
        }
    }
    acc = wave_sum_u64(acc);
    if (lane == 0 && acc) atomicAdd(total, (unsigned long long)acc);
}

// ------------------------------------------------------------------ the kernel

template <bool PV>
__global__ __launch_bounds__(kThreads) void k_count(
    const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ col,
    const uint32_t *__restrict__ cptr, const uint32_t *__restrict__ cbeg,
    const uint4 *__restrict__ er, const uint32_t *__restrict__ item_v_a,
    const uint32_t *__restrict__ item_off_a, const uint32_t *__restrict__ n_items_a_ptr,
    const uint32_t *__restrict__ item_v_b, const uint32_t *__restrict__ item_off_b,
    const uint32_t *__restrict__ n_items_b_ptr, uint32_t *__restrict__ queue_a,
    uint32_t *__restrict__ queue_b, unsigned long long *__restrict__ total,
    unsigned long long *__restrict__ tpv, uint32_t n1, uint32_t p0, uint32_t wave_bits,
    uint32_t block_bits, uint32_t block_list, uint32_t kitem_a, uint32_t kitem_b,
    const uint16_t *__restrict__ hcol, const uint32_t *__restrict__ hrow, uint32_t hbase,
    const int32_t *__restrict__ status) {
    // 8 KiB aligned: a wave slice's base has zero low bits, so bitmap addresses OR it in
    __shared__ __attribute__((aligned(kSliceWords * 4))) uint32_t s_mem[kLdsWords];
    __shared__ WaveScratch s_ws[kWaves];
    __shared__ uint32_t s_item;
    if (*status) return;
    const uint32_t t = threadIdx.x, w = t / kWave, lane = lane_id();
    WaveScratch &ws = s_ws[w];
    const InEdgeSegs segs{cbeg, er};
    for (uint32_t i = t; i < kLdsWords; i += kThreads) s_mem[i] = 0;
    uint64_t acc = 0;

    // phase 1: workgroup items
    const uint32_t n_items_b = *n_items_b_ptr;
    for (;;) {
        __syncthreads();
        if (t == 0) s_item = atomicAdd(queue_b, 1u);
        __syncthreads();
        uint32_t q = s_item;
        if (q >= n_items_b) break;
        q = n_items_b - 1 - q;
        const ItemRange it = item_range(q, kitem_b, n1, item_v_b, item_off_b, cptr, row_ptr);
        const uint32_t first = it.e0 + w * kWave, step = kWaves * kWave;
        if (it.v >= p0) {  // a panel of middle vertices P = it.v, ...
            const uint32_t P = it.v, np = min(kPanel, n1 - 1 - P);
            if (!PV) {
                for (uint32_t j = w; j < np; j += kWaves)
                    for (uint32_t i = row_ptr[P + j] + lane; i < row_ptr[P + j + 1]; i += kWave)
                        atomicOr(&s_mem[col[i] - P], 1u << j);
                __syncthreads();
                const PanelSegs psegs{cbeg, er};
                uint32_t cnt = 0;
                if (P >= hbase) {  // the suffixes are in hcol
                    const PanelHighProbe probe{s_mem, P - hbase};
                    cnt += stream_t(first, it.e1, step, psegs, col, hcol, hbase, probe, ws);
                } else {  // no high region: 32-bit entries
                    const PanelProbe probe{s_mem, P, n1 - 2 - P};
                    for (uint32_t eb = first; eb < it.e1; eb += step)
                        cnt += run_batch<false>(eb, it.e1, psegs, col, probe, ws, nullptr, tpv);
                }
                acc += cnt;
                __syncthreads();
                for (uint32_t j = w; j < np; j += kWaves)
                    for (uint32_t i = row_ptr[P + j] + lane; i < row_ptr[P + j + 1]; i += kWave)
                        s_mem[col[i] - P] = 0;
            }
            continue;
        }
        const uint32_t lo = col[it.r0];
        const uint32_t span = col[it.r0 + it.d - 1] - lo;
        // 0 = bitmap, 1 = LDS list, 2 = global list (block_bits <= kBlockBits, block_list <=
        // kBlockList, or kBlockListPV for per-vertex counts)
        const int mode = (!PV && span < block_bits) ? 0 : (it.d <= block_list) ? 1 : 2;
        if (mode == 0) {
            for (uint32_t i = t; i < it.d; i += kThreads) {
                const uint32_t o = col[it.r0 + i] - lo;
                atomicOr(&s_mem[o >> 5], 1u << (o & 31u));
            }
        } else if (mode == 1) {
            for (uint32_t i = t; i < it.d; i += kThreads) s_mem[i] = col[it.r0 + i];
        }
        __syncthreads();
        uint32_t cnt = 0;
        if (mode == 0) {
            const BitmapProbe probe{s_mem, lo, span};
            if constexpr (PV) {
                for (uint32_t eb = first; eb < it.e1; eb += step)
                    cnt += run_batch<true>(eb, it.e1, segs, col, probe, ws, nullptr, tpv);
            } else {
                cnt += stream_t(first, it.e1, step, segs, col, hcol, hbase, probe, ws);
            }
        } else if (mode == 1) {
            const ListProbe probe{s_mem, it.d};
            uint32_t *tc = PV ? s_mem + kBlockListPV : nullptr;
            if constexpr (PV) {
                for (uint32_t eb = first; eb < it.e1; eb += step)
                    cnt += run_batch<true>(eb, it.e1, segs, col, probe, ws, tc, tpv);
            } else {
                cnt += stream_t(first, it.e1, step, segs, col, hcol, hbase, probe, ws);
            }
        } else {
            const ListProbe probe{col + it.r0, it.d};
            if constexpr (PV) {
                for (uint32_t eb = first; eb < it.e1; eb += step)
                    cnt += run_batch<true>(eb, it.e1, segs, col, probe, ws, nullptr, tpv);
            } else {
                cnt += stream_t(first, it.e1, step, segs, col, hcol, hbase, probe, ws);
            }
        }
        if (PV) {
            uint64_t wave_hits = wave_sum_u64(cnt);
            if (lane == 0 && wave_hits) atomicAdd(&tpv[it.v], (unsigned long long)wave_hits);
        }
        acc += cnt;
        __syncthreads();
        if (mode == 0) {
            for (uint32_t i = t; i < it.d; i += kThreads) s_mem[(col[it.r0 + i] - lo) >> 5] = 0;
        } else if (mode == 1) {
            for (uint32_t i = t; i < it.d; i += kThreads) {
                s_mem[i] = 0;
                if (PV) {
                    uint32_t c = s_mem[kBlockListPV + i];
                    if (c) {
                        atomicAdd(&tpv[col[it.r0 + i]], (unsigned long long)c);
                        s_mem[kBlockListPV + i] = 0;
                    }
                }
            }
        }
    }
    __syncthreads();

    // phase 2: wave items, each wave in its own LDS slice
    uint32_t *mem = s_mem + w * kSliceWords;
    // the high-region bitmap ORs the slice's address into its word offsets (requested by the
    // alignment of s_mem; otherwise the span bitmap takes its items)
    const bool slices_aligned = (lds_addr(s_mem) & (kSliceWords * 4 - 1)) == 0;
    const uint32_t n_items_a = *n_items_a_ptr;
    WaveQueue<kClaimWave> wq;
    for (uint32_t q; wq.pop(queue_a, n_items_a, q);) {
        q = n_items_a - 1 - q;
        const ItemRange it = item_range(q, kitem_a, n1, item_v_a, item_off_a, cptr, row_ptr);
        uint32_t cnt = 0;
        if (!PV) {
            const uint32_t lo = col[it.r0];
            const uint32_t span = col[it.r0 + it.d - 1] - lo;
            if (span < wave_bits && it.v >= hbase && slices_aligned) {
                // bitmap over the whole high region (N+(v) lies in it; the slice holds 2^16
                // bits); every in-edge suffix is high
                for (uint32_t i = lane; i < it.d; i += kWave) {
                    const uint32_t x = col[it.r0 + i] - hbase;
                    atomicOr(&mem[x >> 5], 1u << (x & 31u));
                }
                wave_lds_sync();
                const HighBitmapProbe probe{lds_addr(mem)};
                cnt += stream_t(it.e0, it.e1, kWave, segs, col, hcol, hbase, probe, ws);
                for (uint32_t i = lane; i < it.d; i += kWave)
                    mem[(col[it.r0 + i] - hbase) >> 5] = 0;
            } else if (span < wave_bits) {  // bitmap over the span
                for (uint32_t i = lane; i < it.d; i += kWave) {
                    const uint32_t o = col[it.r0 + i] - lo;
                    atomicOr(&mem[o >> 5], 1u << (o & 31u));
                }
                wave_lds_sync();
                const BitmapProbe probe{mem, lo, span};
                cnt += stream_t(it.e0, it.e1, kWave, segs, col, hcol, hbase, probe, ws);
                for (uint32_t i = lane; i < it.d; i += kWave)
                    mem[(col[it.r0 + i] - lo) >> 5] = 0;
            } else if (hbase + 1 < n1 && slices_aligned) {
                // a wide span (a list of at most wave_list_max <= kSliceWords entries, see
                // k_items): the suffixes' entries below hbase against N+(v)'s entries below
                // hbase as a sorted list in the slice, then their entries >= hbase against
                // N+(v)'s in the high-region bitmap (no pass for a part N+(v) lacks)
                const uint32_t hr = hrow[it.v];
                const uint32_t dlo = hr == ~0u ? it.d : hr - it.r0;
                if (dlo > 0) {
                    for (uint32_t i = lane; i < dlo; i += kWave) mem[i] = col[it.r0 + i];
                    wave_lds_sync();
                    const ListProbe lp{mem, dlo};
                    cnt += stream_t<1>(it.e0, it.e1, kWave, segs, col, hcol, hbase, lp, ws);
                    for (uint32_t i = lane; i < dlo; i += kWave) mem[i] = 0;
                    wave_lds_sync();
                }
                for (uint32_t i = dlo + lane; i < it.d; i += kWave) {
                    const uint32_t x = col[it.r0 + i] - hbase;
                    atomicOr(&mem[x >> 5], 1u << (x & 31u));
                }
                wave_lds_sync();
                if (dlo < it.d) {
                    const HighMaskedProbe probe{HighBitmapProbe{lds_addr(mem)}};
                    cnt += stream_t<2>(it.e0, it.e1, kWave, segs, col, hcol, hbase, probe, ws);
                }
                for (uint32_t i = dlo + lane; i < it.d; i += kWave)
                    mem[(col[it.r0 + i] - hbase) >> 5] = 0;
            } else {  // a wide span, but a list that fits the slice (see k_items)
                for (uint32_t i = lane; i < it.d; i += kWave) mem[i] = col[it.r0 + i];
                wave_lds_sync();
                const ListProbe probe{mem, it.d};
                cnt += stream_t(it.e0, it.e1, kWave, segs, col, hcol, hbase, probe, ws);
                for (uint32_t i = lane; i < it.d; i += kWave) mem[i] = 0;
            }
            wave_lds_sync();
        } else {
            uint32_t *list = mem, *tc = mem + kWaveListPV;
            for (uint32_t i = lane; i < it.d; i += kWave) list[i] = col[it.r0 + i];
            wave_lds_sync();
            const ListProbe probe{list, it.d};
            for (uint32_t eb = it.e0; eb < it.e1; eb += kWave)
                cnt += run_batch<true>(eb, it.e1, segs, col, probe, ws, tc, tpv);
            for (uint32_t i = lane; i < it.d; i += kWave) {
                uint32_t c = tc[i];
                if (c) {
                    atomicAdd(&tpv[list[i]], (unsigned long long)c);
                    tc[i] = 0;
                }
            }
            uint64_t item_hits = wave_sum_u64(cnt);
            if (lane == 0 && item_hits) atomicAdd(&tpv[it.v], (unsigned long long)item_hits);
            wave_lds_sync();
        }
        acc += cnt;
    }
    acc = wave_sum_u64(acc);
    if (lane == 0 && acc) atomicAdd(total, (unsigned long long)acc);
}

// ------------------------------------------------------------------ batched kernel

// Light segments of the batched kernel.  Segment i of [eb, e1) is edge e = eb + i (u -> v) of
// the forward CSR, kept when 2 <= d+(u) <= light_max: it streams the whole list N+(v) and
// looks every element up in N+(u), which the caller staged in LDS (`win` holds fcol from
// position wbase on; binary search, the list is short).  Returns the hits of this lane's own
// segment (at most d+(u)); per-vertex counts go to global counters: T(w) per hit, T(u) and
// T(v) per segment.
template <bool PV>
__device__ __forceinline__ uint32_t run_light(uint32_t eb, uint32_t e1,
                                              const uint32_t *__restrict__ frp,
                                              const uint32_t *__restrict__ fcol,
                                              const uint32_t *__restrict__ fsrc,
                                              const uint32_t *__restrict__ gid,
                                              const uint32_t *win, uint32_t wbase,
                                              WaveScratch &ws,
                                              unsigned long long *__restrict__ tpv,
                                              uint32_t light_max, uint32_t &graph) {
    const uint32_t lane = lane_id();
    const uint32_t e = eb + lane;
    uint32_t b = 0, en = 0, lo = 0, d = 0, u = 0, v = 0;
    graph = 0xFFFFFFFFu;
    if (e < e1) {  // two rounds of independent loads
        u = fsrc[e];
        v = fcol[e];
        const uint32_t r0 = frp[u], r1 = frp[u + 1];
        b = frp[v];
        en = frp[v + 1];
        graph = gid[u];
        d = r1 - r0;
        lo = r0 - wbase;
        if (d < 2 || d > light_max) d = b = en = lo = 0;
    }
    const uint32_t a0 = b & ~3u;
    const uint32_t p = (d && en > b) ? (en - a0 + kLightPiece - 1) / kLightPiece : 0u;
    const uint32_t incl = wave_incl_scan(p);
    const uint32_t Q = wave_bcast(incl, kWave - 1);
    ws.off[lane] = incl - p;
    ws.beg[lane] = a0;
    ws.first[lane] = b;
    ws.end[lane] = en;
    ws.tag[lane] = lo;
    ws.aux[lane] = d;
    ws.cnt[lane] = 0;
    wave_lds_sync();
    for (uint32_t q0 = 0; q0 < Q; q0 += kWave) {
        const uint32_t q = q0 + lane;
        if (q < Q) {
            uint32_t k = 0;
#pragma unroll
            for (uint32_t step = 32; step; step >>= 1)
                if (ws.off[k + step] <= q) k += step;
            const uint32_t start = ws.beg[k] + (q - ws.off[k]) * kLightPiece;
            const uint32_t first = ws.first[k], stop = ws.end[k];
            const uint4 *p4 = reinterpret_cast<const uint4 *>(fcol + start);
            uint32_t wv[kLightPiece];
#pragma unroll
            for (uint32_t j = 0; j < kLightPiece / 4; ++j) {
                const uint4 x = p4[j];
                wv[4 * j] = x.x;
                wv[4 * j + 1] = x.y;
                wv[4 * j + 2] = x.z;
                wv[4 * j + 3] = x.w;
            }
            const uint32_t *list = win + ws.tag[k];
            const uint32_t dl = ws.aux[k];  // >= 2
            const uint32_t lo_i = first > start ? first - start : 0u;
            const uint32_t hi_i = min(stop - start, kLightPiece);
            // the piece's lookups as binary searches in lockstep (one list per lane)
            uint32_t base[kLightPiece];
#pragma unroll
            for (uint32_t i = 0; i < kLightPiece; ++i) base[i] = 0;
            for (uint32_t n_left = dl; n_left > 1;) {
                const uint32_t half = n_left >> 1;
#pragma unroll
                for (uint32_t i = 0; i < kLightPiece; ++i)
                    base[i] = list[base[i] + half - 1] < wv[i] ? base[i] + half : base[i];
                n_left -= half;
            }
            uint32_t packed = 0;
#pragma unroll
            for (uint32_t i = 0; i < kLightPiece; ++i) {
                const uint32_t pos = base[i] + (list[base[i]] < wv[i] ? 1u : 0u);
                packed |= (list[min(pos, dl - 1u)] == wv[i] ? 1u : 0u) << i;
            }
            const uint32_t hmask = hi_i >= 32u ? ~0u : ((1u << hi_i) - 1u);
            packed &= hmask & ~((1u << lo_i) - 1u);
            const uint32_t hits = __popc(packed);
            if (PV) {
#pragma unroll
                for (uint32_t i = 0; i < kLightPiece; ++i)
                    if ((packed >> i) & 1u) atomicAdd(&tpv[wv[i]], 1ull);
            }
            if (hits) atomicAdd(&ws.cnt[k], hits);
        }
    }
    wave_lds_sync();
    const uint32_t h = ws.cnt[lane];
    if (PV && h) {
        atomicAdd(&tpv[u], (unsigned long long)h);
        atomicAdd(&tpv[v], (unsigned long long)h);
    }
    return h;
}

// Batched counting over a disjoint union of small graphs in id space (their oriented lists
// keep the input's id order, no relabelling).  Every triangle is found once, from its first
// vertex u in the order of Section 2.2: for every out-neighbour v of u, the common elements of
// N+(u) and N+(v).
//   heavy items (u with d+(u) > light_max): (u, chunk of up to kitem out-neighbours of u);
//     N+(u) is staged in the wave's LDS slice (bitmap over its id span, or a sorted list) and
//     the whole list N+(v) of every out-neighbour v streams through it.  Hits go to the graph
//     of u; per-vertex counts credit u (per item), v (per segment) and w (LDS counters by
//     list position).
//   light items: chunks of `chunk` consecutive forward edges, one edge per lane (run_light);
//     the lists of the chunk's light rows lie inside the window [e0 - light_max, e1 +
//     light_max) of fcol, which is staged in the wave's slice.  Graph ids are non-decreasing
//     along the edges, so per-graph totals are summed per run of equal graph ids.

template <bool PV>
__global__ __launch_bounds__(kThreads) void k_count_u(const BatchKernelArgs a) {
    __shared__ uint32_t s_mem[kLdsWords];
    __shared__ WaveScratch s_ws[kWaves];
    const uint32_t t = threadIdx.x, w = t / kWave, lane = lane_id();
    WaveScratch &ws = s_ws[w];
    uint32_t *mem = s_mem + w * kSliceWords;
    for (uint32_t i = t; i < kLdsWords; i += kThreads) s_mem[i] = 0;
    __syncthreads();
    const uint32_t *__restrict__ frp = a.frp;
    const uint32_t *__restrict__ fcol = a.fcol;
    const uint32_t n_items = *a.n_items, kitem = *a.kitem;
    unsigned long long *totals = *a.totals_pp;
    unsigned long long *tpv = PV ? *a.tpv_pp : nullptr;
    const OutEdgeSegs segs{frp, fcol};
    WaveQueue<kClaimBatched> wq;
    for (uint32_t q; wq.pop(a.queue, n_items, q);) {
        q = n_items - 1 - q;
        const uint32_t u = a.item_u[q];
        const uint32_t r0 = frp[u], d = frp[u + 1] - r0;
        const uint32_t e0 = r0 + (q - a.item_off[u]) * kitem;
        const uint32_t e1 = min(e0 + kitem, r0 + d);
        uint32_t lo = ~0u, hi = 0;  // the id span of N+(u) (rows of invalid graphs may be
        for (uint32_t i = lane; i < d; i += kWave) {  // unsorted, so take min and max)
            const uint32_t x = fcol[r0 + i];
            lo = min(lo, x);
            hi = max(hi, x);
        }
        for (int o = kWave / 2; o >= 1; o >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, kWave));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, kWave));
        }
        const uint32_t span = hi - lo;
        // 0 = bitmap in the slice, 1 = sorted list in the slice, 2 = sorted list in memory
        // (a.wave_bits <= kWaveBits; a.wave_list <= kSliceWords, or kWaveListPV per vertex)
        const int mode = (!PV && span < a.wave_bits) ? 0 : (d <= a.wave_list) ? 1 : 2;
        uint32_t cnt = 0;
        if (mode == 0) {
            for (uint32_t i = lane; i < d; i += kWave) {
                const uint32_t o = fcol[r0 + i] - lo;
                atomicOr(&mem[o >> 5], 1u << (o & 31u));
            }
            wave_lds_sync();
            const BitmapProbe probe{mem, lo, span};
            for (uint32_t eb = e0; eb < e1; eb += kWave)
                cnt += run_batch<PV>(eb, e1, segs, fcol, probe, ws, nullptr, tpv);
            for (uint32_t i = lane; i < d; i += kWave) mem[(fcol[r0 + i] - lo) >> 5] = 0;
        } else if (mode == 1) {
            uint32_t *list = mem, *tc = PV ? mem + kWaveListPV : nullptr;
            for (uint32_t i = lane; i < d; i += kWave) list[i] = fcol[r0 + i];
            wave_lds_sync();
            const ListProbe probe{list, d};
            for (uint32_t eb = e0; eb < e1; eb += kWave)
                cnt += run_batch<PV>(eb, e1, segs, fcol, probe, ws, tc, tpv);
            for (uint32_t i = lane; i < d; i += kWave) {
                list[i] = 0;
                if (PV && tc[i]) {
                    atomicAdd(&tpv[fcol[r0 + i]], (unsigned long long)tc[i]);
                    tc[i] = 0;
                }
            }
        } else {
            const ListProbe probe{fcol + r0, d};
            for (uint32_t eb = e0; eb < e1; eb += kWave)
                cnt += run_batch<PV>(eb, e1, segs, fcol, probe, ws, nullptr, tpv);
        }
        wave_lds_sync();
        const uint64_t item_hits = wave_sum_u64(cnt);
        if (lane == 0 && item_hits) {
            atomicAdd(&totals[a.gid[u]], (unsigned long long)item_hits);
            if (PV) atomicAdd(&tpv[u], (unsigned long long)item_hits);
        }
    }
    // light chunks
    const uint32_t mf = a.light[0], n_chunks = a.light[1], chunk = *a.chunk;
    WaveQueue<kClaimLight> lq;
    for (uint32_t q; lq.pop(a.queue + 1, n_chunks, q);) {
        const uint32_t e0 = q * chunk, e1 = min(e0 + chunk, mf);
        // the rows of the chunk's first and last edges, clipped to light_max (<= kLightMax)
        // entries around the chunk (a light row that meets the chunk lies inside)
        const uint32_t lm = a.light_max;
        const uint32_t rb = frp[a.fsrc[e0]], re = frp[a.fsrc[e1 - 1] + 1];
        const uint32_t wbase = max(rb, e0 > lm ? e0 - lm : 0u);
        const uint32_t wend = min(re, e1 + lm);
        for (uint32_t i = wbase + lane; i < wend; i += kWave) mem[i - wbase] = fcol[i];
        wave_lds_sync();
        for (uint32_t eb = e0; eb < e1; eb += kWave) {
            uint32_t g;
            uint32_t h =
                run_light<PV>(eb, e1, frp, fcol, a.fsrc, a.gid, mem, wbase, ws, tpv, lm, g);
            // per-graph sums over runs of equal graph ids (non-decreasing along the edges)
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t hv = (uint32_t)__shfl_up((int)h, o, kWave);
                const uint32_t gv = (uint32_t)__shfl_up((int)g, o, kWave);
                if (lane >= (uint32_t)o && gv == g) h += hv;
            }
            const uint32_t gn = (uint32_t)__shfl_down((int)g, 1, kWave);
            if ((lane == kWave - 1 || gn != g) && g != 0xFFFFFFFFu && h)
                atomicAdd(&totals[g], (unsigned long long)h);
        }
        wave_lds_sync();  // the next chunk's window overwrites this one (nothing after the
                          // light chunks needs a zeroed slice)
    }
}

hipError_t launch_count_u(const BatchKernelArgs &a, bool per_vertex, uint32_t grid,
                          hipStream_t s) {
    if (per_vertex)
        hipLaunchKernelGGL(k_count_u<true>, dim3(grid), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_count_u<false>, dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ host side

uint32_t count_wave_span() { return kWaveBits; }
uint32_t count_wave_list(bool per_vertex) { return per_vertex ? kWaveListPV : kSliceWords; }
uint32_t count_block_span() { return kBlockBits; }
uint32_t count_block_list(bool per_vertex) { return per_vertex ? kBlockListPV : kBlockList; }
uint32_t count_item_edges_wave() { return kItemEdgesWave; }
uint32_t count_item_edges_block() { return kItemEdgesBlock; }
uint32_t count_col_pad_bytes() { return kPiece * 4; }
uint32_t count_hcol_pad() { return kPieceHigh - 8; }
uint32_t count_panel() { return kPanel; }
uint32_t count_wgs_per_cu() { return kWgsPerCu; }
uint32_t count_light_max() { return kLightMax; }
uint32_t count_light_chunk_max() { return kLightChunkMax; }
uint32_t count_panel_ranks() { return kPanelRanks; }

hipError_t launch_count(const CountArgs &x, bool per_vertex, hipStream_t s) {
    const dim3 grid(device_cu_count() * kWgsPerCu), block(kThreads);
    if (per_vertex && x.p0 + 1 < x.n1) {  // panels: those that fit first, on their own queue
        hipLaunchKernelGGL(k_count_panel_pv, grid, block, 0, s, x.row_ptr, x.col, x.cptr,
                           x.cbeg, x.er, x.item_v_b, x.item_off_b,
                           x.n_items_b, x.queue_c, x.total, x.tpv, x.n1, x.p0, x.kitem_b,
                           x.hcol, x.hbase, x.status);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (per_vertex)
        hipLaunchKernelGGL(k_count<true>, grid, block, 0, s, x.row_ptr, x.col, x.cptr, x.cbeg,
                           x.er, x.item_v_a, x.item_off_a, x.n_items_a,
                           x.item_v_b, x.item_off_b, x.n_items_b, x.queue_a, x.queue_b, x.total,
                           x.tpv, x.n1, x.p0, x.wave_bits, x.block_bits, x.block_list,
                           x.kitem_a, x.kitem_b, x.hcol, x.hrow, x.hbase, x.status);
    else
        hipLaunchKernelGGL(k_count<false>, grid, block, 0, s, x.row_ptr, x.col, x.cptr, x.cbeg,
                           x.er, x.item_v_a, x.item_off_a, x.n_items_a,
                           x.item_v_b, x.item_off_b, x.n_items_b, x.queue_a, x.queue_b, x.total,
                           x.tpv, x.n1, x.p0, x.wave_bits, x.block_bits, x.block_list,
                           x.kitem_a, x.kitem_b, x.hcol, x.hrow, x.hbase, x.status);
    return hipGetLastError();
}

}  // namespace tc
