/*
 * oracle/forward.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, single-threaded CPU reference for exact triangle counting, written from
 * A. Polak, "Counting Triangles in Large Graphs on GPU" (IPDPS Workshops 2016, arXiv
 * 1503.00576).  Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library; the GPU path neither includes, links nor calls it, and this file
 * includes nothing of the GPU path.
 *
 * What it computes
 *   - oracle_degrees / oracle_oriented_csr / oracle_count: the sequential *forward*
 *     algorithm of Section 2.2 (Schank-Wagner, in Latapy's compact form): a total order on
 *     vertices consistent with degree, every undirected edge kept only in its forward
 *     direction, adjacency lists sorted by vertex number, then one two-pointer merge per
 *     remaining edge; the merges' sizes sum to the triangle count.  Input is the edge array
 *     of Section 3.1.
 *   - oracle_vertex_triangles: the plain definition of the per-vertex count, T(v) = number
 *     of edges joining two neighbours of v, evaluated one vertex at a time.
 *   - oracle_count_sym_csr: the forward algorithm on a symmetric adjacency-list input
 *     (rows sorted), the format the paper contrasts with the edge array in Section 3.1.
 *
 * Readings where the paper leaves a choice open (listed again in the design notes):
 *   - the order: u precedes v iff (deg u, u) < (deg v, v) (ties by identifier, ascending);
 *     order == 1 selects plain identifier order instead (any total order gives the same
 *     total, which the tests use to pin the orientation step);
 *   - degree = full undirected degree;
 *   - edge-array multiplicity: both == 0 lists every undirected edge once in either
 *     orientation; both == 1 is the paper's format (each edge twice, once per direction),
 *     whose degree is the count of entries with the vertex first;
 *   - bad input (identifier outside [0, n), self-loop, repeated edge, or in the two-direction
 *     format an edge without its mirror) is reported, never repaired;
 *   - per-vertex counts: T(v) = number of triangles containing v, so they sum to 3 * total.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    OR_OK = 0,
    OR_E_ARG = 1,
    OR_E_RANGE = 2,
    OR_E_SELF_LOOP = 3,
    OR_E_DUP_EDGE = 4,
    OR_E_ASYMMETRIC = 5,
    OR_E_NOMEM = 6,
    OR_E_UNSORTED = 7
};

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* u precedes v in the total order of Section 2.2 */
static int precedes(int32_t u, int32_t v, const int64_t *deg, int order) {
    if (order == 1) return u < v;
    if (deg[u] != deg[v]) return deg[u] < deg[v];
    return u < v;
}

/* Input checks of Section 3.1 (identifiers in range, no self-loops). */
static int check_ids(int64_t n, int64_t m, const int32_t *edges) {
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || (int64_t)u >= n || (int64_t)v >= n) return OR_E_RANGE;
    }
    for (int64_t i = 0; i < m; ++i)
        if (edges[2 * i] == edges[2 * i + 1]) return OR_E_SELF_LOOP;
    return OR_OK;
}

/* Vertex degrees (the source of the order in Section 2.2).  In the two-direction format
 * every undirected edge contributes one entry with each end first, so counting first ends
 * gives the degree, as the paper does from its node array (Section 3.2, step 5). */
int oracle_degrees(int64_t n, int64_t m, const int32_t *edges, int both, int64_t *deg) {
    if (n < 0 || m < 0 || (m > 0 && !edges) || (n > 0 && !deg)) return OR_E_ARG;
    int st = check_ids(n, m, edges);
    if (st) return st;
    for (int64_t x = 0; x < n; ++x) deg[x] = 0;
    for (int64_t i = 0; i < m; ++i) {
        deg[edges[2 * i]] += 1;
        if (!both) deg[edges[2 * i + 1]] += 1;
    }
    return OR_OK;
}

/* Build sorted adjacency lists (CSR) of the entries selected by `sel`:
 * sel == 0: forward entries s -> t with s preceding t (edges-once input: every edge, turned
 *           forward; two-direction input: only entries already forward),
 * sel == 1: two-direction input only: backward entries, turned around to s -> t.
 * Rows are sorted ascending by vertex number (Section 2.2, last preprocessing step). */
static int build_csr(int64_t n, int64_t m, const int32_t *edges, int both, int order,
                     const int64_t *deg, int sel, int64_t *row_ptr, int32_t **col_out,
                     int64_t *m_out) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return OR_E_NOMEM;
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = edges[2 * i], v = edges[2 * i + 1];
        int fwd = precedes(u, v, deg, order);
        int32_t s;
        if (!both) s = fwd ? u : v;
        else if (sel == 0) { if (!fwd) continue; s = u; }
        else { if (fwd) continue; s = v; }
        cnt[s] += 1;
        k += 1;
    }
    row_ptr[0] = 0;
    for (int64_t x = 0; x < n; ++x) row_ptr[x + 1] = row_ptr[x] + cnt[x];
    int32_t *col = (int32_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int32_t));
    if (!col) { free(cnt); return OR_E_NOMEM; }
    for (int64_t x = 0; x < n; ++x) cnt[x] = row_ptr[x];
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = edges[2 * i], v = edges[2 * i + 1];
        int fwd = precedes(u, v, deg, order);
        int32_t s, t;
        if (!both) { s = fwd ? u : v; t = fwd ? v : u; }
        else if (sel == 0) { if (!fwd) continue; s = u; t = v; }
        else { if (fwd) continue; s = v; t = u; }
        col[cnt[s]++] = t;
    }
    free(cnt);
    for (int64_t x = 0; x < n; ++x) {
        int64_t len = row_ptr[x + 1] - row_ptr[x];
        if (len > 1) qsort(col + row_ptr[x], (size_t)len, sizeof(int32_t), cmp_i32);
    }
    *col_out = col;
    *m_out = k;
    return OR_OK;
}

static int has_adjacent_repeat(int64_t n, const int64_t *row_ptr, const int32_t *col) {
    for (int64_t x = 0; x < n; ++x)
        for (int64_t j = row_ptr[x] + 1; j < row_ptr[x + 1]; ++j)
            if (col[j] == col[j - 1]) return 1;
    return 0;
}

/* Preprocessing phase: degrees, orientation, sorted lists.  On success *col_out is
 * malloc'ed (caller frees) and row_ptr[0..n] is filled. */
static int preprocess(int64_t n, int64_t m, const int32_t *edges, int both, int order,
                      int64_t *deg, int64_t *row_ptr, int32_t **col_out, int64_t *m_fwd) {
    int st = oracle_degrees(n, m, edges, both, deg);
    if (st) return st;
    int32_t *col = NULL;
    st = build_csr(n, m, edges, both, order, deg, 0, row_ptr, &col, m_fwd);
    if (st) return st;
    if (has_adjacent_repeat(n, row_ptr, col)) { free(col); return OR_E_DUP_EDGE; }
    if (both) {
        /* the backward entries, turned around, must be exactly the forward ones */
        int64_t *rp2 = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
        int32_t *col2 = NULL;
        int64_t m2 = 0;
        if (!rp2) { free(col); return OR_E_NOMEM; }
        st = build_csr(n, m, edges, both, order, deg, 1, rp2, &col2, &m2);
        if (st) { free(rp2); free(col); return st; }
        int same = (m2 == *m_fwd) &&
                   memcmp(rp2, row_ptr, ((size_t)n + 1) * sizeof(int64_t)) == 0 &&
                   memcmp(col2, col, (size_t)m2 * sizeof(int32_t)) == 0;
        int dup2 = has_adjacent_repeat(n, rp2, col2);
        free(rp2);
        free(col2);
        if (dup2) { free(col); return OR_E_DUP_EDGE; }
        if (!same) { free(col); return OR_E_ASYMMETRIC; }
    }
    *col_out = col;
    return OR_OK;
}

/* The oriented, sorted adjacency lists as CSR (row_ptr[n+1], col[m_fwd]); col may be NULL
 * to query m_fwd only (col_cap is then ignored). */
int oracle_oriented_csr(int64_t n, int64_t m, const int32_t *edges, int both, int order,
                        int64_t *row_ptr, int32_t *col, int64_t col_cap, int64_t *m_fwd) {
    if (n < 0 || m < 0 || !row_ptr || !m_fwd) return OR_E_ARG;
    int64_t *deg = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!deg) return OR_E_NOMEM;
    int32_t *c = NULL;
    int st = preprocess(n, m, edges, both, order, deg, row_ptr, &c, m_fwd);
    free(deg);
    if (st) return st;
    if (col) {
        if (col_cap < *m_fwd) { free(c); return OR_E_ARG; }
        memcpy(col, c, (size_t)*m_fwd * sizeof(int32_t));
    }
    free(c);
    return OR_OK;
}

/* Counting phase over an oriented CSR: for every edge u -> v the two-pointer merge of the
 * sorted lists N+(u) and N+(v) (Section 2.2); every common element w closes the triangle
 * {u, v, w}, found exactly once. */
static void count_merge(int64_t n, const int64_t *row_ptr, const int32_t *col, uint64_t *total,
                        uint64_t *per_vertex) {
    uint64_t t = 0;
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            int64_t i = row_ptr[u], iend = row_ptr[u + 1];
            int64_t j = row_ptr[v], jend = row_ptr[v + 1];
            while (i < iend && j < jend) {
                int32_t a = col[i], b = col[j];
                if (a < b) {
                    ++i;
                } else if (a > b) {
                    ++j;
                } else {
                    ++t;
                    if (per_vertex) {
                        per_vertex[u] += 1;
                        per_vertex[v] += 1;
                        per_vertex[a] += 1;
                    }
                    ++i;
                    ++j;
                }
            }
        }
    }
    *total = t;
}

/* Exact triangle count (and optionally per-vertex counts, uint64[n]) of an edge array. */
int oracle_count(int64_t n, int64_t m, const int32_t *edges, int both, int order,
                 uint64_t *total, uint64_t *per_vertex) {
    if (n < 0 || m < 0 || !total) return OR_E_ARG;
    int64_t *deg = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *row_ptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!deg || !row_ptr) { free(deg); free(row_ptr); return OR_E_NOMEM; }
    int32_t *col = NULL;
    int64_t m_fwd = 0;
    int st = preprocess(n, m, edges, both, order, deg, row_ptr, &col, &m_fwd);
    free(deg);
    if (st) { free(row_ptr); return st; }
    if (per_vertex) for (int64_t x = 0; x < n; ++x) per_vertex[x] = 0;
    count_merge(n, row_ptr, col, total, per_vertex);
    free(row_ptr);
    free(col);
    return OR_OK;
}

/* Forward algorithm on a symmetric adjacency-list input: row_ptr[n+1] (int64), col (int32)
 * with every undirected edge in both rows and every row strictly ascending.  The degree is
 * the row length; the forward entries of each row are kept in order, so rows stay sorted. */
int oracle_count_sym_csr(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         uint64_t *total, uint64_t *per_vertex) {
    if (n < 0 || !row_ptr || !total || row_ptr[0] != 0) return OR_E_ARG;
    for (int64_t x = 0; x < n; ++x) {
        if (row_ptr[x + 1] < row_ptr[x]) return OR_E_ARG;
        for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j) {
            if (col[j] < 0 || (int64_t)col[j] >= n) return OR_E_RANGE;
            if (col[j] == x) return OR_E_SELF_LOOP;
            if (j > row_ptr[x] && col[j] <= col[j - 1])
                return col[j] == col[j - 1] ? OR_E_DUP_EDGE : OR_E_UNSORTED;
        }
    }
    int64_t m2 = row_ptr[n];
    int32_t *edges = (int32_t *)malloc((size_t)(m2 > 0 ? m2 : 1) * 2 * sizeof(int32_t));
    if (!edges) return OR_E_NOMEM;
    for (int64_t x = 0; x < n; ++x)
        for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j) {
            edges[2 * j] = (int32_t)x;
            edges[2 * j + 1] = col[j];
        }
    /* the two-direction edge array: its checks also catch a missing mirror entry */
    int st = oracle_count(n, m2, edges, 1, 0, total, per_vertex);
    free(edges);
    return st;
}

/* Plain definition, one vertex at a time: T(v) = number of edges {a, b} with both a and b
 * adjacent to v.  Edges are given once (either orientation); the input is assumed valid.
 * Cost per query is the sum of the degrees of v's neighbours. */
int oracle_vertex_triangles(int64_t n, int64_t m, const int32_t *edges, int64_t nq,
                            const int32_t *queries, uint64_t *out) {
    if (n < 0 || m < 0 || nq < 0 || (nq > 0 && (!queries || !out))) return OR_E_ARG;
    int st = check_ids(n, m, edges);
    if (st) return st;
    /* undirected adjacency (both directions) */
    int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc((size_t)(m > 0 ? 2 * m : 1) * sizeof(int32_t));
    uint8_t *mark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!rp || !adj || !mark) { free(rp); free(adj); free(mark); return OR_E_NOMEM; }
    for (int64_t i = 0; i < m; ++i) { rp[edges[2 * i] + 1] += 1; rp[edges[2 * i + 1] + 1] += 1; }
    for (int64_t x = 0; x < n; ++x) rp[x + 1] += rp[x];
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!fill) { free(rp); free(adj); free(mark); return OR_E_NOMEM; }
    memcpy(fill, rp, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = edges[2 * i], v = edges[2 * i + 1];
        adj[fill[u]++] = v;
        adj[fill[v]++] = u;
    }
    free(fill);
    for (int64_t q = 0; q < nq; ++q) {
        int32_t v = queries[q];
        if (v < 0 || (int64_t)v >= n) { st = OR_E_RANGE; break; }
        for (int64_t j = rp[v]; j < rp[v + 1]; ++j) mark[adj[j]] = 1;
        uint64_t c = 0;
        for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
            int32_t a = adj[j];
            for (int64_t k = rp[a]; k < rp[a + 1]; ++k) {
                int32_t b = adj[k];
                if (b > a && mark[b]) ++c; /* each edge {a, b} among N(v) once */
            }
        }
        for (int64_t j = rp[v]; j < rp[v + 1]; ++j) mark[adj[j]] = 0;
        out[q] = c;
    }
    free(rp);
    free(adj);
    free(mark);
    return st;
}
