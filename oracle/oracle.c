/*
 * ORACLE -- test infrastructure, not product code.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no source with the HIP path.
 *
 * Plain CPU computation of the 11 induced 4-vertex graphlet counts of a
 * simple undirected graph G = (V, E), V = {0..n-1}.
 *
 *   - brute_counts(): the plain definition.  Every 4-subset S of V is
 *     classified by the isomorphism class of G[S] (Problem 1 of the paper
 *     counts induced size-4 graphlets; Fig. 1 lists the six connected ones,
 *     g1..g6; the five disconnected classes complete the catalogue of
 *     graphs on four vertices).  O(n^4), tiny graphs only.
 *
 *   - static_counts(): the static recount the baseline of Sec. 4.1 performs
 *     after every batch (a PGD-style count: per-edge triangles, 4-cliques and
 *     4-cycles plus combinatorics, Sec. 3 "PGD Algorithm").  It counts
 *     non-induced copies N_X of every 4-vertex pattern X from per-vertex and
 *     per-edge quantities and inverts the triangular "copies of X inside Y"
 *     relation.  All sums are checked int64 inside a loop body and __int128
 *     across the graph.
 *
 * Class index (output order):
 *   0 P4 (3-path, g1)   1 K1,3 (3-star, g2)   2 C4 (4-cycle, g3)
 *   3 paw (tailed triangle, g4)   4 diamond (g5)   5 K4 (4-clique, g6)
 *   6 K3+K1   7 P3+K1   8 2K2   9 K2+2K1   10 empty
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include <time.h>

typedef __int128 i128;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ---------------------------------------------------------------- helpers */
static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

typedef struct {
    int64_t n, m;
    int64_t* off;   /* n+1 */
    int32_t* adj;   /* 2m, each row sorted ascending */
} adjlist;

/* Builds sorted adjacency rows.  Input must be a simple graph: no loops, no
 * repeated pairs (either orientation).  Returns 0, or -1 on a loop,
 * an id out of range or a repeated pair. */
static int build_adj(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, adjlist* g) {
    g->n = n; g->m = m;
    g->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
        g->off[u + 1]++; g->off[v + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) g->off[v + 1] += g->off[v];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(pos, g->off, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < m; ++i) {
        g->adj[pos[src[i]]++] = dst[i];
        g->adj[pos[dst[i]]++] = src[i];
    }
    free(pos);
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1024) reduction(|:bad)
    for (int64_t v = 0; v < n; ++v) {
        int64_t b = g->off[v], e = g->off[v + 1];
        qsort(g->adj + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        for (int64_t k = b + 1; k < e; ++k) if (g->adj[k] == g->adj[k - 1]) bad = 1;
    }
    return bad ? -1 : 0;
}

static void free_adj(adjlist* g) { free(g->off); free(g->adj); }

static inline int64_t deg(const adjlist* g, int64_t v) { return g->off[v + 1] - g->off[v]; }

static int has_edge(const adjlist* g, int32_t u, int32_t v) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (g->adj[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < g->off[u + 1] && g->adj[lo] == v;
}

static int64_t common_count(const adjlist* g, int32_t u, int32_t v) {
    int64_t a = g->off[u], ae = g->off[u + 1], b = g->off[v], be = g->off[v + 1], c = 0;
    while (a < ae && b < be) {
        if (g->adj[a] < g->adj[b]) ++a;
        else if (g->adj[a] > g->adj[b]) ++b;
        else { ++c; ++a; ++b; }
    }
    return c;
}

static inline int64_t c2(int64_t x) { return x * (x - 1) / 2; }
static inline int64_t c3(int64_t x) { return x * (x - 1) * (x - 2) / 6; }
static inline i128 c2w(i128 x) { return x * (x - 1) / 2; }
static inline i128 c4w(i128 x) { return x * (x - 1) * (x - 2) * (x - 3) / 24; }

static void store128(i128 x, int64_t* hi, uint64_t* lo) {
    *lo = (uint64_t)x;
    *hi = (int64_t)(x >> 64);
}

/* ------------------------------------------------------- brute force ---- */
/* Classification of a 4-vertex graph by (edge count, sorted degrees),
 * which separates all 11 isomorphism classes. */
static int classify(int e, int d0, int d1, int d2, int d3) {
    int d[4] = {d0, d1, d2, d3};
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            if (d[j] < d[i]) { int t = d[i]; d[i] = d[j]; d[j] = t; }
    switch (e) {
    case 0: return 10;
    case 1: return 9;
    case 2: return d[0] == 0 ? 7 : 8;                 /* P3+K1 (0,1,1,2) or 2K2 */
    case 3:
        if (d[0] == 0) return 6;                         /* K3+K1 (0,2,2,2) */
        if (d[3] == 3) return 1;                         /* star (1,1,1,3) */
        return 0;                                        /* P4 (1,1,2,2) */
    case 4: return d[0] == 2 ? 2 : 3;                    /* C4 (2,2,2,2) or paw */
    case 5: return 4;
    case 6: return 5;
    }
    return -1;
}

/* counts[c] = |{S subset of V, |S| = 4, G[S] in class c}| by enumeration.
 * Uses a dense adjacency matrix; n <= 4096. */
int brute_counts(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                 int64_t* hi, uint64_t* lo) {
    if (n > 4096) return -2;
    uint8_t* A = (uint8_t*)calloc((size_t)(n * n + 1), 1);
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) { free(A); return -1; }
        A[u * n + v] = 1; A[v * n + u] = 1;
    }
    i128 cnt[11] = {0};
    #pragma omp parallel
    {
        int64_t loc[11] = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t a = 0; a < n; ++a)
            for (int64_t b = a + 1; b < n; ++b)
                for (int64_t c = b + 1; c < n; ++c)
                    for (int64_t d = c + 1; d < n; ++d) {
                        int ab = A[a * n + b], ac = A[a * n + c], ad = A[a * n + d];
                        int bc = A[b * n + c], bd = A[b * n + d], cd = A[c * n + d];
                        int e = ab + ac + ad + bc + bd + cd;
                        int k = classify(e, ab + ac + ad, ab + bc + bd, ac + bc + cd, ad + bd + cd);
                        loc[k]++;
                    }
        #pragma omp critical
        for (int k = 0; k < 11; ++k) cnt[k] += loc[k];
    }
    free(A);
    for (int k = 0; k < 11; ++k) store128(cnt[k], &hi[k], &lo[k]);
    return 0;
}

/* ------------------------------------------------------- static recount - */
/* Non-induced copy counts of the six connected patterns plus the global
 * terms the disconnected classes need.  sig layout (all exact integers):
 *   0 N_P4  1 N_K13  2 N_C4  3 N_paw  4 N_diamond  5 N_K4  6 T  7 W  8 m
 * Returned as hi/lo halves of __int128.
 *
 * Every edge and every 4-clique is visited once under a fixed total order
 * of the vertices: a precedes b iff (deg a, a) < (deg b, b).  Any total
 * order visits each once; this one makes the row that is scanned the
 * shorter one. */
static inline int precedes(const adjlist* g, int64_t a, int64_t b) {
    int64_t da = deg(g, a), db = deg(g, b);
    return da < db || (da == db && a < b);
}

/* stride > 1 visits only the vertices offset, offset + stride, ... in the
 * three per-vertex loops below (to time a sample of the work; the sums are
 * then partial). */
static int noninduced(const adjlist* g, i128 sig[9], int64_t stride, int64_t offset) {
    const int64_t n = g->n;
    const int64_t ns_v = offset < n ? (n - offset + stride - 1) / stride : 0;
    i128 W = 0, K13 = 0, T3 = 0, P4raw = 0, paw2 = 0, dia = 0, k4 = 0, c4x2 = 0;
    int ovf = 0;

    /* vertex terms: wedges W = sum C(d,2); 3-stars sum C(d,3) */
    #pragma omp parallel
    {
        i128 w = 0, s = 0;
        #pragma omp for schedule(static)
        for (int64_t v = 0; v < n; ++v) { int64_t d = deg(g, v); w += c2(d); s += c3(d); }
        #pragma omp critical
        { W += w; K13 += s; }
    }

    /* edge terms, every edge (u, v) once, at its later endpoint v:
     * t_uv = |N(u) & N(v)| = number of w in N(u) marked as members of N(v).
     *   3T        = sum_e t
     *   N_P4 + 3T = sum_e (d_u - 1)(d_v - 1)   (middle edge, one end each side)
     *   2 N_paw   = sum_e t (d_u + d_v - 4)    (triangle on e, pendant at u or v)
     *   N_diamond = sum_e C(t, 2)              (two triangles sharing e)  */
    #pragma omp parallel
    {
        i128 t3 = 0, p4 = 0, pw = 0, di = 0;
        uint8_t* mark = (uint8_t*)calloc((size_t)n + 1, 1);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < ns_v; ++i) {
            const int64_t v = offset + i * stride;
            for (int64_t q = g->off[v]; q < g->off[v + 1]; ++q) mark[g->adj[q]] = 1;
            for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) {
                int32_t u = g->adj[p];
                if (!precedes(g, u, v)) continue;
                int64_t t = 0;
                for (int64_t q = g->off[u]; q < g->off[u + 1]; ++q) t += mark[g->adj[q]];
                int64_t du = deg(g, u), dv = deg(g, v);
                t3 += t;
                p4 += (i128)(du - 1) * (dv - 1);
                pw += (i128)t * (du + dv - 4);
                di += c2(t);
            }
            for (int64_t q = g->off[v]; q < g->off[v + 1]; ++q) mark[g->adj[q]] = 0;
        }
        free(mark);
        #pragma omp critical
        { T3 += t3; P4raw += p4; paw2 += pw; dia += di; }
    }

    /* 4-cliques {a, b, c, d} with a, b, c, d in that order: counted once, at
     * u = a, v = b, as the edge (c, d) inside S = out(a) & out(b), where
     * out(x) = the neighbours that follow x. */
    {
        int64_t* ooff = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
        for (int64_t u = 0; u < n; ++u) {
            int64_t c = 0;
            for (int64_t p = g->off[u]; p < g->off[u + 1]; ++p) c += precedes(g, u, g->adj[p]);
            ooff[u + 1] = ooff[u] + c;
        }
        int32_t* oadj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ooff[n] + 1));
        #pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t u = 0; u < n; ++u) {
            int64_t k = ooff[u];
            for (int64_t p = g->off[u]; p < g->off[u + 1]; ++p)
                if (precedes(g, u, g->adj[p])) oadj[k++] = g->adj[p];
        }
        #pragma omp parallel
        {
            i128 kk = 0;
            uint8_t* in_a = (uint8_t*)calloc((size_t)n + 1, 1);
            uint8_t* in_s = (uint8_t*)calloc((size_t)n + 1, 1);
            int64_t cap = 16, ns;
            int32_t* S = (int32_t*)malloc(sizeof(int32_t) * cap);
            #pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < ns_v; ++i) {
                const int64_t a = offset + i * stride;
                for (int64_t p = ooff[a]; p < ooff[a + 1]; ++p) in_a[oadj[p]] = 1;
                for (int64_t p = ooff[a]; p < ooff[a + 1]; ++p) {
                    int32_t b = oadj[p];
                    ns = 0;
                    for (int64_t q = ooff[b]; q < ooff[b + 1]; ++q)
                        if (in_a[oadj[q]]) {
                            if (ns == cap) { cap *= 2; S = (int32_t*)realloc(S, sizeof(int32_t) * cap); }
                            S[ns++] = oadj[q];
                        }
                    for (int64_t i = 0; i < ns; ++i) in_s[S[i]] = 1;
                    for (int64_t i = 0; i < ns; ++i)
                        for (int64_t q = ooff[S[i]]; q < ooff[S[i] + 1]; ++q) kk += in_s[oadj[q]];
                    for (int64_t i = 0; i < ns; ++i) in_s[S[i]] = 0;
                }
                for (int64_t p = ooff[a]; p < ooff[a + 1]; ++p) in_a[oadj[p]] = 0;
            }
            free(in_a); free(in_s); free(S);
            #pragma omp critical
            k4 += kk;
        }
        free(ooff); free(oadj);
    }

    /* 4-cycles: N_C4 = 1/2 sum over unordered vertex pairs {v, w} of
     * C(c(v, w), 2), c(v, w) = number of common neighbours, over ALL pairs
     * (adjacent or not): each 4-cycle has two diagonals.  For every vertex v,
     * c[w] counts the common neighbours of v and each w < v (vertex ids). */
    #pragma omp parallel
    {
        int32_t* cnt = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
        i128 acc = 0;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < ns_v; ++i) {
            const int64_t v = offset + i * stride;
            int64_t nt = 0;
            for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) {
                int32_t u = g->adj[p];
                for (int64_t q = g->off[u]; q < g->off[u + 1]; ++q) {
                    int32_t w = g->adj[q];
                    if (w >= v) break;   /* rows are sorted by id */
                    if (cnt[w]++ == 0) touched[nt++] = w;
                }
            }
            for (int64_t i = 0; i < nt; ++i) { acc += c2(cnt[touched[i]]); cnt[touched[i]] = 0; }
        }
        free(cnt); free(touched);
        #pragma omp critical
        c4x2 += acc;
    }

    if (T3 % 3 != 0 || paw2 % 2 != 0 || c4x2 % 2 != 0) ovf = 1;
    i128 T = T3 / 3;
    sig[0] = P4raw - 3 * T;
    sig[1] = K13;
    sig[2] = c4x2 / 2;
    sig[3] = paw2 / 2;
    sig[4] = dia;
    sig[5] = k4;
    sig[6] = T;
    sig[7] = W;
    sig[8] = g->m;
    return ovf ? -3 : 0;
}

/* The same non-induced counts by a second formulation: t_uv by a sorted
 * merge of the two rows for every edge u < v (vertex id order), 4-cliques as
 * u < v < w < x by id with a binary search per pair.  O(sum of d^2) merge
 * steps: kept only so that tests can check the two formulations against
 * each other on graphs too large for brute force. */
static int noninduced_merge(const adjlist* g, i128 sig[9]) {
    const int64_t n = g->n;
    i128 W = 0, K13 = 0, T3 = 0, P4raw = 0, paw2 = 0, dia = 0, k4 = 0, c4x4 = 0;
    int ovf = 0;

    /* vertex terms: wedges W = sum C(d,2); 3-stars sum C(d,3) */
    #pragma omp parallel
    {
        i128 w = 0, s = 0;
        #pragma omp for schedule(static)
        for (int64_t v = 0; v < n; ++v) { int64_t d = deg(g, v); w += c2(d); s += c3(d); }
        #pragma omp critical
        { W += w; K13 += s; }
    }

    /* edge terms: t_uv = |N(u) & N(v)| by sorted merge.
     *   3T        = sum_e t
     *   N_P4 + 3T = sum_e (d_u - 1)(d_v - 1)   (middle edge, one end each side)
     *   2 N_paw   = sum_e t (d_u + d_v - 4)    (triangle on e, pendant at u or v)
     *   N_diamond = sum_e C(t, 2)              (two triangles sharing e)
     *   N_K4      = #{u<v<w<x : all six pairs adjacent}                     */
    #pragma omp parallel
    {
        i128 t3 = 0, p4 = 0, pw = 0, di = 0, kk = 0;
        int64_t* cs = (int64_t*)malloc(sizeof(int64_t) * 16);
        int64_t cap = 16;
        #pragma omp for schedule(dynamic, 256)
        for (int64_t u = 0; u < n; ++u) {
            for (int64_t p = g->off[u]; p < g->off[u + 1]; ++p) {
                int32_t v = g->adj[p];
                if (v <= u) continue;
                int64_t du = deg(g, u), dv = deg(g, v);
                int64_t t = common_count(g, (int32_t)u, v);
                t3 += t;
                p4 += (i128)(du - 1) * (dv - 1);
                pw += (i128)t * (du + dv - 4);
                di += c2(t);
                /* 4-cliques with u < v < w < x: w, x common neighbours above v */
                int64_t k = 0;
                int64_t a = g->off[u], ae = g->off[u + 1], b = g->off[v], be = g->off[v + 1];
                while (a < ae && b < be) {
                    if (g->adj[a] < g->adj[b]) ++a;
                    else if (g->adj[a] > g->adj[b]) ++b;
                    else {
                        if (g->adj[a] > v) {
                            if (k == cap) { cap *= 2; cs = (int64_t*)realloc(cs, sizeof(int64_t) * cap); }
                            cs[k++] = g->adj[a];
                        }
                        ++a; ++b;
                    }
                }
                for (int64_t i = 0; i < k; ++i)
                    for (int64_t j = i + 1; j < k; ++j)
                        if (has_edge(g, (int32_t)cs[i], (int32_t)cs[j])) kk += 1;
            }
        }
        free(cs);
        #pragma omp critical
        { T3 += t3; P4raw += p4; paw2 += pw; dia += di; k4 += kk; }
    }

    /* 4-cycles: for every vertex v, c[w] = number of common neighbours of v
     * and w (w != v), over ALL pairs.  sum_v sum_w C(c[w], 2) counts every
     * 4-cycle four times (two diagonals, each from both ends). */
    #pragma omp parallel
    {
        int32_t* cnt = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
        i128 acc = 0;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            int64_t nt = 0;
            for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) {
                int32_t u = g->adj[p];
                for (int64_t q = g->off[u]; q < g->off[u + 1]; ++q) {
                    int32_t w = g->adj[q];
                    if (w == v) continue;
                    if (cnt[w]++ == 0) touched[nt++] = w;
                }
            }
            for (int64_t i = 0; i < nt; ++i) { acc += c2(cnt[touched[i]]); cnt[touched[i]] = 0; }
        }
        free(cnt); free(touched);
        #pragma omp critical
        c4x4 += acc;
    }

    if (T3 % 3 != 0 || paw2 % 2 != 0 || c4x4 % 4 != 0) ovf = 1;
    i128 T = T3 / 3;
    sig[0] = P4raw - 3 * T;
    sig[1] = K13;
    sig[2] = c4x4 / 4;
    sig[3] = paw2 / 2;
    sig[4] = dia;
    sig[5] = k4;
    sig[6] = T;
    sig[7] = W;
    sig[8] = g->m;
    return ovf ? -3 : 0;
}

/* Induced counts from non-induced counts.  Every induced 4-vertex subgraph
 * of class Y contains a fixed number of copies of pattern X; the relation is
 * triangular (ordered by edge count), so it inverts by back-substitution:
 *   copies in (P4 star C4 paw dia K4):
 *     P4:   1    0    4    2   6   12
 *     star: 0    1    0    1   2    4
 *     C4:   0    0    1    0   1    3
 *     paw:  0    0    0    1   4   12
 *     dia:  0    0    0    0   1    6
 *     K4:   0    0    0    0   0    1
 * The disconnected classes come from global totals over all 4-subsets:
 *   T (n-3)          = sum_S #triangles in G[S]
 *   W (n-3)          = sum_S #2-paths  in G[S]
 *   C(m,2) - W       = sum_S #pairs of disjoint edges in G[S]
 *   m C(n-2, 2)      = sum_S #edges in G[S]
 *   C(n,4)           = sum_S 1                                          */
static void invert(int64_t n, const i128 s[9], i128 I[11]) {
    const i128 Np4 = s[0], Nst = s[1], Nc4 = s[2], Npaw = s[3], Ndia = s[4], Nk4 = s[5];
    const i128 T = s[6], W = s[7], m = s[8], nn = n;
    I[5] = Nk4;
    I[4] = Ndia - 6 * I[5];
    I[3] = Npaw - 4 * I[4] - 12 * I[5];
    I[2] = Nc4 - I[4] - 3 * I[5];
    I[0] = Np4 - 2 * I[3] - 4 * I[2] - 6 * I[4] - 12 * I[5];
    I[1] = Nst - I[3] - 2 * I[4] - 4 * I[5];
    /* triangles: K3+K1 1, paw 1, diamond 2, K4 4 */
    I[6] = T * (nn - 3) - I[3] - 2 * I[4] - 4 * I[5];
    /* 2-paths: P3+K1 1, K3+K1 3, star 3, P4 2, C4 4, paw 5, diamond 8, K4 12 */
    I[7] = W * (nn - 3) - 3 * I[6] - 3 * I[1] - 2 * I[0] - 4 * I[2] - 5 * I[3] - 8 * I[4] - 12 * I[5];
    /* disjoint edge pairs: 2K2 1, P4 1, C4 2, paw 1, diamond 2, K4 3 */
    I[8] = (c2w(m) - W) - I[0] - 2 * I[2] - I[3] - 2 * I[4] - 3 * I[5];
    /* edges: K2+2K1 1, 2K2 2, P3+K1 2, K3+K1 3, star 3, P4 3, C4 4, paw 4, dia 5, K4 6 */
    I[9] = m * c2w(nn - 2) - 2 * I[8] - 2 * I[7] - 3 * I[6] - 3 * I[1] - 3 * I[0]
         - 4 * I[2] - 4 * I[3] - 5 * I[4] - 6 * I[5];
    i128 rest = 0;
    for (int k = 0; k < 10; ++k) rest += I[k];
    I[10] = c4w(nn) - rest;
}

/* counts (hi/lo halves) of the 11 classes; sig (hi/lo) of the 9 terms. */
int static_counts(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                  int64_t* hi, uint64_t* lo, int64_t* sig_hi, uint64_t* sig_lo) {
    adjlist g;
    if (build_adj(n, m, src, dst, &g) != 0) { free_adj(&g); return -1; }
    i128 sig[9], I[11];
    int rc = noninduced(&g, sig, 1, 0);
    free_adj(&g);
    if (rc) return rc;
    invert(n, sig, I);
    for (int k = 0; k < 11; ++k) store128(I[k], &hi[k], &lo[k]);
    if (sig_hi) for (int k = 0; k < 9; ++k) store128(sig[k], &sig_hi[k], &sig_lo[k]);
    return 0;
}

/* Same output as static_counts, through the merge formulation. */
int static_counts_merge(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        int64_t* hi, uint64_t* lo) {
    adjlist g;
    if (build_adj(n, m, src, dst, &g) != 0) { free_adj(&g); return -1; }
    i128 sig[9], I[11];
    int rc = noninduced_merge(&g, sig);
    free_adj(&g);
    if (rc) return rc;
    invert(n, sig, I);
    for (int k = 0; k < 11; ++k) store128(I[k], &hi[k], &lo[k]);
    return 0;
}

/* Timing of a sample of static_counts' work (no counts): the adjacency
 * build in full, then the per-vertex loops over the vertices offset,
 * offset + stride, ...  secs[0] = build, secs[1] = sampled loops. */
int static_counts_sample_time(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              int64_t stride, int64_t offset, double* secs) {
    if (stride < 1 || offset < 0) return -2;
    double t0 = now_s();
    adjlist g;
    if (build_adj(n, m, src, dst, &g) != 0) { free_adj(&g); return -1; }
    double t1 = now_s();
    i128 sig[9];
    (void)noninduced(&g, sig, stride, offset);
    double t2 = now_s();
    free_adj(&g);
    secs[0] = t1 - t0;
    secs[1] = t2 - t1;
    return 0;
}

/* ------------------------------------------------- 3-vertex graphlets -- */
/* Induced 3-vertex counts, order: 0 triangle, 1 induced 2-path (wedge),
 * 2 one edge + isolated vertex, 3 empty.  Sec. 3: PGD counts the graphlets
 * of size 3 as well as size 4. */

/* By enumeration of all C(n,3) subsets (n <= 4096). */
int brute3_counts(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t* hi, uint64_t* lo) {
    if (n > 4096) return -2;
    uint8_t* A = (uint8_t*)calloc((size_t)(n * n + 1), 1);
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) { free(A); return -1; }
        A[u * n + v] = 1; A[v * n + u] = 1;
    }
    i128 cnt[4] = {0};
    #pragma omp parallel
    {
        int64_t loc[4] = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t a = 0; a < n; ++a)
            for (int64_t b = a + 1; b < n; ++b)
                for (int64_t c = b + 1; c < n; ++c) {
                    int e = A[a * n + b] + A[a * n + c] + A[b * n + c];
                    loc[3 - e]++;   /* 3 edges -> 0 (triangle), ..., 0 edges -> 3 (empty) */
                }
        #pragma omp critical
        for (int k = 0; k < 4; ++k) cnt[k] += loc[k];
    }
    free(A);
    for (int k = 0; k < 4; ++k) store128(cnt[k], &hi[k], &lo[k]);
    return 0;
}

/* From the static recount's totals: T triangles, W = sum_v C(d_v, 2) 2-paths
 * (a triangle holds three), m edges; every triple with an edge is counted
 * by its edges in m (n - 2). */
int static_counts3(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t* hi, uint64_t* lo) {
    adjlist g;
    if (build_adj(n, m, src, dst, &g) != 0) { free_adj(&g); return -1; }
    i128 sig[9];
    int rc = noninduced(&g, sig, 1, 0);
    free_adj(&g);
    if (rc) return rc;
    const i128 T = sig[6], W = sig[7], mm = sig[8], nn = n;
    i128 I[4];
    I[0] = T;
    I[1] = W - 3 * T;
    I[2] = mm * (nn - 2) - 2 * I[1] - 3 * I[0];
    I[3] = nn * (nn - 1) * (nn - 2) / 6 - I[0] - I[1] - I[2];
    for (int k = 0; k < 4; ++k) store128(I[k], &hi[k], &lo[k]);
    return 0;
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
