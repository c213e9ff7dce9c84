/*
 * glo_oracle.c -- CPU oracle for exact 2-, 3- and 4-node graphlet counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this code.  It shares nothing with the GPU library: no headers, no
 * helpers, no tables.  It is deliberately plain and slow.
 *
 * Four methods live here:
 *
 *  (1) brute_*  -- the definition (Section 3, Definitions 1-3 and Problem 1): every 3- and
 *      4-vertex subset is classified by the induced subgraph it spans.  Per-edge counts
 *      enumerate every vertex pair outside the edge.  Feasible for a few hundred vertices.
 *
 *  (2) glo_*    -- the paper's edge-centric method (Section 4): for each edge the hash
 *      Psi with per-edge unique tags (Alg. "3-Graphlets" and Section 4.5), the
 *      neighbour-iteration scans for cliques (Alg. "Clique") and cycles (Alg. "Cycle"),
 *      then the local counts, the unrestricted counts C3..C16 (Section 4.5) and the global
 *      frequencies X1..X17 (Section 4.6).  Readings taken where the text is garbled:
 *        - local x5 is n - x4 - |T| - 2 (the printed sign of |T| contradicts C5);
 *        - C9 sums |T|*(|S_u|+|S_v|), not the triple product;
 *        - X11 uses C11, not C9;
 *        - the cycle scan tests for the S_v tag (lambda_1, kept by neighbours of v that
 *          are not neighbours of u), since lambda_2 marks S_u itself;
 *        - the clique scan counts each unordered adjacent pair of T once (sequential
 *          reading of the parallel loop);
 *        - |T| + |S_u| = d_u - 1 (v is excluded).
 *      The remaining 4-node per-edge counts (chordal cycle, tailed triangle, 3-star,
 *      4-path and the disconnected ones) follow from a partition of V \ {u,v} into
 *      T, S_u, S_v and D (neither endpoint) and the edge counts between those classes,
 *      derived from |T|, the clique and cycle counts, three extra scan counters and
 *      vertex triangle / neighbour-degree sums.  glo_count_range runs the same pass over a
 *      block of edges, so that a long run can proceed (and be checked) block by block.
 *
 *  (3) glo_global_substructures -- global counts only, for graphs far too large for (2):
 *      every unrestricted count of Section 4.5 follows from the triangles on each edge
 *      (by definition, |N(u) & N(v)|), the number of 4-cliques and the number of 4-cycles,
 *      each counted once at its lowest vertex in the order of P1; Section 4.6 then gives
 *      X1..X17.  Pinned against (1) and (2) on every graph the tests draw.
 *
 *  (4) glo_per_edge_substructures -- per-edge and global counts for graphs too large for
 *      (2): the per-edge terms that (2) gets from tag scans (4-cliques, T-S_u and T-S_v
 *      edges, S_u-S_v edges, degree sum over T) are recovered from per-edge counts of
 *      triangles, 4-cliques, 4-cycles and triangle-weighted sums, each sub-structure
 *      enumerated once; the class-pair formulas of (2) then give the 13 local counts.
 *      Pinned against (1) and (2) on every graph the tests draw.
 *
 * Edge numbering (shared convention of the C interface, re-implemented here): edge k is
 * the k-th CSR entry (i, col[j]) with i < col[j] in row-major order.
 *
 * Per-edge output is 13 slots x m (slot-major), slots in graphlet order
 *   0:H3 triangle 1:H4 2-star 2:H5 3-node-1-edge 3:H7 4-clique 4:H8 chordal-cycle
 *   5:H9 tailed-triangle 6:H10 4-cycle 7:H11 3-star 8:H12 4-path 9:H13 4-node-1-triangle
 *   10:H14 4-node-2-edge 11:H15 4-node-2-star 12:H16 4-node-1-edge
 * Global output is 17 graphlets x (lo, hi) 64-bit words of an unsigned 128-bit count.
 */
#define _GNU_SOURCE   /* qsort_r */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_INEXACT -2   /* a division that must be exact was not: a bug */
#define ORC_E_NEGATIVE -3  /* a count came out negative: a bug */
#define ORC_E_NOMEM -4

/* ------------------------------------------------------------------------------------ */
/* small helpers                                                                         */
/* ------------------------------------------------------------------------------------ */

static i128 choose2(i128 x) { return x < 2 ? 0 : x * (x - 1) / 2; }
static i128 choose3(i128 x) { return x < 3 ? 0 : x * (x - 1) * (x - 2) / 6; }
static i128 choose4(i128 x) { return x < 4 ? 0 : x * (x - 1) * (x - 2) * (x - 3) / 24; }

static void put128(uint64_t* out, int i, i128 v) {
    u128 u = (u128)v;
    out[2 * i] = (uint64_t)u;
    out[2 * i + 1] = (uint64_t)(u >> 64);
}

/* edge list in the shared numbering */
static int64_t build_edges(int64_t n, const int64_t* rp, const int32_t* col,
                           int32_t* eu, int32_t* ev) {
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = rp[i]; j < rp[i + 1]; j++)
            if ((int64_t)col[j] > i) {
                if (eu) { eu[k] = (int32_t)i; ev[k] = col[j]; }
                k++;
            }
    return k;
}

/* ------------------------------------------------------------------------------------ */
/* (1) brute force from the definition                                                   */
/* ------------------------------------------------------------------------------------ */

/* Graphlet id (1-based, Table 1) of the induced subgraph on k vertices given its
 * adjacency bits.  Classification of 4-vertex graphs by edge count and sorted degree
 * sequence, which separates the 11 isomorphism classes. */
static int classify3(int e) {
    switch (e) { case 3: return 3; case 2: return 4; case 1: return 5; default: return 6; }
}

static int classify4(int e, int deg[4]) {
    int d[4] = {deg[0], deg[1], deg[2], deg[3]};
    for (int i = 1; i < 4; i++)
        for (int j = i; j > 0 && d[j - 1] > d[j]; j--) { int t = d[j]; d[j] = d[j - 1]; d[j - 1] = t; }
    switch (e) {
    case 6: return 7;
    case 5: return 8;
    case 4: return (d[0] == 2) ? 10 : 9;           /* (2,2,2,2) cycle, (1,2,2,3) tailed */
    case 3:
        if (d[0] == 0) return 13;                  /* triangle + isolated */
        if (d[3] == 3) return 11;                  /* star */
        return 12;                                 /* path */
    case 2: return (d[0] == 1) ? 14 : 15;          /* two disjoint edges, or wedge + K1 */
    case 1: return 16;
    default: return 17;
    }
}

static inline int adjbit(const uint8_t* A, int64_t n, int64_t a, int64_t b) { return A[a * n + b]; }

int brute_count(int64_t n, const int64_t* rp, const int32_t* col,
                uint64_t* X /* [17] */, uint64_t* per_edge /* [13*m] or NULL */) {
    if (n < 0 || n > 4096 || !rp || (!col && rp[n] > 0) || !X) return ORC_E_ARG;
    uint8_t* A = (uint8_t*)calloc((size_t)(n > 0 ? n * n : 1), 1);
    if (!A) return ORC_E_NOMEM;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = rp[i]; j < rp[i + 1]; j++) A[i * n + col[j]] = 1;
    uint64_t cnt[18] = {0};
    for (int64_t a = 0; a < n; a++)
        for (int64_t b = a + 1; b < n; b++) {
            cnt[adjbit(A, n, a, b) ? 1 : 2]++;
            for (int64_t c = b + 1; c < n; c++) {
                int e3 = adjbit(A, n, a, b) + adjbit(A, n, a, c) + adjbit(A, n, b, c);
                cnt[classify3(e3)]++;
                for (int64_t d = c + 1; d < n; d++) {
                    int64_t v[4] = {a, b, c, d};
                    int deg[4] = {0, 0, 0, 0}, e = 0;
                    for (int x = 0; x < 4; x++)
                        for (int y = x + 1; y < 4; y++)
                            if (adjbit(A, n, v[x], v[y])) { e++; deg[x]++; deg[y]++; }
                    cnt[classify4(e, deg)]++;
                }
            }
        }
    for (int i = 0; i < 17; i++) X[i] = cnt[i + 1];
    if (per_edge) {
        int64_t m = build_edges(n, rp, col, NULL, NULL);
        int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
        int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
        if (!eu || !ev) { free(A); free(eu); free(ev); return ORC_E_NOMEM; }
        build_edges(n, rp, col, eu, ev);
        /* graphlet id -> per-edge slot */
        static const int slot_of[18] = {-1, -1, -1, 0, 1, 2, -1, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, -1};
        memset(per_edge, 0, sizeof(uint64_t) * 13 * (size_t)m);
        for (int64_t k = 0; k < m; k++) {
            int64_t a = eu[k], b = ev[k];
            for (int64_t w = 0; w < n; w++) {
                if (w == a || w == b) continue;
                int e3 = 1 + adjbit(A, n, a, w) + adjbit(A, n, b, w);
                per_edge[(size_t)slot_of[classify3(e3)] * m + k]++;
                for (int64_t r = w + 1; r < n; r++) {
                    if (r == a || r == b) continue;
                    int64_t v[4] = {a, b, w, r};
                    int deg[4] = {0, 0, 0, 0}, e = 0;
                    for (int x = 0; x < 4; x++)
                        for (int y = x + 1; y < 4; y++)
                            if (adjbit(A, n, v[x], v[y])) { e++; deg[x]++; deg[y]++; }
                    per_edge[(size_t)slot_of[classify4(e, deg)] * m + k]++;
                }
            }
        }
        free(eu); free(ev);
    }
    free(A);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* (2) the paper's edge-centric method                                                   */
/* ------------------------------------------------------------------------------------ */

/* Preprocessing P1/P3 (Section 4.2): vertices are ordered by (degree, id) ascending; for
 * an edge the endpoint called v is the later one in that order, so d_v >= d_u.  The
 * order is only used to name the endpoints, so it is applied as a comparison rather than
 * a physical relabelling. */
static inline int ranks_above(const int64_t* deg, int64_t a, int64_t b) {
    return deg[a] > deg[b] || (deg[a] == deg[b] && a > b);
}

/* Per-vertex pre-pass: tri[x] = edges among N(x) (triangles at x), sdeg[x] = sum of the
 * degrees of x's neighbours.  Plain neighbour iteration with a mark array. */
static int vertex_terms(int64_t n, const int64_t* rp, const int32_t* col, const int64_t* deg,
                        const uint8_t* want, int64_t* tri, int64_t* sdeg, int nthreads) {
    int fail = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t* mark = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        if (!mark) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t x = 0; x < n; x++) {
            if (!mark || (want && !want[x])) continue;
            int64_t tag = x + 1;
            int64_t s = 0, c = 0;
            for (int64_t j = rp[x]; j < rp[x + 1]; j++) { mark[col[j]] = tag; s += deg[col[j]]; }
            for (int64_t j = rp[x]; j < rp[x + 1]; j++) {
                int64_t y = col[j];
                for (int64_t k = rp[y]; k < rp[y + 1]; k++)
                    if (mark[col[k]] == tag) c++;
            }
            tri[x] = c / 2;   /* every edge among N(x) was seen from both of its ends */
            sdeg[x] = s;
        }
        free(mark);
    }
    return fail ? ORC_E_NOMEM : ORC_OK;
}

typedef struct {
    int64_t t, su, sv, D;     /* |T|, |S_u|, |S_v|, vertices adjacent to neither */
    int64_t K;                /* edges inside T: 4-cliques on the edge  (X_{k,7})  */
    int64_t Q;                /* edges between S_u and S_v: 4-cycles     (X_{k,10}) */
    int64_t au, av;           /* edges T-S_u and T-S_v                             */
    int64_t sigT;             /* sum of degrees over T                             */
} edge_terms;

/* One edge neighbourhood: Alg. "3-Graphlets" builds T and S_u with the tags
 * lambda1 (neighbours of v), lambda2 (S_u) and lambda3 (T); Alg. "Clique" scans N(w) for
 * w in T (extended to also count tags lambda2 and lambda1, i.e. T-S_u and T-S_v edges),
 * Alg. "Cycle" scans N(w) for w in S_u counting neighbours still tagged lambda1 (S_v). */
static void edge_neighbourhood(int64_t u, int64_t v, const int64_t* rp, const int32_t* col,
                               const int64_t* deg, int64_t* psi, int64_t* Tbuf, int64_t* Sbuf,
                               int64_t serial, edge_terms* out) {
    const int64_t l1 = 3 * serial + 1, l2 = 3 * serial + 2, l3 = 3 * serial + 3;
    int64_t nt = 0, ns = 0;
    for (int64_t j = rp[v]; j < rp[v + 1]; j++)
        if (col[j] != u) psi[col[j]] = l1;
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
        int64_t w = col[j];
        if (w == v) continue;
        if (psi[w] == l1) { Tbuf[nt++] = w; psi[w] = l3; }
        else { Sbuf[ns++] = w; psi[w] = l2; }
    }
    int64_t twoK = 0, au = 0, av = 0, sig = 0, Q = 0;
    for (int64_t i = 0; i < nt; i++) {
        int64_t w = Tbuf[i];
        sig += deg[w];
        for (int64_t j = rp[w]; j < rp[w + 1]; j++) {
            int64_t tag = psi[col[j]];
            if (tag == l3) twoK++;
            else if (tag == l2) au++;
            else if (tag == l1) av++;
        }
    }
    for (int64_t i = 0; i < ns; i++) {
        int64_t w = Sbuf[i];
        for (int64_t j = rp[w]; j < rp[w + 1]; j++)
            if (psi[col[j]] == l1) Q++;
    }
    out->t = nt;
    out->su = ns;
    out->sv = deg[v] - 1 - nt;
    out->K = twoK / 2;
    out->Q = Q;
    out->au = au;
    out->av = av;
    out->sigT = sig;
}

/* The 13 local counts of an edge from its terms (class-pair edge counts, see header). */
static int local_counts(const edge_terms* e, int64_t n, int64_t m, int64_t du, int64_t dv,
                        int64_t tri_u, int64_t tri_v, int64_t sdeg_u, int64_t sdeg_v,
                        int64_t out[13]) {
    int64_t t = e->t, su = e->su, sv = e->sv, K = e->K, Q = e->Q, au = e->au, av = e->av;
    int64_t D = n - 2 - t - su - sv;
    int64_t Esu = tri_u - t - K - au;               /* edges inside S_u */
    int64_t Esv = tri_v - t - K - av;               /* edges inside S_v */
    int64_t ETD = e->sigT - 2 * t - 2 * K - au - av;
    int64_t sig_u = sdeg_u - dv - e->sigT;          /* sum of degrees over S_u */
    int64_t sig_v = sdeg_v - du - e->sigT;
    int64_t ESuD = sig_u - su - 2 * Esu - au - Q;
    int64_t ESvD = sig_v - sv - 2 * Esv - av - Q;
    int64_t EDD = m - 1 - 2 * t - su - sv -
                  (K + Esu + Esv + au + av + Q + ETD + ESuD + ESvD);
    out[0] = t;
    out[1] = su + sv;
    out[2] = D;
    out[3] = K;
    out[4] = (t * (t - 1) / 2 - K) + au + av;
    out[5] = (t * su - au) + (t * sv - av) + ETD + Esu + Esv;
    out[6] = Q;
    out[7] = (su * (su - 1) / 2 - Esu) + (sv * (sv - 1) / 2 - Esv);
    out[8] = (su * sv - Q) + ESuD + ESvD;
    out[9] = t * D - ETD;
    out[10] = EDD;
    out[11] = (su + sv) * D - ESuD - ESvD;
    out[12] = D * (D - 1) / 2 - EDD;
    if (D < 0 || Esu < 0 || Esv < 0 || ETD < 0 || ESuD < 0 || ESvD < 0 || EDD < 0)
        return ORC_E_NEGATIVE;
    for (int i = 0; i < 13; i++)
        if (out[i] < 0) return ORC_E_NEGATIVE;
    return ORC_OK;
}

/* Global frequencies from the unrestricted counts (Section 4.6). */
static int global_from_unrestricted(int64_t n, int64_t m, const i128 C[17], i128 X[18]) {
#define EXACT(num, den, dst) do { i128 _n = (num); if (_n % (den) != 0 || _n < 0) return ORC_E_INEXACT; dst = _n / (den); } while (0)
    X[1] = m;
    X[2] = choose2(n) - m;
    EXACT(C[3], 3, X[3]);
    EXACT(C[4], 2, X[4]);
    X[5] = C[5];
    X[6] = choose3(n) - X[3] - X[4] - X[5];
    EXACT(C[7], 6, X[7]);
    X[8] = C[8] - C[7];
    EXACT(C[9] - 4 * X[8], 2, X[9]);
    EXACT(C[10], 4, X[10]);
    EXACT(C[11] - X[9], 3, X[11]);
    X[12] = C[12] - C[10];
    EXACT(C[13] - X[9], 3, X[13]);
    EXACT(C[14] - 6 * X[7] - 4 * X[8] - 2 * X[9] - 4 * X[10] - 2 * X[12], 2, X[14]);
    EXACT(C[15] - 2 * X[12], 2, X[15]);
    X[16] = C[16] - 2 * X[14];
    i128 s = 0;
    for (int i = 7; i <= 16; i++) s += X[i];
    X[17] = choose4(n) - s;
    for (int i = 1; i <= 17; i++)
        if (X[i] < 0) return ORC_E_NEGATIVE;
    return ORC_OK;
#undef EXACT
}

/* Edge order Pi (Section 4.3): heaviest edges first, by d_u + d_v, ties by id, over the
 * caller's edges [k0, k1); workers take one edge at a time (chunk b = 1, the paper's CPU
 * setting). */
static int heaviest_first(const int32_t* eu, const int32_t* ev, const int64_t* deg,
                          int64_t k0, int64_t k1, int64_t* order) {
    int64_t maxkey = 0;
    for (int64_t k = k0; k < k1; k++) {
        int64_t key = deg[eu[k]] + deg[ev[k]];
        if (key > maxkey) maxkey = key;
    }
    int64_t* bucket = (int64_t*)calloc((size_t)(maxkey + 2), sizeof(int64_t));
    if (!bucket) return ORC_E_NOMEM;
    for (int64_t k = k0; k < k1; k++) bucket[maxkey - (deg[eu[k]] + deg[ev[k]])]++;
    int64_t acc = 0;
    for (int64_t b = 0; b <= maxkey; b++) { int64_t c = bucket[b]; bucket[b] = acc; acc += c; }
    for (int64_t k = k0; k < k1; k++) order[bucket[maxkey - (deg[eu[k]] + deg[ev[k]])]++] = k;
    free(bucket);
    return ORC_OK;
}

/* The edge-centric pass over the caller's edges [k0, k1) in the order Pi: per edge its
 * neighbourhood (Alg. "3-Graphlets", "Clique", "Cycle"), its 13 local counts (written to
 * per_edge[i * stride + k - k0] when per_edge is given) and its terms of the unrestricted
 * counts C3..C16 (Section 4.5), summed into Csum. */
static int edge_pass(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const int64_t* deg,
                     const int32_t* eu, const int32_t* ev, const int64_t* tri, const int64_t* sdeg,
                     int64_t k0, int64_t k1, int nthreads, i128 Csum[17], uint64_t* per_edge,
                     int64_t stride) {
    memset(Csum, 0, sizeof(i128) * 17);
    if (k1 <= k0) return ORC_OK;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k1 - k0));
    if (!order) return ORC_E_NOMEM;
    int rc = heaviest_first(eu, ev, deg, k0, k1, order);
    if (rc) { free(order); return rc; }
    int fail = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t* psi = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        int64_t* Tb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t* Sb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        i128 loc[17];
        memset(loc, 0, sizeof(loc));
        int64_t serial = 0;
        int lfail = (!psi || !Tb || !Sb) ? ORC_E_NOMEM : 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < k1 - k0; q++) {
            if (lfail) continue;
            int64_t k = order[q];
            int64_t a = eu[k], b = ev[k];
            int64_t v = ranks_above(deg, a, b) ? a : b;
            int64_t u = (v == a) ? b : a;
            edge_terms e;
            edge_neighbourhood(u, v, rp, col, deg, psi, Tb, Sb, serial++, &e);
            int64_t x[13];
            int r = local_counts(&e, n, m, deg[u], deg[v], tri[u], tri[v], sdeg[u], sdeg[v], x);
            if (r) { lfail = r; continue; }
            if (per_edge)
                for (int i = 0; i < 13; i++) per_edge[(size_t)i * stride + (k - k0)] = (uint64_t)x[i];
            /* unrestricted counts (Section 4.5) */
            i128 t = e.t, s = e.su + e.sv, D = x[2];
            loc[3] += t;
            loc[4] += s;
            loc[5] += D;
            loc[7] += e.K;
            loc[8] += choose2(t);
            loc[9] += t * s;
            loc[10] += e.Q;
            loc[11] += choose2(e.su) + choose2(e.sv);
            loc[12] += (i128)e.su * e.sv;
            loc[13] += t * D;
            loc[14] += (i128)(m - deg[u] - deg[v] + 1);
            loc[15] += s * D;
            loc[16] += choose2(D);
        }
#pragma omp critical
        {
            for (int i = 0; i < 17; i++) Csum[i] += loc[i];
            if (lfail) fail = lfail;
        }
        free(psi); free(Tb); free(Sb);
    }
    free(order);
    return fail;
}

/* Full count: global X1..X17 (as 17 x (lo,hi)), optional unrestricted sums C (index 3..16
 * meaningful, same layout), optional per-edge counts [13][m]. */
int glo_count(int64_t n, const int64_t* rp, const int32_t* col, int nthreads,
              uint64_t* Xout, uint64_t* Cout, uint64_t* per_edge) {
    if (n < 0 || !rp || !Xout || nthreads < 1) return ORC_E_ARG;
    int64_t m = build_edges(n, rp, col, NULL, NULL);
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* tri = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t* sdeg = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    int rc = ORC_OK;
    if (!eu || !ev || !deg || !tri || !sdeg) { rc = ORC_E_NOMEM; goto done; }
    build_edges(n, rp, col, eu, ev);
    for (int64_t x = 0; x < n; x++) deg[x] = rp[x + 1] - rp[x];
    rc = vertex_terms(n, rp, col, deg, NULL, tri, sdeg, nthreads);
    if (rc) goto done;
    {
        i128 Csum[17];
        rc = edge_pass(n, m, rp, col, deg, eu, ev, tri, sdeg, 0, m, nthreads, Csum, per_edge, m);
        if (rc) goto done;
        i128 X[18];
        rc = global_from_unrestricted(n, m, Csum, X);
        if (rc) goto done;
        for (int i = 0; i < 17; i++) put128(Xout, i, X[i + 1]);
        if (Cout)
            for (int i = 0; i < 17; i++) put128(Cout, i, Csum[i]);
    }
done:
    free(eu); free(ev); free(deg); free(tri); free(sdeg);
    return rc;
}

/* The same pass restricted to the caller's edges [k0, k1): their terms of the unrestricted
 * counts (C3..C16, as 17 x (lo,hi), index 3..16 meaningful; the sums over a partition of
 * [0, m) add up to glo_count's) and, when per_edge is given, their 13 local counts
 * ([13][k1 - k0], slot-major).  Lets a long run proceed block by block. */
int glo_count_range(int64_t n, const int64_t* rp, const int32_t* col, int nthreads,
                    int64_t k0, int64_t k1, uint64_t* Cout, uint64_t* per_edge) {
    if (n < 0 || !rp || !Cout || nthreads < 1) return ORC_E_ARG;
    int64_t m = build_edges(n, rp, col, NULL, NULL);
    if (k0 < 0 || k1 < k0 || k1 > m) return ORC_E_ARG;
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* tri = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t* sdeg = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    uint8_t* want = (uint8_t*)calloc((size_t)(n + 1), 1);
    int rc = ORC_OK;
    if (!eu || !ev || !deg || !tri || !sdeg || !want) { rc = ORC_E_NOMEM; goto done; }
    build_edges(n, rp, col, eu, ev);
    for (int64_t x = 0; x < n; x++) deg[x] = rp[x + 1] - rp[x];
    for (int64_t k = k0; k < k1; k++) { want[eu[k]] = 1; want[ev[k]] = 1; }
    rc = vertex_terms(n, rp, col, deg, want, tri, sdeg, nthreads);
    if (rc) goto done;
    {
        i128 Csum[17];
        rc = edge_pass(n, m, rp, col, deg, eu, ev, tri, sdeg, k0, k1, nthreads, Csum, per_edge, k1 - k0);
        if (rc) goto done;
        for (int i = 0; i < 17; i++) put128(Cout, i, Csum[i]);
    }
done:
    free(eu); free(ev); free(deg); free(tri); free(sdeg); free(want);
    return rc;
}

/* Global counts X1..X17 from unrestricted sums C (17 x (lo,hi) as glo_count_range returns
 * them, summed over a partition of the edges), Section 4.6. */
int glo_global_from_c(int64_t n, int64_t m, const uint64_t* Cin, uint64_t* Xout) {
    if (n < 0 || m < 0 || !Cin || !Xout) return ORC_E_ARG;
    i128 C[17], X[18];
    for (int i = 0; i < 17; i++) C[i] = (i128)(((u128)Cin[2 * i + 1] << 64) | (u128)Cin[2 * i]);
    int rc = global_from_unrestricted(n, m, C, X);
    if (rc) return rc;
    for (int i = 0; i < 17; i++) put128(Xout, i, X[i + 1]);
    return ORC_OK;
}

/* Per-edge counts for selected edges only (no global sums).  Vertex terms are computed
 * just for the endpoints involved, so this runs on graphs far too large for glo_count. */
int glo_count_edges(int64_t n, const int64_t* rp, const int32_t* col, int nthreads,
                    const int64_t* eids, int64_t k, uint64_t* out /* [13][k] */) {
    if (n < 0 || !rp || nthreads < 1 || (k > 0 && (!eids || !out))) return ORC_E_ARG;
    int64_t m = build_edges(n, rp, col, NULL, NULL);
    for (int64_t i = 0; i < k; i++)
        if (eids[i] < 0 || eids[i] >= m) return ORC_E_ARG;
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* tri = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t* sdeg = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    uint8_t* want = (uint8_t*)calloc((size_t)(n + 1), 1);
    int rc = ORC_OK;
    if (!eu || !ev || !deg || !tri || !sdeg || !want) { rc = ORC_E_NOMEM; goto done; }
    build_edges(n, rp, col, eu, ev);
    for (int64_t x = 0; x < n; x++) deg[x] = rp[x + 1] - rp[x];
    for (int64_t i = 0; i < k; i++) { want[eu[eids[i]]] = 1; want[ev[eids[i]]] = 1; }
    rc = vertex_terms(n, rp, col, deg, want, tri, sdeg, nthreads);
    if (rc) goto done;
    {
        int fail = 0;
#pragma omp parallel num_threads(nthreads)
        {
            int64_t* psi = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
            int64_t* Tb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
            int64_t* Sb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
            int64_t serial = 0;
            int lfail = (!psi || !Tb || !Sb) ? ORC_E_NOMEM : 0;
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < k; i++) {
                if (lfail) continue;
                int64_t a = eu[eids[i]], b = ev[eids[i]];
                int64_t v = ranks_above(deg, a, b) ? a : b;
                int64_t u = (v == a) ? b : a;
                edge_terms e;
                edge_neighbourhood(u, v, rp, col, deg, psi, Tb, Sb, serial++, &e);
                int64_t x[13];
                int r = local_counts(&e, n, m, deg[u], deg[v], tri[u], tri[v], sdeg[u], sdeg[v], x);
                if (r) { lfail = r; continue; }
                for (int s = 0; s < 13; s++) out[(size_t)s * k + i] = (uint64_t)x[s];
            }
#pragma omp critical
            { if (lfail) fail = lfail; }
            free(psi); free(Tb); free(Sb);
        }
        rc = fail;
    }
done:
    free(eu); free(ev); free(deg); free(tri); free(sdeg); free(want);
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* (3) global counts from three plainly defined sub-counts, for graphs too large for (2)  */
/* ------------------------------------------------------------------------------------ */
/*
 * Every count of Sections 4.5-4.6 follows from the triangles on each edge, the number of
 * 4-cliques and the number of (not necessarily induced) 4-cycles, besides n, m and the
 * degrees:
 *   - t_e = |N(u) & N(v)|, the triangles on edge e = (u, v), by definition;
 *   - a 4-clique has one lowest vertex a in the order of P1 (degree, then id), and its other
 *     three vertices form a triangle among the neighbours of a ranked above a;
 *   - a 4-cycle has one lowest vertex y; its opposite vertex x and both middle vertices rank
 *     above y, so with c(y, x) = the common neighbours of y and x ranked above y, the
 *     4-cycles number the sum over pairs y < x (in rank) of C(c(y, x), 2).
 * Per edge, s_u = d_u - 1 - t, s_v = d_v - 1 - t and D = n - 2 - t - s_u - s_v give every
 * unrestricted count except C7 and C10; C7 = 6 #K4 (each 4-clique holds 6 edges, each with
 * the other two vertices in T and adjacent), X8 = C8 - C7 (Section 4.6), and since an
 * induced 4-cycle holds one 4-cycle, a chordal cycle one and a 4-clique three,
 * X10 = #C4 - X8 - 3 X7 and C10 = 4 X10.  The rest is Section 4.6 as in (2).
 * per_edge3, when given, receives the three per-edge counts of Section 4.5 that depend on
 * t and the degrees alone: [0] triangles (H3) t, [1] 2-stars (H4) s_u + s_v, [2] H5 = D,
 * slot-major [3][m] in the shared numbering.  work, when given, receives #K4 and #C4 as two
 * (lo, hi) pairs.
 */
static int rank_less(const int64_t* deg, int64_t a, int64_t b) { return ranks_above(deg, b, a); }

int glo_global_substructures(int64_t n, const int64_t* rp, const int32_t* col, int nthreads,
                             uint64_t* Xout, uint64_t* per_edge3, uint64_t* work) {
    if (n < 0 || !rp || !Xout || nthreads < 1) return ORC_E_ARG;
    int64_t m = build_edges(n, rp, col, NULL, NULL);
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* hstart = (int64_t*)calloc((size_t)(n + 2), sizeof(int64_t));   /* edges by higher end */
    int64_t* hedge = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t* ustart = (int64_t*)calloc((size_t)(n + 2), sizeof(int64_t));   /* upward neighbours */
    int32_t* up = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    uint32_t* tcnt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m + 1));
    int rc = ORC_OK;
    if (!eu || !ev || !deg || !hstart || !hedge || !ustart || !up || !tcnt) { rc = ORC_E_NOMEM; goto done; }
    build_edges(n, rp, col, eu, ev);
    for (int64_t x = 0; x < n; x++) deg[x] = rp[x + 1] - rp[x];
    /* each edge listed at its higher-ranked endpoint; N+(x) = neighbours ranked above x */
    for (int64_t k = 0; k < m; k++) {
        int64_t hi = ranks_above(deg, eu[k], ev[k]) ? eu[k] : ev[k];
        int64_t lo = (hi == eu[k]) ? ev[k] : eu[k];
        hstart[hi + 1]++;
        ustart[lo + 1]++;
    }
    for (int64_t x = 0; x < n; x++) { hstart[x + 1] += hstart[x]; ustart[x + 1] += ustart[x]; }
    {
        int64_t* fh = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t* fu = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        if (!fh || !fu) { free(fh); free(fu); rc = ORC_E_NOMEM; goto done; }
        memcpy(fh, hstart, sizeof(int64_t) * (size_t)n);
        memcpy(fu, ustart, sizeof(int64_t) * (size_t)n);
        for (int64_t k = 0; k < m; k++) {
            int64_t hi = ranks_above(deg, eu[k], ev[k]) ? eu[k] : ev[k];
            int64_t lo = (hi == eu[k]) ? ev[k] : eu[k];
            hedge[fh[hi]++] = k;
            up[fu[lo]++] = (int32_t)hi;
        }
        free(fh); free(fu);
    }
    i128 k4 = 0, c4 = 0;
    int fail = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t* mark = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t* mark2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        uint32_t* cnt = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
        int32_t* L = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
        i128 lk4 = 0, lc4 = 0;
        int lfail = (!mark || !mark2 || !cnt || !touched || !L) ? ORC_E_NOMEM : 0;
        if (!lfail)
            for (int64_t x = 0; x < n; x++) { mark[x] = -1; mark2[x] = -1; }
        int64_t serial = 0;
        /* triangles on every edge: N(v) marked once per higher endpoint v, N(u) probed */
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; v++) {
            if (lfail || hstart[v] == hstart[v + 1]) continue;
            for (int64_t j = rp[v]; j < rp[v + 1]; j++) mark[col[j]] = v;
            for (int64_t q = hstart[v]; q < hstart[v + 1]; q++) {
                int64_t k = hedge[q];
                int64_t u = (eu[k] == v) ? ev[k] : eu[k];
                uint32_t c = 0;
                for (int64_t j = rp[u]; j < rp[u + 1]; j++) c += (mark[col[j]] == v);
                tcnt[k] = c;
            }
        }
        /* 4-cliques at their lowest vertex a: triangles b < c < d inside N+(a) */
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < n; a++) {
            if (lfail) continue;
            for (int64_t j = ustart[a]; j < ustart[a + 1]; j++) mark[up[j]] = n + a;
            for (int64_t j = ustart[a]; j < ustart[a + 1]; j++) {
                int64_t b = up[j];
                int64_t nl = 0;
                serial++;
                for (int64_t q = ustart[b]; q < ustart[b + 1]; q++)
                    if (mark[up[q]] == n + a) { L[nl++] = up[q]; mark2[up[q]] = serial; }
                for (int64_t i = 0; i < nl; i++) {
                    int64_t c = L[i];
                    for (int64_t q = ustart[c]; q < ustart[c + 1]; q++) lk4 += (mark2[up[q]] == serial);
                }
            }
        }
        /* 4-cycles at their lowest vertex y: wedges y - w - x with w and x ranked above y */
#pragma omp for schedule(dynamic, 64)
        for (int64_t y = 0; y < n; y++) {
            if (lfail) continue;
            int64_t nt = 0;
            for (int64_t j = ustart[y]; j < ustart[y + 1]; j++) {
                int64_t w = up[j];
                for (int64_t q = rp[w]; q < rp[w + 1]; q++) {
                    int64_t x = col[q];
                    if (x == y || !rank_less(deg, y, x)) continue;
                    if (cnt[x]++ == 0) touched[nt++] = (int32_t)x;
                }
            }
            for (int64_t i = 0; i < nt; i++) { lc4 += choose2(cnt[touched[i]]); cnt[touched[i]] = 0; }
        }
#pragma omp critical
        {
            k4 += lk4;
            c4 += lc4;
            if (lfail) fail = lfail;
        }
        free(mark); free(mark2); free(cnt); free(touched); free(L);
    }
    if (fail) { rc = fail; goto done; }
    {
        i128 C[17], X[18];
        memset(C, 0, sizeof(C));
        for (int64_t k = 0; k < m; k++) {
            const int64_t du = deg[eu[k]], dv = deg[ev[k]];
            const i128 t = tcnt[k], su = du - 1 - (int64_t)tcnt[k], sv = dv - 1 - (int64_t)tcnt[k];
            const i128 D = (i128)n - 2 - t - su - sv;
            if (su < 0 || sv < 0 || D < 0) { rc = ORC_E_NEGATIVE; goto done; }
            C[3] += t;
            C[4] += su + sv;
            C[5] += D;
            C[8] += choose2(t);
            C[9] += t * (su + sv);
            C[11] += choose2(su) + choose2(sv);
            C[12] += su * sv;
            C[13] += t * D;
            C[14] += (i128)(m - du - dv + 1);
            C[15] += (su + sv) * D;
            C[16] += choose2(D);
            if (per_edge3) {
                per_edge3[k] = (uint64_t)t;
                per_edge3[(size_t)m + k] = (uint64_t)(su + sv);
                per_edge3[2 * (size_t)m + k] = (uint64_t)D;
            }
        }
        C[7] = 6 * k4;
        const i128 x8 = C[8] - C[7];
        const i128 x10 = c4 - x8 - 3 * k4;
        if (x8 < 0 || x10 < 0) { rc = ORC_E_NEGATIVE; goto done; }
        C[10] = 4 * x10;
        rc = global_from_unrestricted(n, m, C, X);
        if (rc) goto done;
        for (int i = 0; i < 17; i++) put128(Xout, i, X[i + 1]);
        if (work) {
            put128(work, 0, k4);
            put128(work, 1, c4);
        }
    }
done:
    free(eu); free(ev); free(deg); free(hstart); free(hedge); free(ustart); free(up); free(tcnt);
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* (4) per-edge counts from plainly defined per-edge sub-counts, for graphs too large     */
/*     for (2)                                                                            */
/* ------------------------------------------------------------------------------------ */
/*
 * The terms that (2) obtains per edge e = (u, v) by tag scans (Section 4.5) are counts with
 * plain definitions, and each can be gathered from sub-structures enumerated once each:
 *   t      = |N(u) & N(v)|, by definition (marks of N(v), probes of N(u));
 *   K      = the 4-cliques that contain e: every 4-clique is enumerated once at its lowest
 *            vertex in the order of P1 and credited to its six edges;
 *   P      = the 4-cycles (not necessarily induced) that contain e: every 4-cycle is
 *            enumerated once at its lowest vertex y, as two middles w, w' that are both
 *            adjacent to y and to the opposite vertex x, and credited to its four edges;
 *   gu, gv = sums over w in T of t(w, u) and of t(w, v): every triangle is enumerated once
 *            and credits each of its edges with the triangle counts of its other two edges;
 *   sigT   = the sum of d_w over w in T: every triangle credits each of its edges with the
 *            degree of its third vertex.
 * The tag counts of (2) follow from these: for w in T, N(w) & N(u) holds v, the neighbours
 * of w inside T and those inside S_u, so gu = t + 2K + a_u (likewise gv with S_v); a 4-cycle
 * through e is a path u - r - w - v whose middle pair (r, w) is an ordered adjacent pair of
 * T (2K of them), a T-S_v or S_u-T pair (a_v + a_u), or an S_u-S_v pair (Q), so
 * P = 2K + a_u + a_v + Q.  The 13 local counts, the unrestricted sums and X1..X17 then
 * come from the same class-pair formulas as (2) (local_counts, Sections 4.5-4.6).
 * Pinned against (1) and (2) on every graph the tests draw.
 *
 * Neighbour lists are copied in descending P1 rank (Section 4.2, P2) so that the wedge
 * scans stop at the first vertex not ranked above y.  per_edge receives [13][m] (slot-
 * major, shared numbering), Xout 17 x (lo, hi), work #K4 and #C4 as two (lo, hi) pairs.
 */
typedef struct { int32_t v; int64_t e; } nbr_entry;

/* qsort_r comparator: neighbours in descending P1 rank */
static int by_rank_desc(const void* pa, const void* pb, void* ctx) {
    const int64_t* deg = (const int64_t*)ctx;
    const int64_t a = ((const nbr_entry*)pa)->v, b = ((const nbr_entry*)pb)->v;
    if (a == b) return 0;
    return ranks_above(deg, a, b) ? -1 : 1;
}

#define ADD(arr, k, val) __atomic_fetch_add(&(arr)[k], (val), __ATOMIC_RELAXED)

int glo_per_edge_substructures(int64_t n, const int64_t* rp, const int32_t* col, int nthreads,
                               uint64_t* Xout, uint64_t* per_edge, uint64_t* work) {
    if (n < 0 || !rp || !Xout || nthreads < 1) return ORC_E_ARG;
    const int64_t m = build_edges(n, rp, col, NULL, NULL);
    const int64_t nn = n > 0 ? n : 1, mm = m > 0 ? m : 1;
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)mm);
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)mm);
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)nn);
    int64_t* seid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * mm));   /* CSR slot -> edge */
    int32_t* rcol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * mm));   /* rows, rank-descending */
    int64_t* reid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * mm));
    int64_t* nup = (int64_t*)calloc((size_t)nn, sizeof(int64_t));           /* |N+(x)| */
    int64_t* tE = (int64_t*)calloc((size_t)mm, sizeof(int64_t));
    int64_t* KE = (int64_t*)calloc((size_t)mm, sizeof(int64_t));
    int64_t* PE = (int64_t*)calloc((size_t)mm, sizeof(int64_t));
    int64_t* guE = (int64_t*)calloc((size_t)mm, sizeof(int64_t));
    int64_t* gvE = (int64_t*)calloc((size_t)mm, sizeof(int64_t));
    int64_t* sgE = (int64_t*)calloc((size_t)mm, sizeof(int64_t));
    int64_t* tri = (int64_t*)calloc((size_t)nn, sizeof(int64_t));
    int64_t* sdeg = (int64_t*)calloc((size_t)nn, sizeof(int64_t));
    int rc = ORC_OK;
    i128 k4 = 0, c4 = 0;
    if (!eu || !ev || !deg || !seid || !rcol || !reid || !nup || !tE || !KE || !PE || !guE ||
        !gvE || !sgE || !tri || !sdeg) { rc = ORC_E_NOMEM; goto done; }
    build_edges(n, rp, col, eu, ev);
    for (int64_t x = 0; x < n; x++) deg[x] = rp[x + 1] - rp[x];
    /* slot -> edge id: the edge (i, j), i < j, is numbered in row i; row j finds it there */
    {
        int64_t k = 0;
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = rp[i]; j < rp[i + 1]; j++)
                if ((int64_t)col[j] > i) seid[j] = k++;
        int fail = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = rp[i]; j < rp[i + 1]; j++) {
                int64_t o = col[j];
                if (o > i) continue;
                int64_t f = -1;
                for (int64_t q = rp[o]; q < rp[o + 1]; q++)   /* row o holds i once */
                    if (col[q] == i) { f = seid[q]; break; }
                if (f < 0) {
#pragma omp atomic write
                    fail = 1;
                }
                seid[j] = f;
            }
        if (fail) { rc = ORC_E_ARG; goto done; }   /* not symmetric */
    }
    /* rank-descending copy of every row; N+(x) is its prefix of vertices ranked above x */
    {
        int64_t dmax = 0;
        for (int64_t x = 0; x < n; x++) dmax = deg[x] > dmax ? deg[x] : dmax;
        int fail = 0;
#pragma omp parallel num_threads(nthreads)
        {
            nbr_entry* tmp = (nbr_entry*)malloc(sizeof(nbr_entry) * (size_t)(dmax + 1));
            if (!tmp) {
#pragma omp atomic write
                fail = 1;
            }
#pragma omp for schedule(dynamic, 256)
            for (int64_t x = 0; x < n; x++) {
                if (!tmp) continue;
                const int64_t b = rp[x], len = rp[x + 1] - rp[x];
                for (int64_t j = 0; j < len; j++) { tmp[j].v = col[b + j]; tmp[j].e = seid[b + j]; }
                qsort_r(tmp, (size_t)len, sizeof(nbr_entry), by_rank_desc, (void*)deg);
                int64_t c = 0;
                for (int64_t j = 0; j < len; j++) { rcol[b + j] = tmp[j].v; reid[b + j] = tmp[j].e; }
                while (c < len && ranks_above(deg, rcol[b + c], x)) c++;
                nup[x] = c;
            }
            free(tmp);
        }
        if (fail) { rc = ORC_E_NOMEM; goto done; }
    }
    int fail = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t* mark = (int64_t*)malloc(sizeof(int64_t) * (size_t)nn);
        int64_t* markE = (int64_t*)malloc(sizeof(int64_t) * (size_t)nn);
        int64_t* mark2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)nn);
        int64_t* mark2E = (int64_t*)malloc(sizeof(int64_t) * (size_t)nn);
        int64_t* cnt = (int64_t*)calloc((size_t)nn, sizeof(int64_t));
        int64_t* accA = (int64_t*)calloc((size_t)nn, sizeof(int64_t));
        int64_t* accB = (int64_t*)calloc((size_t)nn, sizeof(int64_t));
        int32_t* L = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
        int64_t* LE = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        i128 lk4 = 0, lc4 = 0;
        int lfail = (!mark || !markE || !mark2 || !mark2E || !cnt || !accA || !accB || !L || !LE)
                        ? ORC_E_NOMEM : 0;
        if (!lfail)
            for (int64_t x = 0; x < n; x++) { mark[x] = -1; mark2[x] = -1; }
        /* triangles on every edge, t = |N(u) & N(v)|: N(x) marked once, every edge (x, y)
         * with y ranked below x probed through N(y) */
#pragma omp for schedule(dynamic, 64)
        for (int64_t x = 0; x < n; x++) {
            if (lfail) continue;
            for (int64_t j = rp[x]; j < rp[x + 1]; j++) mark[col[j]] = x;
            for (int64_t j = rp[x]; j < rp[x + 1]; j++) {
                int64_t y = col[j];
                if (!ranks_above(deg, x, y)) continue;
                int64_t c = 0;
                for (int64_t q = rp[y]; q < rp[y + 1]; q++) c += (mark[col[q]] == x);
                tE[seid[j]] = c;
            }
        }
        /* per vertex: triangles at x (= half the sum of t over its edges) and the sum of its
         * neighbours' degrees */
#pragma omp for schedule(dynamic, 256)
        for (int64_t x = 0; x < n; x++) {
            int64_t s = 0, c = 0;
            for (int64_t j = rp[x]; j < rp[x + 1]; j++) { s += deg[col[j]]; c += tE[seid[j]]; }
            sdeg[x] = s;
            tri[x] = c / 2;
        }
        /* triangles {a, b, c} and 4-cliques {a, b, c, d}, a < b < c < d in rank, at their lowest
         * vertex a */
#pragma omp for schedule(dynamic, 16)
        for (int64_t a = 0; a < n; a++) {
            if (lfail) continue;
            const int64_t ba = rp[a];
            for (int64_t j = 0; j < nup[a]; j++) { mark[rcol[ba + j]] = n + a; markE[rcol[ba + j]] = reid[ba + j]; }
            for (int64_t j = 0; j < nup[a]; j++) {
                const int64_t b = rcol[ba + j], eab = reid[ba + j], bb = rp[b];
                int64_t nl = 0;
                for (int64_t q = 0; q < nup[b]; q++) {
                    const int64_t c = rcol[bb + q];
                    if (mark[c] != n + a) continue;
                    L[nl] = (int32_t)c;
                    LE[nl++] = reid[bb + q];
                    mark2[c] = n + b;   /* c is above b and in N+(a) */
                    mark2E[c] = reid[bb + q];
                }
                int64_t kab = 0;
                for (int64_t i = 0; i < nl; i++) {
                    const int64_t c = L[i], ebc = LE[i], eac = markE[c], bc0 = rp[c];
                    /* triangle {a, b, c}: gather credits (edge ab's u-side endpoint is a) */
                    const int64_t tab = tE[eab], tac = tE[eac], tbc = tE[ebc];
                    ADD(guE, eab, tac); ADD(gvE, eab, tbc); ADD(sgE, eab, deg[c]);
                    ADD(guE, eac, tab); ADD(gvE, eac, tbc); ADD(sgE, eac, deg[b]);
                    ADD(guE, ebc, tab); ADD(gvE, ebc, tac); ADD(sgE, ebc, deg[a]);
                    /* 4-cliques {a, b, c, d}, d above c, adjacent to a and b; each credits
                     * its six edges: ab, ac, ad summed per vertex over a's iteration (accA),
                     * bc, bd over b's (accB), cd directly */
                    int64_t kc = 0;
                    for (int64_t q = 0; q < nup[c]; q++) {
                        const int64_t d = rcol[bc0 + q];
                        if (mark2[d] != n + b) continue;
                        kc++;
                        accA[d]++;
                        accB[d]++;
                        ADD(KE, reid[bc0 + q], 1);
                    }
                    kab += kc;
                    accA[c] += kc;
                    accB[c] += kc;
                }
                lk4 += kab;
                if (kab) ADD(KE, eab, kab);
                for (int64_t i = 0; i < nl; i++) {
                    const int64_t c = L[i];
                    if (accB[c]) ADD(KE, mark2E[c], accB[c]);
                    accB[c] = 0;
                    mark2[c] = -1;
                }
            }
            for (int64_t j = 0; j < nup[a]; j++) {
                const int64_t x = rcol[ba + j];
                if (accA[x]) ADD(KE, markE[x], accA[x]);
                accA[x] = 0;
            }
        }
        /* 4-cycles at their lowest vertex y: middles w (above y, adjacent to y), opposite
         * x (above y, adjacent to w); c(y, x) middles give C(c, 2) cycles, and each of the
         * edges (y, w), (w, x) lies on c - 1 of them */
#pragma omp for schedule(dynamic, 16)
        for (int64_t y = 0; y < n; y++) {
            if (lfail) continue;
            const int64_t by = rp[y];
            for (int pass = 0; pass < 3; pass++)
                for (int64_t j = 0; j < nup[y]; j++) {
                    const int64_t w = rcol[by + j], eyw = reid[by + j], bw = rp[w];
                    int64_t credit = 0;
                    for (int64_t q = 0; q < deg[w] && ranks_above(deg, rcol[bw + q], y); q++) {
                        const int64_t x = rcol[bw + q];
                        if (pass == 0) cnt[x]++;
                        else if (pass == 1) {
                            ADD(PE, reid[bw + q], cnt[x] - 1);
                            credit += cnt[x] - 1;
                        } else if (cnt[x] > 0) {
                            lc4 += choose2(cnt[x]);
                            cnt[x] = 0;
                        }
                    }
                    if (pass == 1) ADD(PE, eyw, credit);
                }
        }
#pragma omp critical
        {
            k4 += lk4;
            c4 += lc4;
            if (lfail) fail = lfail;
        }
        free(mark); free(markE); free(mark2); free(mark2E); free(cnt); free(accA); free(accB);
        free(L); free(LE);
    }
    if (fail) { rc = fail; goto done; }
    {
        i128 C[17];
        memset(C, 0, sizeof(C));
        for (int64_t k = 0; k < m; k++) {
            const int64_t a = eu[k], b = ev[k];
            const int64_t v = ranks_above(deg, a, b) ? a : b, u = (v == a) ? b : a;
            /* the enumeration credited g to each edge's lower endpoint as gu */
            edge_terms e;
            e.t = tE[k];
            e.su = deg[u] - 1 - e.t;
            e.sv = deg[v] - 1 - e.t;
            e.K = KE[k];
            e.au = guE[k] - e.t - 2 * e.K;
            e.av = gvE[k] - e.t - 2 * e.K;
            e.Q = PE[k] - 2 * e.K - e.au - e.av;
            e.sigT = sgE[k];
            if (e.su < 0 || e.sv < 0 || e.au < 0 || e.av < 0 || e.Q < 0) { rc = ORC_E_NEGATIVE; goto done; }
            int64_t x[13];
            rc = local_counts(&e, n, m, deg[u], deg[v], tri[u], tri[v], sdeg[u], sdeg[v], x);
            if (rc) goto done;
            if (per_edge)
                for (int i = 0; i < 13; i++) per_edge[(size_t)i * m + k] = (uint64_t)x[i];
            i128 t = e.t, s = e.su + e.sv, D = x[2];
            C[3] += t;
            C[4] += s;
            C[5] += D;
            C[7] += e.K;
            C[8] += choose2(t);
            C[9] += t * s;
            C[10] += e.Q;
            C[11] += choose2(e.su) + choose2(e.sv);
            C[12] += (i128)e.su * e.sv;
            C[13] += t * D;
            C[14] += (i128)(m - deg[u] - deg[v] + 1);
            C[15] += s * D;
            C[16] += choose2(D);
        }
        /* each 4-clique has six edges, each 4-cycle four */
        if (C[7] != 6 * k4) { rc = ORC_E_INEXACT; goto done; }
        {
            i128 sp = 0;
            for (int64_t k = 0; k < m; k++) sp += PE[k];
            if (sp != 4 * c4) { rc = ORC_E_INEXACT; goto done; }
        }
        i128 X[18];
        rc = global_from_unrestricted(n, m, C, X);
        if (rc) goto done;
        for (int i = 0; i < 17; i++) put128(Xout, i, X[i + 1]);
        if (work) {
            put128(work, 0, k4);
            put128(work, 1, c4);
        }
    }
done:
    free(eu); free(ev); free(deg); free(seid); free(rcol); free(reid); free(nup); free(tE); free(KE);
    free(PE); free(guE); free(gvE); free(sgE); free(tri); free(sdeg);
    return rc;
}
#undef ADD
