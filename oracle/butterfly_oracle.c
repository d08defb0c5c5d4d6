/*
 * Butterfly ORACLE — test infrastructure only (same rules as ktruss_oracle.c:
 * plain single-threaded C99, no code shared with the GPU library; only tests,
 * the smoke check and the benchmark's CPU baseline may load it).
 *
 * The paper's closing section names butterfly counting on bipartite graphs as
 * another motif-counting problem its fine-grained decomposition may serve.
 * A bipartite graph has sides U (nu vertices) and V (nv vertices) and edges
 * between them, given as CSR rows over U with ascending, distinct columns in
 * [0, nv).  A butterfly is a 4-cycle u1 - v1 - u2 - v2 with u1 != u2 in U and
 * v1 != v2 in V (a complete 2x2 biclique).  Outputs:
 *   count[e]  the butterflies containing edge e (CSR position), and
 *   total     the butterflies of the graph.
 *
 * Written from the definition: two distinct U vertices u1, u2 with c common
 * neighbours span C(c, 2) butterflies (one per pair of common neighbours),
 * and each edge (u1, v) or (u2, v) with v common lies in c - 1 of them.  The
 * oracle visits every pair u1 < u2 that shares a neighbour (found through
 * the V-side lists), intersects the two sorted rows, and adds these numbers.
 */
#include <stdint.h>
#include <stdlib.h>

#define ORC_OK 0
#define ORC_INVALID (-1)
#define ORC_NOMEM (-5)

static int check_bipartite(int32_t nu, int32_t nv, const int32_t* rowptr, const int32_t* col) {
    if (nu < 0 || nv < 0 || !rowptr || rowptr[0] != 0) return ORC_INVALID;
    for (int32_t u = 0; u < nu; ++u) {
        if (rowptr[u + 1] < rowptr[u]) return ORC_INVALID;
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            if (col[e] < 0 || col[e] >= nv) return ORC_INVALID;
            if (e > rowptr[u] && col[e] <= col[e - 1]) return ORC_INVALID;
        }
    }
    return ORC_OK;
}

int orc_butterflies(int32_t nu, int32_t nv, const int32_t* rowptr, const int32_t* col, int64_t* count,
                    int64_t* total) {
    if (check_bipartite(nu, nv, rowptr, col) != ORC_OK || !total) return ORC_INVALID;
    const int64_t m = rowptr[nu];
    if (m > 0 && !count) return ORC_INVALID;
    /* V-side lists: for every v the U vertices adjacent to it */
    int64_t* voff = (int64_t*)calloc((size_t)nv + 1, sizeof(int64_t));
    int32_t* vadj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nv + 1));
    int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nu + 1));
    int32_t* pairs = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nu + 1));
    if (!voff || !vadj || !fill || !seen || !pairs) {
        free(voff); free(vadj); free(fill); free(seen); free(pairs);
        return ORC_NOMEM;
    }
    for (int64_t e = 0; e < m; ++e) voff[col[e] + 1]++;
    for (int32_t v = 0; v < nv; ++v) voff[v + 1] += voff[v];
    for (int32_t v = 0; v <= nv; ++v) fill[v] = voff[v];
    for (int32_t u = 0; u < nu; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) vadj[fill[col[e]]++] = u;
    for (int32_t u = 0; u < nu; ++u) seen[u] = -1;
    for (int64_t e = 0; e < m; ++e) count[e] = 0;
    int64_t tot = 0;
    for (int32_t u1 = 0; u1 < nu; ++u1) {
        /* every u2 > u1 sharing a neighbour with u1, once */
        int32_t np = 0;
        for (int64_t e = rowptr[u1]; e < rowptr[u1 + 1]; ++e) {
            const int32_t v = col[e];
            for (int64_t k = voff[v]; k < voff[v + 1]; ++k) {
                const int32_t u2 = vadj[k];
                if (u2 > u1 && seen[u2] != u1) {
                    seen[u2] = u1;
                    pairs[np++] = u2;
                }
            }
        }
        for (int32_t k = 0; k < np; ++k) {
            const int32_t u2 = pairs[k];
            /* c = common neighbours of u1 and u2 (merge of two sorted rows) */
            int64_t c = 0;
            int64_t a = rowptr[u1], ae = rowptr[u1 + 1], b = rowptr[u2], be = rowptr[u2 + 1];
            while (a < ae && b < be) {
                if (col[a] < col[b]) ++a;
                else if (col[b] < col[a]) ++b;
                else { ++c; ++a; ++b; }
            }
            if (c < 2) continue;
            tot += c * (c - 1) / 2;
            a = rowptr[u1]; b = rowptr[u2];
            while (a < ae && b < be) {
                if (col[a] < col[b]) ++a;
                else if (col[b] < col[a]) ++b;
                else { count[a] += c - 1; count[b] += c - 1; ++a; ++b; }
            }
        }
    }
    *total = tot;
    free(voff); free(vadj); free(fill); free(seen); free(pairs);
    return ORC_OK;
}
