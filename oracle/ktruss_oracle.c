/*
 * K-truss ORACLE — test infrastructure only.
 *
 * A plain, slow, single-threaded C99 implementation of what the GPU library
 * computes, written from the paper (Blanco, Low, Kim, "Exploration of
 * Fine-Grained Parallelism for Load Balancing Eager K-truss on GPU and CPU",
 * HPEC 2019).  It shares no code, header or table with the library under
 * paper_2009_07929_amd/; only tests, the smoke check and the benchmark's CPU
 * baseline may load it.  No SIMD intrinsics, no threads.
 *
 * What is computed (Section I; Section II-A, Algorithm 1):
 *   The K-truss is the largest edge set in which every edge lies in at least
 *   K-2 triangles whose three edges are all in the set.  Algorithm 1 reaches
 *   it by repeating  S <- (A^T A) o A ;  M <- S >= K-2 ;  A <- A o M  until M
 *   no longer changes, and returns S (which is then the support inside the
 *   truss; removed edges carry 0).
 *
 * Two independent modes:
 *   mode R (orc_truss_recompute): Algorithm 1 written out: every pass
 *     recomputes every alive edge's support as |N(u) ∩ N(v)| over the alive
 *     subgraph, then removes the edges below K-2.
 *   mode P (orc_truss_peel): triangles are enumerated once, then each pass
 *     removes the edges below K-2 one at a time and decrements the supports of
 *     the other two edges of every triangle that removal destroys.  The passes
 *     are level-synchronous, so the pass count equals mode R's.
 *
 * Readings of the paper used here:
 *   - keep S >= K-2, drop S < K-2 (Algorithm 1, the mask line);
 *   - the pass count includes the final pass that removes nothing; an empty
 *     graph or K <= 2 takes one pass;
 *   - supports of removed edges are 0, survivors carry their support in the
 *     final truss (Algorithm 1 returns S after the last pass);
 *   - input preparation (Section IV-A only says the graphs are made
 *     upper-triangular): drop self-loops and duplicate pairs, treat pairs as
 *     undirected, relabel vertices by ascending degree with ties broken by
 *     the original id, and store the upper triangle (column > row) as CSR
 *     with ascending columns.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_INVALID (-1)
#define ORC_CAPACITY (-3)
#define ORC_NOMEM (-5)

/* ------------------------------------------------------------------ helpers */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

typedef struct { int64_t key; int32_t id; } vkey;

static int cmp_vkey(const void* a, const void* b) {
    const vkey* x = (const vkey*)a;
    const vkey* y = (const vkey*)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->id > y->id) - (x->id < y->id);
}

/* ------------------------------------------------------ canonical CSR input */

/*
 * Canonicalise raw pairs into the upper-triangular CSR the method works on.
 * order: 0 keeps ids, 1 relabels by ascending degree, 2 by descending degree
 * (ties by original id).  new_to_old (may be NULL) receives the relabelling.
 * col must hold `cap` entries; npairs always suffices.
 */
int orc_canonical_csr(const int32_t* src, const int32_t* dst, int64_t npairs, int32_t n,
                      int32_t order, int32_t* rowptr, int32_t* col, int64_t cap,
                      int32_t* new_to_old, int64_t* m_out) {
    if (n < 0 || npairs < 0 || order < 0 || order > 2 || !rowptr || !m_out) return ORC_INVALID;
    if (npairs > 0 && (!src || !dst || !col)) return ORC_INVALID;
    for (int64_t k = 0; k < npairs; ++k)
        if (src[k] < 0 || src[k] >= n || dst[k] < 0 || dst[k] >= n) return ORC_INVALID;

    /* 1. undirected, loop-free, duplicate-free edge keys (min, max) */
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(npairs > 0 ? npairs : 1));
    if (!key) return ORC_NOMEM;
    int64_t nk = 0;
    for (int64_t k = 0; k < npairs; ++k) {
        int32_t u = src[k], v = dst[k];
        if (u == v) continue;
        uint32_t lo = (uint32_t)(u < v ? u : v), hi = (uint32_t)(u < v ? v : u);
        key[nk++] = ((uint64_t)lo << 32) | hi;
    }
    qsort(key, (size_t)nk, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    for (int64_t k = 0; k < nk; ++k)
        if (k == 0 || key[k] != key[k - 1]) key[m++] = key[k];
    if (m > cap) { free(key); *m_out = m; return ORC_CAPACITY; }

    /* 2. degrees and relabelling */
    int32_t* old_to_new = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    vkey* vk = (vkey*)malloc(sizeof(vkey) * (size_t)(n > 0 ? n : 1));
    if (!old_to_new || !vk) { free(key); free(old_to_new); free(vk); return ORC_NOMEM; }
    for (int32_t v = 0; v < n; ++v) { vk[v].key = 0; vk[v].id = v; }
    for (int64_t k = 0; k < m; ++k) {
        vk[(int32_t)(key[k] >> 32)].key++;
        vk[(int32_t)(key[k] & 0xffffffffu)].key++;
    }
    if (order == 0) {
        for (int32_t v = 0; v < n; ++v) vk[v].key = 0;
    } else if (order == 2) {
        for (int32_t v = 0; v < n; ++v) vk[v].key = -vk[v].key;
    }
    qsort(vk, (size_t)n, sizeof(vkey), cmp_vkey);
    for (int32_t i = 0; i < n; ++i) {
        old_to_new[vk[i].id] = i;
        if (new_to_old) new_to_old[i] = vk[i].id;
    }

    /* 3. relabel, orient so that row < column, sort by (row, column) */
    for (int64_t k = 0; k < m; ++k) {
        int32_t a = old_to_new[(int32_t)(key[k] >> 32)];
        int32_t b = old_to_new[(int32_t)(key[k] & 0xffffffffu)];
        uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
        key[k] = ((uint64_t)lo << 32) | hi;
    }
    qsort(key, (size_t)m, sizeof(uint64_t), cmp_u64);

    /* 4. CSR */
    for (int32_t i = 0; i <= n; ++i) rowptr[i] = 0;
    for (int64_t k = 0; k < m; ++k) rowptr[(int32_t)(key[k] >> 32) + 1]++;
    for (int32_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
    for (int64_t k = 0; k < m; ++k) col[k] = (int32_t)(key[k] & 0xffffffffu);
    *m_out = m;
    free(key);
    free(old_to_new);
    free(vk);
    return ORC_OK;
}

/* ------------------------------------------------- symmetric adjacency lists */

/* Full (both directions) adjacency of the upper-triangular CSR: for every
 * vertex its neighbours in ascending order with the id of the connecting edge. */
typedef struct {
    int32_t n;
    int64_t* off;   /* n+1 */
    int32_t* nbr;   /* 2m */
    int64_t* eid;   /* 2m */
} sym_adj;

static void sym_free(sym_adj* a) {
    free(a->off);
    free(a->nbr);
    free(a->eid);
}

static int sym_build(int32_t n, const int32_t* rowptr, const int32_t* col, sym_adj* a) {
    const int64_t m = rowptr[n];
    a->n = n;
    a->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    a->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    a->eid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!a->off || !a->nbr || !a->eid || !fill) { sym_free(a); free(fill); return ORC_NOMEM; }
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            a->off[u + 1]++;
            a->off[col[e] + 1]++;
        }
    for (int32_t v = 0; v < n; ++v) a->off[v + 1] += a->off[v];
    for (int32_t v = 0; v <= n; ++v) fill[v] = a->off[v];
    /* Rows are visited in ascending order and columns ascend within a row, so
     * each list is filled in ascending neighbour order: first the smaller
     * neighbours (as the column side of earlier rows), then the row's own. */
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            int32_t v = col[e];
            a->nbr[fill[u]] = v; a->eid[fill[u]++] = e;
            a->nbr[fill[v]] = u; a->eid[fill[v]++] = e;
        }
    free(fill);
    return ORC_OK;
}

static int check_csr(int32_t n, const int32_t* rowptr, const int32_t* col) {
    if (n < 0 || !rowptr) return ORC_INVALID;
    if (rowptr[0] != 0) return ORC_INVALID;
    for (int32_t u = 0; u < n; ++u) {
        if (rowptr[u + 1] < rowptr[u]) return ORC_INVALID;
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            if (col[e] <= u || col[e] >= n) return ORC_INVALID;
            if (e > rowptr[u] && col[e] <= col[e - 1]) return ORC_INVALID;
        }
    }
    return ORC_OK;
}

/* Calls visit(ctx, e1, e2) for every common neighbour w of u and v, where e1
 * is the edge (u,w) and e2 the edge (v,w): a merge of the two sorted lists. */
typedef void (*visit_fn)(void* ctx, int64_t e1, int64_t e2);

static void for_common(const sym_adj* a, int32_t u, int32_t v, visit_fn visit, void* ctx) {
    int64_t p = a->off[u], pe = a->off[u + 1];
    int64_t q = a->off[v], qe = a->off[v + 1];
    while (p < pe && q < qe) {
        const int32_t x = a->nbr[p], y = a->nbr[q];
        if (x < y) ++p;
        else if (y < x) ++q;
        else {
            visit(ctx, a->eid[p], a->eid[q]);
            ++p;
            ++q;
        }
    }
}

typedef struct { const uint8_t* alive; int32_t count; } count_ctx;

static void count_visit(void* c, int64_t e1, int64_t e2) {
    count_ctx* x = (count_ctx*)c;
    if (x->alive[e1] && x->alive[e2]) x->count++;
}

/* Number of common neighbours w of u and v such that edges (u,w) and (v,w) are
 * both alive. */
static int32_t common_alive(const sym_adj* a, const uint8_t* alive, int32_t u, int32_t v) {
    count_ctx c = {alive, 0};
    for_common(a, u, v, count_visit, &c);
    return c.count;
}

/* ------------------------------------------------ one support computation */

/*
 * support[e] = number of triangles of the alive subgraph that contain edge e,
 * for alive e; 0 for dead e.  This is one evaluation of S = (A^T A) o A
 * (Algorithm 1, first line of the loop) on the alive edges.  alive may be NULL
 * (every edge alive).
 */
int orc_supports(int32_t n, const int32_t* rowptr, const int32_t* col, const uint8_t* alive,
                 int32_t* support) {
    if (check_csr(n, rowptr, col) != ORC_OK || !support) return ORC_INVALID;
    const int64_t m = rowptr[n];
    uint8_t* al = (uint8_t*)malloc((size_t)m + 1);
    if (!al) return ORC_NOMEM;
    for (int64_t e = 0; e < m; ++e) al[e] = alive ? (alive[e] != 0) : 1;
    sym_adj a;
    if (sym_build(n, rowptr, col, &a) != ORC_OK) { free(al); return ORC_NOMEM; }
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
            support[e] = al[e] ? common_alive(&a, al, u, col[e]) : 0;
    sym_free(&a);
    free(al);
    return ORC_OK;
}

/*
 * support[k] = number of triangles containing edge edges[k] (the whole graph
 * alive): the definition of one support evaluation, S = (A^T A) o A, read at
 * the listed edges only.  Used to time the oracle on a sample of a graph too
 * large for a full run: loop_ns (may be NULL) receives the wall time of the
 * per-edge loop alone (after the adjacency is built).
 */
int orc_supports_of(int32_t n, const int32_t* rowptr, const int32_t* col, const int64_t* edges,
                    int64_t count, int32_t* support, int64_t* loop_ns) {
    if (check_csr(n, rowptr, col) != ORC_OK || count < 0 || (count > 0 && (!edges || !support)))
        return ORC_INVALID;
    const int64_t m = rowptr[n];
    for (int64_t k = 0; k < count; ++k)
        if (edges[k] < 0 || edges[k] >= m) return ORC_INVALID;
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    uint8_t* al = (uint8_t*)malloc((size_t)m + 1);
    sym_adj a;
    if (!eu || !al || sym_build(n, rowptr, col, &a) != ORC_OK) { free(eu); free(al); return ORC_NOMEM; }
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) eu[e] = u;
    for (int64_t e = 0; e < m; ++e) al[e] = 1;
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int64_t k = 0; k < count; ++k) support[k] = common_alive(&a, al, eu[edges[k]], col[edges[k]]);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (loop_ns) *loop_ns = (int64_t)(t1.tv_sec - t0.tv_sec) * 1000000000 + (t1.tv_nsec - t0.tv_nsec);
    sym_free(&a);
    free(eu);
    free(al);
    return ORC_OK;
}

/* ------------------------------------------------------- mode R: recompute */

/*
 * Algorithm 1 as printed: recompute S on the alive subgraph, mask the edges
 * with S >= K-2, drop the rest, stop when a pass drops nothing.
 * alive_init (may be NULL = all edges) is the starting edge set.
 */
int orc_truss_recompute(int32_t n, const int32_t* rowptr, const int32_t* col, int32_t K,
                        const uint8_t* alive_init, uint8_t* mask, int32_t* support,
                        int32_t* rounds) {
    if (check_csr(n, rowptr, col) != ORC_OK || !mask || !support || !rounds) return ORC_INVALID;
    const int64_t m = rowptr[n];
    uint8_t* alive = (uint8_t*)malloc((size_t)m + 1);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    sym_adj a;
    if (!alive || !S || sym_build(n, rowptr, col, &a) != ORC_OK) {
        free(alive); free(S); return ORC_NOMEM;
    }
    for (int64_t e = 0; e < m; ++e) alive[e] = alive_init ? (alive_init[e] != 0) : 1;
    int32_t r = 0;
    for (;;) {
        ++r;
        for (int32_t u = 0; u < n; ++u)
            for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
                S[e] = alive[e] ? common_alive(&a, alive, u, col[e]) : 0;
        int64_t dropped = 0;
        for (int64_t e = 0; e < m; ++e)
            if (alive[e] && (int64_t)S[e] < (int64_t)K - 2) ++dropped;
        if (dropped == 0) break;
        for (int64_t e = 0; e < m; ++e)
            if (alive[e] && (int64_t)S[e] < (int64_t)K - 2) alive[e] = 0;
    }
    for (int64_t e = 0; e < m; ++e) {
        mask[e] = alive[e];
        support[e] = alive[e] ? S[e] : 0;
    }
    *rounds = r;
    sym_free(&a);
    free(alive);
    free(S);
    return ORC_OK;
}

/* ----------------------------------------------------------- mode P: peel */

typedef struct { const uint8_t* alive; int32_t* S; } peel_ctx;

/* Triangle (u, v, w) is destroyed by removing (u, v): if (u,w) and (v,w) are
 * still present, each loses one triangle. */
static void peel_visit(void* c, int64_t e1, int64_t e2) {
    peel_ctx* x = (peel_ctx*)c;
    if (x->alive[e1] && x->alive[e2]) { x->S[e1]--; x->S[e2]--; }
}

/*
 * Same result as mode R, different route: count every alive edge's triangles
 * once, then in each pass take the frontier F = {alive e : S[e] < K-2}; if F is
 * empty stop.  Otherwise remove the frontier edges one at a time; removing
 * e = (u,v) destroys each triangle (u,v,w) whose edges (u,w) and (v,w) have not
 * yet been removed, and the supports of those two edges drop by one.  Edges of
 * F not yet removed still count as present, so every destroyed triangle is
 * charged exactly once and the supports left on the survivors equal a fresh
 * recount on the surviving subgraph.
 */
int orc_truss_peel(int32_t n, const int32_t* rowptr, const int32_t* col, int32_t K,
                   const uint8_t* alive_init, uint8_t* mask, int32_t* support, int32_t* rounds) {
    if (check_csr(n, rowptr, col) != ORC_OK || !mask || !support || !rounds) return ORC_INVALID;
    const int64_t m = rowptr[n];
    uint8_t* alive = (uint8_t*)malloc((size_t)m + 1);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    int64_t* frontier = (int64_t*)malloc(sizeof(int64_t) * ((size_t)m + 1));
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    sym_adj a;
    if (!alive || !S || !frontier || !eu || sym_build(n, rowptr, col, &a) != ORC_OK) {
        free(alive); free(S); free(frontier); free(eu); return ORC_NOMEM;
    }
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) eu[e] = u;
    for (int64_t e = 0; e < m; ++e) alive[e] = alive_init ? (alive_init[e] != 0) : 1;
    for (int64_t e = 0; e < m; ++e) S[e] = alive[e] ? common_alive(&a, alive, eu[e], col[e]) : 0;

    int32_t r = 0;
    for (;;) {
        ++r;
        int64_t nf = 0;
        for (int64_t e = 0; e < m; ++e)
            if (alive[e] && (int64_t)S[e] < (int64_t)K - 2) frontier[nf++] = e;
        if (nf == 0) break;
        for (int64_t f = 0; f < nf; ++f) {
            const int64_t e = frontier[f];
            const int32_t u = eu[e], v = col[e];
            alive[e] = 0;
            peel_ctx c = {alive, S};
            for_common(&a, u, v, peel_visit, &c);
        }
    }
    for (int64_t e = 0; e < m; ++e) {
        mask[e] = alive[e];
        support[e] = alive[e] ? S[e] : 0;
    }
    *rounds = r;
    sym_free(&a);
    free(alive);
    free(S);
    free(frontier);
    free(eu);
    return ORC_OK;
}
