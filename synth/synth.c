/*
 * Seeded synthetic graph generators (raw vertex-pair lists).
 *
 * This file holds input generation only: it produces unordered vertex pairs
 * (possibly with self-loops and duplicates) and nothing of the K-truss method.
 * Both the CPU oracle tests and the GPU path consume its output; neither side's
 * arithmetic lives here.
 *
 * Randomness: a counter-based generator.  Every draw is a pure function of
 * (seed, stream, counter) built from the SplitMix64 output function (Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014), so results do not depend on thread count or call order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* 64 random bits for (seed, stream, counter). */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return mix64(mix64(seed * GOLDEN + stream + 1) ^ (ctr * GOLDEN + 0x632be59bd9b4e019ULL));
}

/* uniform double in [0, 1) */
static inline double unif(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return (double)(draw(seed, stream, ctr) >> 11) * 0x1.0p-53;
}

/* uniform integer in [0, bound), bound > 0 (multiply-shift; bias < 2^-32 for bound < 2^32) */
static inline uint64_t below(uint64_t seed, uint64_t stream, uint64_t ctr, uint64_t bound) {
    uint64_t x = draw(seed, stream, ctr) >> 32;
    return (x * bound) >> 32;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) without per-level noise:
 * n = 2^scale vertices, npairs = 2^scale * edge_factor pairs.  At each of the
 * `scale` levels (most significant bit first) a quadrant is chosen with
 * probabilities (a, b, c, 1-a-b-c): a -> (0,0), b -> (0,1), c -> (1,0),
 * d -> (1,1) for the (src bit, dst bit).
 */
int synth_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c,
               uint64_t seed, int32_t* src, int32_t* dst) {
    if (scale < 1 || scale > 30 || edge_factor < 1) return -1;
    const int64_t npairs = ((int64_t)1 << scale) * edge_factor;
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < npairs; ++k) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            double r = unif(seed, 0, (uint64_t)k * 64u + (uint64_t)l);
            uint32_t sb = r >= ab;
            uint32_t db = (r >= a && r < ab) || r >= abc;
            u = (u << 1) | sb;
            v = (v << 1) | db;
        }
        src[k] = (int32_t)u;
        dst[k] = (int32_t)v;
    }
    return 0;
}

/*
 * `size` distinct vertices drawn uniformly from [0, n) (rejection on a bitmap),
 * written to verts[size].  The clique's pairs are formed by the caller.
 */
int synth_distinct_vertices(int32_t n, int32_t size, uint64_t seed, int32_t* verts) {
    if (size < 0 || size > n) return -1;
    uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
    if (!seen) return -5;
    uint64_t ctr = 0;
    for (int32_t i = 0; i < size;) {
        int32_t v = (int32_t)below(seed, 1, ctr++, (uint64_t)n);
        if (!seen[v]) { seen[v] = 1; verts[i++] = v; }
    }
    free(seen);
    return 0;
}

/*
 * Chung-Lu graph: weights w_i = (i+1)^(-1/(gamma-1)), scaled so that they sum to
 * n*dbar and capped at n-1; npairs = round(n*dbar/2) pairs whose endpoints are
 * drawn independently with probability proportional to w (inverse CDF).
 * Returns the number of pairs written (<= cap), or < 0 on error.
 */
int64_t synth_chung_lu(int32_t n, double gamma, double dbar, uint64_t seed,
                       int32_t* src, int32_t* dst, int64_t cap) {
    if (n < 2 || gamma <= 1.0 || dbar <= 0) return -1;
    const int64_t npairs = (int64_t)llround((double)n * dbar / 2.0);
    if (npairs > cap) return -3;
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* cdf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!w || !cdf) { free(w); free(cdf); return -5; }
    double sum = 0;
    for (int32_t i = 0; i < n; ++i) { w[i] = pow((double)(i + 1), -1.0 / (gamma - 1.0)); sum += w[i]; }
    const double scale = (double)n * dbar / sum;
    double acc = 0;
    for (int32_t i = 0; i < n; ++i) {
        double wi = w[i] * scale;
        if (wi > (double)(n - 1)) wi = (double)(n - 1);
        acc += wi;
        cdf[i] = acc;
    }
    for (int64_t k = 0; k < npairs; ++k) {
        for (int side = 0; side < 2; ++side) {
            double r = unif(seed, 2, (uint64_t)k * 2u + (uint64_t)side) * acc;
            int32_t lo = 0, hi = n - 1;           /* first i with cdf[i] > r */
            while (lo < hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] > r) hi = mid; else lo = mid + 1;
            }
            if (side == 0) src[k] = lo; else dst[k] = lo;
        }
    }
    free(w);
    free(cdf);
    return npairs;
}

/*
 * Per-graph parameters of the many-small-graphs workload, graph g of a batch
 * seeded with `seed`: n log-uniform in [nmin, nmax], gamma uniform in
 * [2.1, 3.0], mean degree uniform in [4, 64], K uniform in {3..8}.
 */
void synth_batch_params(uint64_t seed, int32_t g, int32_t nmin, int32_t nmax,
                        int32_t* n, double* gamma, double* dbar, int32_t* K) {
    const double l0 = log((double)nmin), l1 = log((double)nmax);
    double r0 = unif(seed, 3, (uint64_t)g * 8u + 0);
    double r1 = unif(seed, 3, (uint64_t)g * 8u + 1);
    double r2 = unif(seed, 3, (uint64_t)g * 8u + 2);
    int32_t nn = (int32_t)llround(exp(l0 + r0 * (l1 - l0)));
    if (nn < nmin) nn = nmin;
    if (nn > nmax) nn = nmax;
    *n = nn;
    *gamma = 2.1 + 0.9 * r1;
    *dbar = 4.0 + 60.0 * r2;
    *K = 3 + (int32_t)below(seed, 3, (uint64_t)g * 8u + 3, 6);
}

/*
 * Barabasi-Albert preferential attachment: a seed clique on m+1 vertices, then
 * each new vertex v attaches to m distinct earlier vertices, each chosen with
 * probability proportional to its current degree (uniform pick from the list of
 * edge endpoints, rejecting repeats).  Writes (m+1)m/2 + (n-m-1)m pairs.
 */
int64_t synth_ba(int32_t n, int32_t m, uint64_t seed, int32_t* src, int32_t* dst, int64_t cap) {
    if (m < 1 || n <= m + 1) return -1;
    const int64_t total = (int64_t)(m + 1) * m / 2 + (int64_t)(n - m - 1) * m;
    if (total > cap) return -3;
    int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * total));
    int32_t* pick = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    if (!ends || !pick) { free(ends); free(pick); return -5; }
    int64_t ne = 0, k = 0;
    for (int32_t u = 0; u <= m; ++u)
        for (int32_t v = u + 1; v <= m; ++v) {
            src[k] = u; dst[k] = v; ++k;
            ends[ne++] = u; ends[ne++] = v;
        }
    uint64_t ctr = 0;
    for (int32_t v = m + 1; v < n; ++v) {
        const int64_t avail = ne;            /* attach only to edges present before v */
        int32_t got = 0;
        while (got < m) {
            int32_t t = ends[below(seed, 4, ctr++, (uint64_t)avail)];
            int dup = 0;
            for (int32_t j = 0; j < got; ++j) dup |= (pick[j] == t);
            if (!dup) pick[got++] = t;
        }
        for (int32_t j = 0; j < m; ++j) {
            src[k] = v; dst[k] = pick[j]; ++k;
            ends[ne++] = v; ends[ne++] = pick[j];
        }
    }
    free(ends);
    free(pick);
    return k;
}
