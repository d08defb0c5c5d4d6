// Host-side input preparation: raw pairs -> canonical upper-triangular CSR.
//
// Section IV-A of the paper says only that the input graphs are made
// upper-triangular.  This builder also drops self-loops and repeated pairs and
// relabels vertices (by ascending degree by default), which bounds every
// row's out-degree in the upper triangle and so the length of the lists the
// support tasks intersect.
//
// Sorting uses an LSD radix sort over the packed key  row * n + col  (fewer
// than 2*log2(n) significant bits), 16-bit digits.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace {

int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

// Sorts keys[0..k) whose values are below 2^bits.
void radix_sort(std::vector<uint64_t>& keys, size_t k, int bits) {
    if (k < 2 || bits == 0) return;
    std::vector<uint64_t> tmp(k);
    std::vector<size_t> hist(1u << 16);
    uint64_t* a = keys.data();
    uint64_t* b = tmp.data();
    for (int shift = 0; shift < bits; shift += 16) {
        std::fill(hist.begin(), hist.end(), 0);
        for (size_t i = 0; i < k; ++i) hist[(a[i] >> shift) & 0xffffu]++;
        size_t run = 0;
        for (size_t d = 0; d < hist.size(); ++d) {
            size_t c = hist[d];
            hist[d] = run;
            run += c;
        }
        for (size_t i = 0; i < k; ++i) b[hist[(a[i] >> shift) & 0xffffu]++] = a[i];
        std::swap(a, b);
    }
    if (a != keys.data()) std::memcpy(keys.data(), a, k * sizeof(uint64_t));
}

}  // namespace

extern "C" int32_t ktruss_build_csr(const int32_t* src, const int32_t* dst, int64_t npairs, int32_t n,
                                    int32_t order, int32_t* rowptr, int32_t* col, int64_t col_capacity,
                                    int32_t* new_to_old, int64_t* m_out) {
    kt::clear_error();
    if (n < 0 || npairs < 0) return kt::fail(KTRUSS_E_INVALID, "n (%d) and npairs (%lld) must be >= 0", n, (long long)npairs);
    if (order < 0 || order > 2) return kt::fail(KTRUSS_E_INVALID, "order must be 0, 1 or 2 (got %d)", order);
    if (!rowptr || !m_out || (npairs > 0 && (!src || !dst))) return kt::fail(KTRUSS_E_INVALID, "null pointer argument");
    if (n > INT32_MAX - 1) return kt::fail(KTRUSS_E_OVERFLOW, "n too large");
    try {
        const uint64_t un = (uint64_t)n;
        std::vector<uint64_t> key((size_t)npairs);
        size_t k = 0;
        for (int64_t i = 0; i < npairs; ++i) {
            const int32_t u = src[i], v = dst[i];
            if (u < 0 || u >= n || v < 0 || v >= n)
                return kt::fail(KTRUSS_E_INVALID, "pair %lld = (%d, %d) has an id outside [0, %d)", (long long)i, u, v, n);
            if (u == v) continue;
            const uint64_t lo = (uint64_t)std::min(u, v), hi = (uint64_t)std::max(u, v);
            key[k++] = lo * un + hi;
        }
        const int bits = n > 0 ? bits_for(un * un) : 0;
        radix_sort(key, k, bits);
        size_t m = 0;
        for (size_t i = 0; i < k; ++i)
            if (i == 0 || key[i] != key[i - 1]) key[m++] = key[i];
        *m_out = (int64_t)m;
        if ((int64_t)m > (int64_t)INT32_MAX - 1) return kt::fail(KTRUSS_E_OVERFLOW, "edge count %zu too large", m);
        if ((int64_t)m > col_capacity) return kt::fail(KTRUSS_E_CAPACITY, "col capacity %lld < m = %zu", (long long)col_capacity, m);
        if (m > 0 && !col) return kt::fail(KTRUSS_E_INVALID, "col is null");

        // relabel: new label = rank of (degree, original id) in the chosen order
        std::vector<int32_t> o2n((size_t)n), n2o((size_t)n);
        if (order == 0) {
            for (int32_t v = 0; v < n; ++v) o2n[v] = n2o[v] = v;
        } else {
            std::vector<int32_t> deg((size_t)n, 0);
            int32_t maxdeg = 0;
            for (size_t i = 0; i < m; ++i) {
                const int32_t lo = (int32_t)(key[i] / un), hi = (int32_t)(key[i] % un);
                maxdeg = std::max(maxdeg, std::max(++deg[lo], ++deg[hi]));
            }
            // counting sort by degree; scanning ids upward keeps ties by id
            std::vector<int64_t> start((size_t)maxdeg + 2, 0);
            for (int32_t v = 0; v < n; ++v) {
                const int32_t d = order == 1 ? deg[v] : maxdeg - deg[v];
                start[(size_t)d + 1]++;
            }
            for (size_t d = 0; d + 1 < start.size(); ++d) start[d + 1] += start[d];
            for (int32_t v = 0; v < n; ++v) {
                const int32_t d = order == 1 ? deg[v] : maxdeg - deg[v];
                const int32_t pos = (int32_t)start[(size_t)d]++;
                n2o[pos] = v;
                o2n[v] = pos;
            }
            for (size_t i = 0; i < m; ++i) {
                const int32_t a = o2n[key[i] / un], b = o2n[key[i] % un];
                key[i] = (uint64_t)std::min(a, b) * un + (uint64_t)std::max(a, b);
            }
            radix_sort(key, m, bits);
        }
        for (int32_t v = 0; v <= n; ++v) rowptr[v] = 0;
        for (size_t i = 0; i < m; ++i) {
            rowptr[key[i] / un + 1]++;
            col[i] = (int32_t)(key[i] % un);
        }
        for (int32_t v = 0; v < n; ++v) rowptr[v + 1] += rowptr[v];
        if (new_to_old && n > 0) std::memcpy(new_to_old, n2o.data(), sizeof(int32_t) * (size_t)n);
        return KTRUSS_OK;
    } catch (const std::bad_alloc&) {
        return kt::fail(KTRUSS_E_NOMEM, "host allocation failed while building the CSR");
    }
}
