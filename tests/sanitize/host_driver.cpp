// Host-side sanitizer harness (AddressSanitizer + UndefinedBehaviorSanitizer):
// drives the library's host CSR builder and every oracle routine over seeded
// random pair lists (self-loops, duplicates, isolated vertices, both
// orientations), the error paths included, and checks that the builder
// equals the oracle's canonicalisation and that the oracle's two truss modes
// agree.  Built with g++/gcc by tests/test_host_sanitizers.py; CPU only.
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/ktruss.h"

// The builder reports errors through the library's error helpers, which live
// in the HIP translation unit; this harness provides host stand-ins.
namespace kt {
int32_t fail(int32_t code, const char*, ...) { return code; }
void clear_error() {}
}  // namespace kt

extern "C" {
int orc_canonical_csr(const int32_t* src, const int32_t* dst, int64_t npairs, int32_t n, int32_t order,
                      int32_t* rowptr, int32_t* col, int64_t cap, int32_t* new_to_old, int64_t* m_out);
int orc_supports(int32_t n, const int32_t* rowptr, const int32_t* col, const uint8_t* alive, int32_t* support);
int orc_truss_recompute(int32_t n, const int32_t* rowptr, const int32_t* col, int32_t K, const uint8_t* alive_init,
                        uint8_t* mask, int32_t* support, int32_t* rounds);
int orc_truss_peel(int32_t n, const int32_t* rowptr, const int32_t* col, int32_t K, const uint8_t* alive_init,
                   uint8_t* mask, int32_t* support, int32_t* rounds);
int orc_supports_of(int32_t n, const int32_t* rowptr, const int32_t* col, const int64_t* edges, int64_t count,
                    int32_t* support, int64_t* loop_ns);
}

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next_u64() {  // xorshift64
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                 \
        }                                                             \
    } while (0)

static int one_graph(int32_t n, int64_t npairs, int dense_core) {
    std::vector<int32_t> s((size_t)npairs), d((size_t)npairs);
    for (int64_t i = 0; i < npairs; ++i) {
        // a dense core on the first vertices makes triangles and hubs
        const int32_t span = (dense_core && (i & 1)) ? (n < 24 ? n : 24) : n;
        s[(size_t)i] = (int32_t)(next_u64() % (uint64_t)span);
        d[(size_t)i] = (int32_t)(next_u64() % (uint64_t)span);
    }
    for (int order = 0; order < 3; ++order) {
        std::vector<int32_t> rp((size_t)n + 1), col((size_t)(npairs > 0 ? npairs : 1)), n2o((size_t)(n > 0 ? n : 1));
        std::vector<int32_t> orp((size_t)n + 1), ocol((size_t)(npairs > 0 ? npairs : 1)), on2o((size_t)(n > 0 ? n : 1));
        int64_t m = -1, om = -1;
        CHECK(ktruss_build_csr(s.data(), d.data(), npairs, n, order, rp.data(), col.data(), (int64_t)col.size(),
                               n2o.data(), &m) == KTRUSS_OK);
        CHECK(orc_canonical_csr(s.data(), d.data(), npairs, n, order, orp.data(), ocol.data(), (int64_t)ocol.size(),
                                on2o.data(), &om) == 0);
        CHECK(m == om);
        CHECK(std::memcmp(rp.data(), orp.data(), sizeof(int32_t) * ((size_t)n + 1)) == 0);
        CHECK(m == 0 || std::memcmp(col.data(), ocol.data(), sizeof(int32_t) * (size_t)m) == 0);
        CHECK(n == 0 || std::memcmp(n2o.data(), on2o.data(), sizeof(int32_t) * (size_t)n) == 0);
        if (m > 0) {  // capacity one short: the needed size comes back
            int64_t m2 = -1;
            CHECK(ktruss_build_csr(s.data(), d.data(), npairs, n, order, rp.data(), col.data(), m - 1, nullptr,
                                   &m2) == KTRUSS_E_CAPACITY);
            CHECK(m2 == m);
        }
        if (order != 1) continue;
        std::vector<int32_t> sup((size_t)(m > 0 ? m : 1)), sup2((size_t)(m > 0 ? m : 1));
        CHECK(orc_supports(n, rp.data(), col.data(), nullptr, sup.data()) == 0);
        std::vector<int64_t> edges;
        for (int64_t e = 0; e < m; e += 3) edges.push_back(e);
        int64_t ns = 0;
        CHECK(orc_supports_of(n, rp.data(), col.data(), edges.data(), (int64_t)edges.size(), sup2.data(), &ns) == 0);
        for (size_t k = 0; k < edges.size(); ++k) CHECK(sup2[k] == sup[(size_t)edges[k]]);
        for (int32_t K = 2; K <= 8; ++K) {
            std::vector<uint8_t> mr((size_t)(m > 0 ? m : 1)), mp((size_t)(m > 0 ? m : 1));
            std::vector<int32_t> sr((size_t)(m > 0 ? m : 1)), sp((size_t)(m > 0 ? m : 1));
            int32_t rr = 0, rpp = 0;
            CHECK(orc_truss_recompute(n, rp.data(), col.data(), K, nullptr, mr.data(), sr.data(), &rr) == 0);
            CHECK(orc_truss_peel(n, rp.data(), col.data(), K, nullptr, mp.data(), sp.data(), &rpp) == 0);
            CHECK(rr == rpp);
            CHECK(m == 0 || (std::memcmp(mr.data(), mp.data(), (size_t)m) == 0 &&
                             std::memcmp(sr.data(), sp.data(), sizeof(int32_t) * (size_t)m) == 0));
            // restart from the result: nothing moves
            CHECK(orc_truss_peel(n, rp.data(), col.data(), K, mp.data(), mr.data(), sr.data(), &rr) == 0);
            CHECK(rr == 1 && (m == 0 || std::memcmp(sr.data(), sp.data(), sizeof(int32_t) * (size_t)m) == 0));
        }
    }
    return 0;
}

int main() {
    const int32_t sizes[][2] = {{0, 0}, {1, 3}, {5, 0}, {7, 40}, {40, 300}, {200, 3000}, {1000, 6000}, {3000, 30000}};
    for (const auto& sz : sizes)
        for (int core = 0; core < 2; ++core)
            if (one_graph(sz[0], sz[1], core)) return 1;
    // error paths of the builder: bad ids, bad order, null pointers
    int32_t s[2] = {0, 5}, d[2] = {1, 2}, rp[6], col[2];
    int64_t m = 0;
    CHECK(ktruss_build_csr(s, d, 2, 5, 1, rp, col, 2, nullptr, &m) == KTRUSS_E_INVALID);
    CHECK(ktruss_build_csr(s, d, 2, 6, 3, rp, col, 2, nullptr, &m) == KTRUSS_E_INVALID);
    CHECK(ktruss_build_csr(nullptr, d, 2, 6, 1, rp, col, 2, nullptr, &m) == KTRUSS_E_INVALID);
    CHECK(ktruss_build_csr(s, d, -1, 6, 1, rp, col, 2, nullptr, &m) == KTRUSS_E_INVALID);
    CHECK(orc_canonical_csr(s, d, 2, 5, 1, rp, col, 2, nullptr, &m) != 0);
    std::printf("sanitizer harness ok\n");
    return 0;
}
