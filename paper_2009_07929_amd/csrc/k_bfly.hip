// Butterfly counting on a bipartite graph with the fine-grained, eager
// decomposition of the support pass: the paper's closing section names
// butterflies (4-cycles of a bipartite graph, its smallest dense motif) as a
// further problem for the same task mapping.
//
// Sides U and V; a butterfly is u1 - v1 - u2 - v2 with u1 != u2, v1 != v2.
// Pick the "pair" side P and the "centre" side C (the other one) so that the
// wedges p1 - c - p2 centred on C are the fewer (sum over c of deg(c)(deg(c)-1)).
// For a pair vertex p1 let w(p1, p2) be the number of centres the two share;
// the pair spans C(w, 2) butterflies and every edge (c, p1) with c shared lies
// in w - 1 of them.  So the butterflies of edge (c, p1) are
//   sum over p2 in N(c), p2 != p1, of (w(p1, p2) - 1),
// and the total is half the sum over ordered pairs of C(w, 2).
//
// One task per pair vertex p1 (or per window of p2 labels when p1 has many
// wedges): a workgroup walks p1's wedges (every c in N(p1), every p2 in N(c))
// twice.  The first walk counts w(p1, .) in LDS (an open-addressing hash when
// the wedges fit, else a dense window of labels); the second walk sums
// w(p1, p2) - 1 per centre c and adds it to the count of edge (c, p1) with
// one atomic per edge and task.  Every edge's count is written from its own
// pair vertex's tasks, so no task updates another vertex's edges.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

constexpr int kBfThreads = 256;
constexpr int kBfWaves = kBfThreads / 64;
constexpr int kBfHashCap = 4096;                  // LDS hash slots: keys + counts, 32 KB
constexpr int64_t kBfHashWedges = kBfHashCap / 2; // wedges of a pair vertex that the hash takes (load <= 1/2)
constexpr int kBfWin = 2 * kBfHashCap;           // labels per dense window (int32 counts over the same 32 KB)

struct BfCtl {
    int32_t err;
    int32_t pad;
    unsigned long long ticket;   // next task of the persistent kernel
    unsigned long long pairs2;   // sum over ordered pairs of C(w, 2): twice the butterflies
    unsigned long long wedges_u; // sum over u of deg(u) (deg(u) - 1) / 2
    unsigned long long wedges_v; // same over v
};

// ---- input checks: rowptr over U monotone from 0 to m; columns in [0, nv),
// strictly ascending inside each row
__global__ __launch_bounds__(kBlock) void k_bf_check_ptr(const int32_t* __restrict__ rowptr, int32_t nu, int32_t m,
                                                       BfCtl* ctl) {
    const int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (u > nu) return;
    const int32_t v = rowptr[u];
    int bad = 0;
    if (v < 0 || v > m) bad |= 1;
    if (u == 0 && v != 0) bad |= 2;
    if (u == nu && v != m) bad |= 4;
    if (u < nu && rowptr[u + 1] < v) bad |= 8;
    if (bad) atomicOr(&ctl->err, bad);
}

__global__ __launch_bounds__(kBlock) void k_bf_check_cols(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, int32_t nu, int32_t nv,
                                                        int32_t m, BfCtl* ctl) {
    if (ctl->err) return;  // rowptr is not walked unless it is valid
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int32_t c = col[e];
    int bad = (c < 0 || c >= nv) ? 16 : 0;
    // row of e: last u with rowptr[u] <= e
    int32_t lo = 0, hi = nu;
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (rowptr[mid] <= e) lo = mid;
        else hi = mid;
    }
    if (e > rowptr[lo] && col[e - 1] >= c) bad |= 32;
    if (bad) atomicOr(&ctl->err, bad);
}

// Wedges centred on each side: sum of C(deg, 2).
__global__ __launch_bounds__(kBlock) void k_bf_side_wedges(const int32_t* __restrict__ ptr, int32_t n,
                                                         unsigned long long* __restrict__ acc) {
    __shared__ long long s_w[kBlock / 64];
    long long w = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const long long d = ptr[v + 1] - ptr[v];
        w += d * (d - 1) / 2;
    }
    w = block_sum64<kBlock>(w, s_w);
    if (threadIdx.x == 0 && w) atomicAdd(acc, (unsigned long long)w);
}

struct BfSide {
    int32_t nP;
    const int32_t* ptrP;  // pair side: neighbours (centres) of each pair vertex, ascending
    const int32_t* adjP;
    const int32_t* eidP;  // edge id of entry q of adjP, or null: q itself
    const int32_t* ptrC;  // centre side: neighbours (pair vertices) of each centre, ascending
    const int32_t* adjC;
};

// W(p) = wedges of pair vertex p = sum over c in N(p) of deg(c) - 1; one wave per p.
__global__ __launch_bounds__(kBlock) void k_bf_pair_wedges(BfSide sd, int64_t* __restrict__ W) {
    const int lane = __lane_id();
    const int32_t nw = (int32_t)(gridDim.x * (kBlock / 64));
    for (int32_t p = (int32_t)((blockIdx.x * kBlock + threadIdx.x) >> 6); p < sd.nP; p += nw) {
        long long w = 0;
        for (int32_t q = sd.ptrP[p] + lane; q < sd.ptrP[p + 1]; q += 64) {
            const int32_t c = sd.adjP[q];
            w += sd.ptrC[c + 1] - sd.ptrC[c] - 1;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
        if (lane == 0) W[p] = w;
    }
}

__device__ __forceinline__ uint32_t bf_hash(int32_t x) {
    uint32_t h = (uint32_t)x * 0x9E3779B1u;  // Fibonacci hashing: the top bits mix all of x
    return h >> (32 - 12);                   // 4096 = 2^12 slots
}
static_assert(kBfHashCap == 4096, "bf_hash keeps 12 bits");

// Tasks of the pass: pair vertex p1 with W(p1) wedges is one task (hash) if
// W(p1) <= kBfHashWedges, else ceil(nP / kBfWin) tasks, one per window of
// p2 labels; off[p] (int64) is the first task of p, off[nP] the total.
__global__ __launch_bounds__(kBfThreads) void k_bfly(BfSide sd, const int64_t* __restrict__ W,
                                                   const int64_t* __restrict__ off, BfCtl* ctl,
                                                   unsigned long long* __restrict__ count) {
    __shared__ int32_t s_lds[2 * kBfHashCap];  // hash: keys [0, cap) and counts [cap, 2 cap); window: counts
    __shared__ long long s_red[kBfWaves];
    __shared__ long long s_ticket;
    const int t = threadIdx.x, lane = t & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int32_t nP = sd.nP;
    const int64_t ntask = off[nP];
    int32_t* s_key = s_lds;
    int32_t* s_cnt = s_lds + kBfHashCap;
    if (t == 0) s_ticket = (long long)atomicAdd(&ctl->ticket, 1ull);
    __syncthreads();
    for (;;) {
        const int64_t task = s_ticket;
        if (task >= ntask) break;
        // pair vertex of the task: last p with off[p] <= task
        int32_t lo = 0, hi = nP;
        while (hi - lo > 1) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (off[mid] <= task) lo = mid;
            else hi = mid;
        }
        const int32_t p1 = lo;
        const bool hashed = W[p1] <= kBfHashWedges;
        const int32_t wlo = hashed ? 0 : (int32_t)((task - off[p1]) * kBfWin);
        const int32_t whi = hashed ? nP : (int32_t)min((int64_t)wlo + kBfWin, (int64_t)nP);
        if (hashed) {
            for (int i = t; i < kBfHashCap; i += kBfThreads) {
                s_key[i] = -1;
                s_cnt[i] = 0;
            }
        } else {
            for (int i = t; i < kBfWin; i += kBfThreads) s_lds[i] = 0;
        }
        __syncthreads();
        const int32_t a0 = sd.ptrP[p1], a1 = sd.ptrP[p1 + 1];
        // walk 1: w(p1, p2) for every p2 of the task's labels
        for (int32_t q = a0 + wave; q < a1; q += kBfWaves) {
            const int32_t c = sd.adjP[q];
            const int32_t c1 = sd.ptrC[c + 1];
            int32_t c0 = sd.ptrC[c];
            if (!hashed) c0 += lower_bound_i32(sd.adjC + c0, c1 - c0, wlo);
            for (int32_t j0 = c0; j0 < c1; j0 += 64) {
                const int32_t j = j0 + lane;
                const int32_t p2 = j < c1 ? sd.adjC[j] : INT32_MAX;
                if (__ballot(p2 < whi) == 0) break;  // ascending: the rest lies past the window
                if (p2 < whi && p2 != p1) {
                    if (hashed) {
                        uint32_t h = bf_hash(p2);
                        for (;;) {
                            const int32_t k = atomicCAS(&s_key[h], -1, p2);
                            if (k == -1 || k == p2) {
                                atomicAdd(&s_cnt[h], 1);
                                break;
                            }
                            h = (h + 1) & (kBfHashCap - 1);
                        }
                    } else {
                        atomicAdd(&s_lds[p2 - wlo], 1);
                    }
                }
            }
        }
        __syncthreads();
        // walk 2: edge (c, p1) gains the sum over its p2 of w(p1, p2) - 1
        for (int32_t q = a0 + wave; q < a1; q += kBfWaves) {
            const int32_t c = sd.adjP[q];
            const int32_t c1 = sd.ptrC[c + 1];
            int32_t c0 = sd.ptrC[c];
            if (!hashed) c0 += lower_bound_i32(sd.adjC + c0, c1 - c0, wlo);
            long long s = 0;
            for (int32_t j0 = c0; j0 < c1; j0 += 64) {
                const int32_t j = j0 + lane;
                const int32_t p2 = j < c1 ? sd.adjC[j] : INT32_MAX;
                if (__ballot(p2 < whi) == 0) break;
                if (p2 < whi && p2 != p1) {
                    int32_t w;
                    if (hashed) {
                        uint32_t h = bf_hash(p2);
                        while (s_key[h] != p2) h = (h + 1) & (kBfHashCap - 1);  // inserted by walk 1
                        w = s_cnt[h];
                    } else {
                        w = s_lds[p2 - wlo];
                    }
                    s += w - 1;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
            if (lane == 0 && s) atomicAdd(&count[sd.eidP ? sd.eidP[q] : q], (unsigned long long)s);
        }
        // the task's pairs: sum of C(w, 2)
        long long pairs = 0;
        if (hashed) {
            for (int i = t; i < kBfHashCap; i += kBfThreads)
                if (s_key[i] >= 0) pairs += (long long)s_cnt[i] * (s_cnt[i] - 1) / 2;
        } else {
            for (int i = t; i < kBfWin; i += kBfThreads) pairs += (long long)s_lds[i] * (s_lds[i] - 1) / 2;
        }
        pairs = block_sum64<kBfThreads>(pairs, s_red);
        if (t == 0) {
            if (pairs) atomicAdd(&ctl->pairs2, (unsigned long long)pairs);
            s_ticket = (long long)atomicAdd(&ctl->ticket, 1ull);
        }
        __syncthreads();  // LDS and the ticket are read again by the next task
    }
}

__global__ void k_bf_ctl_reset(BfCtl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctl = BfCtl{};
}

__global__ __launch_bounds__(kBlock) void k_bf_zero_u64(unsigned long long* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) a[i] = 0ull;
}

// Workspace of a bipartite graph (256-byte aligned regions).
struct BfLayout {
    size_t vptr, vadj, veid, tk0, tk1, tv0, tv1, hist, blockcnt, blockoff, blockcnt2, blockoff2, W, off, ctl, total;
};

BfLayout bf_layout(int32_t nu, int32_t nv, int64_t m) {
    BfLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += (bytes + 255) & ~(size_t)255;
        return r;
    };
    const size_t em = sizeof(int32_t) * (size_t)(m > 0 ? m : 1);
    const size_t np = (size_t)(nu > nv ? nu : nv) + 1;
    L.vptr = take(sizeof(int32_t) * ((size_t)nv + 1));
    L.vadj = take(em);
    L.veid = take(em);
    L.tk0 = take(em);
    L.tk1 = take(em);
    L.tv0 = take(em);
    L.tv1 = take(em);
    L.hist = take(sizeof(int32_t) * (256 * (((size_t)m + kRsTile - 1) / kRsTile) + 1));
    L.blockcnt = take(sizeof(int32_t) * kMaxScanBlocks);
    L.blockoff = take(sizeof(int32_t) * kMaxScanBlocks);
    L.blockcnt2 = take(sizeof(int32_t) * 2 * kMaxScanBlocks);
    L.blockoff2 = take(sizeof(int32_t) * 2 * kMaxScanBlocks);
    L.W = take(sizeof(int64_t) * np);
    L.off = take(sizeof(int64_t) * np);
    L.ctl = take(sizeof(BfCtl));
    L.total = o;
    return L;
}

}  // namespace
}  // namespace kt

using namespace kt;

extern "C" {

int64_t ktruss_butterfly_workspace_bytes(int32_t nu, int32_t nv, int64_t m) {
    clear_error();
    if (nu < 0 || nv < 0 || m < 0) return fail(KTRUSS_E_INVALID, "sizes must be >= 0");
    if (nu > INT32_MAX - 1 || nv > INT32_MAX - 1 || m > INT32_MAX - 1)
        return fail(KTRUSS_E_OVERFLOW, "nu, nv or m above INT32_MAX - 1");
    return (int64_t)bf_layout(nu, nv, m).total;
}

int32_t ktruss_butterflies(const ktruss_bipartite* g, int64_t* count, int64_t* total, void* stream) {
    clear_error();
    if (!g || !total) return fail(KTRUSS_E_INVALID, "graph or total is null");
    if (g->nu < 0 || g->nv < 0 || g->m < 0) return fail(KTRUSS_E_INVALID, "sizes must be >= 0");
    if (g->nu > INT32_MAX - 1 || g->nv > INT32_MAX - 1 || g->m > INT32_MAX - 1)
        return fail(KTRUSS_E_OVERFLOW, "nu, nv or m above INT32_MAX - 1");
    if (!g->rowptr || (g->m > 0 && (!g->col || !count))) return fail(KTRUSS_E_INVALID, "rowptr/col/count is null");
    const BfLayout L = bf_layout(g->nu, g->nv, g->m);
    if (!g->work) return fail(KTRUSS_E_INVALID, "workspace is null");
    if (((uintptr_t)g->work & 255u) != 0) return fail(KTRUSS_E_INVALID, "workspace must be 256-byte aligned");
    if (g->work_bytes < (int64_t)L.total)
        return fail(KTRUSS_E_CAPACITY, "workspace has %lld bytes, needs %lld", (long long)g->work_bytes,
                    (long long)L.total);
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)g->work;
    BfCtl* ctl = (BfCtl*)(base + L.ctl);
    const int32_t nu = g->nu, nv = g->nv, m = (int32_t)g->m;
    k_bf_ctl_reset<<<1, 64, 0, s>>>(ctl);
    k_bf_check_ptr<<<grid_for((int64_t)nu + 1), kBlock, 0, s>>>(g->rowptr, nu, m, ctl);
    if (m > 0) k_bf_check_cols<<<grid_for(m), kBlock, 0, s>>>(g->rowptr, g->col, nu, nv, m, ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "butterfly checks");
    BfCtl h{};
    e = hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "butterfly check readback");
    if (h.err)
        return fail(KTRUSS_E_INVALID,
                    "malformed bipartite CSR (check bits 0x%x: 1 rowptr range, 2 rowptr[0], 4 rowptr[nu]!=m, "
                    "8 rowptr not monotone, 16 column outside [0, nv), 32 columns not ascending)",
                    h.err);
    *total = 0;
    if (m == 0) return KTRUSS_OK;
    // V-side lists: a stable transpose (ascending u inside each v, with the U-row positions as edge ids)
    Scratch sc{};
    sc.rs_hist = (int32_t*)(base + L.hist);
    sc.blockcnt = (int32_t*)(base + L.blockcnt);
    sc.blockoff = (int32_t*)(base + L.blockoff);
    sc.blockcnt2 = (int32_t*)(base + L.blockcnt2);
    sc.blockoff2 = (int32_t*)(base + L.blockoff2);
    int32_t* vptr = (int32_t*)(base + L.vptr);
    int32_t* vadj = (int32_t*)(base + L.vadj);  // first the sorted V keys, then the U vertex of every entry
    int32_t* veid = (int32_t*)(base + L.veid);
    int32_t* tk[2] = {(int32_t*)(base + L.tk0), (int32_t*)(base + L.tk1)};
    int32_t* tv[2] = {(int32_t*)(base + L.tv0), (int32_t*)(base + L.tv1)};
    e = launch_radix_transpose(g->col, m, nv, vadj, veid, vptr, tk, tv, sc, s);
    if (e == hipSuccess) e = launch_rows_of(g->rowptr, nu, veid, m, vadj, s);
    if (e != hipSuccess) return fail_hip(e, "butterfly transpose");
    // the side whose centred wedges are fewer is the centre side
    k_bf_side_wedges<<<min(grid_for(nu), 1024u), kBlock, 0, s>>>(g->rowptr, nu, &ctl->wedges_u);
    k_bf_side_wedges<<<min(grid_for(nv), 1024u), kBlock, 0, s>>>(vptr, nv, &ctl->wedges_v);
    e = hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "butterfly side readback");
    BfSide sd{};
    if (h.wedges_u <= h.wedges_v) {  // centres U, pairs V
        sd = BfSide{nv, vptr, vadj, veid, g->rowptr, g->col};
    } else {  // centres V, pairs U
        sd = BfSide{nu, g->rowptr, g->col, nullptr, vptr, vadj};
    }
    int64_t* W = (int64_t*)(base + L.W);
    int64_t* off = (int64_t*)(base + L.off);
    k_bf_pair_wedges<<<min(grid_for((int64_t)sd.nP * 64), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(sd, W);
    const int64_t nwin = ((int64_t)sd.nP + kBfWin - 1) / kBfWin;
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_bf_task_offsets(W, sd.nP, kBfHashWedges, nwin, off, sc, s);
    if (e != hipSuccess) return fail_hip(e, "butterfly tasks");
    k_bf_zero_u64<<<min(grid_for(m), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>((unsigned long long*)count, m);
    k_bfly<<<256 * 4, kBfThreads, 0, s>>>(sd, W, off, ctl, (unsigned long long*)count);  // 4 workgroups per CU fit
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "butterfly pass");
    *total = (int64_t)(h.pairs2 / 2);
    return KTRUSS_OK;
}

}  // extern "C"
