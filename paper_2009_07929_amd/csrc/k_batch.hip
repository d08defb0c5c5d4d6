// Batched form: many independent graphs run as one disjoint union.
//
// The union of the K-trusses of disjoint graphs is the truss of their union
// (no triangle spans two graphs), so one fixpoint loop over the concatenated
// CSR computes every graph's truss, provided the prune threshold is the one of
// the edge's own graph (K_g - 2, looked up through the edge's row).  Pass
// counts are per graph: a graph is finished at its first pass that removes
// none of its edges.  At that pass its surviving edges are written to the
// outputs and dropped from the working set, so finished graphs cost nothing in
// later passes and the loop ends when no edge is left.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

// Per graph: its vertex range is [vert_off[g], vert_off[g+1]); checks K_g >= 2
// and the offsets (err bit 32).
__global__ __launch_bounds__(kBlock) void k_batch_graphs(const int32_t* __restrict__ vert_off,
                                                       const int32_t* __restrict__ K, int32_t G, int32_t n_total,
                                                       Ctl* ctl) {
    const int32_t g = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (g >= G) return;
    const int32_t v0 = vert_off[g], v1 = vert_off[g + 1];
    const bool bad = v0 < 0 || v1 < v0 || v1 > n_total || (g == 0 && v0 != 0) || (g == G - 1 && v1 != n_total) ||
                     K[g] < 2;
    if (bad) atomicOr(&ctl->err, 32);
}

// One thread per vertex: its graph (last g with vert_off[g] <= v, by binary
// search over the checked offsets) and that graph's threshold.
__global__ __launch_bounds__(kBlock) void k_batch_vertices(const int32_t* __restrict__ vert_off,
                                                         const int32_t* __restrict__ K, int32_t G, int32_t n_total,
                                                         int32_t* __restrict__ gidv, int32_t* __restrict__ thrv,
                                                         const Ctl* __restrict__ ctl) {
    if (ctl->err) return;
    const int32_t v = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (v >= n_total) return;
    int32_t lo = 0, hi = G;  // vert_off[lo] <= v < vert_off[hi]
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (vert_off[mid] <= v) lo = mid;
        else hi = mid;
    }
    gidv[v] = lo;
    thrv[v] = K[lo] - 2;
}

// Every edge must stay inside its graph (err bit 64).
__global__ __launch_bounds__(kBlock) void k_batch_edges(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                      int32_t m, const int32_t* __restrict__ vert_off,
                                                      const int32_t* __restrict__ gidv, Ctl* ctl) {
    if (ctl->err) return;
    const int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (e >= m) return;
    if (col[e] >= vert_off[gidv[src[e]] + 1]) atomicOr(&ctl->err, 64);
}

__global__ __launch_bounds__(kBlock) void k_batch_reset(int32_t G, int32_t* __restrict__ rounds,
                                                      uint8_t* __restrict__ graph_done, uint8_t* __restrict__ done_now,
                                                      int32_t* __restrict__ low_cnt) {
    const int32_t g = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (g >= G) return;
    rounds[g] = 0;
    graph_done[g] = 0;
    done_now[g] = 0;
    low_cnt[g] = 0;
}

// After a support pass over buffer p: for every unfinished graph, count the
// edges below its threshold (a workgroup per graph, grid-stride over graphs).
// None: the graph finishes now.  Either way the pass counts for it.
__global__ __launch_bounds__(kBlock) void k_batch_status(Buf x, const int32_t* __restrict__ vert_off, int32_t G,
                                                       const int32_t* __restrict__ K, int32_t* __restrict__ rounds,
                                                       uint8_t* __restrict__ graph_done, uint8_t* __restrict__ done_now,
                                                       const Ctl* __restrict__ ctl) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl->done) return;
    for (int32_t g = (int32_t)blockIdx.x; g < G; g += (int32_t)gridDim.x) {
        if (graph_done[g]) {
            if (threadIdx.x == 0) done_now[g] = 0;
            continue;
        }
        const int32_t e0 = x.rowptr[vert_off[g]], e1 = x.rowptr[vert_off[g + 1]];
        const int32_t thr = K[g] - 2;
        int low = 0;
        for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) low += x.S[e] < thr;
        low = block_sum<kBlock>(low, s_wave);
        if (threadIdx.x == 0) {
            rounds[g] += 1;
            const bool fin = low == 0;
            done_now[g] = fin ? 1 : 0;
            if (fin) graph_done[g] = 1;
        }
    }
}

}  // namespace

hipError_t launch_batch_setup(const BatchCtx& b, int32_t G, int32_t n_total, const int32_t* K, const int32_t* src,
                              const int32_t* col, int32_t m, Ctl* ctl, hipStream_t s) {
    if (G > 0) k_batch_graphs<<<grid_for(G), kBlock, 0, s>>>(b.vert_off, K, G, n_total, ctl);
    if (G > 0 && n_total > 0)
        k_batch_vertices<<<grid_for(n_total), kBlock, 0, s>>>(b.vert_off, K, G, n_total, b.gidv, b.thrv, ctl);
    if (m > 0) k_batch_edges<<<grid_for(m), kBlock, 0, s>>>(src, col, m, b.vert_off, b.gidv, ctl);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchCtx& b, int32_t G, int32_t* rounds, hipStream_t s) {
    if (G > 0) k_batch_reset<<<grid_for(G), kBlock, 0, s>>>(G, rounds, b.graph_done, b.done_now, b.low_cnt);
    return hipGetLastError();
}

hipError_t launch_batch_status(const Buf& x, const BatchCtx& b, int32_t G, const int32_t* K, int32_t* rounds,
                               const Ctl* ctl, hipStream_t s) {
    if (G > 0) {
        const int32_t grid = G < kStreamMaxGrid ? G : kStreamMaxGrid;
        k_batch_status<<<grid, kBlock, 0, s>>>(x, b.vert_off, G, K, rounds, b.graph_done, b.done_now, ctl);
    }
    return hipGetLastError();
}

}  // namespace kt
