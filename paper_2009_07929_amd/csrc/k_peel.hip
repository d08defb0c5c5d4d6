// Incremental support maintenance: the decrement form of Algorithm 1's
// recompute line (Section II-A).  After a prune, the survivors keep their
// supports (the compaction copies them) and every triangle of the round's
// alive graph that loses at least one edge is charged exactly once, by its
// removed edge with the smallest position: each of the triangle's surviving
// edges loses one support.  A survivor's support then equals the number of
// triangles it still closes, which is what a recomputation on the new alive
// graph would give, so the fixpoint, the supports and the pass count are
// those of the recompute loop.
//
// The task of removed edge f = (u, v), u < v, lists every triangle (u, v, w)
// of the round's alive graph from the full neighbourhoods of u and v: the
// out-row of a vertex holds its larger neighbours, its in-edge list (the
// transpose, entries ordered by row) its smaller ones, both ascending.  The
// third vertex w lies below v (u's in-list followed by its out-row before f,
// against v's in-list) or above v (u's out-row after f, Algorithm 3's tail,
// against v's out-row).  One wave per removed edge: the lanes walk the shorter
// list of each pair and binary-search the longer one, or, when both fit in 64
// lanes, compare one list against the other held in registers.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

// Every common value of two ascending lists A = [a0, a1) and B = [b0, b1),
// given by value and edge accessors, is passed to hit(edge in A, edge in B).
// The lanes walk the shorter list and binary-search the longer.
template <class VA, class EA, class VB, class EB, class H>
__device__ __forceinline__ void wave_common(int32_t a0, int32_t a1, VA va, EA ea, int32_t b0, int32_t b1, VB vb,
                                            EB eb, H hit) {
    if (a0 >= a1 || b0 >= b1) return;
    const int lane = __lane_id();
    if (a1 - a0 <= 64 && b1 - b0 <= 64) {
        // both lists fit one element per lane: B's elements are broadcast to
        // every lane in turn and compared with the lane's element of A
        const int32_t la = a1 - a0, lb = b1 - b0;
        const int32_t va_l = lane < la ? va(a0 + lane) : -1;
        const int32_t vb_l = lane < lb ? vb(b0 + lane) : -2;
        for (int32_t j = 0; j < lb; ++j) {
            const int32_t y = __shfl(vb_l, j);
            if (lane < la && va_l == y) hit(ea(a0 + lane), eb(b0 + j));
        }
        return;
    }
    const bool walk_a = a1 - a0 <= b1 - b0;
    const int32_t w0 = walk_a ? a0 : b0, w1 = walk_a ? a1 : b1;
    const int32_t s0 = walk_a ? b0 : a0, s1 = walk_a ? b1 : a1;
    for (int32_t base = w0; base < w1; base += 64) {
        const int32_t q = base + lane;
        if (q >= w1) continue;
        const int32_t val = walk_a ? va(q) : vb(q);
        int32_t lo = s0, len = s1 - s0;
        while (len > 0) {
            const int32_t half = len >> 1;
            const int32_t y = walk_a ? vb(lo + half) : va(lo + half);
            if (y < val) {
                lo += half + 1;
                len -= half + 1;
            } else {
                len = half;
            }
        }
        if (lo < s1 && (walk_a ? vb(lo) : va(lo)) == val) {
            if (walk_a) hit(ea(q), eb(lo));
            else hit(ea(lo), eb(q));
        }
    }
}

// Every triangle (f, e1, e2) of removed edge f = (u, v) in the lists of x and
// c is passed to charge(e1, e2) (entries of removed edges included: the
// charge rule tells them apart).  One wave.
template <class Charge>
__device__ __forceinline__ void peel_triangles(const Buf& x, const Csc& c, int32_t f, Charge charge) {
    const int32_t* __restrict__ col = x.col;
    const int32_t* __restrict__ csrc = c.src;
    const int32_t* __restrict__ cedge = c.edge;
    const int32_t u = x.src[f], v = col[f];
    const int32_t ru0 = x.rowptr[u], ru1 = x.rowptr[u + 1];
    const int32_t rv0 = x.rowptr[v], rv1 = x.rowptr[v + 1];
    const int32_t cu0 = c.ptr[u], cu1 = c.ptr[u + 1];
    const int32_t cv0 = c.ptr[v], cv1 = c.ptr[v + 1];
    // w < v: u's neighbours below v, its in-list (w < u) followed by its
    // out-row before f (u < w < v), all ascending, against v's in-list (every
    // neighbour of v below v; u itself is not in the first list)
    const int32_t nin = cu1 - cu0;
    auto low_val = [&](int32_t q) { return q < nin ? csrc[cu0 + q] : col[ru0 + (q - nin)]; };
    auto low_edge = [&](int32_t q) { return q < nin ? cedge[cu0 + q] : ru0 + (q - nin); };
    auto in_val = [&](int32_t q) { return csrc[q]; };
    auto in_edge = [&](int32_t q) { return cedge[q]; };
    wave_common(0, nin + (f - ru0), low_val, low_edge, cv0, cv1, in_val, in_edge, charge);
    // w > v: edges (u, w) and (v, w): u's tail after f against v's out-row
    auto row_val = [&](int32_t q) { return col[q]; };
    auto row_edge = [&](int32_t q) { return q; };
    wave_common(f + 1, ru1, row_val, row_edge, rv0, rv1, row_val, row_edge, charge);
}

// ---- in-place rounds.  Between compactions the edges keep their positions
// and their state lives in S: a support (>= 0) for an alive edge, kDying for
// a removed one; the round's liveness words tell the edges removed by this
// round's prune from those removed earlier.  A round marks the removed edges
// and lists them, decides, and peels; nothing is moved, so the in-edge lists
// need no remap.

// One thread: the round's bookkeeping (pass count, fixpoint, survivors) and,
// with ratio > 0, whether the frontier is left to a recomputation.
// The peel's work is the listed frontier; removed edges in no triangle cost
// it nothing, so the comparison with ratio x the survivors counts the listed.
__global__ void k_state_decide(Ctl* ctl, int p, float ratio) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || ctl->done) return;
    const int32_t removed = ctl->removed_now, nf = ctl->front_n;
    ctl->rounds += 1;
    ctl->need_support = 0;
    if (removed == 0) {
        ctl->done = 1;
        ctl->final_buf = p;
        return;
    }
    ctl->kept -= removed;
    ctl->removed_total += removed;
    if (ratio > 0.f && (double)nf > (double)ratio * (double)ctl->kept) ctl->need_support = 1;
}

// The liveness of an edge comes from the round's LiveWords (a table 1/16 the
// size of S, written by the marking), not from S itself.
__global__ __launch_bounds__(kBlock) void k_peel_state(Buf x, Csc c, const int32_t* __restrict__ frontier,
                                                     const LiveWord* __restrict__ livew,
                                                     const Ctl* __restrict__ ctl) {
    if (ctl->done || ctl->need_support) return;
    const int32_t nf = ctl->front_n;
    int32_t* __restrict__ S = x.S;
    const int32_t nw = (int32_t)(gridDim.x * (kBlock / 64));
    for (int32_t wid = (int32_t)((blockIdx.x * kBlock + threadIdx.x) >> 6); wid < nf; wid += nw) {
        const int32_t f = frontier[wid];
        auto charge = [&](int32_t e1, int32_t e2) {
            if (e1 < 0 || e2 < 0) return;  // tombstones of the in-lists: removed before the last compaction
            const LiveWord w1 = livew[e1 >> 6], w2 = livew[e2 >> 6];
            const int b1 = e1 & 63, b2 = e2 & 63;
            if (((w1.dead >> b1) | (w2.dead >> b2)) & 1ull) return;  // not a triangle of this round
            const bool y1 = (w1.dying >> b1) & 1ull, y2 = (w2.dying >> b2) & 1ull;
            if ((y1 && e1 < f) || (y2 && e2 < f)) return;
            if (!y1) atomicSub(&S[e1], 1);
            if (!y2) atomicSub(&S[e2], 1);
        };
        peel_triangles(x, c, f, charge);
    }
}

}  // namespace

hipError_t launch_state_round(const Buf& x, const Csc& c, int32_t thr, const BatchCtx& b, int32_t G,
                              int32_t* frontier, Scratch& sc, Ctl* ctl, int p, float ratio, int32_t m_hint,
                              hipStream_t s) {
    // an empty buffer still takes the round's bookkeeping (it ends the run)
    const hipError_t e = launch_state_mark(x, b, G, thr, frontier, sc, ctl, p, m_hint, s);
    if (e != hipSuccess) return e;
    k_state_decide<<<1, 64, 0, s>>>(ctl, p, ratio);
    if (m_hint > 0) {
        const unsigned grid = min(grid_for((int64_t)m_hint * 64), (unsigned)kStreamMaxGrid);
        k_peel_state<<<grid, kBlock, 0, s>>>(x, c, frontier, reinterpret_cast<const LiveWord*>(sc.keepw), ctl);
    }
    return hipGetLastError();
}



}  // namespace kt
