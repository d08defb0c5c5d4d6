// Prune + compaction between support passes.
//
// The alive edge tasks of buffer p are filtered, order-preserving, into buffer
// 1-p: a keep flag per element, a per-workgroup count, one workgroup scanning
// the counts, then a scatter whose positions come from a wave ballot + mbcnt
// prefix and the wave totals.  Every old position's new position is recorded
// (xscan; ~q for a dropped element) so that row pointers, and the in-edge
// lists that point at edge positions, can be remapped without another search.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

// ---- keep predicates and emitters

// Prune-round keep test of edge e of buffer x: S[e] >= K-2, with K the
// graph's own K in the batched form, where edges of graphs that finished in
// this pass are not kept but written to the outputs.
__device__ __forceinline__ bool round_keep(const Buf& x, const BatchCtx& b, int32_t thr, int32_t e) {
    if (!b.thrv) return x.S[e] >= thr;
    const int32_t v = x.src[e];
    if (b.done_now[b.gidv[v]]) return false;
    return x.S[e] >= b.thrv[v];
}

// A policy reads what element i needs once (load), decides on it (keep) and
// writes the survivor (emit) or handles the dropped element (drop).  The
// recompute loop's prune: supports restart at 0 for the next pass.
struct CsrRound {
    Buf x, y;
    int32_t thr;
    BatchCtx b;
    __device__ int32_t load(int32_t e) const { return e; }
    __device__ bool keep(int32_t e) const { return round_keep(x, b, thr, e); }
    __device__ void drop(int32_t e, int32_t, int32_t) const {
        // an edge of a graph finished in this pass leaves the working set
        // without leaving its truss
        const bool finished = b.thrv && b.done_now[b.gidv[x.src[e]]];
        if (finished) {
            const int32_t c = x.eid[e];
            b.mask[c] = 1;
            b.support[c] = x.S[e];
        }
    }
    __device__ void emit(int32_t e, int32_t, int32_t q) const {
        y.col[q] = x.col[e];
        y.src[q] = x.src[e];
        y.eid[q] = x.eid[e];
        y.S[q] = 0;
    }
};

// In-place rounds' compaction (between rounds, after the peel): the alive
// edges (S >= 0) keep their supports; in the batched form the edges of
// finished graphs are written to the outputs and leave.
struct CsrLive {
    Buf x, y;
    BatchCtx b;
    __device__ int32_t load(int32_t e) const { return e; }
    __device__ bool finished(int32_t e) const { return b.thrv && b.graph_done[b.gidv[x.src[e]]]; }
    __device__ bool keep(int32_t e) const { return x.S[e] >= 0 && !finished(e); }
    __device__ void drop(int32_t e, int32_t, int32_t) const {
        if (x.S[e] >= 0) {  // alive, in a finished graph
            const int32_t c = x.eid[e];
            b.mask[c] = 1;
            b.support[c] = x.S[e];
        }
    }
    __device__ void emit(int32_t e, int32_t, int32_t q) const {
        y.col[q] = x.col[e];
        y.src[q] = x.src[e];
        y.eid[q] = x.eid[e];
        y.S[q] = x.S[e];
    }
};

// CSR element e; keep = the caller's alive flag of its canonical edge.
struct CsrAlive {
    Buf x, y;
    const uint8_t* alive_can;
    __device__ int32_t load(int32_t e) const { return e; }
    __device__ bool keep(int32_t e) const { return alive_can[x.eid[e]] != 0; }
    __device__ void drop(int32_t, int32_t, int32_t) const {}
    __device__ void emit(int32_t e, int32_t, int32_t q) const {
        y.col[q] = x.col[e];
        y.src[q] = x.src[e];
        y.eid[q] = x.eid[e];
        y.S[q] = 0;
    }
};

// ---- generic stable filter

// Workgroup chunks of [0, N): multiples of kBlock, so that every wave's 64
// elements form one keep word.
__device__ __forceinline__ void chunk_of(int32_t N, int32_t& lo, int32_t& hi) {
    const int32_t G = (int32_t)gridDim.x;
    const int64_t chunk = (((int64_t)N + G - 1) / G + kBlock - 1) / kBlock * kBlock;
    lo = (int32_t)min((int64_t)blockIdx.x * chunk, (int64_t)N);
    hi = (int32_t)min((int64_t)lo + chunk, (int64_t)N);
}

template <class P>
__global__ __launch_bounds__(kBlock) void k_filter_count(P pol, const Ctl* __restrict__ ctl, int p, int round,
                                                       int32_t* __restrict__ blockcnt) {
    __shared__ int s_wave[kBlock / 64];
    if (round && ctl->done) return;
    int32_t lo, hi;
    chunk_of(ctl->m_buf[p], lo, hi);
    int c = 0;
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kBlock) c += pol.keep(pol.load(i));
    c = block_sum<kBlock>(c, s_wave);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = c;
}

// Exclusive scan of the G per-workgroup counts into blockoff (one workgroup
// of kScanThreads); returns the total.
__device__ __forceinline__ int scan_block_counts(const int32_t* __restrict__ blockcnt, int32_t* __restrict__ blockoff,
                                                 int32_t G, int* s_wave) {
    constexpr int PER = kMaxScanBlocks / kScanThreads;
    const int t = threadIdx.x;
    int v[PER];
    int local = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = t * PER + j;
        v[j] = idx < G ? blockcnt[idx] : 0;
        local += v[j];
    }
    int total;
    int run = block_excl_sum<kScanThreads>(local, s_wave, total);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = t * PER + j;
        if (idx < G) blockoff[idx] = run;
        run += v[j];
    }
    return total;
}

// update: 0 = only the scan; 1 = prune-round bookkeeping (pass count,
// fixpoint flag, survivor count); 2 = set the survivor count of buffer 1-p;
// 3 = batched prune round (pass count, survivor count; the run ends in
// k_batch_end once nothing is kept).
__global__ __launch_bounds__(kScanThreads) void k_filter_scan(const int32_t* __restrict__ blockcnt,
                                                            int32_t* __restrict__ blockoff, int32_t G, Ctl* ctl,
                                                            int p, int update, int round,
                                                            int32_t* __restrict__ xscan) {
    __shared__ int s_wave[kScanThreads / 64];
    if (round && ctl->done) return;
    const int t = threadIdx.x;
    const int total = scan_block_counts(blockcnt, blockoff, G, s_wave);
    if (t == 0) {
        const int32_t N = ctl->m_buf[p];
        xscan[N] = total;
        if (update == 1) {
            ctl->rounds += 1;
            const int32_t removed = N - total;
            ctl->kept = total;
            if (removed == 0) {
                ctl->done = 1;
                ctl->final_buf = p;
            } else {
                ctl->m_buf[1 - p] = total;
                ctl->removed_total += removed;
            }
        } else if (update == 2 || update == 3) {
            if (update == 3) ctl->rounds += 1;
            ctl->kept = total;
            ctl->m_buf[1 - p] = total;
            if (update == 3) ctl->removed_total += N - total;
        }
    }
}

template <class P>
__global__ __launch_bounds__(kBlock) void k_filter_scatter(P pol, const Ctl* __restrict__ ctl, int p, int round,
                                                         const int32_t* __restrict__ blockoff,
                                                         int32_t* __restrict__ xscan, KeepWord* __restrict__ keepw) {
    __shared__ int s_wave[kBlock / 64];
    if (round && ctl->done) return;
    int32_t lo, hi;
    chunk_of(ctl->m_buf[p], lo, hi);
    int32_t base = blockoff[blockIdx.x];
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const bool in = i < hi;
        const int32_t v = in ? pol.load(i) : 0;
        const bool k = in && pol.keep(v);
        int tot;
        const int32_t q = base + block_excl_flag<kBlock>(k, s_wave, tot);
        const unsigned long long kb = __ballot(k);
        if (__lane_id() == 0 && in) keepw[i >> 6] = KeepWord{kb, q, 0};  // i is the word's first element
        if (in) {
            xscan[i] = k ? q : ~q;  // new position; ~ marks a dropped element
            if (k) pol.emit(v, i, q);
            else pol.drop(v, i, q);
        }
        base += tot;
    }
}

// new_ptr[s] = the new position of old_ptr[s] for s in [0, n]
__global__ __launch_bounds__(kBlock) void k_ptr_remap(const int32_t* __restrict__ old_ptr, int32_t* __restrict__ new_ptr,
                                                    int32_t n, const int32_t* __restrict__ xscan,
                                                    const Ctl* __restrict__ ctl, int round) {
    if (round && ctl->done) return;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > n) return;
    const int32_t v = xscan[old_ptr[s]];
    new_ptr[s] = v < 0 ? ~v : v;
}

__global__ __launch_bounds__(kBlock) void k_zero_rows(int32_t* __restrict__ a, int32_t n, const Ctl* __restrict__ ctl,
                                                    int round) {
    if (round && ctl->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = 0;
}

// In-edge lists after the CSR filter, in place: every entry's edge position
// becomes the edge's new position (keep_rank: q for a kept edge, ~q for a
// removed one); entries of removed edges, and tombstones, stay -1.  The alive
// entries of every row kappa are counted on the way (alive_in, zeroed
// before): the lists are grouped by kappa (key), so a wave-level segmented
// sum adds each run and its last lane issues one atomic per run piece (a
// wave inside one run: a popcount and one atomic).
__global__ __launch_bounds__(kBlock) void k_csc_remap(int32_t* __restrict__ cedge, const int32_t* __restrict__ ckey,
                                                    const KeepWord* __restrict__ keepw, int32_t* __restrict__ alive_in,
                                                    const Ctl* __restrict__ ctl, int round) {
    if (round && ctl->done) return;
    const int32_t N = ctl->csc_m;
    const int lane = __lane_id();
    const int32_t stride = (int32_t)(gridDim.x * kBlock);
    // wave-uniform loop: lanes take 64 consecutive entries
    for (int32_t c0 = (int32_t)(blockIdx.x * kBlock + (threadIdx.x & ~63u)); c0 < N; c0 += stride) {
        const int32_t c = c0 + lane;
        int32_t key = -1, v = 0;
        if (c < N) {
            const int32_t e = cedge[c];
            if (e >= 0) {
                const int32_t q = keep_rank(keepw, e);
                cedge[c] = q >= 0 ? q : -1;
                v = q >= 0;
            }
            key = ckey[c];
        }
        // keys never decrease along the lists (-1 past the end): equal keys at
        // both ends put the wave in one row's list, counted by one popcount
        const int32_t k_first = __builtin_amdgcn_readfirstlane(key);
        if (k_first >= 0 && k_first == __builtin_amdgcn_readlane(key, 63)) {
            const int32_t n_alive = (int32_t)__popcll(__ballot(v != 0));
            if (lane == 0 && n_alive) atomicAdd(&alive_in[k_first], n_alive);
            continue;
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(v, o);
            const int32_t kk = __shfl_up(key, o);
            if (lane >= o && kk == key) v += u;
        }
        const int32_t next = __shfl_down(key, 1);
        if (c < N && v && (lane == 63 || next != key)) atomicAdd(&alive_in[key], v);
    }
}

// ---- packing of the in-edge lists.  Tombstones keep every per-entry kernel
// at the run's edge count; once they outnumber the alive entries
// (kCscPackRatio), the lists are compacted in order (count, scan, scatter
// into scratch, row pointers remapped, copied back), so that later passes
// cost the alive count.  Decided on the device: replayed rounds pack too.
constexpr int kCscPackRatio = 2;

__global__ void k_csc_pack_decide(Ctl* ctl, int p, int round) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int32_t alive = ctl->m_buf[1 - p];
    ctl->csc_pack = !(round && ctl->done) && alive > 0 && (int64_t)ctl->csc_m > (int64_t)kCscPackRatio * alive;
}

__global__ __launch_bounds__(kBlock) void k_csc_pack_count(Csc c, const Ctl* __restrict__ ctl,
                                                         int32_t* __restrict__ blockcnt) {
    __shared__ int s_wave[kBlock / 64];
    if (!ctl->csc_pack) return;
    int32_t lo, hi;
    chunk_of(ctl->csc_m, lo, hi);
    int k = 0;
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kBlock) k += c.edge[i] >= 0;
    k = block_sum<kBlock>(k, s_wave);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = k;
}

__global__ __launch_bounds__(kScanThreads) void k_csc_pack_scan(const int32_t* __restrict__ blockcnt,
                                                              int32_t* __restrict__ blockoff, int32_t G, Ctl* ctl,
                                                              int32_t* __restrict__ cscan) {
    __shared__ int s_wave[kScanThreads / 64];
    if (!ctl->csc_pack) return;
    const int total = scan_block_counts(blockcnt, blockoff, G, s_wave);
    if (threadIdx.x == 0) {
        cscan[ctl->csc_m] = total;
        ctl->csc_next = total;
    }
}

__global__ __launch_bounds__(kBlock) void k_csc_pack_scatter(Csc c, Csc t, const Ctl* __restrict__ ctl,
                                                           const int32_t* __restrict__ blockoff,
                                                           int32_t* __restrict__ cscan) {
    __shared__ int s_wave[kBlock / 64];
    if (!ctl->csc_pack) return;
    int32_t lo, hi;
    chunk_of(ctl->csc_m, lo, hi);
    int32_t base = blockoff[blockIdx.x];
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const bool in = i < hi;
        const int32_t e = in ? c.edge[i] : -1;
        const bool k = e >= 0;
        int tot;
        const int32_t q = base + block_excl_flag<kBlock>(k, s_wave, tot);
        if (in) {
            cscan[i] = k ? q : ~q;
            if (k) {
                t.edge[q] = e;
                t.src[q] = c.src[i];
                t.key[q] = c.key[i];
            }
        }
        base += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_csc_pack_ptr(const int32_t* __restrict__ old_ptr,
                                                       int32_t* __restrict__ new_ptr, int32_t n,
                                                       const int32_t* __restrict__ cscan, const Ctl* __restrict__ ctl) {
    if (!ctl->csc_pack) return;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > n) return;
    const int32_t v = cscan[old_ptr[s]];
    new_ptr[s] = v < 0 ? ~v : v;
}

__global__ __launch_bounds__(kBlock) void k_csc_pack_copy(Csc c, Csc t, int32_t n, const Ctl* __restrict__ ctl) {
    if (!ctl->csc_pack) return;
    const int32_t N = ctl->csc_next;
    const int32_t stride = (int32_t)(gridDim.x * kBlock);
    for (int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x); i < N; i += stride) {
        c.edge[i] = t.edge[i];
        c.src[i] = t.src[i];
        c.key[i] = t.key[i];
    }
    for (int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x); i <= n; i += stride) c.ptr[i] = t.ptr[i];
}

__global__ void k_csc_pack_end(Ctl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && ctl->csc_pack) {
        ctl->csc_m = ctl->csc_next;
        ctl->csc_pack = 0;
    }
}

// ---- marking of an in-place round: the same count / scan / scatter as the
// filter, writing only the removed edges' positions (in position order) and
// their marks.
// The threshold of edge e: the run's, or its graph's in the batched form.
__device__ __forceinline__ int32_t state_thr(const Buf& x, const BatchCtx& b, int32_t thr, int32_t e) {
    return b.thrv ? b.thrv[x.src[e]] : thr;
}
__device__ __forceinline__ bool state_dying(int32_t d, int32_t thr) { return d >= 0 && d < thr; }

// Batched form: whether the wave's positions [w0, w1] all lie in one graph
// that has finished.  Its edges no longer change, so the wave skips them (no
// read of S, no marks): finished graphs stop costing a pass over their edges.
__device__ __forceinline__ bool state_wave_done(const Buf& x, const BatchCtx& b, int32_t w0, int32_t w1) {
    if (!b.thrv || w0 > w1) return false;
    const int32_t g0 = b.gidv[x.src[w0]], g1 = b.gidv[x.src[w1]];
    return g0 == g1 && b.graph_done[g0];
}

// A removed edge with support 0 lies in no triangle of the round's graph, so
// it destroys none: it is marked but not listed for the peel.
__device__ __forceinline__ bool state_listed(int32_t d) { return d > 0; }

// Per workgroup chunk: the removed edges (blockcnt2) and those listed for the
// peel (blockcnt, scanned into frontier positions).  This pass reads every
// support once and writes the round's liveness words (removed earlier: S < 0;
// removed now), which the scatter then reads instead of the supports; in the
// batched form it also counts each graph's removed edges.
__global__ __launch_bounds__(kBlock) void k_state_count(Buf x, BatchCtx b, const Ctl* __restrict__ ctl, int p,
                                                      int32_t thr, int32_t* __restrict__ blockcnt,
                                                      int32_t* __restrict__ blockcnt2,
                                                      LiveWord* __restrict__ livew) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl->done) return;
    int32_t lo, hi;
    chunk_of(ctl->m_buf[p], lo, hi);
    const int lane = __lane_id();
    int c = 0, r = 0;
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const int32_t w0 = i - lane;  // the wave's first position (a multiple of 64)
        // a wave inside one finished graph reads nothing and removes nothing
        const bool gone = state_wave_done(x, b, w0, min(w0 + 63, hi - 1));
        const int32_t d = i < hi && !gone ? x.S[i] : kDying;
        const bool kr = i < hi && !gone && state_dying(d, state_thr(x, b, thr, i));  // removed
        const bool k = kr && state_listed(d);                                          // listed for the peel
        r += kr;
        c += k;
        if (b.thrv && !gone) {
            // per-graph counts of the removed edges: a graph's edges are
            // consecutive, so the graph ids along the wave never decrease (-1
            // past the end).  Equal ids at both ends put the whole wave in one
            // graph (the usual case): one popcount and one atomic.  Otherwise
            // a segmented sum over the wave gives one atomic per graph piece.
            const int32_t key = i < hi ? b.gidv[x.src[i]] : -1;
            const int32_t k_first = __builtin_amdgcn_readfirstlane(key);
            const int32_t k_last = __builtin_amdgcn_readlane(key, 63);
            if (k_first == k_last && k_first >= 0) {
                const int32_t n_kr = (int32_t)__popcll(__ballot(kr));
                if (lane == 0 && n_kr) atomicAdd(&b.low_cnt[k_first], n_kr);
            } else {
                int32_t v = kr ? 1 : 0;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int32_t u = __shfl_up(v, o);
                    const int32_t kk = __shfl_up(key, o);
                    if (lane >= o && kk == key) v += u;
                }
                const int32_t next = __shfl_down(key, 1);
                if (i < hi && v && (lane == 63 || next != key)) atomicAdd(&b.low_cnt[key], v);
            }
        }
        const unsigned long long dead = __ballot(i < hi && d < 0);
        const unsigned long long dying = __ballot(kr);
        if (lane == 0 && w0 < hi) livew[w0 >> 6] = LiveWord{dead, dying};
    }
    c = block_sum<kBlock>(c, s_wave);
    r = block_sum<kBlock>(r, s_wave);
    if (threadIdx.x == 0) {
        blockcnt[blockIdx.x] = c;
        blockcnt2[blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_state_scan(const int32_t* __restrict__ blockcnt,
                                                           const int32_t* __restrict__ blockcnt2,
                                                           int32_t* __restrict__ blockoff, int32_t G, Ctl* ctl) {
    __shared__ int s_wave[kScanThreads / 64];
    if (ctl->done) return;
    const int total = scan_block_counts(blockcnt, blockoff, G, s_wave);
    int removed = 0;
    for (int32_t j = (int32_t)threadIdx.x; j < G; j += kScanThreads) removed += blockcnt2[j];
    removed = block_sum<kScanThreads>(removed, s_wave);
    if (threadIdx.x == 0) {
        ctl->front_n = total;
        ctl->removed_now = removed;
    }
}

// The removed edges of the round (from the liveness words) get S = kDying and
// the listed ones their frontier slots, in position order.
__global__ __launch_bounds__(kBlock) void k_state_scatter(Buf x, const Ctl* __restrict__ ctl, int p,
                                                        const int32_t* __restrict__ blockoff,
                                                        int32_t* __restrict__ frontier,
                                                        const LiveWord* __restrict__ livew) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl->done) return;
    int32_t lo, hi;
    chunk_of(ctl->m_buf[p], lo, hi);
    int32_t base = blockoff[blockIdx.x];
    const int lane = __lane_id();
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const int32_t w0 = i - lane;
        const unsigned long long dying = w0 < hi ? livew[w0 >> 6].dying : 0ull;
        const bool kr = i < hi && ((dying >> lane) & 1ull);
        const int32_t d = kr ? x.S[i] : 0;
        const bool k = kr && state_listed(d);
        int tot;
        const int32_t q = base + block_excl_flag<kBlock>(k, s_wave, tot);
        if (kr) x.S[i] = kDying;
        if (k) frontier[q] = i;
        base += tot;
    }
}

// Batched form: the run ends after the pass that leaves no edge.
__global__ void k_batch_end(Ctl* ctl, int p) {
    if (threadIdx.x == 0 && !ctl->done && ctl->m_buf[1 - p] == 0) {
        ctl->done = 1;
        ctl->final_buf = 1 - p;
    }
}

int32_t filter_grid(int32_t m_hint) {
    int64_t g = ((int64_t)m_hint + 8 * kBlock - 1) / (8 * kBlock);
    if (g < 1) g = 1;
    if (g > kMaxScanBlocks) g = kMaxScanBlocks;
    return (int32_t)g;
}

template <class P>
void run_filter(const P& pol, Ctl* ctl, int p, int update, int round, int32_t* blockcnt, int32_t* blockoff,
                int32_t* xscan, KeepWord* keepw, int32_t m_hint, hipStream_t s) {
    const int32_t G = filter_grid(m_hint);
    k_filter_count<P><<<G, kBlock, 0, s>>>(pol, ctl, p, round, blockcnt);
    k_filter_scan<<<1, kScanThreads, 0, s>>>(blockcnt, blockoff, G, ctl, p, update, round, xscan);
    k_filter_scatter<P><<<G, kBlock, 0, s>>>(pol, ctl, p, round, blockoff, xscan, keepw);
}

// Batched form, after the marking: every unfinished graph counts the pass,
// and finishes if the round removes none of its edges (its edges then stay
// put: nothing in the graph changes any more).  Runs before the round's
// fixpoint check, so the last round counts too.
__global__ __launch_bounds__(kBlock) void k_state_graphs(BatchCtx b, int32_t G, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t g = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (g >= G) return;
    if (!b.graph_done[g]) {
        b.rounds[g] += 1;
        if (b.low_cnt[g] == 0) b.graph_done[g] = 1;
    }
    b.low_cnt[g] = 0;
}

}  // namespace

hipError_t launch_state_mark(const Buf& x, const BatchCtx& b, int32_t G, int32_t thr, int32_t* frontier, Scratch& sc,
                             Ctl* ctl, int p, int32_t m_hint, hipStream_t s) {
    const int32_t grid = filter_grid(m_hint);
    LiveWord* livew = reinterpret_cast<LiveWord*>(sc.keepw);
    k_state_count<<<grid, kBlock, 0, s>>>(x, b, ctl, p, thr, sc.blockcnt, sc.blockcnt2, livew);
    k_state_scan<<<1, kScanThreads, 0, s>>>(sc.blockcnt, sc.blockcnt2, sc.blockoff, grid, ctl);
    k_state_scatter<<<grid, kBlock, 0, s>>>(x, ctl, p, sc.blockoff, frontier, livew);
    if (b.thrv && G > 0) k_state_graphs<<<grid_for(G), kBlock, 0, s>>>(b, G, ctl);
    return hipGetLastError();
}

hipError_t launch_compact(const Buf& x, const Buf& y, const Csc* cx, const Csc* cy, int32_t n, int mode, int32_t thr,
                          const uint8_t* alive_can, const BatchCtx& b, Scratch& sc, Ctl* ctl, int p, int32_t m_hint,
                          int32_t csc_hint, hipStream_t s) {
    const int round = mode != 1;  // modes 0, 2, 3 skip their work once the run is done
    const bool batch = b.thrv != nullptr;
    if (mode == 0) {
        run_filter(CsrRound{x, y, thr, b}, ctl, p, batch ? 3 : 1, 1, sc.blockcnt, sc.blockoff, sc.xscan, sc.keepw,
                   m_hint, s);
    } else if (mode == 2) {
        run_filter(CsrRound{x, y, thr, b}, ctl, p, 2, 1, sc.blockcnt, sc.blockoff, sc.xscan, sc.keepw, m_hint, s);
    } else if (mode == 3) {
        run_filter(CsrLive{x, y, b}, ctl, p, 2, 1, sc.blockcnt, sc.blockoff, sc.xscan, sc.keepw, m_hint, s);
    } else {
        run_filter(CsrAlive{x, y, alive_can}, ctl, p, 2, 0, sc.blockcnt, sc.blockoff, sc.xscan, sc.keepw, m_hint, s);
    }
    k_ptr_remap<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(x.rowptr, y.rowptr, n, sc.xscan, ctl, round);
    if (cx && csc_hint > 0) {  // the in-edge lists (one set: cy names the same arrays) and alive in-edge counts
        k_zero_rows<<<grid_for(n), kBlock, 0, s>>>(sc.alive_in, n, ctl, round);
        k_csc_remap<<<min(grid_for(csc_hint), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(cx->edge, cx->key, sc.keepw,
                                                                                         sc.alive_in, ctl, round);
        // packing when tombstones dominate; scratch that the next preparation rebuilds holds the packed copy
        const Csc t{sc.wave_tasks, sc.thread_tasks, sc.ctail, sc.itemoff};
        const int32_t G = filter_grid(csc_hint);
        k_csc_pack_decide<<<1, 64, 0, s>>>(ctl, p, round);
        k_csc_pack_count<<<G, kBlock, 0, s>>>(*cx, ctl, sc.blockcnt);
        k_csc_pack_scan<<<1, kScanThreads, 0, s>>>(sc.blockcnt, sc.blockoff, G, ctl, sc.cxscan);
        k_csc_pack_scatter<<<G, kBlock, 0, s>>>(*cx, t, ctl, sc.blockoff, sc.cxscan);
        k_csc_pack_ptr<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(cx->ptr, t.ptr, n, sc.cxscan, ctl);
        k_csc_pack_copy<<<min(grid_for(csc_hint), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(*cx, t, n, ctl);
        k_csc_pack_end<<<1, 64, 0, s>>>(ctl);
    }
    (void)cy;
    if (batch && mode == 0) k_batch_end<<<1, 64, 0, s>>>(ctl, p);
    return hipGetLastError();
}

}  // namespace kt
