// Device kernels of the K-truss hot path for gfx950 (CDNA4, wave64).
//
// Working graph: the alive edges, compacted in canonical order into one of
// two buffers (Buf).  A prune round reads buffer p and writes the survivors
// into buffer 1-p; the control block (Ctl) on the device says how many edges
// each buffer holds and whether the fixpoint has been reached, so that every
// kernel of a round can be enqueued (or replayed from a graph) without a host
// round trip, and turns into a no-op once a pass has removed nothing.
#include "kernels.h"

namespace kt {

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive prefix of `flag` over a kBlock-thread workgroup (ballot + mbcnt
// inside each wave, wave totals through LDS).  `total` receives the count.
__device__ __forceinline__ int block_excl_prefix(bool flag, int* s_wave, int& total) {
    const uint64_t bal = __ballot(flag);
    const int w = threadIdx.x >> 6;
    const int pre = (int)lanes_below(bal);
    if (__lane_id() == 0) s_wave[w] = __popcll(bal);
    __syncthreads();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        const int c = s_wave[i];
        wpre += i < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return wpre + pre;
}

__device__ __forceinline__ int block_sum(int v, int* s_wave) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) s_wave[w] = v;
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) tot += s_wave[i];
    __syncthreads();
    return tot;
}

static inline unsigned grid_for(int64_t items, int per_block = kBlock) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

// ------------------------------------------------------ validation, set-up

__global__ void k_ctl_reset(Ctl* ctl, int32_t m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->m_buf[0] = m;
        ctl->m_buf[1] = 0;
        ctl->done = 0;
        ctl->final_buf = 0;
        ctl->rounds = 0;
        ctl->err = 0;
        ctl->kept = m;
        ctl->pad = 0;
        ctl->removed_total = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_validate_rowptr(const int32_t* __restrict__ rowptr, int32_t n, int32_t m,
                                                          Ctl* ctl) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > n) return;
    const int32_t v = rowptr[s];
    int bad = 0;
    if (v < 0 || v > m) bad |= 1;
    if (s == 0 && v != 0) bad |= 2;
    if (s == n && v != m) bad |= 4;
    if (s < n && rowptr[s + 1] < v) bad |= 8;
    if (bad) atomicOr(&ctl->err, bad);
}

// One thread per row: columns strictly ascending, above the diagonal, below n.
// Also writes each edge's row into src_out.  Skipped when rowptr is invalid,
// so a malformed rowptr is never walked.
__global__ __launch_bounds__(kBlock) void k_validate_rows(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, int32_t n,
                                                        int32_t* __restrict__ src_out, Ctl* ctl) {
    if (ctl->err) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t b = rowptr[i], e = rowptr[i + 1];
    int32_t prev = (int32_t)i;
    int bad = 0;
    for (int32_t p = b; p < e; ++p) {
        const int32_t c = col[p];
        bad |= (c <= prev) | (c >= n);
        prev = c;
        src_out[p] = (int32_t)i;
    }
    if (bad) atomicOr(&ctl->err, 16);
}

__global__ __launch_bounds__(kBlock) void k_init_eid_s(int32_t* __restrict__ eid, int32_t* __restrict__ S, int32_t m) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < m) {
        eid[e] = (int32_t)e;
        S[e] = 0;
    }
}

hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m, int32_t* src_out,
                           Ctl* ctl, hipStream_t s) {
    k_ctl_reset<<<1, 64, 0, s>>>(ctl, m);
    k_validate_rowptr<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(rowptr, n, m, ctl);
    if (n > 0) k_validate_rows<<<grid_for(n), kBlock, 0, s>>>(rowptr, col, n, src_out, ctl);
    return hipGetLastError();
}

// Buffer `b` := the whole input graph (its src was written by validation).
hipError_t launch_init_run(const Buf& b, const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m, Ctl* ctl,
                           hipStream_t s) {
    (void)ctl;
    hipError_t e = hipMemcpyAsync(b.rowptr, rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (m > 0) {
        e = hipMemcpyAsync(b.col, col, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        k_init_eid_s<<<grid_for(m), kBlock, 0, s>>>(b.eid, b.S, m);
    }
    return hipGetLastError();
}

// --------------------------------------------------- support: thread/edge

// One thread per alive edge e = (i, k): merge the part of row i after e with
// row k (both ascending).  Every common column w closes the triangle
// (i, k, w): the supports of (i, w) and (k, w) are bumped atomically where the
// merge finds them, and e's own support once with the triangle count.  This
// is the task of Algorithm 3 (one per non-zero), in the merge form the
// paper's Kokkos listing uses.
__global__ __launch_bounds__(kBlock) void k_support_thread_edge(const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ col,
                                                              const int32_t* __restrict__ src, int32_t* S,
                                                              const Ctl* __restrict__ ctl, int p) {
    if (ctl->done) return;
    const int32_t m_r = ctl->m_buf[p];
    const int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (e >= m_r) return;
    const int32_t i = src[e];
    const int32_t k = col[e];
    int32_t a = e + 1;
    const int32_t ae = rowptr[i + 1];
    int32_t b = rowptr[k];
    const int32_t be = rowptr[k + 1];
    int32_t cnt = 0;
    if (a < ae && b < be) {
        int32_t x = col[a], y = col[b];
        for (;;) {
            if (x == y) {
                atomicAdd(&S[a], 1);
                atomicAdd(&S[b], 1);
                ++cnt;
                if (++a >= ae || ++b >= be) break;
                x = col[a];
                y = col[b];
            } else if (x < y) {
                if (++a >= ae) break;
                x = col[a];
            } else {
                if (++b >= be) break;
                y = col[b];
            }
        }
    }
    if (cnt) atomicAdd(&S[e], cnt);
}

hipError_t launch_support_thread_edge(const Buf& x, const Ctl* ctl, int p, int32_t m_hint, hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    k_support_thread_edge<<<grid_for(m_hint), kBlock, 0, s>>>(x.rowptr, x.col, x.src, x.S, ctl, p);
    return hipGetLastError();
}

// ----------------------------------------------------- prune + compaction

template <int MODE>
__device__ __forceinline__ bool keep_edge(const Buf& x, const uint8_t* __restrict__ alive_can, int32_t thr, int32_t e) {
    if (MODE == 0) return x.S[e] >= thr;
    return alive_can[x.eid[e]] != 0;
}

// Blocks split the alive range into G contiguous chunks; count survivors per chunk.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_count_keep(Buf x, const uint8_t* __restrict__ alive_can, int32_t thr,
                                                     const Ctl* __restrict__ ctl, int p, int32_t* __restrict__ blockcnt) {
    __shared__ int s_wave[kBlock / 64];
    if (MODE == 0 && ctl->done) return;
    const int32_t m_r = ctl->m_buf[p];
    const int32_t G = (int32_t)gridDim.x;
    const int32_t chunk = (int32_t)(((int64_t)m_r + G - 1) / G);
    const int32_t lo = (int32_t)min((int64_t)blockIdx.x * chunk, (int64_t)m_r);
    const int32_t hi = (int32_t)min((int64_t)lo + chunk, (int64_t)m_r);
    int c = 0;
    for (int32_t e = lo + (int32_t)threadIdx.x; e < hi; e += kBlock) c += keep_edge<MODE>(x, alive_can, thr, e);
    c = block_sum(c, s_wave);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = c;
}

// One workgroup: exclusive scan of the G chunk counts; records the survivor
// count and, for a prune round, the pass count and the fixpoint flag.
template <int MODE>
__global__ __launch_bounds__(kScanThreads) void k_scan_counts(const int32_t* __restrict__ blockcnt,
                                                            int32_t* __restrict__ blockoff, int32_t G, Ctl* ctl, int p,
                                                            int32_t* __restrict__ xscan) {
    __shared__ int s_wave[kScanThreads / 64];
    if (MODE == 0 && ctl->done) return;
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
    // inclusive scan of `local` across the workgroup
    int inc = local;
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    const int w = t >> 6;
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    int wbase = 0, total = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
        const int c = s_wave[i];
        wbase += i < w ? c : 0;
        total += c;
    }
    int run = wbase + inc - local;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = t * PER + j;
        if (idx < G) blockoff[idx] = run;
        run += v[j];
    }
    if (t == 0) {
        const int32_t m_r = ctl->m_buf[p];
        xscan[m_r] = total;
        ctl->kept = total;
        if (MODE == 0) {
            ctl->rounds += 1;
            const int32_t removed = m_r - total;
            if (removed == 0) {
                ctl->done = 1;
                ctl->final_buf = p;
            } else {
                ctl->m_buf[1 - p] = total;
                ctl->removed_total += removed;
            }
        } else {
            ctl->m_buf[1 - p] = total;
        }
    }
}

// Scatter the survivors of buffer p into buffer 1-p (order preserved) and
// record every old position's new position in xscan.  Within each 256-edge
// tile, positions come from a wave ballot + mbcnt prefix and the wave totals.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_compact(Buf x, Buf y, const uint8_t* __restrict__ alive_can, int32_t thr,
                                                  const Ctl* __restrict__ ctl, int p,
                                                  const int32_t* __restrict__ blockoff, int32_t* __restrict__ xscan) {
    __shared__ int s_wave[kBlock / 64];
    if (MODE == 0 && ctl->done) return;
    const int32_t m_r = ctl->m_buf[p];
    const int32_t G = (int32_t)gridDim.x;
    const int32_t chunk = (int32_t)(((int64_t)m_r + G - 1) / G);
    const int32_t lo = (int32_t)min((int64_t)blockIdx.x * chunk, (int64_t)m_r);
    const int32_t hi = (int32_t)min((int64_t)lo + chunk, (int64_t)m_r);
    int32_t base = blockoff[blockIdx.x];
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t e = t0 + (int32_t)threadIdx.x;
        const bool in = e < hi;
        const bool k = in && keep_edge<MODE>(x, alive_can, thr, e);
        int tot;
        const int q = base + block_excl_prefix(k, s_wave, tot);
        if (in) {
            xscan[e] = q;
            if (k) {
                y.col[q] = x.col[e];
                y.src[q] = x.src[e];
                y.eid[q] = x.eid[e];
                y.S[q] = 0;
            }
        }
        base += tot;
    }
}

// New row pointers: row s of the new buffer starts where its first old
// position went.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_rowptr(const int32_t* __restrict__ old_rowptr, int32_t* __restrict__ new_rowptr,
                                                 int32_t n, const int32_t* __restrict__ xscan, const Ctl* __restrict__ ctl) {
    if (MODE == 0 && ctl->done) return;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > n) return;
    new_rowptr[s] = xscan[old_rowptr[s]];
}

static inline int32_t compact_grid(int32_t m_hint) {
    int64_t g = ((int64_t)m_hint + 8 * kBlock - 1) / (8 * kBlock);
    if (g < 1) g = 1;
    if (g > kMaxScanBlocks) g = kMaxScanBlocks;
    return (int32_t)g;
}

hipError_t launch_compact(const Buf& x, const Buf& y, int32_t n, int mode, int32_t thr, const uint8_t* alive_can,
                          int32_t* xscan, int32_t* blockcnt, int32_t* blockoff, Ctl* ctl, int p, int32_t m_hint,
                          hipStream_t s) {
    const int32_t G = compact_grid(m_hint);
    if (mode == 0) {
        k_count_keep<0><<<G, kBlock, 0, s>>>(x, alive_can, thr, ctl, p, blockcnt);
        k_scan_counts<0><<<1, kScanThreads, 0, s>>>(blockcnt, blockoff, G, ctl, p, xscan);
        k_compact<0><<<G, kBlock, 0, s>>>(x, y, alive_can, thr, ctl, p, blockoff, xscan);
        k_rowptr<0><<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(x.rowptr, y.rowptr, n, xscan, ctl);
    } else {
        k_count_keep<1><<<G, kBlock, 0, s>>>(x, alive_can, thr, ctl, p, blockcnt);
        k_scan_counts<1><<<1, kScanThreads, 0, s>>>(blockcnt, blockoff, G, ctl, p, xscan);
        k_compact<1><<<G, kBlock, 0, s>>>(x, y, alive_can, thr, ctl, p, blockoff, xscan);
        k_rowptr<1><<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(x.rowptr, y.rowptr, n, xscan, ctl);
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------- outputs

__global__ void k_set_final(Ctl* ctl, int f) {
    if (threadIdx.x == 0) ctl->final_buf = f;
}

hipError_t launch_set_final(Ctl* ctl, int f, hipStream_t s) {
    k_set_final<<<1, 64, 0, s>>>(ctl, f);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_scatter_out(Buf b0, Buf b1, const Ctl* __restrict__ ctl,
                                                      uint8_t* __restrict__ mask, int32_t* __restrict__ support) {
    const int f = ctl->final_buf;
    const Buf& b = f ? b1 : b0;
    const int32_t m_f = ctl->m_buf[f];
    const int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (e >= m_f) return;
    const int32_t c = b.eid[e];
    if (mask) mask[c] = 1;
    support[c] = b.S[e];
}

hipError_t launch_scatter_out(const Buf& b0, const Buf& b1, const Ctl* ctl, uint8_t* mask, int32_t* support,
                              int32_t m_hint, hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    k_scatter_out<<<grid_for(m_hint), kBlock, 0, s>>>(b0, b1, ctl, mask, support);
    return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long* p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__global__ __launch_bounds__(kBlock) void k_prune_canonical(const int32_t* __restrict__ support, uint8_t* __restrict__ alive,
                                                          int32_t m, int32_t thr, unsigned long long* removed) {
    __shared__ int s_wave[kBlock / 64];
    const int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    int gone = 0;
    if (e < m) {
        const bool was = alive[e] != 0;
        const bool keep = was && support[e] >= thr;
        alive[e] = keep ? 1 : 0;
        gone = was && !keep;
    }
    if (removed) {
        gone = block_sum(gone, s_wave);
        if (threadIdx.x == 0 && gone) atomicAdd(removed, (unsigned long long)gone);
    }
}

hipError_t launch_prune_canonical(const int32_t* support, uint8_t* alive, int32_t m, int32_t thr,
                                  unsigned long long* removed, hipStream_t s) {
    if (removed) k_zero_u64<<<1, 64, 0, s>>>(removed);
    if (m > 0) k_prune_canonical<<<grid_for(m), kBlock, 0, s>>>(support, alive, m, thr, removed);
    return hipGetLastError();
}

}  // namespace kt
