// Input validation, working-buffer set-up, outputs and the stateless prune.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

__global__ void k_ctl_reset(Ctl* ctl, int32_t m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->m_buf[0] = m;
        ctl->m_buf[1] = 0;
        ctl->done = 0;
        ctl->need_support = 0;
        ctl->final_buf = 0;
        ctl->rounds = 0;
        ctl->err = 0;
        ctl->kept = m;
        ctl->n_items = 0;
        ctl->n_wave = 0;
        ctl->n_thread = 0;
        ctl->item_next = 0;
        ctl->n_active = 0;
        ctl->n_samples = 0;
        ctl->csc_m = m;
        ctl->csc_pack = 0;
        ctl->csc_next = m;
        ctl->merge_work = 0ull;
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

// Columns of every row strictly ascending, above the diagonal and below n;
// also writes the row of every edge.  Every workgroup takes a tile of
// kValTile consecutive edges: two of its lanes find the rows of the tile's
// first and last edge by binary search over rowptr (already checked
// monotone, so a malformed rowptr is never walked), every row in between
// marks the tile slot where it starts (the largest row wins, so empty rows
// give way), and a max-scan over the tile gives every edge its row.  The
// lanes then check their 8 consecutive edges.
constexpr int kValSpan = 16;
constexpr int kValPer = 8;
constexpr int kValTile = kBlock * kValPer;
constexpr int kValMaxGrid = 2048;  // workgroups (tiles strided over them)

// tally: also accumulates the input statistic of the light-graph gate into
// ctl->merge_work: the tail of every edge's row after it, exactly (summed per
// row as d (d - 1) / 2 by the tile holding the row's first edge), plus the
// length of row kappa (the edge's column) sampled on every edge whose position
// is a multiple of kValSpan and weighted by the edge count of that span.
__global__ __launch_bounds__(kBlock) void k_validate_rows(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, int32_t n, int32_t m,
                                                        int32_t* __restrict__ src_out, Ctl* ctl, bool tally) {
    __shared__ int32_t s_row[kValTile];
    __shared__ int32_t s_r[2];
    __shared__ int32_t s_wmax[kBlock / 64];
    __shared__ unsigned long long s_work[kBlock / 64];
    if (ctl->err & 15) return;  // rowptr's own checks (bit 16 is this kernel's, set concurrently)
    const int t = threadIdx.x, lane = __lane_id(), wv = t >> 6;
    unsigned long long work = 0ull;
    int bad = 0;
    // tiles strided over the grid: one atomic per workgroup for the statistic
    for (int64_t q0 = (int64_t)blockIdx.x * kValTile; q0 < m; q0 += (int64_t)gridDim.x * kValTile) {
        const int32_t p0 = (int32_t)q0;
        const int32_t cnt = (int32_t)min((int64_t)kValTile, (int64_t)m - q0);
        __syncthreads();  // the previous tile is done with s_row, s_r and s_wmax
        if (t < 2) {      // last row i with rowptr[i] <= x, with rowptr[lo] <= x < rowptr[hi]
            const int32_t x = t == 0 ? p0 : p0 + cnt - 1;
            int32_t lo = 0, hi = n;
            while (hi - lo > 1) {
                const int32_t mid = lo + ((hi - lo) >> 1);
                if (rowptr[mid] <= x) lo = mid;
                else hi = mid;
            }
            s_r[t] = lo;
        }
#pragma unroll
        for (int j = 0; j < kValPer; ++j) s_row[t * kValPer + j] = -1;
        __syncthreads();
        const int32_t r0 = s_r[0], r1 = s_r[1];
        if (t == 0) {
            s_row[0] = r0;
            if (tally && rowptr[r0] == p0) {  // the statistic's tail part, per row: sum of its tails d (d - 1) / 2
                const uint64_t d = (uint64_t)(rowptr[r0 + 1] - p0);
                work += d * (d - 1) / 2;
            }
        }
        for (int32_t r = r0 + 1 + t; r <= r1; r += kBlock) {  // rows starting inside the tile
            const int32_t q = rowptr[r] - p0;
            if (q > 0 && q < cnt) atomicMax(&s_row[q], r);
            if (tally) {
                const uint64_t d = (uint64_t)(rowptr[r + 1] - rowptr[r]);
                work += d * (d - 1) / 2;
            }
        }
        __syncthreads();
        // inclusive max-scan: 8 slots per lane, then across lanes and waves
        int32_t v[kValPer];
        int32_t run = -1;
#pragma unroll
        for (int j = 0; j < kValPer; ++j) {
            run = max(run, s_row[t * kValPer + j]);
            v[j] = run;
        }
        int32_t incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(incl, o);
            if (lane >= o) incl = max(incl, u);
        }
        if (lane == 63) s_wmax[wv] = incl;
        __syncthreads();
        int32_t before = __shfl_up(incl, 1);
        if (lane == 0) before = -1;
        for (int i = 0; i < wv; ++i) before = max(before, s_wmax[i]);
        // the row of the slot before this lane's first (for the first-of-row test)
        int32_t prev_row = before;
#pragma unroll
        for (int j = 0; j < kValPer; ++j) {
            const int32_t i = t * kValPer + j;
            const int32_t row = max(before, v[j]);
            if (i < cnt) {
                const int32_t p = p0 + i;
                const bool first = i == 0 ? rowptr[row] == p : row != prev_row;
                const int32_t prev = first ? row : col[p - 1];
                const int32_t cv = col[p];
                const bool b = (cv <= prev) | (cv >= n);
                bad |= b;
                src_out[p] = row;
                if (tally && !b && p % kValSpan == 0)
                    work += (unsigned long long)(min(p + kValSpan, m) - p) *
                            (unsigned long long)(rowptr[cv + 1] - rowptr[cv]);
            }
            prev_row = row;
        }
    }
    if (bad) atomicOr(&ctl->err, 16);
    if (tally) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) work += __shfl_xor(work, o);
        if (lane == 0) s_work[wv] = work;
        __syncthreads();
        if (t == 0) {
            unsigned long long tot = 0ull;
#pragma unroll
            for (int i = 0; i < kBlock / 64; ++i) tot += s_work[i];
            if (tot) atomicAdd(&ctl->merge_work, tot);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_init_eid_s(int32_t* __restrict__ eid, int32_t* __restrict__ S, int32_t m) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < m) {
        eid[e] = (int32_t)e;
        S[e] = 0;
    }
}

// Survivors of a decomposition level (buffer f of the fixpoint) get trussness K.
__global__ __launch_bounds__(kBlock) void k_mark_level(Buf b, const Ctl* __restrict__ ctl, int f, int32_t K,
                                                     int32_t* __restrict__ trussness) {
    const int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (e < ctl->m_buf[f] && b.S[e] >= 0) trussness[b.eid[e]] = K;  // S < 0: removed in place
}

__global__ __launch_bounds__(kBlock) void k_fill_value(int32_t* __restrict__ a, int32_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = v;
}

// Next decomposition level: the fixpoint flag is cleared so that the rounds
// continue from the final buffer.
__global__ void k_ctl_restart(Ctl* ctl) {
    if (threadIdx.x == 0) {
        ctl->done = 0;
        ctl->need_support = 0;
    }
}

__global__ void k_set_final(Ctl* ctl, int f) {
    if (threadIdx.x == 0) ctl->final_buf = f;
}

__global__ __launch_bounds__(kBlock) void k_scatter_out(Buf b0, Buf b1, const Ctl* __restrict__ ctl,
                                                      uint8_t* __restrict__ mask, int32_t* __restrict__ support) {
    const int f = ctl->final_buf;
    const Buf& b = f ? b1 : b0;
    const int32_t m_f = ctl->m_buf[f];
    const int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (e >= m_f) return;
    const int32_t v = b.S[e];
    if (v < 0) return;  // removed by an in-place round (outputs were zeroed)
    const int32_t c = b.eid[e];
    if (mask) mask[c] = 1;
    support[c] = v;
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
        gone = block_sum<kBlock>(gone, s_wave);
        if (threadIdx.x == 0 && gone) atomicAdd(removed, (unsigned long long)gone);
    }
}

}  // namespace

hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m, int32_t* src_out,
                           Ctl* ctl, bool tally, hipStream_t s) {
    k_ctl_reset<<<1, 64, 0, s>>>(ctl, m);
    k_validate_rowptr<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(rowptr, n, m, ctl);
    if (n > 0 && m > 0)
        k_validate_rows<<<(unsigned)min(((int64_t)m + kValTile - 1) / kValTile, (int64_t)kValMaxGrid), kBlock, 0,
                          s>>>(rowptr, col, n, m, src_out, ctl, tally);
    return hipGetLastError();
}

// Buffer `b` := the whole input graph (its src was written by validation).
hipError_t launch_init_run(const Buf& b, const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m,
                           hipStream_t s) {
    hipError_t e = hipMemcpyAsync(b.rowptr, rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (m > 0) {
        e = hipMemcpyAsync(b.col, col, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        k_init_eid_s<<<grid_for(m), kBlock, 0, s>>>(b.eid, b.S, m);
    }
    return hipGetLastError();
}

hipError_t launch_mark_level(const Buf& b, const Ctl* ctl, int f, int32_t m_hint, int32_t K, int32_t* trussness,
                             hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    k_mark_level<<<grid_for(m_hint), kBlock, 0, s>>>(b, ctl, f, K, trussness);
    return hipGetLastError();
}

hipError_t launch_fill_value(int32_t* a, int32_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_value<<<grid_for(n), kBlock, 0, s>>>(a, n, v);
    return hipGetLastError();
}

hipError_t launch_ctl_restart(Ctl* ctl, hipStream_t s) {
    k_ctl_restart<<<1, 64, 0, s>>>(ctl);
    return hipGetLastError();
}

hipError_t launch_set_final(Ctl* ctl, int f, hipStream_t s) {
    k_set_final<<<1, 64, 0, s>>>(ctl, f);
    return hipGetLastError();
}

hipError_t launch_scatter_out(const Buf& b0, const Buf& b1, const Ctl* ctl, uint8_t* mask, int32_t* support,
                              int32_t m_hint, hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    k_scatter_out<<<grid_for(m_hint), kBlock, 0, s>>>(b0, b1, ctl, mask, support);
    return hipGetLastError();
}

hipError_t launch_prune_canonical(const int32_t* support, uint8_t* alive, int32_t m, int32_t thr,
                                  unsigned long long* removed, hipStream_t s) {
    if (removed) k_zero_u64<<<1, 64, 0, s>>>(removed);
    if (m > 0) k_prune_canonical<<<grid_for(m), kBlock, 0, s>>>(support, alive, m, thr, removed);
    return hipGetLastError();
}

}  // namespace kt
