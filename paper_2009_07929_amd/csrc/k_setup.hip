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

// One thread per row: columns strictly ascending, above the diagonal, below n.
// Also writes each edge's row into src_out.  Skipped when rowptr is invalid,
// so a malformed rowptr is never walked.
// Columns of every row strictly ascending, above the diagonal and below n;
// also writes the row of every edge.  Each thread takes kValSpan consecutive
// edges, finds the row of the first by binary search over rowptr (already
// checked monotone) and walks on, so long rows cost no more than short ones.
constexpr int kValSpan = 16;

// tally: also accumulates the input statistic of the light-graph gate into
// ctl->merge_work: the tail of every edge's row after it, exactly, plus the
// length of row kappa (the edge's column) sampled on the first edge of every
// span of kValSpan edges and weighted by the span's edge count.
__global__ __launch_bounds__(kBlock) void k_validate_rows(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, int32_t n, int32_t m,
                                                        int32_t* __restrict__ src_out, Ctl* ctl, bool tally) {
    if (ctl->err) return;
    const int64_t p0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kValSpan;
    unsigned long long work = 0ull;
    if (p0 < m) {
        // row = last i with rowptr[i] <= p0
        int32_t lo = 0, hi = n;  // rowptr[lo] <= p0 < rowptr[hi]
        while (hi - lo > 1) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (rowptr[mid] <= p0) lo = mid;
            else hi = mid;
        }
        int32_t row = lo, next = rowptr[row + 1];
        const int32_t p1 = (int32_t)min(p0 + kValSpan, (int64_t)m);
        int bad = 0;
        for (int32_t p = (int32_t)p0; p < p1; ++p) {
            while (p >= next) next = rowptr[++row + 1];
            const int32_t prev = p == rowptr[row] ? row : col[p - 1];
            const int32_t c = col[p];
            const bool b = (c <= prev) | (c >= n);
            bad |= b;
            src_out[p] = row;
            if (tally && !b) {
                work += (unsigned long long)(next - p - 1);
                if (p == p0) work += (unsigned long long)(p1 - p0) * (unsigned long long)(rowptr[c + 1] - rowptr[c]);
            }
        }
        if (bad) atomicOr(&ctl->err, 16);
    }
    if (tally) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) work += __shfl_xor(work, o);
        if (__lane_id() == 0 && work) atomicAdd(&ctl->merge_work, work);
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
    if (e < ctl->m_buf[f]) trussness[b.eid[e]] = K;
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
    const int32_t c = b.eid[e];
    if (mask) mask[c] = 1;
    support[c] = b.S[e];
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
        k_validate_rows<<<grid_for(((int64_t)m + kValSpan - 1) / kValSpan), kBlock, 0, s>>>(rowptr, col, n, m, src_out,
                                                                                           ctl, tally);
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
