// Scheduling structures of the support pass.
//
// Algorithm 3's task (i, j) selects row kappa = a12(j) of A22 and updates
// S(kappa, :).  Grouping the tasks by kappa lets one workgroup stage row kappa
// once in LDS for all the tasks that select it ("hub rows").  This file builds
//   - the in-edge lists (for every kappa, the edge positions whose column is
//     kappa: a CSR transpose), once per run; prune rounds compact them;
//   - per pass, the work lists of the kernel variants: hub items
//     (kappa, chunk of its in-edges) and the remaining edge tasks split into
//     wavefront-per-edge and thread-per-edge lists, by the static degree
//     heuristic or by per-row bins chosen by the cost model.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* __restrict__ a, int32_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_indeg(const int32_t* __restrict__ col, int32_t m, int32_t* __restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < m) atomicAdd(&cnt[col[e]], 1);
}

__global__ __launch_bounds__(kBlock) void k_csc_scatter(const int32_t* __restrict__ col, int32_t m,
                                                      const int32_t* __restrict__ cptr, int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ cedge) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int32_t k = col[e];
    cedge[cptr[k] + atomicAdd(&cursor[k], 1)] = (int32_t)e;
}

// ---- device-wide exclusive scan of f(0..N-1) into out[0..N], out[N] = total

struct FromArray {
    const int32_t* a;
    __device__ int32_t operator()(int32_t i) const { return a[i]; }
};

__device__ __forceinline__ void span_of(int32_t N, int32_t& lo, int32_t& hi) {
    const int32_t G = (int32_t)gridDim.x;
    const int32_t chunk = (int32_t)(((int64_t)N + G - 1) / G);
    lo = (int32_t)min((int64_t)blockIdx.x * chunk, (int64_t)N);
    hi = (int32_t)min((int64_t)lo + chunk, (int64_t)N);
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_partial(F f, int32_t N, const Ctl* __restrict__ ctl,
                                                       int32_t* __restrict__ blockcnt) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl && ctl->done) return;
    int32_t lo, hi;
    span_of(N, lo, hi);
    int c = 0;
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kBlock) c += f(i);
    c = block_sum<kBlock>(c, s_wave);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = c;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int32_t* __restrict__ blockcnt,
                                                            int32_t* __restrict__ blockoff, int32_t G,
                                                            const Ctl* __restrict__ ctl) {
    __shared__ int s_wave[kScanThreads / 64];
    if (ctl && ctl->done) return;
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
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_write(F f, int32_t N, const Ctl* __restrict__ ctl,
                                                     const int32_t* __restrict__ blockoff, int32_t* __restrict__ out,
                                                     int32_t* total_dst) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl && ctl->done) return;
    int32_t lo, hi;
    span_of(N, lo, hi);
    int32_t base = blockoff[blockIdx.x];
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const int v = i < hi ? f(i) : 0;
        int tot;
        const int32_t pre = block_excl_sum<kBlock>(v, s_wave, tot);
        if (i < hi) out[i] = base + pre;
        base += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        out[N] = base;
        if (total_dst) *total_dst = base;
    }
}

int32_t scan_grid(int32_t N) {
    int64_t g = ((int64_t)N + 8 * kBlock - 1) / (8 * kBlock);
    if (g < 1) g = 1;
    if (g > kMaxScanBlocks) g = kMaxScanBlocks;
    return (int32_t)g;
}

template <class F>
void device_scan(const F& f, int32_t N, const Ctl* ctl, Scratch& sc, int32_t* out, int32_t* total_dst, hipStream_t s) {
    const int32_t G = scan_grid(N);
    k_scan_partial<F><<<G, kBlock, 0, s>>>(f, N, ctl, sc.blockcnt);
    k_scan_blocks<<<1, kScanThreads, 0, s>>>(sc.blockcnt, sc.blockoff, G, ctl);
    k_scan_write<F><<<G, kBlock, 0, s>>>(f, N, ctl, sc.blockoff, out, total_dst);
}

// ---- hub items

// Number of hub items of row kappa: its in-edges cut into chunks of kHubChunk.
struct HubChunks {
    const int32_t* rowptr;
    const int32_t* cptr;
    const uint8_t* is_hub;  // per row, or null = every row with work
    __device__ int32_t operator()(int32_t k) const {
        const int32_t indeg = cptr[k + 1] - cptr[k];
        const int32_t d = rowptr[k + 1] - rowptr[k];
        if (indeg == 0 || d == 0) return 0;
        if (is_hub && !is_hub[k]) return 0;
        return (indeg + kHubChunk - 1) / kHubChunk;
    }
};

__global__ __launch_bounds__(kBlock) void k_hub_items(HubChunks f, int32_t n, const int32_t* __restrict__ itemoff,
                                                    int32_t* __restrict__ item_kappa, int32_t* __restrict__ item_c0,
                                                    const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k == 0) const_cast<Ctl*>(ctl)->item_next = 0;
    if (k >= n) return;
    const int32_t nch = f((int32_t)k);
    const int32_t o = itemoff[k];
    const int32_t c0 = f.cptr[k];
    for (int32_t j = 0; j < nch; ++j) {
        item_kappa[o + j] = (int32_t)k;
        item_c0[o + j] = c0 + j * kHubChunk;
    }
}

// ---- static degree heuristic: which rows kappa are hub rows

__global__ __launch_bounds__(kBlock) void k_heuristic_bins(const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ cptr, int32_t n,
                                                         int32_t hub_min_in, uint8_t* __restrict__ is_hub,
                                                         const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int32_t indeg = cptr[k + 1] - cptr[k];
    const int32_t d = rowptr[k + 1] - rowptr[k];
    is_hub[k] = (d > 0 && indeg >= hub_min_in) ? 1 : 0;
}

// ---- remaining edge tasks: wavefront-per-edge vs thread-per-edge lists

// Class of in-edge list entry c: 0 = handled by a hub item, 1 = wavefront,
// 2 = thread.  Merge length of the task = tail of its row + |N+(kappa)|.
struct TaskClass {
    Buf x;
    Csc c;
    const uint8_t* is_hub;
    int32_t wave_min;
    __device__ int cls(int32_t i) const {
        const int32_t e = c.edge[i];
        const int32_t k = x.col[e];
        if (is_hub[k]) return 0;
        const int32_t tail = x.rowptr[x.src[e] + 1] - e - 1;
        const int32_t d = x.rowptr[k + 1] - x.rowptr[k];
        if (tail == 0 || d == 0) return 0;  // no triangle can close on this task
        return (tail + d >= wave_min) ? 1 : 2;
    }
};

__global__ __launch_bounds__(kBlock) void k_task_count(TaskClass tc, const Ctl* __restrict__ ctl, int p,
                                                     int32_t* __restrict__ cnt2) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl->done) return;
    int32_t lo, hi;
    span_of(ctl->m_buf[p], lo, hi);
    int a = 0, b = 0;
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kBlock) {
        const int k = tc.cls(i);
        a += k == 1;
        b += k == 2;
    }
    a = block_sum<kBlock>(a, s_wave);
    b = block_sum<kBlock>(b, s_wave);
    if (threadIdx.x == 0) {
        cnt2[blockIdx.x] = a;
        cnt2[kMaxScanBlocks + blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_task_scan(const int32_t* __restrict__ cnt2, int32_t* __restrict__ off2,
                                                          int32_t G, Ctl* ctl) {
    __shared__ int s_wave[kScanThreads / 64];
    if (ctl->done) return;
    constexpr int PER = kMaxScanBlocks / kScanThreads;
    const int t = threadIdx.x;
    for (int list = 0; list < 2; ++list) {
        const int32_t* c = cnt2 + list * kMaxScanBlocks;
        int32_t* o = off2 + list * kMaxScanBlocks;
        int v[PER];
        int local = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int idx = t * PER + j;
            v[j] = idx < G ? c[idx] : 0;
            local += v[j];
        }
        int total;
        int run = block_excl_sum<kScanThreads>(local, s_wave, total);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int idx = t * PER + j;
            if (idx < G) o[idx] = run;
            run += v[j];
        }
        if (t == 0) {
            if (list == 0) ctl->n_wave = total;
            else ctl->n_thread = total;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_task_scatter(TaskClass tc, const Ctl* __restrict__ ctl, int p,
                                                       const int32_t* __restrict__ off2,
                                                       int32_t* __restrict__ wave_tasks,
                                                       int32_t* __restrict__ thread_tasks) {
    __shared__ int s_wave[kBlock / 64];
    if (ctl->done) return;
    int32_t lo, hi;
    span_of(ctl->m_buf[p], lo, hi);
    int32_t ba = off2[blockIdx.x], bb = off2[kMaxScanBlocks + blockIdx.x];
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const int k = i < hi ? tc.cls(i) : 0;
        int ta, tb;
        const int32_t qa = ba + block_excl_flag<kBlock>(k == 1, s_wave, ta);
        const int32_t qb = bb + block_excl_flag<kBlock>(k == 2, s_wave, tb);
        if (k == 1) wave_tasks[qa] = tc.c.edge[i];
        if (k == 2) thread_tasks[qb] = tc.c.edge[i];
        ba += ta;
        bb += tb;
    }
}

}  // namespace

hipError_t launch_build_csc(const Buf& b, const Csc& c, int32_t n, int32_t m, Scratch& sc, hipStream_t s) {
    k_fill_i32<<<grid_for(n), kBlock, 0, s>>>(sc.tmp_n, n, 0);
    if (m > 0) k_indeg<<<grid_for(m), kBlock, 0, s>>>(b.col, m, sc.tmp_n);
    device_scan(FromArray{sc.tmp_n}, n, nullptr, sc, c.ptr, nullptr, s);
    k_fill_i32<<<grid_for(n), kBlock, 0, s>>>(sc.tmp_n, n, 0);
    if (m > 0) k_csc_scatter<<<grid_for(m), kBlock, 0, s>>>(b.col, m, c.ptr, sc.tmp_n, c.edge);
    return hipGetLastError();
}

hipError_t launch_prepare_pass(const Buf& x, const Csc& c, int32_t n, int sched, const ktruss_tuning& t,
                               const uint8_t* learned_hub, Scratch& sc, Ctl* ctl, int p, int32_t m_hint,
                               hipStream_t s) {
    const uint8_t* is_hub = nullptr;
    if (sched == KTRUSS_SCHED_HEURISTIC) {
        const int32_t hub_min_in = t.hub_min_work > 0 ? t.hub_min_work : kDefaultHubMinIn;
        k_heuristic_bins<<<grid_for(n), kBlock, 0, s>>>(x.rowptr, c.ptr, n, hub_min_in, sc.is_hub, ctl);
        is_hub = sc.is_hub;
    } else if (sched == KTRUSS_SCHED_LEARNED) {
        is_hub = learned_hub;
    }
    // hub items (every row with work under FORCE_HUB)
    HubChunks hc{x.rowptr, c.ptr, is_hub};
    device_scan(hc, n, ctl, sc, sc.itemoff, &ctl->n_items, s);
    k_hub_items<<<grid_for(n), kBlock, 0, s>>>(hc, n, sc.itemoff, sc.item_kappa, sc.item_c0, ctl);
    if (is_hub) {
        const int32_t wave_min = t.wave_min_work > 0 ? t.wave_min_work : kDefaultWaveMin;
        TaskClass tc{x, c, is_hub, wave_min};
        const int32_t G = scan_grid(m_hint);
        k_task_count<<<G, kBlock, 0, s>>>(tc, ctl, p, sc.blockcnt2);
        k_task_scan<<<1, kScanThreads, 0, s>>>(sc.blockcnt2, sc.blockoff2, G, ctl);
        k_task_scatter<<<G, kBlock, 0, s>>>(tc, ctl, p, sc.blockoff2, sc.wave_tasks, sc.thread_tasks);
    }
    return hipGetLastError();
}

}  // namespace kt
