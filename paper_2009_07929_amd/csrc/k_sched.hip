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

// ---- the same scan in 64 bits (hit-word offsets), out[N] = total

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan64_partial(F f, int32_t N, const Ctl* __restrict__ ctl,
                                                         long long* __restrict__ blockcnt) {
    __shared__ long long s_wave[kBlock / 64];
    if (ctl && ctl->done) return;
    int32_t lo, hi;
    span_of(N, lo, hi);
    long long c = 0;
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kBlock) c += f(i);
    c = block_sum64<kBlock>(c, s_wave);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = c;
}

__global__ __launch_bounds__(kScanThreads) void k_scan64_blocks(const long long* __restrict__ blockcnt,
                                                              long long* __restrict__ blockoff, int32_t G,
                                                              const Ctl* __restrict__ ctl) {
    __shared__ long long s_wave[kScanThreads / 64];
    if (ctl && ctl->done) return;
    constexpr int PER = kMaxScanBlocks / kScanThreads;
    const int t = threadIdx.x;
    long long v[PER];
    long long local = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = t * PER + j;
        v[j] = idx < G ? blockcnt[idx] : 0;
        local += v[j];
    }
    long long total;
    long long run = block_excl_sum64<kScanThreads>(local, s_wave, total);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = t * PER + j;
        if (idx < G) blockoff[idx] = run;
        run += v[j];
    }
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan64_write(F f, int32_t N, const Ctl* __restrict__ ctl,
                                                       const long long* __restrict__ blockoff,
                                                       int64_t* __restrict__ out) {
    __shared__ long long s_wave[kBlock / 64];
    if (ctl && ctl->done) return;
    int32_t lo, hi;
    span_of(N, lo, hi);
    long long base = blockoff[blockIdx.x];
    for (int32_t t0 = lo; t0 < hi; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const long long v = i < hi ? f(i) : 0;
        long long tot;
        const long long pre = block_excl_sum64<kBlock>(v, s_wave, tot);
        if (i < hi) out[i] = base + pre;
        base += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[N] = base;
}

// The per-workgroup partials live in the paired count / offset scratch
// (2 * kMaxScanBlocks int32 each, 256-byte aligned).
template <class F>
void device_scan64(const F& f, int32_t N, const Ctl* ctl, Scratch& sc, int64_t* out, hipStream_t s) {
    const int32_t G = scan_grid(N);
    long long* cnt = reinterpret_cast<long long*>(sc.blockcnt2);
    long long* off = reinterpret_cast<long long*>(sc.blockoff2);
    k_scan64_partial<F><<<G, kBlock, 0, s>>>(f, N, ctl, cnt);
    k_scan64_blocks<<<1, kScanThreads, 0, s>>>(cnt, off, G, ctl);
    k_scan64_write<F><<<G, kBlock, 0, s>>>(f, N, ctl, off, out);
}

// Hit words of the tasks of row i (tails d-1 .. 0).
struct RowWords {
    const int32_t* rowptr;
    __device__ long long operator()(int32_t i) const { return hit_words_upto(rowptr[i + 1] - rowptr[i] - 1); }
};

// ---- in-edge lists by a stable LSD radix sort of (column, edge) pairs
//
// 8-bit digits.  Per pass: every workgroup histograms the digits of its tile
// of kRsTile pairs (LDS counters); the digit-major table of those histograms is
// scanned; then every workgroup ranks its tile in order (equal digits within
// a wave by eight ballots, one per digit bit, and across sub-rounds and waves
// through LDS counts), reorders it by digit in LDS and writes each digit's
// run out contiguously.  Stable, so every column's list stays in ascending
// edge order; no global atomics.

constexpr int kRsItems = kRsTile / kBlock;

__global__ __launch_bounds__(kBlock) void k_rs_hist(const int32_t* __restrict__ keys, int32_t N, int shift,
                                                  int32_t nblk, int32_t* __restrict__ hist) {
    __shared__ int s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int32_t base = (int32_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int32_t e = base + j * kBlock + (int32_t)threadIdx.x;
        if (e < N) atomicAdd(&s_h[(keys[e] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = s_h[threadIdx.x];
}

// vals == nullptr: the values are the positions themselves (first pass).
// Every wave ranks a contiguous quarter of the tile (16 sub-rounds of 64
// pairs) against its own LDS digit counters; the tile is then reordered by
// digit in LDS and written out, so that each digit's run of the tile leaves
// as consecutive stores rather than one scattered store per pair.
// kRow: a second value (the edge's row) travels with every pair, read from
// rows (indexed like vals) and written to rows_out.
template <bool kRow>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const int32_t* __restrict__ keys, const int32_t* __restrict__ vals,
                                                     const int32_t* __restrict__ rows, int32_t N, int shift,
                                                     int32_t nblk, const int32_t* __restrict__ off,
                                                     int32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out,
                                                     int32_t* __restrict__ rows_out) {
    constexpr int kWaves = kBlock / 64;
    constexpr int kPerWave = kRsTile / kWaves;
    // one staging array, reused for keys, values and rows in turn, and the
    // digit of every sorted slot: a small LDS footprint keeps several
    // workgroups per CU, whose loads overlap each other's ranking
    __shared__ int32_t s_x[kRsTile];
    __shared__ uint8_t s_d[kRsTile];
    __shared__ int s_cnt[kWaves][256];  // per-wave digit counts, then each wave's offset within its digit
    __shared__ int s_loc[256];          // first tile-local slot of every digit
    __shared__ int s_glob[256];         // first output position of every digit's run of this tile
    __shared__ int s_ws[kWaves];
    const int t = threadIdx.x, w = t >> 6, lane = __lane_id();
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s_cnt[i][t] = 0;
    s_glob[t] = off[(int64_t)t * nblk + blockIdx.x];
    const int32_t tile0 = (int32_t)blockIdx.x * kRsTile;
    const int32_t base = tile0 + w * kPerWave;
    const uint64_t lt = (1ull << lane) - 1ull;
    int32_t kreg[kRsItems], vreg[kRsItems], rreg[kRow ? kRsItems : 1];
    int rank[kRsItems];
    // every load of the wave's quarter first, then the ranking
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int32_t e = base + j * 64 + lane;
        const bool valid = e < N;
        kreg[j] = valid ? keys[e] : 0;
        vreg[j] = valid ? (vals ? vals[e] : e) : 0;
        if constexpr (kRow) rreg[j] = valid ? rows[e] : 0;
    }
    __syncthreads();  // counters cleared
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const bool valid = base + j * 64 + lane < N;
        const int d = (kreg[j] >> shift) & 255;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot(valid && ((d >> b) & 1));
            match &= ((d >> b) & 1) ? bb : ~bb;
        }
        const int r = __popcll(match & lt);
        const int before = s_cnt[w][d];
        __builtin_amdgcn_wave_barrier();  // every lane has read the count before its leader advances it
        if (valid && r == 0) s_cnt[w][d] = before + __popcll(match);
        __builtin_amdgcn_wave_barrier();
        rank[j] = valid ? before + r : -1;
    }
    __syncthreads();
    // digit t: per-wave offsets and the tile-local start (exclusive scan over digits)
    int tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        const int c = s_cnt[i][t];
        s_cnt[i][t] = tot;
        tot += c;
    }
    int incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_ws[w] = incl;
    __syncthreads();
    int wpre = 0;
    for (int i = 0; i < w; ++i) wpre += s_ws[i];
    s_loc[t] = wpre + incl - tot;
    __syncthreads();
    // sorted slot of every pair
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        if (rank[j] < 0) continue;
        const int d = (kreg[j] >> shift) & 255;
        rank[j] += s_loc[d] + s_cnt[w][d];
        s_d[rank[j]] = (uint8_t)d;
    }
    const int32_t nvalid = min((int32_t)kRsTile, N - tile0);
    // one array at a time: stage in sorted order, then write each digit's run
    auto pass = [&](const int32_t* reg, int32_t* __restrict__ out) {
#pragma unroll
        for (int j = 0; j < kRsItems; ++j)
            if (rank[j] >= 0) s_x[rank[j]] = reg[j];
        __syncthreads();
        for (int i = t; i < nvalid; i += kBlock) {
            const int d = s_d[i];
            out[s_glob[d] + (i - s_loc[d])] = s_x[i];
        }
        __syncthreads();  // s_x is read before the next array overwrites it
    };
    pass(kreg, keys_out);
    pass(vreg, vals_out);
    if constexpr (kRow) pass(rreg, rows_out);
}

// cptr[k] = first position of the sorted keys holding a value >= k, k in [0, n]
__global__ __launch_bounds__(kBlock) void k_col_ptr(const int32_t* __restrict__ sorted, int32_t m, int32_t n,
                                                  int32_t* __restrict__ cptr) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > n) return;
    cptr[k] = lower_bound_i32(sorted, m, (int32_t)k);
}

// Tail length of the task of every in-edge list entry of the pass: the part
// of row i after the edge (Algorithm 3's a12(j+1:)); 0 for a tombstone.
__global__ __launch_bounds__(kBlock) void k_task_tails(Buf x, Csc c, const Ctl* __restrict__ ctl,
                                                     int32_t* __restrict__ ctail) {
    if (ctl->done) return;
    const int32_t nc = ctl->csc_m;
    for (int32_t q = (int32_t)(blockIdx.x * kBlock + threadIdx.x); q < nc; q += (int32_t)(gridDim.x * kBlock)) {
        const int32_t e = c.edge[q];
        ctail[q] = e < 0 ? 0 : x.rowptr[c.src[q] + 1] - e - 1;
    }
}

// Alive in-edges of every row kappa at the start of a run: the list lengths.
// After every prune the in-place remap of the lists recounts them.
__global__ __launch_bounds__(kBlock) void k_alive_in_init(const int32_t* __restrict__ cptr, int32_t n,
                                                        int32_t* __restrict__ alive_in) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) alive_in[k] = cptr[k + 1] - cptr[k];
}

// ---- hub items

// Number of hub items of row kappa: its in-edges cut into chunks of kHubChunk.
struct HubChunks {
    const int32_t* rowptr;
    const int32_t* cptr;
    const int32_t* alive_in;  // alive in-edges per row (the lists also hold tombstones)
    const uint8_t* is_hub;    // per row, or null = every row with work
    const int32_t* chunk_sz;  // tasks per item of each row (<= kHubChunk), or null = chunk_all
    int32_t chunk_all;
    __device__ int32_t size(int32_t k) const { return chunk_sz ? chunk_sz[k] : chunk_all; }
    __device__ int32_t operator()(int32_t k) const {
        const int32_t indeg = cptr[k + 1] - cptr[k];
        const int32_t d = rowptr[k + 1] - rowptr[k];
        if (alive_in[k] == 0 || d == 0) return 0;
        if (is_hub && !is_hub[k]) return 0;
        const int32_t cs = size(k);
        return (indeg + cs - 1) / cs;
    }
};

__global__ __launch_bounds__(kBlock) void k_hub_items(HubChunks f, const int32_t* __restrict__ col, int32_t n,
                                                    const int32_t* __restrict__ itemoff, HubItem* __restrict__ items,
                                                    uint8_t* __restrict__ hub_row, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k == 0) const_cast<Ctl*>(ctl)->item_next = 0;
    if (k >= n) return;
    const int32_t nch = f((int32_t)k);
    hub_row[k] = nch > 0 ? 1 : 0;
    if (nch == 0) return;
    const int32_t o = itemoff[k];
    const int32_t c0 = f.cptr[k], cend = f.cptr[k + 1];
    const int32_t cs = f.size((int32_t)k);
    const int32_t rs = f.rowptr[k], d = f.rowptr[k + 1] - rs;
    const int32_t last = col[rs + d - 1];
    for (int32_t j = 0; j < nch; ++j) {
        HubItem h;
        h.k = (int32_t)k;
        h.c0 = c0 + j * cs;
        h.c1 = min(c0 + (j + 1) * cs, cend);
        h.rs = rs;
        h.d = d;
        h.last = last;
        h.pad0 = h.pad1 = 0;
        items[o + j] = h;
    }
}

// ---- learned schedule: per-row features and cost-model bins

// Rows kappa that carry support work in the current pass (in-edges and a
// non-empty row).
// Rows whose hit words k_hit_sum_long sums.
struct LongRow {
    const int32_t* rowptr;
    __device__ int32_t operator()(int32_t i) const {
        const int32_t d = rowptr[i + 1] - rowptr[i];
        return (d > kHitLongMin && d <= kHitLongMax) ? 1 : 0;
    }
};

__global__ __launch_bounds__(kBlock) void k_long_list(LongRow f, int32_t n, const int32_t* __restrict__ off,
                                                    int32_t* __restrict__ list, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && f((int32_t)i)) list[off[i]] = (int32_t)i;
}

struct ActiveRow {
    const int32_t* rowptr;
    const int32_t* alive_in;  // alive in-edges per row
    __device__ int32_t operator()(int32_t k) const {
        return (alive_in[k] > 0 && rowptr[k + 1] > rowptr[k]) ? 1 : 0;
    }
};

__global__ __launch_bounds__(kBlock) void k_active_list(ActiveRow f, int32_t n, const int32_t* __restrict__ off,
                                                      int32_t* __restrict__ list, const Ctl* __restrict__ ctl) {
    if (ctl && ctl->done) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n && f((int32_t)k)) list[off[k]] = (int32_t)k;
}

// For every row kappa: sum over its in-edges (i, kappa) of the out-degree of
// row i ("sum of neighbour out-degrees").  The in-edge lists are grouped by
// kappa, so a wave-level segmented scan adds each run and its last lane
// issues one atomic per run piece.
__global__ __launch_bounds__(kBlock) void k_in_outdeg_sum(Buf x, Csc c, int32_t m, unsigned long long* __restrict__ sum) {
    const int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    const int lane = __lane_id();
    int32_t key = -1;
    long long v = 0;
    if (i < m) {
        const int32_t r = c.src[i];
        key = c.key[i];
        v = x.rowptr[r + 1] - x.rowptr[r];
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(v, o);
        const int32_t kk = __shfl_up(key, o);
        if (lane >= o && kk == key) v += u;
    }
    const int32_t next = __shfl_down(key, 1);
    const bool tail = lane == 63 || next != key;
    if (i < m && tail) atomicAdd(&sum[key], (unsigned long long)v);
}

// Features of active row kappa (the cost model's inputs): out-degree,
// log2 out-degree, log2 of the sum of in-neighbour out-degrees, pass index,
// fraction of the input's edges still alive.
__device__ __forceinline__ void row_features(const int32_t* rowptr, const unsigned long long* insum, int32_t k,
                                             int32_t pass, float alive, float* f) {
    const float d = (float)(rowptr[k + 1] - rowptr[k]);
    f[0] = d * (1.f / 1024.f);
    f[1] = log2f(1.f + d) * (1.f / 12.f);
    f[2] = log2f(1.f + (float)insum[k]) * (1.f / 24.f);
    f[3] = (float)pass * (1.f / 32.f);
    f[4] = alive;
}

__global__ __launch_bounds__(kBlock) void k_row_features(const int32_t* __restrict__ rowptr,
                                                       const unsigned long long* __restrict__ insum,
                                                       const int32_t* __restrict__ list, const Ctl* __restrict__ ctl,
                                                       int p, int32_t m0, float* __restrict__ feats) {
    if (ctl->done) return;
    const int32_t a = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (a >= ctl->n_active) return;
    float f[KTRUSS_MLP_IN];
    row_features(rowptr, insum, list[a], ctl->rounds, (float)ctl->m_buf[p] / (float)(m0 > 0 ? m0 : 1), f);
#pragma unroll
    for (int i = 0; i < KTRUSS_MLP_IN; ++i) feats[(int64_t)a * KTRUSS_MLP_IN + i] = f[i];
}

// Bins from the cost model's prediction for each active row: log2 of the
// row's wave-cycles on the hub kernel minus log2 of them on the wavefront
// kernel.  A row predicted at most `thr` is a hub row (items of the common
// chunk size); the others' tasks go to the wavefront / thread lists.
__global__ __launch_bounds__(kBlock) void k_learned_bins(const int32_t* __restrict__ list, const float* __restrict__ pred,
                                                       float thr, uint8_t* __restrict__ is_hub,
                                                       const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t a = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (a >= ctl->n_active) return;
    is_hub[list[a]] = pred[a] <= thr ? 1 : 0;  // a NaN prediction leaves the row off the hub kernel
}

__global__ __launch_bounds__(kBlock) void k_fill_u8(uint8_t* __restrict__ a, int32_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long* __restrict__ a, int32_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

// Training rows from a timed pass: features of every active row and its
// measured support cycles as log2(1 + cycles), appended while capacity lasts.
__global__ __launch_bounds__(kBlock) void k_append_costs(const int32_t* __restrict__ list, const float* __restrict__ feats,
                                                       const unsigned long long* __restrict__ cycles, int32_t capacity,
                                                       float* __restrict__ out_x, float* __restrict__ out_y,
                                                       Ctl* ctl) {
    if (ctl->done) return;
    const int32_t n_act = ctl->n_active;
    const int32_t base = ctl->n_samples;
    const int32_t a = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (a < n_act && base + a < capacity) {
        const int32_t k = list[a];
#pragma unroll
        for (int i = 0; i < KTRUSS_MLP_IN; ++i)
            out_x[(int64_t)(base + a) * KTRUSS_MLP_IN + i] = feats[(int64_t)a * KTRUSS_MLP_IN + i];
        out_y[base + a] = log2f(1.f + (float)cycles[k]);
    }
}

__global__ void k_advance_samples(Ctl* ctl, int32_t capacity) {
    if (threadIdx.x == 0 && !ctl->done) ctl->n_samples = min(ctl->n_samples + ctl->n_active, capacity);
}

// ---- static degree heuristic: which rows kappa are hub rows

__global__ __launch_bounds__(kBlock) void k_heuristic_bins(const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ alive_in, int32_t n,
                                                         int32_t hub_min_in, uint8_t* __restrict__ is_hub,
                                                         const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int32_t indeg = alive_in[k];
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
        const int32_t k = c.key[i];
        if (is_hub[k]) return 0;
        const int32_t e = c.edge[i];
        if (e < 0) return 0;  // tombstone of a removed edge
        const int32_t tail = x.rowptr[c.src[i] + 1] - e - 1;
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
    span_of(ctl->csc_m, lo, hi);
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
    span_of(ctl->csc_m, lo, hi);
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

// Stable transpose of CSR columns by the radix sort above (8-bit digits,
// as many passes as n's bits need): keys_out gets the columns in ascending
// order, vals_out the position holding each (ascending within a column), and
// ptr[k] (k in [0, n]) the first entry with a column >= k.  tk, tv: two
// int32[m] ping-pong buffers each, distinct from the outputs; uses
// sc.rs_hist, sc.blockcnt and sc.blockoff.  rows (optional): one more value
// per position, carried into rows_out in the same order (tr: its two
// ping-pong buffers).
hipError_t launch_radix_transpose(const int32_t* keys, int32_t m, int32_t n, int32_t* keys_out, int32_t* vals_out,
                                  int32_t* ptr, int32_t* const tk[2], int32_t* const tv[2], Scratch& sc,
                                  hipStream_t s, const int32_t* rows, int32_t* rows_out, int32_t* const tr[2]) {
    if (m == 0) {
        k_fill_i32<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(ptr, n + 1, 0);
        return hipGetLastError();
    }
    int bits = 0;
    while (bits < 31 && ((int64_t)(n - 1) >> bits) != 0) ++bits;
    const int passes = bits <= 8 ? 1 : (bits + 7) / 8;
    const int32_t nblk = (int32_t)(((int64_t)m + kRsTile - 1) / kRsTile);
    const int32_t nh = 256 * nblk;
    const int32_t* kin = keys;
    const int32_t* vin = nullptr;
    const int32_t* rin = rows;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const bool last = p == passes - 1;
        int32_t* kout = last ? keys_out : tk[p & 1];
        int32_t* vout = last ? vals_out : tv[p & 1];
        k_rs_hist<<<nblk, kBlock, 0, s>>>(kin, m, shift, nblk, sc.rs_hist);
        device_scan(FromArray{sc.rs_hist}, nh, nullptr, sc, sc.rs_hist, nullptr, s);
        if (rows) {
            int32_t* rout = last ? rows_out : tr[p & 1];
            k_rs_scatter<true><<<nblk, kBlock, 0, s>>>(kin, vin, rin, m, shift, nblk, sc.rs_hist, kout, vout, rout);
            rin = rout;
        } else {
            k_rs_scatter<false><<<nblk, kBlock, 0, s>>>(kin, vin, nullptr, m, shift, nblk, sc.rs_hist, kout, vout,
                                                        nullptr);
        }
        kin = kout;
        vin = vout;
    }
    k_col_ptr<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(kin, m, n, ptr);
    return hipGetLastError();
}

// In-edge lists of buffer b: the transpose of its columns, with every
// entry's row carried through the sort.
hipError_t launch_build_csc(const Buf& b, const Csc& c, int32_t n, int32_t m, Scratch& sc, hipStream_t s) {
    if (m == 0) {
        k_fill_i32<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(c.ptr, n + 1, 0);
        k_fill_i32<<<grid_for((int64_t)n + 1), kBlock, 0, s>>>(sc.alive_in, n + 1, 0);
        return hipGetLastError();
    }
    // ping-pong buffers: scratch that the first pass rebuilds (the hit words hold at least 8 m words)
    int32_t* const tk[2] = {sc.xscan, sc.wave_tasks};
    int32_t* const tv[2] = {sc.cxscan, sc.thread_tasks};
    int32_t* const tr[2] = {sc.ctail, (int32_t*)sc.hitw};
    hipError_t e = launch_radix_transpose(b.col, m, n, c.key, c.edge, c.ptr, tk, tv, sc, s, b.src, c.src, tr);
    if (e != hipSuccess) return e;
    k_alive_in_init<<<grid_for(n), kBlock, 0, s>>>(c.ptr, n, sc.alive_in);
    return hipGetLastError();
}

// Row (last r with rowptr[r] <= e) of the positions pos[0 .. m).
__global__ __launch_bounds__(kBlock) void k_rows_of(const int32_t* __restrict__ rowptr, int32_t nrows,
                                                  const int32_t* __restrict__ pos, int32_t m,
                                                  int32_t* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    const int32_t e = pos[j];
    int32_t lo = 0, hi = nrows;
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (rowptr[mid] <= e) lo = mid;
        else hi = mid;
    }
    out[j] = lo;
}

hipError_t launch_rows_of(const int32_t* rowptr, int32_t nrows, const int32_t* pos, int32_t m, int32_t* out,
                          hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_rows_of<<<grid_for(m), kBlock, 0, s>>>(rowptr, nrows, pos, m, out);
    return hipGetLastError();
}

// Butterfly tasks of pair vertex p: none without wedges, one when its W(p)
// wedges fit the hash, else one per window of labels.
struct BfTasks {
    const int64_t* W;
    int64_t hash_max, nwin;
    __device__ long long operator()(int32_t p) const {
        const int64_t w = W[p];
        return w == 0 ? 0 : (w <= hash_max ? 1 : nwin);
    }
};

hipError_t launch_bf_task_offsets(const int64_t* W, int32_t nP, int64_t hash_max, int64_t nwin, int64_t* off,
                                  Scratch& sc, hipStream_t s) {
    device_scan64(BfTasks{W, hash_max, nwin}, nP, nullptr, sc, off, s);
    return hipGetLastError();
}

hipError_t launch_in_outdeg_sum(const Buf& x, const Csc& c, int32_t n, int32_t m, Scratch& sc, hipStream_t s) {
    k_fill_u64<<<grid_for(n), kBlock, 0, s>>>(sc.insum, n);
    if (m > 0) k_in_outdeg_sum<<<grid_for(m), kBlock, 0, s>>>(x, c, m, sc.insum);
    return hipGetLastError();
}

hipError_t launch_append_costs(Scratch& sc, int32_t n, int32_t capacity, float* out_x, float* out_y, Ctl* ctl,
                               hipStream_t s) {
    k_append_costs<<<grid_for(n), kBlock, 0, s>>>(sc.act_list, sc.feats, sc.cycles, capacity, out_x, out_y, ctl);
    k_advance_samples<<<1, 64, 0, s>>>(ctl, capacity);
    k_fill_u64<<<grid_for(n), kBlock, 0, s>>>(sc.cycles, n);
    return hipGetLastError();
}

hipError_t launch_prepare_pass(const Buf& x, const Csc& c, int32_t n, int sched, const ktruss_tuning& t,
                               const float* mlp, int32_t m0, bool features, Scratch& sc, Ctl* ctl, int p,
                               int32_t m_hint, hipStream_t s) {
    const uint8_t* is_hub = nullptr;
    const int32_t* chunk = nullptr;
    const bool learned = sched == KTRUSS_SCHED_LEARNED && mlp;
    // task tails (the in-edge lists hold tombstones of removed edges)
    if (m_hint > 0)
        k_task_tails<<<min(grid_for(m0), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, c, ctl, sc.ctail);
    // first hit word of every row's tasks (a 64-bit scan of the rows' word counts)
    device_scan64(RowWords{x.rowptr}, n, ctl, sc, sc.hwoff, s);
    // the rows whose hit words are summed per row
    device_scan(LongRow{x.rowptr}, n, ctl, sc, sc.long_off, &ctl->n_long, s);
    if (n > 0) k_long_list<<<grid_for(n), kBlock, 0, s>>>(LongRow{x.rowptr}, n, sc.long_off, sc.long_rows, ctl);
    if (sched == kSchedSampleWave) {  // cost sampling: no hub rows, every task on the wavefront kernel
        k_fill_u8<<<grid_for(n), kBlock, 0, s>>>(sc.is_hub, n, 0);
        is_hub = sc.is_hub;
    }
    if (sched == KTRUSS_SCHED_HEURISTIC || (sched == KTRUSS_SCHED_LEARNED && !mlp)) {
        const int32_t hub_min_in = t.hub_min_work > 0 ? t.hub_min_work : kDefaultHubMinIn;
        k_heuristic_bins<<<grid_for(n), kBlock, 0, s>>>(x.rowptr, sc.alive_in, n, hub_min_in, sc.is_hub, ctl);
        is_hub = sc.is_hub;
    }
    if (learned || features) {
        // rows with work, their features (and, learned, the cost model's bins)
        device_scan(ActiveRow{x.rowptr, sc.alive_in}, n, ctl, sc, sc.act_off, &ctl->n_active, s);
        k_active_list<<<grid_for(n), kBlock, 0, s>>>(ActiveRow{x.rowptr, sc.alive_in}, n, sc.act_off, sc.act_list,
                                                      ctl);
        k_row_features<<<grid_for(n), kBlock, 0, s>>>(x.rowptr, sc.insum, sc.act_list, ctl, p, m0, sc.feats);
    }
    if (learned) {
        hipError_t e = launch_mlp_forward_dev(mlp, sc.feats, &ctl->n_active, n, sc.pred, s);
        if (e != hipSuccess) return e;
        const float thr = t.learned_hub_min != 0.f ? t.learned_hub_min : kDefaultLearnedHubMax;
        k_fill_u8<<<grid_for(n), kBlock, 0, s>>>(sc.is_hub, n, 0);
        k_learned_bins<<<grid_for(n), kBlock, 0, s>>>(sc.act_list, sc.pred, thr, sc.is_hub, ctl);
        is_hub = sc.is_hub;
    }
    // hub items (every row with work under FORCE_HUB)
    int32_t chunk_all = t.hub_chunk_tasks > 0 ? t.hub_chunk_tasks : kHubChunk;
    chunk_all = max(kMinLearnedChunk, min(chunk_all, kHubChunk));  // item capacity assumes >= kMinLearnedChunk
    HubChunks hc{x.rowptr, c.ptr, sc.alive_in, is_hub, chunk, chunk_all};
    device_scan(hc, n, ctl, sc, sc.itemoff, &ctl->n_items, s);
    k_hub_items<<<grid_for(n), kBlock, 0, s>>>(hc, x.col, n, sc.itemoff, sc.items, sc.hub_row, ctl);
    if (is_hub) {
        const int32_t wave_min = sched == kSchedSampleWave ? 0 : (t.wave_min_work > 0 ? t.wave_min_work : kDefaultWaveMin);
        TaskClass tc{x, c, is_hub, wave_min};
        const int32_t G = scan_grid(m0);  // the in-edge lists keep the run's m entries
        k_task_count<<<G, kBlock, 0, s>>>(tc, ctl, p, sc.blockcnt2);
        k_task_scan<<<1, kScanThreads, 0, s>>>(sc.blockcnt2, sc.blockoff2, G, ctl);
        k_task_scatter<<<G, kBlock, 0, s>>>(tc, ctl, p, sc.blockoff2, sc.wave_tasks, sc.thread_tasks);
    }
    return hipGetLastError();
}

}  // namespace kt
