// Support computation (Algorithm 1's S = (A^T A) o A on the alive edges) by
// eager fine-grained tasks, Algorithm 3: the task of edge e = (i, kappa), at
// position j of row i, intersects the part of row i after j (a12(j+1:)) with
// row kappa of A22.  Each common column w closes the triangle (i, kappa, w),
// found exactly once (from its two smallest labels), and all three supports
// are incremented: S(i,kappa) (s12(j)), S(i,w) (s12(j+1:)) and S(kappa,w)
// (S(kappa,:)).  Integer atomics commute, so every variant below produces the
// same S bit for bit; they differ only in how tasks map onto the GPU.
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

__device__ __forceinline__ void thread_task(const Buf& x, int32_t e);
__device__ __forceinline__ void wave_task(const Buf& x, int32_t e);

// ------------------------------------------------------ thread-per-edge
// One thread per task: a merge of the two ascending lists (the mapping of the
// paper's Kokkos listing).  `tasks` = null means tasks 0..count-1 are the edge
// positions themselves.
__global__ __launch_bounds__(kBlock) void k_support_thread(Buf x, const int32_t* __restrict__ tasks,
                                                         const int32_t* __restrict__ count, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t nt = *count;
    for (int32_t t = (int32_t)(blockIdx.x * kBlock + threadIdx.x); t < nt; t += (int32_t)(gridDim.x * kBlock))
        thread_task(x, tasks ? tasks[t] : t);
}

__device__ __forceinline__ void thread_task(const Buf& x, int32_t e) {
    const int32_t* __restrict__ col = x.col;
    const int32_t i = x.src[e];
    const int32_t k = col[e];
    int32_t a = e + 1;
    const int32_t ae = x.rowptr[i + 1];
    int32_t b = x.rowptr[k];
    const int32_t be = x.rowptr[k + 1];
    int32_t cnt = 0;
    if (a < ae && b < be) {
        int32_t u = col[a], v = col[b];
        for (;;) {
            if (u == v) {
                atomicAdd(&x.S[a], 1);
                atomicAdd(&x.S[b], 1);
                ++cnt;
                if (++a >= ae || ++b >= be) break;
                u = col[a];
                v = col[b];
            } else if (u < v) {
                if (++a >= ae) break;
                u = col[a];
            } else {
                if (++b >= be) break;
                v = col[b];
            }
        }
    }
    if (cnt) atomicAdd(&x.S[e], cnt);
}

// ---------------------------------------------------- wavefront-per-edge
// One wave per task.  The 64 lanes walk the shorter of the two lists and
// binary-search each element in the other (both ascending, in global memory;
// the first search steps of all lanes hit the same lines).  Hits bump the two
// other edges' supports; the wave total goes to S[e] once.
__global__ __launch_bounds__(kBlock) void k_support_wave(Buf x, const int32_t* __restrict__ tasks,
                                                       const int32_t* __restrict__ count, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t nt = *count;
    const int32_t nw = (int32_t)(gridDim.x * (kBlock / 64));
    for (int32_t wid = (int32_t)((blockIdx.x * kBlock + threadIdx.x) >> 6); wid < nt; wid += nw)
        wave_task(x, tasks ? tasks[wid] : wid);
}

__device__ __forceinline__ void wave_task(const Buf& x, int32_t e) {
    const int lane = __lane_id();
    const int32_t* __restrict__ col = x.col;
    const int32_t i = x.src[e];
    const int32_t k = col[e];
    const int32_t a0 = e + 1, a1 = x.rowptr[i + 1];     // tail of row i
    const int32_t b0 = x.rowptr[k], b1 = x.rowptr[k + 1];  // row kappa
    if (a0 >= a1 || b0 >= b1) return;
    const int32_t la = a1 - a0, lb = b1 - b0;
    // walk list W (positions w0..w1), search list F (f0..f1)
    const bool walk_tail = la <= lb;
    const int32_t w0 = walk_tail ? a0 : b0, w1 = walk_tail ? a1 : b1;
    const int32_t f0 = walk_tail ? b0 : a0, flen = walk_tail ? lb : la;
    const int32_t fmin = col[f0], fmax = col[f0 + flen - 1];
    int cnt = 0;
    for (int32_t base = w0; base < w1; base += 64) {
        const int32_t pos = base + lane;
        const bool in = pos < w1;
        const int32_t v = in ? col[pos] : INT32_MAX;
        const bool cand = in && v >= fmin && v <= fmax;
        if (__ballot(in && v <= fmax) == 0) break;  // ascending: nothing further can match
        if (cand) {
            const int32_t q = f0 + lower_bound_i32(col + f0, flen, v);
            if (col[q] == v) {
                atomicAdd(&x.S[pos], 1);
                atomicAdd(&x.S[q], 1);
                ++cnt;
            }
        }
    }
    cnt = wave_sum(cnt);
    if (lane == 0 && cnt) atomicAdd(&x.S[e], cnt);
}

// ------------------------------------------------- workgroup-per-hub-row
// One workgroup per hub item: row kappa of A22 and up to kHubChunk of the
// tasks that select it.  Row kappa is staged once in LDS as a rank bitmap over
// its label span (membership and position of a label with one 64-bit LDS
// read), or as a sorted key array when the span is wide; its supports
// S(kappa, :) accumulate in LDS and are flushed once per item.  Each wave walks
// the tails of its tasks (contiguous, coalesced reads).  The hits of a task's
// tail chunk, which belong to edges (i, w) of other rows' items, are stored as
// one 64-bit word instead of one global atomic per triangle; k_hit_sum adds
// them to S(i, w) row by row after the pass.
enum { kModeBitmap = 0, kModeKeys = 1, kModeGlobal = 2 };

__global__ __launch_bounds__(kHubThreads) void k_support_hub(Buf x, Csc c, const int32_t* __restrict__ item_kappa,
                                                           const int32_t* __restrict__ item_c0,
                                                           const int32_t* __restrict__ item_c1, Ctl* ctl,
                                                           unsigned long long* __restrict__ hitw,
                                                           unsigned long long* __restrict__ cycles) {
    __shared__ uint2 s_bm[kSpanWords];   // rank bitmap {bits, set bits before this word}; or keys
    __shared__ int32_t s_acc[kKeyCap];
    __shared__ int32_t s_e[kHubChunk];
    __shared__ int32_t s_tl[kHubChunk];
    __shared__ int s_wave[kHubThreads / 64];
    __shared__ int32_t s_it;
    if (ctl->done) return;
    const int32_t n_items = ctl->n_items;
    // Persistent: workgroups pull items from a device counter.  Items are laid
    // out by ascending kappa and the heaviest rows carry the largest labels, so
    // they are taken from the end first (longest work first).
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_it = atomicAdd(&ctl->item_next, 1);
        __syncthreads();
        const int32_t it = n_items - 1 - s_it;
        if (it < 0) break;
        const int32_t* __restrict__ col = x.col;
        const int32_t k = item_kappa[it];
        const int32_t c0 = item_c0[it];
        const int32_t c1 = item_c1[it];
        const unsigned long long t_start = cycles ? (unsigned long long)clock64() : 0ull;
        const int32_t ntask = c1 - c0;
        const int32_t rs = x.rowptr[k], d = x.rowptr[k + 1] - rs;
        const int t = threadIdx.x;
        if (t < ntask) {
            const int32_t e = c.edge[c0 + t];
            s_e[t] = e;
            s_tl[t] = x.rowptr[x.src[e] + 1] - e - 1;
        }
        const int32_t last = col[rs + d - 1];
        const int32_t span = last - k;  // labels of row kappa lie in (k, last]
        const int mode = d > kKeyCap ? kModeGlobal : (span <= kSpanCap ? kModeBitmap : kModeKeys);
        int32_t* s_keys = reinterpret_cast<int32_t*>(s_bm);
        if (mode == kModeBitmap) {
            const int32_t nw = (span + 31) >> 5;
            for (int32_t j = t; j < nw; j += kHubThreads) s_bm[j] = make_uint2(0u, 0u);
            __syncthreads();
            for (int32_t q = t; q < d; q += kHubThreads) {
                const int32_t off = col[rs + q] - k - 1;
                atomicOr(&s_bm[off >> 5].x, 1u << (off & 31));
            }
            __syncthreads();
            const int32_t per = (nw + kHubThreads - 1) / kHubThreads;
            const int32_t j0 = t * per, j1 = min(j0 + per, nw);
            int local = 0;
            for (int32_t j = j0; j < j1; ++j) local += __popc(s_bm[j].x);
            int tot;
            int run = block_excl_sum<kHubThreads>(local, s_wave, tot);
            for (int32_t j = j0; j < j1; ++j) {
                s_bm[j].y = (uint32_t)run;
                run += __popc(s_bm[j].x);
            }
        } else if (mode == kModeKeys) {
            for (int32_t q = t; q < d; q += kHubThreads) s_keys[q] = col[rs + q];
        }
        if (mode != kModeGlobal)
            for (int32_t q = t; q < d; q += kHubThreads) s_acc[q] = 0;
        __syncthreads();

        // Each wave walks the 64-element chunks of its tasks (kk = wv, wv + 4,
        // ...) in order, kHubUnroll chunks per step: their loads are issued
        // together, so several tail reads are in flight per wave however
        // short the tails are.
        const int wv = t >> 6, lane = t & 63;
        int32_t kk = wv, ch = 0, e_cur = 0, L_cur = 0;
        auto next_task = [&]() {
            while (kk < ntask && s_tl[kk] <= 0) kk += kHubThreads / 64;
            if (kk < ntask) {
                e_cur = s_e[kk];
                L_cur = s_tl[kk];
            }
        };
        next_task();
        uint32_t acc = 0;  // hits of the current task so far: S(i, kappa)
        while (kk < ntask) {
            int32_t ue[kHubUnroll], uc[kHubUnroll], uL[kHubUnroll], uw[kHubUnroll];
            bool uv[kHubUnroll], ulast[kHubUnroll];
#pragma unroll
            for (int u = 0; u < kHubUnroll; ++u) {
                uv[u] = kk < ntask;
                ue[u] = e_cur;
                uc[u] = ch;
                uL[u] = L_cur;
                ulast[u] = (ch + 1) * 64 >= L_cur;
                if (uv[u]) {
                    if (ulast[u]) {
                        ch = 0;
                        kk += kHubThreads / 64;
                        next_task();
                    } else {
                        ++ch;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kHubUnroll; ++u) {
                const int32_t o = uc[u] * 64 + lane;
                uw[u] = (uv[u] && o < uL[u]) ? col[ue[u] + 1 + o] : INT32_MAX;
            }
#pragma unroll
            for (int u = 0; u < kHubUnroll; ++u) {
                if (!uv[u]) continue;
                const int32_t w = uw[u];
                bool hit = false;
                if (w <= last) {  // beyond the last label of row kappa nothing matches
                    int32_t q = -1;
                    if (mode == kModeBitmap) {
                        const int32_t off = w - k - 1;
                        const uint2 bw = s_bm[off >> 5];
                        const uint32_t bit = (uint32_t)off & 31u;
                        if ((bw.x >> bit) & 1u) q = (int32_t)(bw.y + __popc(bw.x & ((1u << bit) - 1u)));
                    } else if (mode == kModeKeys) {
                        const int32_t qq = lower_bound_i32(s_keys, d, w);
                        if (s_keys[qq] == w) q = qq;
                    } else {
                        const int32_t qq = lower_bound_i32(col + rs, d, w);
                        if (col[rs + qq] == w) q = qq;
                    }
                    if (q >= 0) {
                        hit = true;
                        if (mode != kModeGlobal) atomicAdd(&s_acc[q], 1);
                        else atomicAdd(&x.S[rs + q], 1);
                    }
                }
                // S(i, w): the chunk's hits as one word, summed per row by
                // k_hit_sum; chunks past kHitWords add directly.
                const unsigned long long hb = __ballot(hit);
                if (uc[u] < kHitWords) {
                    if (lane == 0) hitw[(size_t)ue[u] * kHitWords + uc[u]] = hb;
                } else if (hit) {
                    atomicAdd(&x.S[ue[u] + 1 + uc[u] * 64 + lane], 1);
                }
                acc += (uint32_t)__popcll(hb);
                if (ulast[u]) {
                    if (lane == 0 && acc) atomicAdd(&x.S[ue[u]], (int32_t)acc);
                    acc = 0;
                }
            }
        }
        __syncthreads();
        if (mode != kModeGlobal)
            for (int32_t q = t; q < d; q += kHubThreads) {
                const int32_t a = s_acc[q];
                if (a) atomicAdd(&x.S[rs + q], a);
            }
        if (cycles) {  // per-row cost samples for the cost model (shader clock)
            __syncthreads();
            if (t == 0) atomicAdd(&cycles[k], (unsigned long long)clock64() - t_start);
        }
    }
}

// Row-local sum of the hub kernel's hit words: S(i, w) of the edge at
// position p of row i gains one for every earlier task j of row i (a hub task,
// hub_row[col[j]]) whose hit word has the bit of tail offset p - j - 1.  One
// thread per edge; the threads of a row walk the same tasks in step, so the
// task's column, flag and word are shared loads.
__global__ __launch_bounds__(kBlock) void k_hit_sum(Buf x, const unsigned long long* __restrict__ hitw,
                                                  const uint8_t* __restrict__ hub_row,
                                                  const int32_t* __restrict__ count, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t m = *count;
    const int32_t* __restrict__ col = x.col;
    for (int32_t p = (int32_t)(blockIdx.x * kBlock + threadIdx.x); p < m; p += (int32_t)(gridDim.x * kBlock)) {
        const int32_t rs = x.rowptr[x.src[p]];
        int32_t add = 0;
#pragma unroll 4
        for (int32_t j = rs; j < p; ++j) {
            const int32_t off = p - j - 1;  // tail offset of p in task j
            if (off < kHitWords * 64 && hub_row[col[j]])
                add += (int32_t)((hitw[(size_t)j * kHitWords + (off >> 6)] >> (off & 63)) & 1ull);
        }
        if (add) x.S[p] += add;
    }
}

}  // namespace

hipError_t launch_support_thread(const Buf& x, const int32_t* tasks, const int32_t* count_dev, int32_t n_hint,
                                 const Ctl* ctl, hipStream_t s) {
    if (n_hint <= 0) return hipSuccess;
    k_support_thread<<<min(grid_for(n_hint), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, tasks, count_dev, ctl);
    return hipGetLastError();
}

hipError_t launch_support_wave(const Buf& x, const int32_t* tasks, const int32_t* count_dev, int32_t n_hint,
                               const Ctl* ctl, hipStream_t s) {
    if (n_hint <= 0) return hipSuccess;
    k_support_wave<<<min(grid_for((int64_t)n_hint * 64), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, tasks, count_dev, ctl);
    return hipGetLastError();
}

hipError_t launch_support_hub(const Buf& x, const Csc& c, const Scratch& sc, int32_t n_items_hint, Ctl* ctl,
                              unsigned long long* cycles, hipStream_t s) {
    if (n_items_hint <= 0) return hipSuccess;
    k_support_hub<<<min(n_items_hint, kHubMaxGrid), kHubThreads, 0, s>>>(x, c, sc.item_kappa, sc.item_c0, sc.item_c1,
                                                                        ctl, sc.hitw, cycles);
    return hipGetLastError();
}

hipError_t launch_hit_sum(const Buf& x, const Scratch& sc, const int32_t* m_count, int32_t m_hint, const Ctl* ctl,
                          hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    k_hit_sum<<<min(grid_for(m_hint), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, sc.hitw, sc.hub_row, m_count, ctl);
    return hipGetLastError();
}

}  // namespace kt
