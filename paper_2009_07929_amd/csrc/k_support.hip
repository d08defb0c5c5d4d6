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
__device__ __forceinline__ void wave_task(const Buf& x, int32_t e, unsigned long long* cycles);

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
// cycles: when not null (cost sampling), every task's shader cycles are
// added to cycles[kappa] (one wave per task: wave-cycles).
__global__ __launch_bounds__(kBlock) void k_support_wave(Buf x, const int32_t* __restrict__ tasks,
                                                       const int32_t* __restrict__ count, const Ctl* __restrict__ ctl,
                                                       unsigned long long* __restrict__ cycles) {
    if (ctl->done) return;
    const int32_t nt = *count;
    const int32_t nw = (int32_t)(gridDim.x * (kBlock / 64));
    for (int32_t wid = (int32_t)((blockIdx.x * kBlock + threadIdx.x) >> 6); wid < nt; wid += nw)
        wave_task(x, tasks ? tasks[wid] : wid, cycles);
}

__device__ __forceinline__ void wave_task(const Buf& x, int32_t e, unsigned long long* cycles) {
    const int lane = __lane_id();
    const unsigned long long t0 = cycles ? (unsigned long long)clock64() : 0ull;
    const int32_t* __restrict__ col = x.col;
    const int32_t i = x.src[e];
    const int32_t k = col[e];
    const int32_t a0 = e + 1, a1 = x.rowptr[i + 1];     // tail of row i
    const int32_t b0 = x.rowptr[k], b1 = x.rowptr[k + 1];  // row kappa
    if (a0 >= a1 || b0 >= b1) {
        if (cycles && lane == 0) atomicAdd(&cycles[k], (unsigned long long)clock64() - t0);
        return;
    }
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
    if (cycles && lane == 0) atomicAdd(&cycles[k], (unsigned long long)clock64() - t0);
}

constexpr int kHitLongGrid = 2048;  // workgroups of k_hit_sum_long (rows strided over them)
constexpr int kHitLongUnroll = 4;   // word steps whose loads k_hit_sum_long issues together

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
static_assert(kHubChunk <= kHubThreads, "each wave holds at most 64 of an item's tasks in registers");
static_assert(64 % kHubUnroll == 0, "a step's chunk indices jj + u stay within the 64 lanes");

// The task loop of one hub item, for one wave.  The wave's tasks (kk = wave,
// wave + 4, ...; at most 64, lane r holds task r) are cut into 64-element
// chunks of their tails, numbered in task order.  For each block of 64
// chunks every lane first finds its chunk's task (a binary search over the
// lanes' chunk prefix sums) and keeps the chunk's descriptor in registers;
// the wave then processes the block kHubUnroll chunks per step, reading the
// descriptors with readlane: the loads of a step are issued together and no
// per-chunk bookkeeping runs on the scalar unit.  Each chunk's hit word goes
// to its lane and is written once per block with one store; the block's hit
// counts of each task are summed across lanes and added to S(i, kappa) with
// one atomic per task.  In the bitmap case a label beyond row kappa is
// clamped onto a zero guard word, so a lookup needs no compare-and-select.
template <int MODE>
__device__ __forceinline__ void hub_tasks(const Buf& x, unsigned long long* __restrict__ hitw,
                                          const int64_t* __restrict__ hwoff, int64_t hit_cap,
                                          const int32_t* __restrict__ cedge, const int32_t* __restrict__ csrc,
                                          const int32_t* __restrict__ ctail, int32_t c0, int32_t ntask, int32_t k,
                                          int32_t rs, int32_t d, int32_t last, uint32_t guard, const uint2* s_bm,
                                          int32_t* s_acc) {
    const int32_t* __restrict__ col = x.col;
    const int32_t* s_keys = reinterpret_cast<const int32_t*>(s_bm);
    const unsigned long long* s_bm64 = reinterpret_cast<const unsigned long long*>(s_bm);
    const int lane = (int)(threadIdx.x & 63);
    const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));  // wave-uniform
    constexpr int kWaves = kHubThreads / 64;
    const int32_t mine = wv + kWaves * lane;
    int32_t t_e = 0, t_L = 0;
    int64_t t_w = 0;  // first hit word of task r
    if (mine < ntask) {
        t_e = cedge[c0 + mine];
        t_L = ctail[c0 + mine];
        if (t_L > 0) t_w = hwoff[csrc[c0 + mine] + 1] - hit_words_upto(t_L);
    }
    const int32_t t_nc = (t_L + 63) >> 6;          // chunks of task r
    const int32_t t_P = wave_incl_scan(t_nc);       // chunks of tasks 0..r
    const int32_t C = __builtin_amdgcn_readlane(t_P, 63);
    for (int32_t b0 = 0; b0 < C; b0 += 64) {
        // descriptor of chunk j = b0 + lane: its task r (smallest r with
        // t_P[r] > j), the chunk index within the task, start and length
        const int32_t j = b0 + lane;
        int32_t lo = 0, hi = 63;
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const int32_t mid = (lo + hi) >> 1;
            if (__shfl(t_P, mid) > j) hi = mid;
            else lo = mid + 1;
        }
        const bool dv = j < C;
        const int32_t de = __shfl(t_e, lo), dL = __shfl(t_L, lo), dS = __shfl(t_P - t_nc, lo);
        const int32_t dc = dv ? j - dS : 0;                   // chunk index within the task
        const int32_t dbase = dv ? de + 1 + 64 * dc : 0;      // first tail position of the chunk
        const int32_t dlen = dv ? min(64, dL - 64 * dc) : 0;  // elements in the chunk
        const int64_t dw = __shfl(t_w, lo) + dc;               // the chunk's hit word
        const bool dfar = dv && dw >= hit_cap;                  // beyond the capacity: hits add directly
        const unsigned long long far = __ballot(dfar);
        const int32_t nch = min(64, C - b0);
        uint32_t word_lo = 0, word_hi = 0;
        // step j0: the descriptors of chunks j0 .. j0 + kHubUnroll - 1 (readlane;
        // j0 + u <= 63, lanes at or past nch carry dbase = dlen = 0) and their
        // tail loads, unconditional at the chunk's base plus the lane: lanes past
        // a chunk read up to 63 elements further (the column arrays carry that
        // much slack) and are masked when processed
        auto load_step = [&](int32_t j0, int32_t(&ub)[kHubUnroll], int32_t(&ul)[kHubUnroll],
                             int32_t(&uw)[kHubUnroll]) {
#pragma unroll
            for (int u = 0; u < kHubUnroll; ++u) {
                ub[u] = __builtin_amdgcn_readlane(dbase, j0 + u);
                ul[u] = __builtin_amdgcn_readlane(dlen, j0 + u);
            }
#pragma unroll
            for (int u = 0; u < kHubUnroll; ++u) uw[u] = (col + (uint32_t)ub[u])[(uint32_t)lane];  // ub >= 0
        };
        auto process_step = [&](int32_t j0, const int32_t(&ub)[kHubUnroll], const int32_t(&ul)[kHubUnroll],
                                const int32_t(&uw)[kHubUnroll]) {
            unsigned long long hb[kHubUnroll];
            if (MODE == kModeBitmap) {
                // all chunks' bitmap words first (independent LDS reads), then
                // bit tests, ranks and LDS accumulations
                unsigned long long bw[kHubUnroll];
                uint32_t off[kHubUnroll];
#pragma unroll
                for (int u = 0; u < kHubUnroll; ++u) {
                    off[u] = min((uint32_t)(uw[u] - k - 1), guard);
                    bw[u] = s_bm64[off[u] >> 5];
                }
#pragma unroll
                for (int u = 0; u < kHubUnroll; ++u) {
                    const uint32_t bits = (uint32_t)bw[u];
                    const uint32_t bit = __builtin_amdgcn_ubfe(bits, off[u], 1u);
                    // hit mask: two lane compares (v_cmp), the bit test and the chunk's lanes
                    const bool in = (uint32_t)lane < (uint32_t)ul[u];
                    hb[u] = __builtin_amdgcn_uicmp(bit, 0u, 33 /* ne */) &
                            __builtin_amdgcn_uicmp((uint32_t)lane, (uint32_t)ul[u], 36 /* ult */);
                    // the word's high half is the byte offset in s_acc of its first set bit's
                    // entry; ubfe takes its width modulo 32, so the bits below off are counted
                    if (bit && in)
                        atomicAdd(reinterpret_cast<int32_t*>(reinterpret_cast<char*>(s_acc) + (uint32_t)(bw[u] >> 32) +
                                                             (__popc(__builtin_amdgcn_ubfe(bits, 0u, off[u])) << 2)),
                                  1);
                }
            } else {
#pragma unroll
                for (int u = 0; u < kHubUnroll; ++u) {
                    const int32_t w = uw[u];
                    bool hit = false;
                    if (lane < ul[u] && w <= last) {  // beyond the last label of row kappa nothing matches
                        int32_t q = -1;
                        if (MODE == kModeKeys) {
                            const int32_t qq = lower_bound_i32(s_keys, d, w);
                            if (s_keys[qq] == w) q = qq;
                        } else {
                            const int32_t qq = lower_bound_i32(col + rs, d, w);
                            if (col[rs + qq] == w) q = qq;
                        }
                        if (q >= 0) {
                            hit = true;
                            if (MODE != kModeGlobal) atomicAdd(&s_acc[q], 1);
                            else atomicAdd(&x.S[rs + q], 1);
                        }
                    }
                    hb[u] = __ballot(hit);
                }
            }
            // the chunk's hit word goes to its lane
#pragma unroll
            for (int u = 0; u < kHubUnroll; ++u) {
                if (lane == j0 + u) {
                    word_lo = (uint32_t)hb[u];
                    word_hi = (uint32_t)(hb[u] >> 32);
                }
            }
            // S(i, w) of chunks without a hit word
            if (far) {
#pragma unroll
                for (int u = 0; u < kHubUnroll; ++u)
                    if (j0 + u < nch && ((far >> (j0 + u)) & 1ull) && ((hb[u] >> lane) & 1ull))
                        atomicAdd(&x.S[ub[u] + lane], 1);
            }
        };
        for (int32_t jj = 0; jj < nch; jj += kHubUnroll) {
            int32_t ub[kHubUnroll], ul[kHubUnroll], uw[kHubUnroll];
            load_step(jj, ub, ul, uw);
            process_step(jj, ub, ul, uw);
        }
        // block end: lane j writes chunk j's hit word and adds its hits to S(i, kappa)
        const unsigned long long word = ((unsigned long long)word_hi << 32) | word_lo;
        // written once and read once by k_hit_sum: a streaming store keeps L2 for the tails
        if (dv && !dfar) __builtin_nontemporal_store(word, &hitw[dw]);
        // S(i, kappa): the block's chunks of one task sit on consecutive lanes; a
        // segmented sum gives one atomic per task and block instead of one per chunk
        const int32_t key = dv ? de : -1;
        int32_t cnt = dv ? __popcll(word) : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(cnt, o);
            const int32_t kk = __shfl_up(key, o);
            if (lane >= o && kk == key) cnt += u;
        }
        const int32_t next_key = __shfl_down(key, 1);
        if (dv && cnt && (lane == 63 || next_key != key)) atomicAdd(&x.S[de], cnt);
    }
}

__global__ __launch_bounds__(kHubThreads) void k_support_hub(Buf x, Csc c, const HubItem* __restrict__ items,
                                                           const int32_t* __restrict__ ctail, Ctl* ctl,
                                                           unsigned long long* __restrict__ hitw,
                                                           const int64_t* __restrict__ hwoff, int64_t hit_cap,
                                                           unsigned long long* __restrict__ cycles) {
    __shared__ uint2 s_bm[kSpanWords + 1];  // rank bitmap {bits, 4 x set bits before this word} + a zero guard word; or keys
    __shared__ int32_t s_acc[kKeyCap];
    __shared__ int s_wave[kHubThreads / 64];
    __shared__ int32_t s_it;
    if (ctl->done) return;
    const int32_t n_items = ctl->n_items;
    const int t = threadIdx.x;
    const int32_t* __restrict__ col = x.col;
    int32_t* s_keys = reinterpret_cast<int32_t*>(s_bm);
    // Row kappa currently staged in LDS (workgroup-uniform), or cur_k = -1.
    int32_t cur_k = -1, cur_rs = 0, cur_d = 0, cur_last = 0, cur_mode = kModeBitmap;
    uint32_t cur_guard = 0;
    auto flush = [&]() {  // S(kappa, :) accumulated in LDS -> global
        if (cur_k >= 0 && cur_mode != kModeGlobal)
            for (int32_t q = t; q < cur_d; q += kHubThreads) {
                const int32_t a = s_acc[q];
                if (a) atomicAdd(&x.S[cur_rs + q], a);
            }
    };
    // Persistent: workgroups pull tickets from a device counter; a ticket is
    // kHubBatch consecutive items, so the counter sees few atomics.  Items are
    // laid out by ascending kappa and the heaviest rows carry the largest
    // labels, so they are taken from the end first (longest work first).  The
    // items of one row are consecutive: a workgroup that takes several keeps
    // the row staged and its accumulators, and flushes them once.  The next
    // ticket is requested while the current one is processed.
    if (t == 0) s_it = atomicAdd(&ctl->item_next, 1);
    __syncthreads();
    for (;;) {
        const int32_t first = n_items - 1 - __builtin_amdgcn_readfirstlane(s_it) * kHubBatch;
        if (first < 0) break;
        int32_t ticket = 0;
        if (t == 0) ticket = atomicAdd(&ctl->item_next, 1);
        for (int32_t it = first; it > first - kHubBatch && it >= 0; --it) {
            // item fields are workgroup-uniform: keep them in scalar registers
            const HubItem h = items[it];
            const int32_t k = __builtin_amdgcn_readfirstlane(h.k), c0 = __builtin_amdgcn_readfirstlane(h.c0);
            const int32_t ntask = __builtin_amdgcn_readfirstlane(h.c1) - c0;
            const unsigned long long t_start = cycles ? (unsigned long long)clock64() : 0ull;
            if (k != cur_k) {
                __syncthreads();  // every wave is done adding into the previous row's accumulators
                flush();
                cur_k = k;
                cur_rs = __builtin_amdgcn_readfirstlane(h.rs);
                cur_d = __builtin_amdgcn_readfirstlane(h.d);
                cur_last = __builtin_amdgcn_readfirstlane(h.last);
                const int32_t rs = cur_rs, d = cur_d;
                const int32_t span = cur_last - k;  // labels of row kappa lie in (k, last]
                cur_mode = d > kKeyCap ? kModeGlobal : (span <= kSpanCap ? kModeBitmap : kModeKeys);
                __syncthreads();  // the flush and the previous row's tasks are done with LDS
                if (cur_mode == kModeBitmap) {
                    const int32_t nw = (span + 31) >> 5;
                    cur_guard = (uint32_t)nw * 32u;  // labels beyond row kappa read the zero word nw
                    for (int32_t j = t; j <= nw; j += kHubThreads) s_bm[j] = make_uint2(0u, 0u);
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
                    for (int32_t j = j0; j < j1; ++j) {  // byte offset of the word's first entry in s_acc
                        s_bm[j].y = (uint32_t)run * 4u;
                        run += __popc(s_bm[j].x);
                    }
                } else if (cur_mode == kModeKeys) {
                    for (int32_t q = t; q < d; q += kHubThreads) s_keys[q] = col[rs + q];
                }
                if (cur_mode != kModeGlobal)
                    for (int32_t q = t; q < d; q += kHubThreads) s_acc[q] = 0;
                __syncthreads();
            }
            if (cur_mode == kModeBitmap)
                hub_tasks<kModeBitmap>(x, hitw, hwoff, hit_cap, c.edge, c.src, ctail, c0, ntask, k, cur_rs, cur_d, cur_last,
                                   cur_guard, s_bm, s_acc);
            else if (cur_mode == kModeKeys)
                hub_tasks<kModeKeys>(x, hitw, hwoff, hit_cap, c.edge, c.src, ctail, c0, ntask, k, cur_rs, cur_d, cur_last,
                                   cur_guard, s_bm, s_acc);
            else
                hub_tasks<kModeGlobal>(x, hitw, hwoff, hit_cap, c.edge, c.src, ctail, c0, ntask, k, cur_rs, cur_d, cur_last,
                                   cur_guard, s_bm, s_acc);
            if (cycles) {  // per-row cost samples for the cost model (shader clock)
                __syncthreads();
                // wave-cycles: the item held the workgroup's kHubThreads / 64 waves
                if (t == 0) atomicAdd(&cycles[k], ((unsigned long long)clock64() - t_start) * (kHubThreads / 64));
            }
        }
        __syncthreads();  // every thread has read s_it
        if (t == 0) s_it = ticket;
        __syncthreads();
    }
    __syncthreads();  // the last row's tasks are done with LDS
    flush();
}

// 64x64 bit transpose across a wave: lane j holds row j (bit l = entry
// (j, l)); afterwards lane l holds column l (bit j = entry (j, l)).  Six
// butterfly stages swap the off-diagonal blocks of halving size: at stage b a
// lane without bit b of its index keeps the bits whose index lacks bit b and
// takes its partner's (lane xor b) such bits moved up by b; a lane with bit b
// does the mirror image.  The 64-bit rows are handled as two 32-bit halves:
// stage 32 exchanges whole halves (one word sent per lane: the half its
// partner needs), the other stages work within each half.  Partners within
// a row of 16 lanes are read with DPP (quad permutes for 1 and 2, rotates of
// the row for 4 and 8), the partner 16 lanes away with a swizzle and the one
// 32 lanes away with a permute; the move by b is a rotate (the bits it wraps
// around fall outside the kept mask) and the merge one bit-field select.
template <int B>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane) {
    if constexpr (B == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (B == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (B == 4) {
        // row_ror:n reads lane (l - n) mod 16 of the row: n = 4 for lanes with bit 2, 12 for the others
        const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false);
        const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x12C, 0xF, 0xF, false);
        return (lane & 4) ? dn : up;
    } else if constexpr (B == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else {
        static_assert(B == 16, "lanes 32 apart go through the permute in transpose64");
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);  // bit-mask mode: lane xor 16
    }
}

template <int B>
__device__ __forceinline__ void transpose_stage(uint32_t& lo, uint32_t& hi, int lane) {
    constexpr uint32_t m = B == 16 ? 0x0000FFFFu : B == 8 ? 0x00FF00FFu : B == 4 ? 0x0F0F0F0Fu
                         : B == 2 ? 0x33333333u : 0x55555555u;  // the bits whose index lacks bit B
    const bool up = (lane & B) != 0;
    const uint32_t keep = up ? ~m : m;
    const uint32_t rot = up ? (uint32_t)B : (uint32_t)(32 - B);  // rotate right: >> B, or << B
    const uint32_t ylo = lane_xor<B>(lo, lane), yhi = lane_xor<B>(hi, lane);
    lo = (lo & keep) | (__builtin_amdgcn_alignbit(ylo, ylo, rot) & ~keep);
    hi = (hi & keep) | (__builtin_amdgcn_alignbit(yhi, yhi, rot) & ~keep);
}

__device__ __forceinline__ unsigned long long transpose64(unsigned long long v, int lane) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    {  // stage 32: a lane in the lower half takes its partner's low half as its high half, and vice versa
        const bool up = (lane & 32) != 0;
        const uint32_t r = (uint32_t)__shfl_xor((int)(up ? lo : hi), 32);
        if (up) lo = r; else hi = r;
    }
    transpose_stage<16>(lo, hi, lane);
    transpose_stage<8>(lo, hi, lane);
    transpose_stage<4>(lo, hi, lane);
    transpose_stage<2>(lo, hi, lane);
    transpose_stage<1>(lo, hi, lane);
    return ((unsigned long long)hi << 32) | lo;
}

// Column counts of the wave's 64x64 bit matrix (lane l: how many rows have
// bit l), by the transpose and a popcount; nothing to do when every row is
// empty.  Called with the whole wave active.
__device__ __forceinline__ uint32_t column_counts(unsigned long long v, int lane) {
    if (__ballot(v != 0ull) == 0ull) return 0u;
    return (uint32_t)__popcll(transpose64(v, lane));
}

// Row-local sum of the hub kernel's hit words: S(i, w) of the edge at
// position p of row i gains one for every earlier task j of row i (a hub task:
// hub_row[col[j]]) whose hit words have the bit of tail offset p - j - 1.
// One wave per window of 64 positions P0 .. P0+63.  Lane l takes the task at
// P0 + l and shifts its first word so that bit l' stands for position
// P0 + l'; a 64x64 bit transpose and a popcount then give every position the
// hits of the window's own tasks (a task has no hits past its row, so tasks of
// other rows add nothing).  The only earlier tasks that reach into the window
// are those of the row holding P0 when it starts before P0: their words are
// aligned to the window with a funnel shift of two words and summed the same
// way, 64 tasks at a time, back to the start of the row.  A word at or past
// the capacity was never written: its chunk added its hits directly.
__global__ __launch_bounds__(kBlock) void k_hit_sum(Buf x, const unsigned long long* __restrict__ hitw,
                                                  const int64_t* __restrict__ hwoff, int64_t hit_cap,
                                                  const uint8_t* __restrict__ hub_row,
                                                  const int32_t* __restrict__ count, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t m = *count;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t P0l = ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * 64;
    if (P0l >= m) return;  // whole wave
    const int32_t P0 = (int32_t)P0l;
    const int32_t* __restrict__ col = x.col;
    const int32_t p = P0 + lane;
    // rows summed by k_hit_sum_long are left out here (their tasks hit only their own row)
    auto is_long = [](int32_t d) { return d > kHitLongMin && d <= kHitLongMax; };
    unsigned long long v = 0;
    if (p < m && lane < 63) {  // position P0 + lane + 1 is tail offset 0 of task p
        const int32_t i = x.src[p];
        const int32_t re = x.rowptr[i + 1];
        const int32_t L = re - p - 1;
        if (L > 0 && !is_long(re - x.rowptr[i]) && hub_row[col[p]]) {
            const int64_t w = hwoff[i + 1] - hit_words_upto(L);
            if (w < hit_cap) v = hitw[w] << (lane + 1);
        }
    }
    uint32_t add = column_counts(v, lane);
    const int32_t r0 = x.src[P0];  // the row holding P0
    const int32_t r0s = x.rowptr[r0], r0e = x.rowptr[r0 + 1];
    if (r0s < P0 && !is_long(r0e - r0s)) {
        const int64_t rend = hwoff[r0 + 1];
        for (int32_t j0 = r0s; j0 < P0; j0 += 64) {
            const int32_t j = j0 + lane;
            unsigned long long w = 0;
            if (j < P0 && hub_row[col[j]]) {
                const int32_t L = r0e - j - 1;   // tail length of task j (> P0 - j - 1)
                const int32_t t0 = P0 - j - 1;   // tail offset of position P0 (>= 0)
                const int32_t c = t0 >> 6, sft = t0 & 63;
                const int64_t wc = rend - hit_words_upto(L) + c;  // word c exists: 64 c <= t0 < L
                const unsigned long long lo = wc < hit_cap ? hitw[wc] : 0ull;
                const unsigned long long hi = ((c + 1) * 64 < L && wc + 1 < hit_cap) ? hitw[wc + 1] : 0ull;
                w = sft ? ((lo >> sft) | (hi << (64 - sft))) : lo;
            }
            add += column_counts(w, lane);
        }
    }
    if (p < m && add) x.S[p] += (int32_t)add;
}

// Row-local sum of the hit words of one row per workgroup, for rows of length
// d in (kHitLongMin, kHitLongMax], where the windows above would re-read the
// words of a row's earlier tasks once per window.  The row's tasks are taken 64
// at a time (task r = 64 b + lane, relative to the row start); for word c of
// every task of the block, the bits that fall in window b + c (relative
// positions 64 (b + c) ...) and those that spill into window b + c + 1 are
// separated by two shifts, and a 64x64 bit transpose plus a popcount of each
// gives every position of the two windows its count, added in LDS.  The spill
// of word c is carried in a register into the next step, so every word is read
// once and transposed once.  The counts are then added to S(i, w).
__global__ __launch_bounds__(kBlock) void k_hit_sum_long(Buf x, const unsigned long long* __restrict__ hitw,
                                                       const int64_t* __restrict__ hwoff, int64_t hit_cap,
                                                       const uint8_t* __restrict__ hub_row,
                                                       const int32_t* __restrict__ long_rows,
                                                       const Ctl* __restrict__ ctl) {
    __shared__ int32_t s_cnt[kHitLongMax + 64 * (kHitLongUnroll + 1)];
    if (ctl->done) return;
    const int32_t nl = ctl->n_long;
    const int t = threadIdx.x, lane = __lane_id(), wv = t >> 6;
    const int32_t* __restrict__ col = x.col;
    for (int32_t k = (int32_t)blockIdx.x; k < nl; k += (int32_t)gridDim.x) {
        const int32_t i = long_rows[k];
        const int32_t rs = x.rowptr[i], d = x.rowptr[i + 1] - rs;  // kHitLongMin < d <= kHitLongMax
        const int64_t rend = hwoff[i + 1];
        for (int32_t j = t; j < d + 64; j += kBlock) s_cnt[j] = 0;
        __syncthreads();
        const int32_t nb = (d + 63) >> 6;
        for (int32_t b = wv; b < nb; b += kBlock / 64) {
            const int32_t r = 64 * b + lane;
            int32_t nw = 0;
            int64_t w0 = 0;
            if (r < d) {
                const int32_t L = d - 1 - r;
                if (L > 0 && hub_row[col[rs + r]]) {
                    nw = (L + 63) >> 6;
                    w0 = rend - hit_words_upto(L);
                }
            }
            // the block's first task has the longest tail: its word count bounds the steps;
            // window b + c takes the low part of word c and the spill of word c - 1
            const int32_t steps = (d - 1 - 64 * b + 63) >> 6;
            unsigned long long prev = 0ull;
            for (int32_t c0 = 0; c0 <= steps; c0 += kHitLongUnroll) {
                unsigned long long wd[kHitLongUnroll];
#pragma unroll
                for (int u = 0; u < kHitLongUnroll; ++u) {  // the step group's loads first
                    const int32_t c = c0 + u;
                    wd[u] = (c < nw && w0 + c < hit_cap) ? hitw[w0 + c] : 0ull;  // past the capacity: added directly
                }
#pragma unroll
                for (int u = 0; u < kHitLongUnroll; ++u) {
                    const unsigned long long v = (lane == 63 ? 0ull : (wd[u] << (lane + 1))) | (prev >> (63 - lane));
                    prev = wd[u];
                    const uint32_t cnt = column_counts(v, lane);
                    if (cnt) atomicAdd(&s_cnt[64 * (b + c0 + u) + lane], (int32_t)cnt);
                }
            }
        }
        __syncthreads();
        for (int32_t j = t; j < d; j += kBlock) {
            const int32_t a = s_cnt[j];
            if (a) x.S[rs + j] += a;
        }
        __syncthreads();  // the next row clears s_cnt
    }
}

// Measurement aid (profiling only): statistics of the pass just computed,
// added to acc[0 .. kPassStats-1] (see PassStat).  hub_row: the rows kappa
// the hub kernel staged in this pass, or null when it did not run.
__global__ __launch_bounds__(kBlock) void k_pass_work(Buf x, const int32_t* __restrict__ count,
                                                    const uint8_t* __restrict__ hub_row,
                                                    unsigned long long* __restrict__ acc) {
    __shared__ unsigned long long s_v[kPassStats][kBlock / 64];
    const int32_t m = *count;
    unsigned long long v[kPassStats] = {};
    for (int32_t e = (int32_t)(blockIdx.x * kBlock + threadIdx.x); e < m; e += (int32_t)(gridDim.x * kBlock)) {
        const int32_t i = x.src[e], k = x.col[e];
        const uint32_t tail = (uint32_t)(x.rowptr[i + 1] - e - 1);
        v[kStatTail] += tail;
        v[kStatRowK] += (uint32_t)(x.rowptr[k + 1] - x.rowptr[k]);
        v[kStatSupport] += (uint32_t)x.S[e];
        v[kStatEdges] += 1;
        if (hub_row) {
            if (hub_row[k]) {
                v[kStatHubTasks] += 1;
                v[kStatHubTail] += tail;
                v[kStatHubWords] += (tail + 63) >> 6;
            }
            if (hub_row[i]) v[kStatHubStaged] += 1;
        }
    }
#pragma unroll
    for (int j = 0; j < kPassStats; ++j) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o);
        if ((threadIdx.x & 63) == 0) s_v[j][threadIdx.x >> 6] = v[j];
    }
    __syncthreads();
    if (threadIdx.x < kPassStats) {
        unsigned long long t = 0;
        for (int i = 0; i < kBlock / 64; ++i) t += s_v[threadIdx.x][i];
        if (t) atomicAdd(&acc[threadIdx.x], t);
    }
}

}  // namespace

hipError_t launch_pass_work(const Buf& x, const int32_t* m_count, int32_t m_hint, const uint8_t* hub_row,
                            unsigned long long* acc, hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    k_pass_work<<<min(grid_for(m_hint), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, m_count, hub_row, acc);
    return hipGetLastError();
}

hipError_t launch_support_thread(const Buf& x, const int32_t* tasks, const int32_t* count_dev, int32_t n_hint,
                                 const Ctl* ctl, hipStream_t s) {
    if (n_hint <= 0) return hipSuccess;
    k_support_thread<<<min(grid_for(n_hint), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, tasks, count_dev, ctl);
    return hipGetLastError();
}

hipError_t launch_support_wave(const Buf& x, const int32_t* tasks, const int32_t* count_dev, int32_t n_hint,
                               const Ctl* ctl, hipStream_t s, unsigned long long* cycles) {
    if (n_hint <= 0) return hipSuccess;
    k_support_wave<<<min(grid_for((int64_t)n_hint * 64), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, tasks, count_dev, ctl,
                                                                                                  cycles);
    return hipGetLastError();
}

hipError_t launch_support_hub(const Buf& x, const Csc& c, const Scratch& sc, int32_t n_items_hint, Ctl* ctl,
                              unsigned long long* cycles, hipStream_t s) {
    if (n_items_hint <= 0) return hipSuccess;
    k_support_hub<<<min(n_items_hint, kHubMaxGrid), kHubThreads, 0, s>>>(x, c, sc.items, sc.ctail, ctl, sc.hitw,
                                                                        sc.hwoff, sc.hit_cap, cycles);
    return hipGetLastError();
}

hipError_t launch_hit_sum(const Buf& x, const Scratch& sc, const int32_t* m_count, int32_t m_hint, const Ctl* ctl,
                          hipStream_t s) {
    if (m_hint <= 0) return hipSuccess;
    const int64_t windows = ((int64_t)m_hint + 63) / 64;
    const unsigned grid = (unsigned)((windows + kBlock / 64 - 1) / (kBlock / 64));  // one wave per window
    k_hit_sum<<<grid, kBlock, 0, s>>>(x, sc.hitw, sc.hwoff, sc.hit_cap, sc.hub_row, m_count, ctl);
    k_hit_sum_long<<<kHitLongGrid, kBlock, 0, s>>>(x, sc.hitw, sc.hwoff, sc.hit_cap, sc.hub_row, sc.long_rows, ctl);
    return hipGetLastError();
}

}  // namespace kt
