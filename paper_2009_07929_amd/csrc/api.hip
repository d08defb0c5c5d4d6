// C-ABI entry points, argument checks, workspace layout and the round driver.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <utility>
#include <vector>

#include "kernels.h"

namespace kt {

namespace {
thread_local char t_msg[512];
thread_local int32_t t_hip = 0;
}  // namespace

int32_t fail(int32_t code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_msg, sizeof(t_msg), fmt, ap);
    va_end(ap);
    return code;
}

int32_t fail_hip(hipError_t e, const char* what) {
    t_hip = (int32_t)e;
    snprintf(t_msg, sizeof(t_msg), "%s: %s", what, hipGetErrorString(e));
    return KTRUSS_E_HIP;
}

void clear_error() {
    t_msg[0] = 0;
    t_hip = 0;
}

namespace {

// Workspace regions (256-byte aligned) for n vertices, m edges and, in the
// batched form, G graphs.
struct FullLayout {
    Layout L;
    size_t gidv, thrv, graph_done, done_now, low_cnt;
};

FullLayout full_layout(int32_t n, int64_t m, int32_t G) {
    FullLayout F{};
    Layout& L = F.L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t em = sizeof(int32_t) * (size_t)m;
    const size_t em1 = sizeof(int32_t) * ((size_t)m + 1);
    const size_t vn = sizeof(int32_t) * ((size_t)n + 1);
    for (int b = 0; b < 2; ++b) {
        L.col[b] = take(em + sizeof(int32_t) * 64);  // 64 columns of slack: the hub kernel's chunk loads
        L.src[b] = take(em);
        L.eid[b] = take(em);
        L.S[b] = take(em);
        L.rowptr[b] = take(vn);
    }
    L.cedge = take(em);
    L.csrc = take(em);
    L.ckey = take(em);
    L.cptr = take(vn);
    L.xscan = take(em1);
    L.keepw = take(sizeof(KeepWord) * ((size_t)m / 64 + 1));
    L.cxscan = take(em1);
    L.blockcnt = take(sizeof(int32_t) * kMaxScanBlocks);
    L.blockoff = take(sizeof(int32_t) * kMaxScanBlocks);
    L.blockcnt2 = take(sizeof(int32_t) * 2 * kMaxScanBlocks);
    L.blockoff2 = take(sizeof(int32_t) * 2 * kMaxScanBlocks);
    L.alive_in = take(vn);
    L.itemoff = take(vn);
    L.items = take(sizeof(HubItem) * (size_t)item_capacity(n, m));
    L.ctail = take(em);
    L.insum = take(sizeof(unsigned long long) * ((size_t)n + 1));
    L.cycles = take(sizeof(unsigned long long) * ((size_t)n + 1));
    L.act_off = take(vn);
    L.act_list = take(vn);
    L.feats = take(sizeof(float) * KTRUSS_MLP_IN * ((size_t)n + 1));
    L.pred = take(sizeof(float) * ((size_t)n + 1));
    L.chunk_sz = take(vn);
    L.rs_hist = take(sizeof(int32_t) * (256 * (((size_t)m + kRsTile - 1) / kRsTile) + 1));
    L.is_hub = take((size_t)n + 1);
    L.hub_row = take((size_t)n + 1);
    L.hitw = take(sizeof(unsigned long long) * kHitWordsPerEdge * (size_t)m);
    L.hwoff = take(sizeof(int64_t) * ((size_t)n + 1));
    L.wave_tasks = take(em);
    L.thread_tasks = take(em);
    L.long_off = take(vn);
    L.long_rows = take(vn);
    L.ctl = take(sizeof(Ctl));
    if (G > 0) {
        F.gidv = take(vn);
        F.thrv = take(vn);
        F.graph_done = take((size_t)G);
        F.done_now = take((size_t)G);
        F.low_cnt = take(sizeof(int32_t) * (size_t)G);
    }
    L.total = off;
    return F;
}

struct Work {
    Buf b[2];
    Csc c[2];
    Scratch sc;
    Ctl* ctl;
    BatchCtx batch;  // batch.thrv == nullptr for a single graph
};

Work carve(void* work, int32_t n, int64_t m, int32_t G) {
    const FullLayout F = full_layout(n, m, G);
    const Layout& L = F.L;
    char* base = (char*)work;
    Work w{};
    for (int b = 0; b < 2; ++b) {
        w.b[b].col = (int32_t*)(base + L.col[b]);
        w.b[b].src = (int32_t*)(base + L.src[b]);
        w.b[b].eid = (int32_t*)(base + L.eid[b]);
        w.b[b].S = (int32_t*)(base + L.S[b]);
        w.b[b].rowptr = (int32_t*)(base + L.rowptr[b]);
        w.c[b].edge = (int32_t*)(base + L.cedge);  // one set of in-edge lists, remapped in place
        w.c[b].src = (int32_t*)(base + L.csrc);
        w.c[b].key = (int32_t*)(base + L.ckey);
        w.c[b].ptr = (int32_t*)(base + L.cptr);
    }
    w.sc.xscan = (int32_t*)(base + L.xscan);
    w.sc.keepw = (KeepWord*)(base + L.keepw);
    w.sc.cxscan = (int32_t*)(base + L.cxscan);
    w.sc.blockcnt = (int32_t*)(base + L.blockcnt);
    w.sc.blockoff = (int32_t*)(base + L.blockoff);
    w.sc.blockcnt2 = (int32_t*)(base + L.blockcnt2);
    w.sc.blockoff2 = (int32_t*)(base + L.blockoff2);
    w.sc.alive_in = (int32_t*)(base + L.alive_in);
    w.sc.itemoff = (int32_t*)(base + L.itemoff);
    w.sc.items = (HubItem*)(base + L.items);
    w.sc.ctail = (int32_t*)(base + L.ctail);
    w.sc.insum = (unsigned long long*)(base + L.insum);
    w.sc.cycles = (unsigned long long*)(base + L.cycles);
    w.sc.act_off = (int32_t*)(base + L.act_off);
    w.sc.act_list = (int32_t*)(base + L.act_list);
    w.sc.feats = (float*)(base + L.feats);
    w.sc.pred = (float*)(base + L.pred);
    w.sc.chunk_sz = (int32_t*)(base + L.chunk_sz);
    w.sc.rs_hist = (int32_t*)(base + L.rs_hist);
    w.sc.is_hub = (uint8_t*)(base + L.is_hub);
    w.sc.hub_row = (uint8_t*)(base + L.hub_row);
    w.sc.hitw = (unsigned long long*)(base + L.hitw);
    w.sc.hwoff = (int64_t*)(base + L.hwoff);
    w.sc.hit_cap = (int64_t)kHitWordsPerEdge * m;
    w.sc.wave_tasks = (int32_t*)(base + L.wave_tasks);
    w.sc.thread_tasks = (int32_t*)(base + L.thread_tasks);
    w.sc.long_off = (int32_t*)(base + L.long_off);
    w.sc.long_rows = (int32_t*)(base + L.long_rows);
    w.ctl = (Ctl*)(base + L.ctl);
    if (G > 0) {
        w.batch.gidv = (int32_t*)(base + F.gidv);
        w.batch.thrv = (int32_t*)(base + F.thrv);
        w.batch.graph_done = (uint8_t*)(base + F.graph_done);
        w.batch.done_now = (uint8_t*)(base + F.done_now);
        w.batch.low_cnt = (int32_t*)(base + F.low_cnt);
    }
    return w;
}

int32_t check_sizes(int32_t n, int64_t m) {
    if (n < 0 || m < 0) return fail(KTRUSS_E_INVALID, "n (%d) and m (%lld) must be >= 0", n, (long long)m);
    if (n > INT32_MAX - 1 || m > INT32_MAX - 1) return fail(KTRUSS_E_OVERFLOW, "n or m above INT32_MAX - 1");
    return KTRUSS_OK;
}

int32_t check_schedule(int32_t sched) {
    if (sched < KTRUSS_SCHED_PLAIN || sched > KTRUSS_SCHED_COARSE)
        return fail(KTRUSS_E_INVALID, "unknown schedule %d", sched);
    return KTRUSS_OK;
}

int32_t check_work(const void* work, int64_t work_bytes, int64_t need) {
    if (!work) return fail(KTRUSS_E_INVALID, "workspace is null");
    if (((uintptr_t)work & 15u) != 0) return fail(KTRUSS_E_INVALID, "workspace must be 16-byte aligned");
    if (work_bytes < need)
        return fail(KTRUSS_E_CAPACITY, "workspace has %lld bytes, needs %lld", (long long)work_bytes, (long long)need);
    return KTRUSS_OK;
}

int32_t check_graph(const ktruss_graph* g, bool need_work) {
    if (!g) return fail(KTRUSS_E_INVALID, "graph is null");
    int32_t rc = check_sizes(g->n, g->m);
    if (rc != KTRUSS_OK) return rc;
    if (!g->rowptr || (g->m > 0 && !g->col)) return fail(KTRUSS_E_INVALID, "graph rowptr/col is null");
    rc = check_schedule(g->schedule);
    if (rc != KTRUSS_OK) return rc;
    if (g->tuning.incremental < 0 || g->tuning.incremental > 2 || !(g->tuning.peel_ratio >= 0.f))
        return fail(KTRUSS_E_INVALID, "tuning.incremental must be 0, 1 or 2 and peel_ratio >= 0");
    if (need_work) return check_work(g->work, g->work_bytes, (int64_t)full_layout(g->n, g->m, 0).L.total);
    return KTRUSS_OK;
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

// Validates the input CSR on the device (writing each edge's row into
// src_out) and reads the verdict back.  Synchronises s.  merge_work: if not
// null, receives the light-graph gate's statistic (the input's merge length
// summed over its edges, the row-kappa part sampled).
int32_t validate_on_device(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m, const Work& w,
                           int32_t* src_out, hipStream_t s, unsigned long long* merge_work = nullptr) {
    HIP_TRY(launch_validate(rowptr, col, n, m, src_out, w.ctl, merge_work != nullptr, s), "validate launch");
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &w.ctl->err, sizeof(err), hipMemcpyDeviceToHost, s), "validate readback");
    if (merge_work)
        HIP_TRY(hipMemcpyAsync(merge_work, &w.ctl->merge_work, sizeof(*merge_work), hipMemcpyDeviceToHost, s),
                "merge work readback");
    HIP_TRY(hipStreamSynchronize(s), "validate sync");
    if (err)
        return fail(KTRUSS_E_INVALID,
                    "malformed CSR (check bits 0x%x: 1 rowptr range, 2 rowptr[0], 4 rowptr[n]!=m, 8 rowptr not "
                    "monotone, 16 columns not ascending above the diagonal or >= n)",
                    err);
    return KTRUSS_OK;
}

// ---- profiling tallies (process-wide; guarded by a mutex)
// kinds: 0 whole support pass, 1 thread-per-edge, 2 wavefront-per-edge, 3 hub,
// 4 row-local sum of the hub hit words, 5 thread-per-row (coarse schedule)
constexpr int kKinds = 6;
struct Rec {
    int kind;
    hipEvent_t e0, e1;
};
struct Profile {
    std::mutex mu;
    bool on = false;
    std::vector<Rec> recs;  // recorded, not yet read
    std::vector<hipEvent_t> pool;
    int64_t launches[kKinds] = {}, tasks[kKinds] = {}, bytes[kKinds] = {};
    double ms[kKinds] = {};
    unsigned long long* work_dev = nullptr;  // pass statistics (PassStat) on the device current at enable
};

// The pass statistics accumulate in a file-scope device array (one copy per
// GPU) rather than in allocated memory; host code reaches it through the
// address hipGetSymbolAddress reports for the current device.
__device__ __align__(256) unsigned long long g_prof_stats[kPassStats];
Profile& prof() {
    static Profile p;
    return p;
}

hipEvent_t take_event(Profile& P) {
    if (!P.pool.empty()) {
        hipEvent_t e = P.pool.back();
        P.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Event pair around a group of launches, tallied under `kind` when profiling
// (never while a graph is being captured).
struct Timer {
    bool on = false;
    int kind = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

thread_local bool t_capturing = false;

int32_t timer_begin(Timer& t, int kind, int64_t tasks, int64_t bytes, hipStream_t s) {
    if (t_capturing) return KTRUSS_OK;
    Profile& P = prof();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        if (!P.on) return KTRUSS_OK;
        t.e0 = take_event(P);
        t.e1 = take_event(P);
        if (!t.e0 || !t.e1) return fail(KTRUSS_E_HIP, "hipEventCreate failed");
        P.launches[kind] += 1;
        P.tasks[kind] += tasks;
        P.bytes[kind] += bytes;
    }
    t.on = true;
    t.kind = kind;
    HIP_TRY(hipEventRecord(t.e0, s), "profile event");
    return KTRUSS_OK;
}

int32_t timer_end(Timer& t, hipStream_t s) {
    if (!t.on) return KTRUSS_OK;
    HIP_TRY(hipEventRecord(t.e1, s), "profile event");
    Profile& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.recs.push_back(Rec{t.kind, t.e0, t.e1});
    return KTRUSS_OK;
}

template <class F>
int32_t timed_launch(int kind, int64_t tasks, hipStream_t s, F&& launch) {
    if (tasks <= 0) return KTRUSS_OK;
    Timer t;
    int32_t rc = timer_begin(t, kind, tasks, 0, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(launch(), "support launch");
    return timer_end(t, s);
}

// Device accumulator of the profiled passes' merge-model work, or null when
// not profiling (or while capturing a graph).
unsigned long long* profile_work() {
    if (t_capturing) return nullptr;
    Profile& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    return P.on ? P.work_dev : nullptr;
}

// Fixed workspace of ktruss_run_noalloc: a file-scope device array (one copy
// per GPU, resident until the process ends), for callers that cannot
// allocate.  Host code never passes the array's name to a kernel: it takes
// the address hipGetSymbolAddress reports on each device, once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;

int32_t noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(KTRUSS_E_INVALID, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "scratch address");
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return KTRUSS_OK;
}

bool uses_csc(int sched) {
    return sched != KTRUSS_SCHED_PLAIN && sched != KTRUSS_SCHED_FORCE_WAVE && sched != KTRUSS_SCHED_COARSE;
}

// Light-graph gate of the heuristic and learned schedules: an input whose
// mean merge length per edge (row tails exact, row-kappa lengths sampled on
// every 16th edge) is at most plain_max_work (0: the default, negative:
// never) has no task long enough to pay for in-edge lists, staging or
// binning, so the run is thread-per-edge throughout.
bool gated(const ktruss_graph* g) {
    return (g->schedule == KTRUSS_SCHED_HEURISTIC || g->schedule == KTRUSS_SCHED_LEARNED) &&
           g->tuning.plain_max_work >= 0;
}
int schedule_for(const ktruss_graph* g, unsigned long long merge_work) {
    if (!gated(g)) return g->schedule;
    const unsigned long long t = g->tuning.plain_max_work > 0 ? g->tuning.plain_max_work : kDefaultPlainMaxWork;
    return merge_work <= t * (unsigned long long)g->m ? KTRUSS_SCHED_PLAIN : g->schedule;
}

// Grid sizes of one pass: exact counts in host-loop mode, upper bounds when
// the pass is captured in a graph (the kernels read the true counts).
struct PassDims {
    int32_t m;        // alive edges (upper bound)
    int32_t items;    // hub items
    int32_t n_wave;   // wavefront tasks
    int32_t n_thread; // thread tasks
};

// One support pass over buffer p.  cycles: per-row hub timing (cost-model
// samples), or null.
int32_t support_pass(int sched, int32_t n, const Work& w, int p, const PassDims& dm, hipStream_t s,
                     unsigned long long* cycles = nullptr) {
    const Buf& x = w.b[p];
    Timer tp;
    int32_t rc = timer_begin(tp, 0, dm.m, 0, s);
    if (rc != KTRUSS_OK) return rc;
    if (sched == KTRUSS_SCHED_PLAIN) {
        rc = timed_launch(1, dm.m, s, [&] {
            return launch_support_thread(x, nullptr, &w.ctl->m_buf[p], dm.m, w.ctl, s);
        });
    } else if (sched == KTRUSS_SCHED_COARSE) {
        rc = timed_launch(5, dm.m, s, [&] { return launch_support_row(x, n, w.ctl, s); });
    } else if (sched == KTRUSS_SCHED_FORCE_WAVE) {
        rc = timed_launch(2, dm.m, s, [&] {
            return launch_support_wave(x, nullptr, &w.ctl->m_buf[p], dm.m, w.ctl, s);
        });
    } else {
        rc = timed_launch(3, dm.items, s, [&] {
            return launch_support_hub(x, w.c[p], w.sc, dm.items, w.ctl, cycles, s);
        });
        if (rc == KTRUSS_OK && dm.items > 0)
            rc = timed_launch(4, dm.m, s, [&] { return launch_hit_sum(x, w.sc, &w.ctl->m_buf[p], dm.m, w.ctl, s); });
        if (rc == KTRUSS_OK && sched != KTRUSS_SCHED_FORCE_HUB) {
            rc = timed_launch(2, dm.n_wave, s, [&] {
                return launch_support_wave(x, w.sc.wave_tasks, &w.ctl->n_wave, dm.n_wave, w.ctl, s, cycles);
            });
            if (rc == KTRUSS_OK)
                rc = timed_launch(1, dm.n_thread, s, [&] {
                    return launch_support_thread(x, w.sc.thread_tasks, &w.ctl->n_thread, dm.n_thread, w.ctl, s);
                });
        }
    }
    if (rc != KTRUSS_OK) return rc;
    rc = timer_end(tp, s);
    if (rc != KTRUSS_OK) return rc;
    if (unsigned long long* acc = profile_work()) {
        const bool hub = uses_csc(sched) && dm.items > 0;
        HIP_TRY(launch_pass_work(x, &w.ctl->m_buf[p], dm.m, hub ? w.sc.hub_row : nullptr, acc, s), "pass work");
    }
    return KTRUSS_OK;
}

int32_t read_ctl(const Work& w, Ctl& h, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(&h, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "control readback");
    HIP_TRY(hipStreamSynchronize(s), "control sync");
    return KTRUSS_OK;
}

// What one fixpoint run needs besides the workspace.
struct RunSpec {
    int32_t n, m;
    const int32_t* rowptr;
    const int32_t* col;
    int sched;
    ktruss_tuning tuning;
    int32_t thr;             // K - 2 (single graph)
    int32_t G;               // graphs (batched form), 0 otherwise
    const int32_t* K;        // device int32[G] (batched form)
    int32_t* rounds_dev;     // device int32[G] (batched form)
    const float* mlp;        // cost-model parameters (LEARNED schedule)
    int incremental;         // 0 recompute, 1 peel after every prune, 2 peel unless the prune removed too much
    // cost sampling (ktruss_collect_row_costs)
    bool collect;
    int32_t capacity;
    float* out_x;
    float* out_y;
};

RunSpec make_spec(int32_t n, int32_t m, const int32_t* rowptr, const int32_t* col, int sched, const ktruss_tuning& t,
                  const float* mlp) {
    RunSpec r{};
    r.n = n;
    r.m = m;
    r.rowptr = rowptr;
    r.col = col;
    r.sched = sched;
    r.tuning = t;
    r.mlp = mlp;
    r.incremental = t.incremental;
    return r;
}

// In-edge lists: for the hub and binned schedules, and for the incremental
// peel (the full neighbourhoods of a removed edge's ends).
bool csc_needed(const RunSpec& r) { return uses_csc(r.sched) || r.incremental != 0; }

// Incremental mode 2's frontier bound (0 in mode 1: every prune peels).
float peel_ratio_of(const RunSpec& r) {
    return r.incremental == 2 ? (r.tuning.peel_ratio > 0.f ? r.tuning.peel_ratio : kDefaultPeelRatio) : 0.f;
}

bool needs_features(const RunSpec& r) { return r.collect || (r.sched == KTRUSS_SCHED_LEARNED && r.mlp); }

int32_t prepare(const RunSpec& r, Work& w, int p, int32_t m_hint, hipStream_t s) {
    if (!uses_csc(r.sched)) return KTRUSS_OK;
    HIP_TRY(launch_prepare_pass(w.b[p], w.c[p], r.n, r.sched, r.tuning, r.sched == KTRUSS_SCHED_LEARNED ? r.mlp : nullptr,
                                r.m, r.collect, w.sc, w.ctl, p, m_hint, s),
            "prepare pass");
    return KTRUSS_OK;
}

// Work before the first round: buffer 0 := the input, in-edge lists, the
// per-run row statistics of the cost model, the first preparation.
int32_t set_up_run(const RunSpec& r, Work& w, hipStream_t s) {
    HIP_TRY(launch_init_run(w.b[0], r.rowptr, r.col, r.n, r.m, s), "init");
    if (csc_needed(r)) HIP_TRY(launch_build_csc(w.b[0], w.c[0], r.n, r.m, w.sc, s), "in-edge lists");
    if (needs_features(r)) {
        HIP_TRY(launch_in_outdeg_sum(w.b[0], w.c[0], r.n, r.m, w.sc, s), "row statistics");
        hipError_t e = hipMemsetAsync(w.sc.cycles, 0, sizeof(unsigned long long) * ((size_t)r.n + 1), s);
        if (e != hipSuccess) return fail_hip(e, "zero cycles");
    }
    return KTRUSS_OK;
}

// Enqueues one round of the recompute loop (Algorithm 1) reading buffer p:
// support pass, per-graph status (batched form), prune + compaction into
// buffer 1-p, preparation of the next pass.  No host interaction: every kernel
// reads its counts from the control block and does nothing once the fixpoint
// is reached.
int32_t enqueue_round(const RunSpec& r, Work& w, int p, const PassDims& dm, hipStream_t s) {
    int32_t rc = support_pass(r.sched, r.n, w, p, dm, s, r.collect ? w.sc.cycles : nullptr);
    if (rc != KTRUSS_OK) return rc;
    if (r.collect) HIP_TRY(launch_append_costs(w.sc, r.n, r.capacity, r.out_x, r.out_y, w.ctl, s), "cost samples");
    if (r.G > 0) HIP_TRY(launch_batch_status(w.b[p], w.batch, r.G, r.K, r.rounds_dev, w.ctl, s), "batch status");
    const bool csc = csc_needed(r);
    HIP_TRY(launch_compact(w.b[p], w.b[1 - p], csc ? &w.c[p] : nullptr, csc ? &w.c[1 - p] : nullptr, r.n, 0, r.thr,
                           nullptr, w.batch, w.sc, w.ctl, p, dm.m, r.m, s),
            "prune launch");
    return prepare(r, w, 1 - p, dm.m, s);
}

// Host-checked rounds of the recompute loop from buffer p (prepared for a
// support pass, h holding its dimensions) until the fixpoint.
int32_t host_rounds(const RunSpec& r, Work& w, int p, int32_t m_hint, Ctl& h, hipStream_t s) {
    for (;;) {
        const PassDims dm{m_hint, h.n_items, h.n_wave, h.n_thread};
        int32_t rc = enqueue_round(r, w, p, dm, s);
        if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK) return rc;
        if (h.done) return KTRUSS_OK;
        m_hint = h.m_buf[1 - p];
        p ^= 1;
    }
}

// Per-thread private stream for graph capture (default priority).
hipStream_t capture_stream(hipError_t& e) {
    thread_local hipStream_t cs = nullptr;
    e = hipSuccess;
    if (!cs) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    return cs;
}

// In-place rounds: incremental maintenance (not while sampling costs).
bool in_place(const RunSpec& r) { return r.incremental != 0 && !r.collect; }

// In-place rounds replayed from a hipGraph, two per replay, ceil(rps / 2)
// replays between host checks; every round peels (mode 1), so the buffer
// never changes.
int32_t state_rounds_graph(const RunSpec& r, Work& w, int p, int32_t m_hint, Ctl& h, hipStream_t s) {
    hipError_t e;
    hipStream_t cs = capture_stream(e);
    if (e != hipSuccess) return fail_hip(e, "capture stream");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    t_capturing = true;
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = launch_state_round(w.b[p], w.c[p], r.thr, w.batch, r.G, w.sc.thread_tasks, w.sc, w.ctl, p, 0.f, m_hint,
                               cs);
    t_capturing = false;
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail_hip(e, "in-place round capture");
    }
    if (ec != hipSuccess) return fail_hip(ec, "end capture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail_hip(e, "graph instantiate");
    }
    const int replays = (r.tuning.rounds_per_sync + 1) / 2;
    int32_t rc = KTRUSS_OK;
    for (;;) {
        for (int i = 0; i < replays && rc == KTRUSS_OK; ++i) {
            e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) rc = fail_hip(e, "graph launch");
        }
        if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK || h.done) break;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return rc;
}

// In-place rounds from buffer p, whose alive edges hold current supports,
// until the fixpoint (Ctl::final_buf, Ctl::kept: the buffer and its alive
// count).  Each round marks the removed edges in S, counts and peels them
// without moving anything, so the in-edge lists keep their positions.  A
// round whose frontier exceeds ratio x the survivors (mode 2) compacts the
// survivors into the other buffer instead and recomputes their supports
// there.
int32_t state_rounds(const RunSpec& r, Work& w, int p, int32_t m_hint, Ctl& h, hipStream_t s) {
    if (r.tuning.rounds_per_sync >= 2) return state_rounds_graph(r, w, p, m_hint, h, s);
    const float ratio = peel_ratio_of(r);
    for (;;) {
        HIP_TRY(launch_state_round(w.b[p], w.c[p], r.thr, w.batch, r.G, w.sc.thread_tasks, w.sc, w.ctl, p, ratio,
                                   m_hint, s),
                "in-place round");
        int32_t rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK || h.done) return rc;
        if (!h.need_support) {
            // once removed edges fill more than half the buffer, the survivors
            // move (with their supports) to the other buffer, so that marking
            // and peeling stop walking them
            if ((int64_t)2 * h.kept < (int64_t)h.m_buf[p]) {
                HIP_TRY(launch_compact(w.b[p], w.b[1 - p], &w.c[p], &w.c[1 - p], r.n, 3, r.thr, nullptr, w.batch, w.sc,
                                       w.ctl, p, m_hint, r.m, s),
                        "survivor compaction");
                p ^= 1;
                rc = read_ctl(w, h, s);
                if (rc != KTRUSS_OK) return rc;
                m_hint = h.m_buf[p];
            }
            continue;
        }
        HIP_TRY(launch_compact(w.b[p], w.b[1 - p], &w.c[p], &w.c[1 - p], r.n, 2, r.thr, nullptr, w.batch, w.sc, w.ctl,
                               p, m_hint, r.m, s),
                "survivor compaction");
        p ^= 1;
        rc = prepare(r, w, p, m_hint, s);
        if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK) return rc;
        m_hint = h.m_buf[p];
        rc = support_pass(r.sched, r.n, w, p, PassDims{m_hint, h.n_items, h.n_wave, h.n_thread}, s);
        if (rc != KTRUSS_OK) return rc;
    }
}

// Runs rounds from buffer 0 until the fixpoint.  The work before the first
// round (set-up, in-edge lists, first preparation) is already enqueued on s.
int32_t run_rounds(const RunSpec& r, Work& w, hipStream_t s, Ctl& h) {
    int32_t rc;
    h = Ctl{};
    if (uses_csc(r.sched)) {
        rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK) return rc;
    } else {
        h.m_buf[0] = r.m;
    }
    if (in_place(r)) {  // the first support pass, then in-place rounds
        rc = support_pass(r.sched, r.n, w, 0, PassDims{r.m, h.n_items, h.n_wave, h.n_thread}, s);
        return rc == KTRUSS_OK ? state_rounds(r, w, 0, r.m, h, s) : rc;
    }
    const int rps = r.tuning.rounds_per_sync;
    if (rps <= 1) return host_rounds(r, w, 0, r.m, h, s);
    const int p = 0;
    const int32_t m_hint = r.m;
    // hipGraph mode: two rounds (p -> 1-p -> p) captured once with upper-bound
    // grids, replayed ceil(rps / 2) times between host checks.
    hipError_t e;
    hipStream_t cs = capture_stream(e);
    if (e != hipSuccess) return fail_hip(e, "capture stream");
    const PassDims dm{m_hint, kHubMaxGrid, m_hint, m_hint};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    t_capturing = true;
    rc = enqueue_round(r, w, p, dm, cs);
    if (rc == KTRUSS_OK) rc = enqueue_round(r, w, 1 - p, dm, cs);
    t_capturing = false;
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != KTRUSS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return fail_hip(ec, "end capture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail_hip(e, "graph instantiate");
    }
    const int replays = (rps + 1) / 2;
    rc = KTRUSS_OK;
    for (;;) {
        for (int i = 0; i < replays && rc == KTRUSS_OK; ++i) {
            e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) rc = fail_hip(e, "graph launch");
        }
        if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK || h.done) break;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return rc;
}

}  // namespace
}  // namespace kt

using namespace kt;

extern "C" {

const char* ktruss_strerror(int32_t code) {
    switch (code) {
        case KTRUSS_OK: return "ok";
        case KTRUSS_E_INVALID: return "invalid argument";
        case KTRUSS_E_OVERFLOW: return "size overflows int32";
        case KTRUSS_E_CAPACITY: return "buffer too small";
        case KTRUSS_E_HIP: return "HIP runtime error";
        case KTRUSS_E_NOMEM: return "host out of memory";
        default: return "unknown status";
    }
}

const char* ktruss_last_error_message(void) { return t_msg; }
int32_t ktruss_last_hip_error(void) { return t_hip; }
int32_t ktruss_version(void) { return 300; }

int64_t ktruss_workspace_bytes(int32_t n, int64_t m, int32_t flags) {
    clear_error();
    if (flags != 0) return fail(KTRUSS_E_INVALID, "flags must be 0");
    const int32_t rc = check_sizes(n, m);
    if (rc != KTRUSS_OK) return rc;
    return (int64_t)full_layout(n, m, 0).L.total;
}

int64_t ktruss_batch_workspace_bytes(int32_t G, int64_t n_total, int64_t m_total, int32_t flags) {
    clear_error();
    if (flags != 0) return fail(KTRUSS_E_INVALID, "flags must be 0");
    if (G < 0 || n_total < 0) return fail(KTRUSS_E_INVALID, "G and n_total must be >= 0");
    if (n_total > INT32_MAX - 1) return fail(KTRUSS_E_OVERFLOW, "n_total above INT32_MAX - 1");
    const int32_t rc = check_sizes((int32_t)n_total, m_total);
    if (rc != KTRUSS_OK) return rc;
    return (int64_t)full_layout((int32_t)n_total, m_total, G).L.total;
}

int32_t ktruss_profile_enable(int32_t on) {
    clear_error();
    Profile& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& r : P.recs) {
        (void)hipEventSynchronize(r.e1);  // only recycles the pair; timings are dropped
        P.pool.push_back(r.e0);
        P.pool.push_back(r.e1);
    }
    P.recs.clear();
    P.on = on != 0;
    for (int k = 0; k < kKinds; ++k) {
        P.launches[k] = P.tasks[k] = P.bytes[k] = 0;
        P.ms[k] = 0.0;
    }
    if (P.on) {
        void* acc = nullptr;
        hipError_t e = hipGetSymbolAddress(&acc, HIP_SYMBOL(g_prof_stats));
        if (e == hipSuccess) e = hipMemset(acc, 0, sizeof(unsigned long long) * kPassStats);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            P.on = false;
            P.work_dev = nullptr;
            return fail_hip(e, "profile accumulator");
        }
        P.work_dev = (unsigned long long*)acc;
    }
    return KTRUSS_OK;
}

int32_t ktruss_profile_read(int32_t kind, int64_t* launches, double* total_ms, int64_t* tasks, int64_t* bytes) {
    clear_error();
    if (kind < 0 || kind >= kKinds) return fail(KTRUSS_E_INVALID, "profile kind must be 0..%d", kKinds - 1);
    Profile& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& r : P.recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.e0, r.e1);
        if (e != hipSuccess) return fail_hip(e, "profile event read");
        P.ms[r.kind] += ms;
        P.pool.push_back(r.e0);
        P.pool.push_back(r.e1);
    }
    P.recs.clear();
    if (launches) *launches = P.launches[kind];
    if (total_ms) *total_ms = P.ms[kind];
    if (tasks) *tasks = P.tasks[kind];
    if (bytes) {
        *bytes = 0;
        if (kind == 0 && P.work_dev) {
            // merge-model algorithmic bytes of the profiled passes:
            // 4 (3 m + sum of tail and row-kappa lengths) reads + 8 (2 T + m) atomic read-writes
            unsigned long long h[kPassStats] = {};
            hipError_t e = hipMemcpy(h, P.work_dev, sizeof(h), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail_hip(e, "profile accumulator read");
            const int64_t m = (int64_t)h[kStatEdges], T = (int64_t)(h[kStatSupport] / 3);
            *bytes = 4 * (3 * m + (int64_t)(h[kStatTail] + h[kStatRowK])) + 8 * (2 * T + m);
        }
    }
    return KTRUSS_OK;
}

int32_t ktruss_profile_stats(int64_t* out, int32_t len) {
    clear_error();
    if (!out || len < 0) return fail(KTRUSS_E_INVALID, "out is null or len < 0");
    Profile& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    unsigned long long h[kPassStats] = {};
    if (P.work_dev) {
        hipError_t e = hipMemcpy(h, P.work_dev, sizeof(h), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail_hip(e, "profile accumulator read");
    }
    for (int32_t i = 0; i < len && i < kPassStats; ++i) out[i] = (int64_t)h[i];
    return KTRUSS_OK;
}

int32_t ktruss_set_schedule(ktruss_graph* g, int32_t mode, const float* mlp_params, const ktruss_tuning* t) {
    clear_error();
    if (!g) return fail(KTRUSS_E_INVALID, "graph is null");
    const int32_t rc = check_schedule(mode);
    if (rc != KTRUSS_OK) return rc;
    g->schedule = mode;
    g->mlp_params = mlp_params;
    if (t) g->tuning = *t;
    return KTRUSS_OK;
}

int32_t ktruss_validate(const ktruss_graph* g, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    Work w = carve(g->work, g->n, g->m, 0);
    return validate_on_device(g->rowptr, g->col, g->n, (int32_t)g->m, w, w.b[0].src, (hipStream_t)stream);
}

int32_t ktruss_support(const ktruss_graph* g, const uint8_t* alive, int32_t* support, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    if (g->m > 0 && !support) return fail(KTRUSS_E_INVALID, "support is null");
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(g->work, g->n, g->m, 0);
    const int32_t n = g->n, m = (int32_t)g->m;
    unsigned long long merge_work = 0;
    rc = validate_on_device(g->rowptr, g->col, n, m, w, w.b[0].src, s, gated(g) ? &merge_work : nullptr);
    if (rc != KTRUSS_OK) return rc;
    if (m == 0) return KTRUSS_OK;
    const RunSpec r = make_spec(n, m, g->rowptr, g->col, schedule_for(g, merge_work), g->tuning, g->mlp_params);
    const bool csc = uses_csc(r.sched);
    rc = set_up_run(r, w, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(hipMemsetAsync(support, 0, sizeof(int32_t) * (size_t)m, s), "zero support");
    int p = 0;
    if (alive) {
        HIP_TRY(launch_compact(w.b[0], w.b[1], csc ? &w.c[0] : nullptr, csc ? &w.c[1] : nullptr, n, 1, 0, alive,
                               w.batch, w.sc, w.ctl, 0, m, m, s),
                "restrict to alive");
        p = 1;
        HIP_TRY(launch_set_final(w.ctl, 1, s), "final buffer");
    }
    rc = prepare(r, w, p, m, s);
    Ctl h{};
    if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
    if (rc != KTRUSS_OK) return rc;
    const PassDims dm{h.m_buf[p], h.n_items, h.n_wave, h.n_thread};
    rc = support_pass(r.sched, n, w, p, dm, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(launch_scatter_out(w.b[0], w.b[1], w.ctl, nullptr, support, m, s), "scatter");
    HIP_TRY(hipStreamSynchronize(s), "support sync");
    return KTRUSS_OK;
}

int32_t ktruss_prune(const ktruss_graph* g, int32_t K, const int32_t* support, uint8_t* alive, int64_t* removed,
                     void* stream) {
    clear_error();
    int32_t rc = check_graph(g, false);
    if (rc != KTRUSS_OK) return rc;
    if (K < 2) return fail(KTRUSS_E_INVALID, "K must be >= 2 (got %d)", K);
    if (g->m > 0 && (!support || !alive)) return fail(KTRUSS_E_INVALID, "support/alive is null");
    HIP_TRY(launch_prune_canonical(support, alive, (int32_t)g->m, K - 2, (unsigned long long*)removed,
                                   (hipStream_t)stream),
            "prune launch");
    return KTRUSS_OK;
}

int32_t ktruss_run(const ktruss_graph* g, int32_t K, uint8_t* mask, int32_t* support, int32_t* rounds, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    if (K < 2) return fail(KTRUSS_E_INVALID, "K must be >= 2 (got %d)", K);
    if (g->m > 0 && (!mask || !support)) return fail(KTRUSS_E_INVALID, "mask/support is null");
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(g->work, g->n, g->m, 0);
    const int32_t n = g->n, m = (int32_t)g->m;
    unsigned long long merge_work = 0;
    rc = validate_on_device(g->rowptr, g->col, n, m, w, w.b[0].src, s, gated(g) ? &merge_work : nullptr);
    if (rc != KTRUSS_OK) return rc;
    if (m == 0) {
        if (rounds) *rounds = 1;
        return KTRUSS_OK;
    }
    RunSpec r = make_spec(n, m, g->rowptr, g->col, schedule_for(g, merge_work), g->tuning, g->mlp_params);
    r.thr = K - 2;
    rc = set_up_run(r, w, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(hipMemsetAsync(mask, 0, (size_t)m, s), "zero mask");
    HIP_TRY(hipMemsetAsync(support, 0, sizeof(int32_t) * (size_t)m, s), "zero support");
    rc = prepare(r, w, 0, m, s);
    if (rc != KTRUSS_OK) return rc;
    Ctl h{};
    rc = run_rounds(r, w, s, h);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(launch_scatter_out(w.b[0], w.b[1], w.ctl, mask, support, m, s), "scatter");
    HIP_TRY(hipStreamSynchronize(s), "run sync");
    if (rounds) *rounds = h.rounds;
    return KTRUSS_OK;
}

int32_t ktruss_run_noalloc(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* col, int32_t schedule,
                           int32_t K, uint8_t* mask, int32_t* support, int32_t* rounds, void* stream) {
    clear_error();
    int32_t rc = check_sizes(n, m);
    if (rc != KTRUSS_OK) return rc;
    rc = check_schedule(schedule);
    if (rc != KTRUSS_OK) return rc;
    if (schedule == KTRUSS_SCHED_LEARNED) return fail(KTRUSS_E_INVALID, "the learned schedule needs its weights");
    const int64_t need = (int64_t)full_layout(n, m, 0).L.total;
    if (need > (int64_t)kNoAllocScratchBytes)
        return fail(KTRUSS_E_CAPACITY, "graph needs %lld workspace bytes, the fixed scratch holds %lld",
                    (long long)need, (long long)kNoAllocScratchBytes);
    void* work = nullptr;
    rc = noalloc_scratch(&work);
    if (rc != KTRUSS_OK) return rc;
    ktruss_graph g{};
    g.n = n;
    g.m = m;
    g.schedule = schedule;
    g.rowptr = rowptr;
    g.col = col;
    g.work = work;
    g.work_bytes = (int64_t)kNoAllocScratchBytes;
    // host-checked rounds (rounds_per_sync = 0): no graph to instantiate
    return ktruss_run(&g, K, mask, support, rounds, stream);
}

int32_t ktruss_decompose(const ktruss_graph* g, int32_t* trussness, int32_t* k_max, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    if (!k_max) return fail(KTRUSS_E_INVALID, "k_max is null");
    if (g->m > 0 && !trussness) return fail(KTRUSS_E_INVALID, "trussness is null");
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(g->work, g->n, g->m, 0);
    const int32_t n = g->n, m = (int32_t)g->m;
    unsigned long long merge_work = 0;
    rc = validate_on_device(g->rowptr, g->col, n, m, w, w.b[0].src, s, gated(g) ? &merge_work : nullptr);
    if (rc != KTRUSS_OK) return rc;
    *k_max = 0;
    if (m == 0) return KTRUSS_OK;
    RunSpec r = make_spec(n, m, g->rowptr, g->col, schedule_for(g, merge_work), g->tuning, g->mlp_params);
    r.tuning.rounds_per_sync = 0;  // host-checked rounds: each level ends on the host
    r.thr = 1;                     // K = 3
    rc = set_up_run(r, w, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(launch_fill_value(trussness, m, 2, s), "trussness fill");
    rc = prepare(r, w, 0, m, s);
    Ctl h{};
    if (rc == KTRUSS_OK) rc = run_rounds(r, w, s, h);
    if (rc != KTRUSS_OK) return rc;
    const bool inplace = in_place(r);
    for (int32_t K = 3;; ++K) {
        const int f = h.final_buf;
        const int32_t mf = h.m_buf[f];
        if ((inplace ? h.kept : mf) == 0) {
            *k_max = K - 1;
            break;
        }
        HIP_TRY(launch_mark_level(w.b[f], w.ctl, f, mf, K, trussness, s), "level marks");
        // level K + 1 from the survivors of level K: prune with the new
        // threshold (their supports are exact), then rounds until the fixpoint
        r.thr = K - 1;
        HIP_TRY(launch_ctl_restart(w.ctl, s), "level restart");
        if (inplace) {
            rc = state_rounds(r, w, f, mf, h, s);
            if (rc != KTRUSS_OK) return rc;
            continue;
        }
        const bool csc = csc_needed(r);
        HIP_TRY(launch_compact(w.b[f], w.b[1 - f], csc ? &w.c[f] : nullptr, csc ? &w.c[1 - f] : nullptr, r.n, 0, r.thr,
                               nullptr, w.batch, w.sc, w.ctl, f, mf, r.m, s),
                "level prune");
        rc = prepare(r, w, 1 - f, mf, s);
        if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK) return rc;
        // something was removed: recompute rounds from buffer 1-f until the fixpoint
        if (!h.done) rc = host_rounds(r, w, 1 - f, h.m_buf[1 - f], h, s);
        if (rc != KTRUSS_OK) return rc;
    }
    HIP_TRY(hipStreamSynchronize(s), "decompose sync");
    return KTRUSS_OK;
}

int32_t ktruss_run_batched(const ktruss_batch* b, const int32_t* K, uint8_t* mask, int32_t* support,
                           int32_t* rounds, void* stream) {
    clear_error();
    if (!b) return fail(KTRUSS_E_INVALID, "batch is null");
    if (b->G < 0 || b->n_total < 0 || b->m_total < 0) return fail(KTRUSS_E_INVALID, "negative batch sizes");
    if (b->n_total > INT32_MAX - 1) return fail(KTRUSS_E_OVERFLOW, "n_total above INT32_MAX - 1");
    int32_t rc = check_sizes((int32_t)b->n_total, b->m_total);
    if (rc != KTRUSS_OK) return rc;
    rc = check_schedule(b->schedule);
    if (rc != KTRUSS_OK) return rc;
    if (b->tuning.incremental < 0 || b->tuning.incremental > 2 || !(b->tuning.peel_ratio >= 0.f))
        return fail(KTRUSS_E_INVALID, "tuning.incremental must be 0, 1 or 2 and peel_ratio >= 0");
    if (!b->vert_off || !b->rowptr || (b->m_total > 0 && !b->col)) return fail(KTRUSS_E_INVALID, "batch arrays are null");
    if (b->G > 0 && (!K || !rounds)) return fail(KTRUSS_E_INVALID, "K/rounds is null");
    if (b->G == 0 && b->n_total > 0) return fail(KTRUSS_E_INVALID, "vertices but no graphs");
    if (b->m_total > 0 && (!mask || !support)) return fail(KTRUSS_E_INVALID, "mask/support is null");
    const int32_t n = (int32_t)b->n_total, m = (int32_t)b->m_total, G = b->G;
    rc = check_work(b->work, b->work_bytes, (int64_t)full_layout(n, m, G).L.total);
    if (rc != KTRUSS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(b->work, n, m, G);
    w.batch.vert_off = b->vert_off;
    w.batch.mask = mask;
    w.batch.support = support;
    w.batch.rounds = rounds;
    rc = validate_on_device(b->rowptr, b->col, n, m, w, w.b[0].src, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(launch_batch_setup(w.batch, G, n, K, w.b[0].src, b->col, m, w.ctl, s), "batch set-up");
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &w.ctl->err, sizeof(err), hipMemcpyDeviceToHost, s), "batch check readback");
    HIP_TRY(hipStreamSynchronize(s), "batch check sync");
    if (err)
        return fail(KTRUSS_E_INVALID,
                    "malformed batch (check bits 0x%x: 32 vertex offsets or K < 2, 64 edge between graphs)", err);
    HIP_TRY(launch_batch_reset(w.batch, G, rounds, s), "batch reset");
    if (m == 0) {
        // every graph is empty: one pass that removes nothing
        HIP_TRY(launch_init_run(w.b[0], b->rowptr, b->col, n, m, s), "init");
        HIP_TRY(launch_batch_status(w.b[0], w.batch, G, K, rounds, w.ctl, s), "batch status");
        HIP_TRY(hipStreamSynchronize(s), "batch sync");
        return KTRUSS_OK;
    }
    RunSpec r = make_spec(n, m, b->rowptr, b->col, b->schedule, b->tuning, nullptr);
    r.G = G;
    r.K = K;
    r.rounds_dev = rounds;
    rc = set_up_run(r, w, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(hipMemsetAsync(mask, 0, (size_t)m, s), "zero mask");
    HIP_TRY(hipMemsetAsync(support, 0, sizeof(int32_t) * (size_t)m, s), "zero support");
    rc = prepare(r, w, 0, m, s);
    if (rc != KTRUSS_OK) return rc;
    Ctl h{};
    rc = run_rounds(r, w, s, h);
    if (rc != KTRUSS_OK) return rc;
    // in-place rounds leave every graph's truss in the final buffer (the
    // compacting rounds wrote each graph out when it finished)
    if (in_place(r)) HIP_TRY(launch_scatter_out(w.b[0], w.b[1], w.ctl, mask, support, m, s), "scatter");
    HIP_TRY(hipStreamSynchronize(s), "batch sync");
    return KTRUSS_OK;
}

// ---------------------------------------------------------------- cost model

int32_t ktruss_collect_row_costs(const ktruss_graph* g, int32_t K, int32_t variant, float* features, float* costs,
                                 int32_t capacity, int32_t* count, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    if (K < 2) return fail(KTRUSS_E_INVALID, "K must be >= 2 (got %d)", K);
    if (variant != 0 && variant != 1) return fail(KTRUSS_E_INVALID, "variant must be 0 (hub) or 1 (wavefront)");
    if (capacity < 0 || (capacity > 0 && (!features || !costs)) || !count)
        return fail(KTRUSS_E_INVALID, "sample buffers are null or capacity < 0");
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(g->work, g->n, g->m, 0);
    const int32_t n = g->n, m = (int32_t)g->m;
    rc = validate_on_device(g->rowptr, g->col, n, m, w, w.b[0].src, s);
    if (rc != KTRUSS_OK) return rc;
    *count = 0;
    if (m == 0) return KTRUSS_OK;
    ktruss_tuning t = g->tuning;
    t.rounds_per_sync = 0;
    t.incremental = 0;  // every pass is a timed support pass
    RunSpec r = make_spec(n, m, g->rowptr, g->col, variant == 0 ? KTRUSS_SCHED_FORCE_HUB : kSchedSampleWave, t, nullptr);
    r.thr = K - 2;
    r.collect = true;
    r.capacity = capacity;
    r.out_x = features;
    r.out_y = costs;
    rc = set_up_run(r, w, s);
    if (rc == KTRUSS_OK) rc = prepare(r, w, 0, m, s);
    if (rc != KTRUSS_OK) return rc;
    Ctl h{};
    rc = run_rounds(r, w, s, h);
    if (rc != KTRUSS_OK) return rc;
    *count = h.n_samples;
    return KTRUSS_OK;
}

int64_t ktruss_mlp_workspace_bytes(int32_t rows) {
    clear_error();
    if (rows < 0) return fail(KTRUSS_E_INVALID, "rows must be >= 0");
    const int64_t nblk = mlp_grad_blocks(rows);
    return (nblk * KTRUSS_MLP_PARAMS + nblk) * (int64_t)sizeof(float);
}

int32_t ktruss_mlp_forward(const float* params, const float* x, int32_t rows, float* y, void* stream) {
    clear_error();
    if (rows < 0) return fail(KTRUSS_E_INVALID, "rows must be >= 0");
    if (rows > 0 && (!params || !x || !y)) return fail(KTRUSS_E_INVALID, "null pointer");
    HIP_TRY(launch_mlp_forward(params, x, rows, y, (hipStream_t)stream), "mlp forward");
    return KTRUSS_OK;
}

int32_t ktruss_mlp_loss_grad(const float* params, const float* x, const float* target, int32_t rows, float* loss,
                             float* grad, void* work, int64_t work_bytes, void* stream) {
    clear_error();
    if (rows <= 0) return fail(KTRUSS_E_INVALID, "rows must be > 0");
    if (!params || !x || !target || !grad) return fail(KTRUSS_E_INVALID, "null pointer");
    const int64_t need = ktruss_mlp_workspace_bytes(rows);
    const int32_t rc = check_work(work, work_bytes, need);
    if (rc != KTRUSS_OK) return rc;
    const int64_t nblk = mlp_grad_blocks(rows);
    float* partial = (float*)work;
    float* loss_part = partial + nblk * KTRUSS_MLP_PARAMS;
    HIP_TRY(launch_mlp_loss_grad(params, x, target, rows, partial, loss_part, grad, loss, (hipStream_t)stream),
            "mlp gradient");
    return KTRUSS_OK;
}

int32_t ktruss_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream) {
    clear_error();
    if (!params || !grad || !m || !v) return fail(KTRUSS_E_INVALID, "null pointer");
    if (step < 1) return fail(KTRUSS_E_INVALID, "step counts from 1");
    HIP_TRY(launch_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream), "adam");
    return KTRUSS_OK;
}

}  // extern "C"
