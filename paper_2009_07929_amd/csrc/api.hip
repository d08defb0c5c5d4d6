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

Layout layout(int32_t n, int64_t m) {
    Layout L{};
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
        L.col[b] = take(em);
        L.src[b] = take(em);
        L.eid[b] = take(em);
        L.S[b] = take(em);
        L.rowptr[b] = take(vn);
        L.cedge[b] = take(em);
        L.cptr[b] = take(vn);
    }
    L.xscan = take(em1);
    L.cxscan = take(em1);
    L.blockcnt = take(sizeof(int32_t) * kMaxScanBlocks);
    L.blockoff = take(sizeof(int32_t) * kMaxScanBlocks);
    L.blockcnt2 = take(sizeof(int32_t) * 2 * kMaxScanBlocks);
    L.blockoff2 = take(sizeof(int32_t) * 2 * kMaxScanBlocks);
    L.tmp_n = take(vn);
    L.itemoff = take(vn);
    L.item_kappa = take(sizeof(int32_t) * (size_t)item_capacity(n, m));
    L.item_c0 = take(sizeof(int32_t) * (size_t)item_capacity(n, m));
    L.is_hub = take((size_t)n + 1);
    L.wave_tasks = take(em);
    L.thread_tasks = take(em);
    L.ctl = take(sizeof(Ctl));
    L.total = off;
    return L;
}

namespace {

struct Work {
    Buf b[2];
    Csc c[2];
    Scratch sc;
    Ctl* ctl;
};

Work carve(const ktruss_graph* g) {
    const Layout L = layout(g->n, g->m);
    char* base = (char*)g->work;
    Work w{};
    for (int b = 0; b < 2; ++b) {
        w.b[b].col = (int32_t*)(base + L.col[b]);
        w.b[b].src = (int32_t*)(base + L.src[b]);
        w.b[b].eid = (int32_t*)(base + L.eid[b]);
        w.b[b].S = (int32_t*)(base + L.S[b]);
        w.b[b].rowptr = (int32_t*)(base + L.rowptr[b]);
        w.c[b].edge = (int32_t*)(base + L.cedge[b]);
        w.c[b].ptr = (int32_t*)(base + L.cptr[b]);
    }
    w.sc.xscan = (int32_t*)(base + L.xscan);
    w.sc.cxscan = (int32_t*)(base + L.cxscan);
    w.sc.blockcnt = (int32_t*)(base + L.blockcnt);
    w.sc.blockoff = (int32_t*)(base + L.blockoff);
    w.sc.blockcnt2 = (int32_t*)(base + L.blockcnt2);
    w.sc.blockoff2 = (int32_t*)(base + L.blockoff2);
    w.sc.tmp_n = (int32_t*)(base + L.tmp_n);
    w.sc.itemoff = (int32_t*)(base + L.itemoff);
    w.sc.item_kappa = (int32_t*)(base + L.item_kappa);
    w.sc.item_c0 = (int32_t*)(base + L.item_c0);
    w.sc.is_hub = (uint8_t*)(base + L.is_hub);
    w.sc.wave_tasks = (int32_t*)(base + L.wave_tasks);
    w.sc.thread_tasks = (int32_t*)(base + L.thread_tasks);
    w.ctl = (Ctl*)(base + L.ctl);
    return w;
}

int32_t check_sizes(int32_t n, int64_t m) {
    if (n < 0 || m < 0) return fail(KTRUSS_E_INVALID, "n (%d) and m (%lld) must be >= 0", n, (long long)m);
    if (n > INT32_MAX - 1 || m > INT32_MAX - 1) return fail(KTRUSS_E_OVERFLOW, "n or m above INT32_MAX - 1");
    return KTRUSS_OK;
}

int32_t check_graph(const ktruss_graph* g, bool need_work) {
    if (!g) return fail(KTRUSS_E_INVALID, "graph is null");
    const int32_t rc = check_sizes(g->n, g->m);
    if (rc != KTRUSS_OK) return rc;
    if (!g->rowptr || (g->m > 0 && !g->col)) return fail(KTRUSS_E_INVALID, "graph rowptr/col is null");
    if (g->schedule < KTRUSS_SCHED_PLAIN || g->schedule > KTRUSS_SCHED_FORCE_HUB)
        return fail(KTRUSS_E_INVALID, "unknown schedule %d", g->schedule);
    if (need_work) {
        const int64_t need = (int64_t)layout(g->n, g->m).total;
        if (!g->work) return fail(KTRUSS_E_INVALID, "workspace is null");
        if (((uintptr_t)g->work & 15u) != 0) return fail(KTRUSS_E_INVALID, "workspace must be 16-byte aligned");
        if (g->work_bytes < need)
            return fail(KTRUSS_E_CAPACITY, "workspace has %lld bytes, needs %lld", (long long)g->work_bytes, (long long)need);
    }
    return KTRUSS_OK;
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

// Validates the input CSR on the device (writing each edge's row into
// src_out) and reads the verdict back.  Synchronises s.
int32_t validate_on_device(const ktruss_graph* g, const Work& w, int32_t* src_out, hipStream_t s) {
    HIP_TRY(launch_validate(g->rowptr, g->col, g->n, (int32_t)g->m, src_out, w.ctl, s), "validate launch");
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &w.ctl->err, sizeof(err), hipMemcpyDeviceToHost, s), "validate readback");
    HIP_TRY(hipStreamSynchronize(s), "validate sync");
    if (err) return fail(KTRUSS_E_INVALID, "malformed CSR (check bits 0x%x: 1 rowptr range, 2 rowptr[0], 4 rowptr[n]!=m, 8 rowptr not monotone, 16 columns not ascending above the diagonal or >= n)", err);
    return KTRUSS_OK;
}

// ---- profiling tallies (process-wide; guarded by a mutex)
// kinds: 0 whole support pass, 1 thread-per-edge, 2 wavefront-per-edge, 3 hub
constexpr int kKinds = 4;
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
};
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

// Event pair around a group of launches, tallied under `kind` when profiling.
struct Timer {
    bool on = false;
    int kind = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

int32_t timer_begin(Timer& t, int kind, int64_t tasks, int64_t bytes, hipStream_t s) {
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
    int32_t rc = timer_begin(t, kind, tasks, 16 * tasks, s);
    if (rc != KTRUSS_OK) return rc;
    HIP_TRY(launch(), "support launch");
    return timer_end(t, s);
}

bool uses_csc(int sched) { return sched != KTRUSS_SCHED_PLAIN && sched != KTRUSS_SCHED_FORCE_WAVE; }

// One support pass over buffer p.  h holds the host copy of the control
// block after the pass was prepared (task and item counts).
int32_t support_pass(const ktruss_graph* g, const Work& w, int p, int32_t m_hint, const Ctl& h, hipStream_t s) {
    const int sched = g->schedule;
    const Buf& x = w.b[p];
    Timer tp;
    int32_t rc = timer_begin(tp, 0, m_hint, 16 * (int64_t)m_hint + 4 * ((int64_t)g->n + 1), s);
    if (rc != KTRUSS_OK) return rc;
    if (sched == KTRUSS_SCHED_PLAIN) {
        rc = timed_launch(1, m_hint, s, [&] {
            return launch_support_thread(x, nullptr, &w.ctl->m_buf[p], m_hint, w.ctl, s);
        });
    } else if (sched == KTRUSS_SCHED_FORCE_WAVE) {
        rc = timed_launch(2, m_hint, s, [&] {
            return launch_support_wave(x, nullptr, &w.ctl->m_buf[p], m_hint, w.ctl, s);
        });
    } else {
        rc = timed_launch(3, h.n_items, s, [&] {
            return launch_support_hub(x, w.c[p], w.sc.item_kappa, w.sc.item_c0, h.n_items, w.ctl, s);
        });
        if (rc == KTRUSS_OK && sched != KTRUSS_SCHED_FORCE_HUB) {
            rc = timed_launch(2, h.n_wave, s, [&] {
                return launch_support_wave(x, w.sc.wave_tasks, &w.ctl->n_wave, h.n_wave, w.ctl, s);
            });
            if (rc == KTRUSS_OK)
                rc = timed_launch(1, h.n_thread, s, [&] {
                    return launch_support_thread(x, w.sc.thread_tasks, &w.ctl->n_thread, h.n_thread, w.ctl, s);
                });
        }
    }
    if (rc != KTRUSS_OK) return rc;
    return timer_end(tp, s);
}

int32_t read_ctl(const Work& w, Ctl& h, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(&h, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "control readback");
    HIP_TRY(hipStreamSynchronize(s), "control sync");
    return KTRUSS_OK;
}

int32_t prepare(const ktruss_graph* g, const Work& w, int p, int32_t m_hint, hipStream_t s) {
    if (!uses_csc(g->schedule)) return KTRUSS_OK;
    Scratch sc = w.sc;
    HIP_TRY(launch_prepare_pass(w.b[p], w.c[p], g->n, g->schedule, g->tuning, nullptr, sc, w.ctl, p, m_hint, s),
            "prepare pass");
    return KTRUSS_OK;
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
int32_t ktruss_version(void) { return 100; }

int64_t ktruss_workspace_bytes(int32_t n, int64_t m, int32_t flags) {
    clear_error();
    if (flags != 0) return fail(KTRUSS_E_INVALID, "flags must be 0");
    const int32_t rc = check_sizes(n, m);
    if (rc != KTRUSS_OK) return rc;
    return (int64_t)layout(n, m).total;
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
    if (bytes) *bytes = P.bytes[kind];
    return KTRUSS_OK;
}

int32_t ktruss_set_schedule(ktruss_graph* g, int32_t mode, const float* mlp_params, const ktruss_tuning* t) {
    clear_error();
    if (!g) return fail(KTRUSS_E_INVALID, "graph is null");
    if (mode < KTRUSS_SCHED_PLAIN || mode > KTRUSS_SCHED_FORCE_HUB) return fail(KTRUSS_E_INVALID, "unknown schedule %d", mode);
    g->schedule = mode;
    g->mlp_params = mlp_params;
    if (t) g->tuning = *t;
    return KTRUSS_OK;
}

int32_t ktruss_validate(const ktruss_graph* g, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    const Work w = carve(g);
    return validate_on_device(g, w, w.b[0].src, (hipStream_t)stream);
}

int32_t ktruss_support(const ktruss_graph* g, const uint8_t* alive, int32_t* support, void* stream) {
    clear_error();
    int32_t rc = check_graph(g, true);
    if (rc != KTRUSS_OK) return rc;
    if (g->m > 0 && !support) return fail(KTRUSS_E_INVALID, "support is null");
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(g);
    const int32_t n = g->n, m = (int32_t)g->m;
    rc = validate_on_device(g, w, w.b[0].src, s);
    if (rc != KTRUSS_OK) return rc;
    if (m == 0) return KTRUSS_OK;
    const bool csc = uses_csc(g->schedule);
    HIP_TRY(launch_init_run(w.b[0], g->rowptr, g->col, n, m, s), "init");
    if (csc) HIP_TRY(launch_build_csc(w.b[0], w.c[0], n, m, w.sc, s), "in-edge lists");
    HIP_TRY(hipMemsetAsync(support, 0, sizeof(int32_t) * (size_t)m, s), "zero support");
    int p = 0;
    Ctl h{};
    h.m_buf[0] = m;
    if (alive) {
        HIP_TRY(launch_compact(w.b[0], w.b[1], csc ? &w.c[0] : nullptr, csc ? &w.c[1] : nullptr, n, 1, 0, alive, w.sc,
                               w.ctl, 0, m, s),
                "restrict to alive");
        p = 1;
        HIP_TRY(launch_set_final(w.ctl, 1, s), "final buffer");
    }
    rc = prepare(g, w, p, m, s);
    if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
    if (rc != KTRUSS_OK) return rc;
    rc = support_pass(g, w, p, h.m_buf[p], h, s);
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
    Work w = carve(g);
    const int32_t n = g->n, m = (int32_t)g->m;
    rc = validate_on_device(g, w, w.b[0].src, s);
    if (rc != KTRUSS_OK) return rc;
    if (m == 0) {
        if (rounds) *rounds = 1;
        return KTRUSS_OK;
    }
    const bool csc = uses_csc(g->schedule);
    HIP_TRY(launch_init_run(w.b[0], g->rowptr, g->col, n, m, s), "init");
    if (csc) HIP_TRY(launch_build_csc(w.b[0], w.c[0], n, m, w.sc, s), "in-edge lists");
    HIP_TRY(hipMemsetAsync(mask, 0, (size_t)m, s), "zero mask");
    HIP_TRY(hipMemsetAsync(support, 0, sizeof(int32_t) * (size_t)m, s), "zero support");
    int p = 0;
    Ctl h{};
    h.m_buf[0] = m;
    rc = prepare(g, w, 0, m, s);
    if (rc == KTRUSS_OK && csc) rc = read_ctl(w, h, s);
    if (rc != KTRUSS_OK) return rc;
    int32_t m_hint = m;
    for (;;) {
        rc = support_pass(g, w, p, m_hint, h, s);
        if (rc != KTRUSS_OK) return rc;
        HIP_TRY(launch_compact(w.b[p], w.b[1 - p], csc ? &w.c[p] : nullptr, csc ? &w.c[1 - p] : nullptr, n, 0, K - 2,
                               nullptr, w.sc, w.ctl, p, m_hint, s),
                "prune launch");
        rc = prepare(g, w, 1 - p, m_hint, s);
        if (rc == KTRUSS_OK) rc = read_ctl(w, h, s);
        if (rc != KTRUSS_OK) return rc;
        if (h.done) break;
        m_hint = h.m_buf[1 - p];
        p ^= 1;
    }
    HIP_TRY(launch_scatter_out(w.b[0], w.b[1], w.ctl, mask, support, m, s), "scatter");
    HIP_TRY(hipStreamSynchronize(s), "run sync");
    if (rounds) *rounds = h.rounds;
    return KTRUSS_OK;
}

}  // extern "C"
