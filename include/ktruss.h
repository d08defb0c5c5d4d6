/*
 * ktruss.h — C-ABI of the MI355X (gfx950) Eager K-truss library.
 *
 * The method (Blanco, Low, Kim, "Exploration of Fine-Grained Parallelism for
 * Load Balancing Eager K-truss on GPU and CPU", HPEC 2019):
 *   - the K-truss is the largest edge set in which every edge lies in at least
 *     K-2 triangles of the set (Section I);
 *   - it is reached by repeating: compute every edge's support S (its triangle
 *     count), keep the edges with S >= K-2, drop the rest, until a pass drops
 *     nothing (Section II-A, Algorithm 1);
 *   - supports are computed eagerly on the upper-triangular adjacency: each
 *     triangle is found once, from its edge with the two smallest labels, and
 *     increments all three edge supports; one fine-grained task per non-zero
 *     (Section III-B, Algorithm 3).
 *
 * Conventions for every call:
 *   - Return value: KTRUSS_OK (0) or a negative status code below.  No C++
 *     exception crosses this boundary.  ktruss_last_error_message() returns a
 *     thread-local description of the last failure on the calling thread.
 *   - Graphs are upper-triangular CSR in 0-based int32: rowptr[n+1] with
 *     rowptr[0] = 0 and rowptr[n] = m; col[m] with, inside row u, strictly
 *     ascending columns all greater than u and less than n (exactly what
 *     ktruss_build_csr produces).  Edge e is the e-th non-zero of that CSR
 *     ("canonical position"); every per-edge output is indexed by it.
 *   - Ownership: the caller owns every buffer.  Pointers marked "device" are
 *     device memory of the current HIP device; "host" pointers are ordinary
 *     host memory.  The library allocates no device memory: each graph call
 *     works inside the caller's workspace (ktruss_workspace_bytes).
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Calls enqueue work on it; calls that return host scalars
 *     (ktruss_run's round count, ktruss_validate) synchronise that stream
 *     before returning.  Two calls that share a workspace must not overlap.
 */
#ifndef KTRUSS_H
#define KTRUSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define KTRUSS_OK           0
#define KTRUSS_E_INVALID   (-1)  /* null pointer, n < 0, K < 2, id outside [0,n), malformed CSR */
#define KTRUSS_E_OVERFLOW  (-2)  /* n or m above INT32_MAX - 1 */
#define KTRUSS_E_CAPACITY  (-3)  /* an output or workspace is too small; the needed size is reported */
#define KTRUSS_E_HIP       (-4)  /* a HIP runtime call failed; see ktruss_last_hip_error() */
#define KTRUSS_E_NOMEM     (-5)  /* host allocation failed */

/* Support-kernel schedules (ktruss_graph.schedule).  They change speed only:
 * mask, supports and round count are identical under every schedule. */
#define KTRUSS_SCHED_PLAIN      0  /* every edge task on the thread-per-edge merge kernel */
#define KTRUSS_SCHED_HEURISTIC  1  /* static degree heuristic bins rows/edges onto the kernel variants */
#define KTRUSS_SCHED_LEARNED    2  /* MLP cost model bins rows/edges (falls back to HEURISTIC without weights) */
#define KTRUSS_SCHED_FORCE_WAVE 3  /* every edge task on the wavefront-per-edge kernel (an ablation) */
#define KTRUSS_SCHED_FORCE_HUB  4  /* every row kappa with tasks on the workgroup-per-hub-row kernel: the fastest
                                      schedule on the large power-law graphs, the default of the benchmark */
#define KTRUSS_SCHED_COARSE     5  /* one thread per row running its edge tasks in turn: the coarse granularity of
                                      Section III-A's Algorithm 2 (with Algorithm 3's updates of all three
                                      edges), kept as the ablation of the fine-grained path */

/* Tuning knobs (0 = library default). */
typedef struct ktruss_tuning {
    int32_t wave_min_work;   /* heuristic/learned: non-hub edge tasks whose merge length (row tail + row kappa)
                                is at least this use wavefront-per-edge, the others thread-per-edge */
    int32_t hub_min_work;    /* heuristic: rows kappa selected by at least this many tasks are hub rows */
    int32_t hub_chunk_work;  /* unused (kept for the layout) */
    int32_t rounds_per_sync; /* <= 1: host checks the fixpoint after every round (exact grids);
                                >= 2: rounds are captured in a hipGraph and replayed this many at a time */
    float learned_hub_min;   /* learned: rows whose predicted log2 (hub cost / wavefront cost) is at most this
                                are hub rows (0: the default 0) */
    int32_t hub_chunk_tasks; /* heuristic/force-hub/learned: tasks per hub item (clamped to 16..256) */
    int32_t plain_max_work;  /* heuristic/learned: if the input's mean merge length per edge (row tail + row
                                kappa; the row-kappa lengths sampled on edges 0, 16, 32, ... and weighted
                                by 16) is at most this, ktruss_run/ktruss_support use thread-per-edge for
                                every task and build no in-edge lists; 0: default 32, negative: never */
    int32_t incremental;     /* ktruss_run / ktruss_decompose / ktruss_run_batched: 0 recompute every pass's
                                supports (Algorithm 1); 1 after the first pass, keep the survivors' supports and
                                take off each triangle a prune destroys (incremental maintenance; the prunes
                                mark edges in place, nothing is compacted); 2 as 1, except that a prune removing
                                more than peel_ratio x the edges it keeps is followed by a compaction and a
                                recomputation.  Masks, supports and pass counts are the same in every mode.
                                Rounds replayed from a hipGraph (rounds_per_sync >= 2) use mode 1 for 2.  In
                                ktruss_run_batched a graph that finishes keeps its edges in place; they destroy
                                no triangle. */
    float peel_ratio;        /* incremental = 2: the ratio above (0: the default 0.125) */
} ktruss_tuning;

/* Cost model: 5 inputs -> 64 ReLU -> 64 ReLU -> 1 output, FP32.  Parameter
 * vector layout: W1[64x5] (row j: weights into hidden unit j), b1[64],
 * W2[64x64] (row k: weights into second-layer unit k), b2[64], w3[64], b3. */
#define KTRUSS_MLP_IN 5
#define KTRUSS_MLP_HIDDEN 64
#define KTRUSS_MLP_PARAMS 4609

/* A graph resident on the device plus its workspace.  Caller-owned POD. */
typedef struct ktruss_graph {
    int32_t n;                 /* vertices */
    int32_t schedule;          /* KTRUSS_SCHED_* */
    int64_t m;                 /* edges (non-zeros of the upper triangle) */
    const int32_t* rowptr;     /* device, n+1 */
    const int32_t* col;        /* device, m */
    void* work;                /* device, >= ktruss_workspace_bytes(n, m, 0) bytes */
    int64_t work_bytes;
    const float* mlp_params;   /* device, KTRUSS_MLP_PARAMS floats, or NULL (LEARNED schedule only) */
    ktruss_tuning tuning;
} ktruss_graph;

/* ------------------------------------------------------------- diagnostics */
const char* ktruss_strerror(int32_t code);
/* Thread-local text of the last failure on this thread ("" if none). */
const char* ktruss_last_error_message(void);
/* The hipError_t of the last KTRUSS_E_HIP on this thread (0 if none). */
int32_t ktruss_last_hip_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t ktruss_version(void);

/* ------------------------------------------------------------- input prep */
/*
 * ktruss_build_csr — host only; the input preparation of Section IV-A (graphs
 * are made upper-triangular), with the relabelling this library uses.
 *   src, dst      host int32[npairs]: raw vertex pairs, read as undirected;
 *                 self-loops and repeated pairs are dropped.
 *   n             vertex count; every id must lie in [0, n).
 *   order         0 keep ids; 1 relabel by ascending degree (ties: smaller
 *                 original id first) — the default; 2 descending degree.
 *   rowptr        host int32[n+1] out.
 *   col           host int32[col_capacity] out; npairs entries always suffice.
 *   new_to_old    host int32[n] out (new label -> original id), or NULL.
 *   m_out         host int64 out: the edge count m (also set on E_CAPACITY).
 * Errors: E_INVALID (null pointer, n < 0, npairs < 0, id outside [0,n),
 * order outside 0..2), E_OVERFLOW (n or m > INT32_MAX-1), E_CAPACITY
 * (col_capacity < m), E_NOMEM.
 */
int32_t ktruss_build_csr(const int32_t* src, const int32_t* dst, int64_t npairs, int32_t n,
                         int32_t order, int32_t* rowptr, int32_t* col, int64_t col_capacity,
                         int32_t* new_to_old, int64_t* m_out);

/* ---------------------------------------------------------------- device */
/*
 * ktruss_workspace_bytes — device workspace needed by ktruss_validate,
 * ktruss_support and ktruss_run on a graph with n vertices and m edges
 * (flags must be 0).  Returns a negative status on invalid sizes.
 */
int64_t ktruss_workspace_bytes(int32_t n, int64_t m, int32_t flags);

/*
 * ktruss_validate — checks on the device that g's CSR has the canonical form
 * described above.  Synchronises `stream`.  KTRUSS_OK or E_INVALID.
 * ktruss_support and ktruss_run perform the same check first.
 */
int32_t ktruss_validate(const ktruss_graph* g, void* stream);

/*
 * ktruss_support — one evaluation of S = (A^T A) o A (Algorithm 1, first line
 * of the loop) on the alive subgraph, by eager fine-grained tasks (Algorithm 3).
 *   alive    device uint8[m]: non-zero = edge present; NULL = every edge.
 *   support  device int32[m] out: triangles of the alive subgraph containing
 *            edge e if e is alive, else 0.
 * Stateless.  Synchronises `stream` once (input validation).
 */
int32_t ktruss_support(const ktruss_graph* g, const uint8_t* alive, int32_t* support, void* stream);

/*
 * ktruss_prune — Algorithm 1's mask and update lines: alive[e] stays non-zero
 * iff it was non-zero and support[e] >= K-2.
 *   K        >= 2.
 *   support  device int32[m] in.
 *   alive    device uint8[m] in/out (output values are 0/1).
 *   removed  device int64 out (may be NULL): number of edges switched off.
 * Stateless, asynchronous; does not use the workspace.
 */
int32_t ktruss_prune(const ktruss_graph* g, int32_t K, const int32_t* support, uint8_t* alive,
                     int64_t* removed, void* stream);

/*
 * ktruss_run — the whole fixpoint of Algorithm 1: supports, prune, repeat
 * until a pass removes nothing.
 *   K        >= 2.
 *   mask     device uint8[m] out: 1 iff edge e is in the K-truss.
 *   support  device int32[m] out: e's support inside the K-truss, 0 if removed.
 *   rounds   host int32 out (may be NULL): number of support passes, counting
 *            the final pass that removes nothing.
 * Equal, bit for bit, to iterating ktruss_support / ktruss_prune to a
 * fixpoint.  Synchronises `stream`.
 */
int32_t ktruss_run(const ktruss_graph* g, int32_t K, uint8_t* mask, int32_t* support,
                   int32_t* rounds, void* stream);

/*
 * ktruss_run_noalloc — for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes exactly what ktruss_run computes for the graph
 * (n, m, rowptr, col: device, the CSR conventions above) under `schedule`
 * (any but KTRUSS_SCHED_LEARNED) with default tuning and host-checked rounds,
 * but its working memory is a fixed 64 MiB device array inside the library
 * instead of a caller workspace: one copy per GPU, created when the library
 * is loaded and held until the process ends; no allocation happens in the
 * call.  Graphs whose ktruss_workspace_bytes(n, m, 0) exceeds 64 MiB (about
 * 400k edges with 100k vertices) are rejected with KTRUSS_E_CAPACITY before
 * any device work.  mask (device uint8[m]), support (device int32[m]) and
 * rounds (host) as in ktruss_run; synchronises `stream`.  All calls on one
 * GPU share that array: two calls that overlap on the same GPU (from two
 * threads or two streams) race and must not be issued.  The array keeps the
 * last call's contents; every call re-initialises what it reads.
 */
int32_t ktruss_run_noalloc(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* col, int32_t schedule,
                           int32_t K, uint8_t* mask, int32_t* support, int32_t* rounds, void* stream);

/*
 * ktruss_decompose — the trussness of every edge (the K_max analysis of
 * Section IV, for all edges at once): the largest K whose K-truss holds the
 * edge.  Since the (K+1)-truss lies inside the K-truss, each level starts from
 * the previous level's survivors and their supports (already exact for that
 * subgraph): it prunes with the new threshold, and recomputes supports only
 * when something was removed, until the fixpoint.
 *   trussness  device int32[m] out: 2 for an edge in no triangle, else the
 *              largest K >= 3 with the edge in the K-truss.
 *   k_max      host int32 out: the largest trussness (0 for a graph with no
 *              edges): the largest K with a non-empty K-truss.
 * Equal, bit for bit, to the largest K at which ktruss_run keeps the edge.
 * Uses the graph's schedule (host-checked rounds).  Synchronises `stream`.
 */
int32_t ktruss_decompose(const ktruss_graph* g, int32_t* trussness, int32_t* k_max, void* stream);

/* ----------------------------------------------------------- batched form */
/*
 * Many independent graphs in one fixpoint loop.  The graphs are concatenated
 * into one upper-triangular CSR (their disjoint union): graph g owns vertices
 * [vert_off[g], vert_off[g+1]) and its edges are those of its rows, which must
 * not leave that range.  Since no triangle spans two graphs, the union's
 * prune-to-fixpoint (Algorithm 1), with every edge tested against its own
 * graph's K, yields every graph's K-truss.
 */
typedef struct ktruss_batch {
    int32_t G;                 /* graphs */
    int32_t schedule;          /* KTRUSS_SCHED_* */
    int64_t n_total;           /* sum of vertex counts (<= INT32_MAX - 1) */
    int64_t m_total;           /* sum of edge counts (<= INT32_MAX - 1) */
    const int32_t* vert_off;   /* device, G+1, vert_off[0] = 0, vert_off[G] = n_total, non-decreasing */
    const int32_t* rowptr;     /* device, n_total+1: the union CSR (edge offsets of graph g: rowptr[vert_off[g]]) */
    const int32_t* col;        /* device, m_total */
    void* work;                /* device, >= ktruss_batch_workspace_bytes(G, n_total, m_total, 0) bytes */
    int64_t work_bytes;
    ktruss_tuning tuning;
} ktruss_batch;

/* Workspace bytes of ktruss_run_batched (flags must be 0); negative status on invalid sizes. */
int64_t ktruss_batch_workspace_bytes(int32_t G, int64_t n_total, int64_t m_total, int32_t flags);

/*
 * ktruss_run_batched — every graph's K-truss, K per graph.
 *   K        device int32[G], each >= 2.
 *   mask     device uint8[m_total] out, support device int32[m_total] out:
 *            as ktruss_run, indexed by position in the union CSR.
 *   rounds   device int32[G] out: each graph's pass count (as ktruss_run).
 * Results equal G separate ktruss_run calls.  Errors: E_INVALID (null
 * pointers, offsets not covering [0, n_total), an edge between two graphs,
 * some K < 2, malformed CSR), E_OVERFLOW, E_CAPACITY, E_HIP.  Synchronises
 * `stream`.
 */
int32_t ktruss_run_batched(const ktruss_batch* b, const int32_t* K, uint8_t* mask, int32_t* support,
                           int32_t* rounds, void* stream);

/*
 * ktruss_set_schedule — selects the support-kernel schedule of g (sets
 * g->schedule, g->mlp_params and, if t is not NULL, g->tuning).  Results do
 * not depend on it.  E_INVALID for an unknown mode.
 */
int32_t ktruss_set_schedule(ktruss_graph* g, int32_t mode, const float* mlp_params,
                            const ktruss_tuning* t);

/* ------------------------------------------------------ butterfly counting */
/*
 * Butterflies of a bipartite graph: the paper's closing section (Section V)
 * names butterfly counting, the 4-cycle motif of bipartite graphs, as a
 * further problem for its fine-grained decomposition.  Sides U (nu vertices)
 * and V (nv vertices); edges given as CSR rows over U: rowptr[nu+1] from 0 to
 * m, columns in [0, nv) strictly ascending inside each row.  Edge e is the
 * e-th non-zero.  A butterfly is u1 - v1 - u2 - v2 with u1 != u2, v1 != v2.
 */
typedef struct ktruss_bipartite {
    int32_t nu, nv;
    int64_t m;
    const int32_t* rowptr;   /* device, nu+1 */
    const int32_t* col;      /* device, m */
    void* work;              /* device, >= ktruss_butterfly_workspace_bytes(nu, nv, m) bytes, 256-byte aligned */
    int64_t work_bytes;
} ktruss_bipartite;

/* Workspace bytes of ktruss_butterflies (negative status on bad sizes). */
int64_t ktruss_butterfly_workspace_bytes(int32_t nu, int32_t nv, int64_t m);
/*
 * count (device int64[m]): the butterflies containing each edge; total
 * (host): the butterflies of the graph.  For two vertices of one side with w
 * common neighbours, the pair spans C(w, 2) butterflies and each of its 2w
 * edges lies in w - 1 of them; the sums are exact integers, identical from
 * run to run.  E_INVALID for a malformed CSR (checked on the device before
 * any counting), E_CAPACITY for a short workspace.  Synchronises `stream`.
 */
int32_t ktruss_butterflies(const ktruss_bipartite* g, int64_t* count, int64_t* total, void* stream);

/* ------------------------------------------------------------- profiling */
/*
 * Kernel timing, a measurement aid.  While enabled (on != 0), the support
 * launches issued by ktruss_support / ktruss_run in this process are bracketed
 * by HIP events recorded on the call's stream and tallied by kind:
 *   0  the whole support pass (all variants of one pass);
 *   1  thread-per-edge launches, 2 wavefront-per-edge launches, 3 hub-row
 *      launches (tasks = edge tasks, or hub items for kind 3);
 *   4  the row-local sum that adds the hub kernel's per-task hit words to
 *      S(i, w) (tasks = alive edges);
 *   5  thread-per-row launches of the coarse schedule (tasks = alive edges).
 * Enabling (or disabling) clears the tallies.  Returns KTRUSS_OK.
 */
int32_t ktruss_profile_enable(int32_t on);
/*
 * Reads the tallies of `kind` since the last enable: launches, summed time in
 * milliseconds (synchronises on the recorded events) and tasks.  `bytes` is
 * set for kind 0 only (0 otherwise): the algorithmic bytes of the profiled
 * passes under the merge model of Algorithm 3, 4 (3 m + W) bytes read plus
 * 8 (2 T + m) bytes of support read-modify-writes, with m the alive edges, W
 * the sum over them of |tail of the edge in its row| + |row kappa| and T the
 * triangles (the sum of the supports over 3), summed over the passes.
 * Any out pointer may be NULL.  E_INVALID for a kind outside 0..5.
 */
int32_t ktruss_profile_read(int32_t kind, int64_t* launches, double* total_ms, int64_t* tasks, int64_t* bytes);
/*
 * Statistics of the support passes profiled since the last enable, summed
 * over the passes (Algorithm 3's tasks of each pass): out[0] alive edges
 * (tasks), out[1] sum of their tail lengths |a12(j+1:)|, out[2] sum of their
 * row-kappa lengths, out[3] sum of the supports (3 x triangles); for the
 * tasks the workgroup-per-hub-row kernel ran: out[4] their count, out[5]
 * their tail sum, out[6] their 64-bit hit words (sum of ceil(tail / 64)),
 * out[7] the row-kappa elements it staged in LDS.  Writes min(len, 8)
 * values (host int64).  The statistics live in a fixed device array of the
 * library (no allocation) on the device current at ktruss_profile_enable;
 * profiling on two devices at once is not supported.
 */
int32_t ktruss_profile_stats(int64_t* out, int32_t len);

/* ------------------------------------------------------------- cost model */
/*
 * The LEARNED schedule decides, for every row kappa of A22 that the tasks of
 * a pass select (Algorithm 3), which kernel variant runs those tasks: the
 * workgroup-per-hub-row kernel or the per-edge kernels.  Section III-B notes
 * that grouping work exactly can cost as much as the work; the cost model
 * predicts instead, from five features of the row (its out-degree, log2 of
 * it, log2 of the sum of the out-degrees of the rows whose tasks select it,
 * the pass index, the fraction of the input's edges still alive), the log2
 * ratio of the row's cost on the hub kernel to its cost on the
 * wavefront-per-edge kernel (both in wave-cycles).  Rows predicted at most
 * tuning.learned_hub_min (default 0: the hub kernel is cheaper) become hub
 * rows, in items of tuning.hub_chunk_tasks tasks; the tasks of the others go
 * to the wavefront- or thread-per-edge kernel by merge length.  Scheduling
 * only: results never depend on the model.  The model is trained on samples
 * from ktruss_collect_row_costs with the calls below.
 */

/*
 * ktruss_collect_row_costs — runs the fixpoint of g for K with every task on
 * one kernel variant (variant 0: workgroup-per-hub-row, 1: wavefront-per-edge),
 * timed per row with the shader clock, and appends one sample per active row
 * and pass: features (device float[capacity*5]) and the measured cost as
 * log2(1 + wave-cycles) (device float[capacity]; a hub item's cycles count
 * once per wave of its workgroup).  Both variants visit the same rows in the
 * same order, so their samples pair up.  count (host) receives the number of
 * samples written (at most capacity).  The truss itself is not output.
 * Synchronises `stream`.
 */
int32_t ktruss_collect_row_costs(const ktruss_graph* g, int32_t K, int32_t variant, float* features, float* costs,
                                 int32_t capacity, int32_t* count, void* stream);

/* Scratch bytes needed by ktruss_mlp_loss_grad for `rows` samples. */
int64_t ktruss_mlp_workspace_bytes(int32_t rows);
/* y[r] = network(x[r*5 .. r*5+4]) for r < rows.  params, x, y: device. */
int32_t ktruss_mlp_forward(const float* params, const float* x, int32_t rows, float* y, void* stream);
/*
 * Mean squared error L = mean_r (y[r] - target[r])^2 and its gradient with
 * respect to all KTRUSS_MLP_PARAMS parameters (device float out; loss may be
 * NULL).  work: device scratch of ktruss_mlp_workspace_bytes(rows) bytes.
 * The reduction order is fixed (results are deterministic).
 */
int32_t ktruss_mlp_loss_grad(const float* params, const float* x, const float* target, int32_t rows, float* loss,
                             float* grad, void* work, int64_t work_bytes, void* stream);
/* One Adam step (Kingma and Ba): m, v device float[KTRUSS_MLP_PARAMS] state; step counts from 1. */
int32_t ktruss_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KTRUSS_H */
