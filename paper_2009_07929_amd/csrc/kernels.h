// Launch wrappers of the device kernels.  All are asynchronous on `s` and
// return the hipError_t of the launch.
#pragma once

#include "common.h"

namespace kt {

// ---- input validation and set-up (k_setup.hip)
hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m, int32_t* src_out,
                           Ctl* ctl, bool tally, hipStream_t s);
hipError_t launch_init_run(const Buf& b, const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m,
                           hipStream_t s);
hipError_t launch_set_final(Ctl* ctl, int f, hipStream_t s);
hipError_t launch_mark_level(const Buf& b, const Ctl* ctl, int f, int32_t m_hint, int32_t K, int32_t* trussness,
                             hipStream_t s);
hipError_t launch_fill_value(int32_t* a, int32_t n, int32_t v, hipStream_t s);
hipError_t launch_ctl_restart(Ctl* ctl, hipStream_t s);
hipError_t launch_scatter_out(const Buf& b0, const Buf& b1, const Ctl* ctl, uint8_t* mask, int32_t* support,
                              int32_t m_hint, hipStream_t s);
hipError_t launch_prune_canonical(const int32_t* support, uint8_t* alive, int32_t m, int32_t thr,
                                  unsigned long long* removed, hipStream_t s);

// ---- prune + compaction of buffer p into buffer 1-p (k_compact.hip)
// mode 0: keep = S[e] >= thr (a prune round: updates the pass count and the
// fixpoint flag); mode 1: keep = alive_can[eid[e]] != 0 (restriction to a
// caller's alive set); mode 2: keep = S[e] >= thr without the round's
// bookkeeping (the survivors of in-place rounds, before a recomputation);
// mode 3: keep = S[e] >= 0 with the supports (in-place rounds shedding their
// removed edges, and in the batched form writing out finished graphs).
// The in-edge lists are compacted too when cx, cy are given.
// With a batch context (b.thrv set) the threshold is per vertex, edges of
// graphs finished in this pass are written to the outputs and dropped, and
// the run ends when no edge is left.  m_hint bounds the alive edges, csc_hint
// the in-edge list entries (the run's m: removed edges stay as tombstones).
hipError_t launch_compact(const Buf& x, const Buf& y, const Csc* cx, const Csc* cy, int32_t n, int mode, int32_t thr,
                          const uint8_t* alive_can, const BatchCtx& b, Scratch& sc, Ctl* ctl, int p, int32_t m_hint,
                          int32_t csc_hint, hipStream_t s);
// One in-place prune round of incremental maintenance on buffer x (k_peel.hip;
// no compaction): removed edges marked and listed in frontier, bookkeeping in
// ctl, then their triangles peeled unless ratio > 0 and the frontier exceeds
// ratio x the survivors (ctl->need_support).
// With a batch context (b.thrv set) the threshold is per graph and every
// unfinished graph counts the pass, finishing when none of its edges goes.
hipError_t launch_state_round(const Buf& x, const Csc& c, int32_t thr, const BatchCtx& b, int32_t G,
                              int32_t* frontier, Scratch& sc, Ctl* ctl, int p, float ratio, int32_t m_hint,
                              hipStream_t s);
// Its marking (k_compact.hip): alive edges of x with S < thr become kDying,
// those with S > 0 are listed in frontier (Ctl::front_n of them; Ctl::
// removed_now counts all), the round's liveness words are written; the
// batched form's per-graph pass counts.
hipError_t launch_state_mark(const Buf& x, const BatchCtx& b, int32_t G, int32_t thr, int32_t* frontier, Scratch& sc,
                             Ctl* ctl, int p, int32_t m_hint, hipStream_t s);

// ---- batched form (k_batch.hip)
hipError_t launch_batch_setup(const BatchCtx& b, int32_t G, int32_t n_total, const int32_t* K, const int32_t* src,
                              const int32_t* col, int32_t m, Ctl* ctl, hipStream_t s);
hipError_t launch_batch_reset(const BatchCtx& b, int32_t G, int32_t* rounds, hipStream_t s);
hipError_t launch_batch_status(const Buf& x, const BatchCtx& b, int32_t G, const int32_t* K, int32_t* rounds,
                               const Ctl* ctl, hipStream_t s);

// ---- scheduling structures (k_sched.hip)
// Stable transpose of CSR columns (radix sort of (column, position) pairs):
// columns ascending into keys_out, their positions into vals_out, ptr[0..n].
// tk, tv: int32[m] ping-pong buffers distinct from the outputs.
hipError_t launch_radix_transpose(const int32_t* keys, int32_t m, int32_t n, int32_t* keys_out, int32_t* vals_out,
                                  int32_t* ptr, int32_t* const tk[2], int32_t* const tv[2], Scratch& sc,
                                  hipStream_t s, const int32_t* rows = nullptr, int32_t* rows_out = nullptr,
                                  int32_t* const tr[2] = nullptr);
// out[j] = the row of CSR position pos[j].
hipError_t launch_rows_of(const int32_t* rowptr, int32_t nrows, const int32_t* pos, int32_t m, int32_t* out,
                          hipStream_t s);
// Butterfly task offsets: off[p] = sum over q < p of the tasks of pair vertex
// q (0 without wedges, 1 if W(q) <= hash_max, else nwin), off[nP] = total.
hipError_t launch_bf_task_offsets(const int64_t* W, int32_t nP, int64_t hash_max, int64_t nwin, int64_t* off,
                                  Scratch& sc, hipStream_t s);
hipError_t launch_build_csc(const Buf& b, const Csc& c, int32_t n, int32_t m, Scratch& sc, hipStream_t s);
// Work lists of one support pass over buffer p: hub items (all rows with
// work under FORCE_HUB; the hub rows of the heuristic or of `learned_hub`
// otherwise) and, except under FORCE_HUB, the wavefront / thread task lists.
// mlp: cost-model parameters (LEARNED; null falls back to the heuristic);
// features: also build the active-row list and features (cost sampling);
// m0: the input's edge count (alive-fraction feature).
hipError_t launch_prepare_pass(const Buf& x, const Csc& c, int32_t n, int sched, const ktruss_tuning& t,
                               const float* mlp, int32_t m0, bool features, Scratch& sc, Ctl* ctl, int p,
                               int32_t m_hint, hipStream_t s);

// ---- support kernels (k_support.hip); count_dev points at the task count
hipError_t launch_support_thread(const Buf& x, const int32_t* tasks, const int32_t* count_dev, int32_t n_hint,
                                 const Ctl* ctl, hipStream_t s);
hipError_t launch_support_row(const Buf& x, int32_t n, const Ctl* ctl, hipStream_t s);
// cycles: per-row wave-cycles of the tasks (cost sampling), or null
hipError_t launch_support_wave(const Buf& x, const int32_t* tasks, const int32_t* count_dev, int32_t n_hint,
                               const Ctl* ctl, hipStream_t s, unsigned long long* cycles = nullptr);
// cycles: per-row wave-cycles of the hub items (cost-model samples: shader clock x 4 waves), or null
hipError_t launch_support_hub(const Buf& x, const Csc& c, const Scratch& sc, int32_t n_items_hint, Ctl* ctl,
                              unsigned long long* cycles, hipStream_t s);
// Profiling: statistics of the pass just computed (PassStat), added to
// acc[0 .. kPassStats-1]; hub_row: rows the hub kernel staged, or null.
hipError_t launch_pass_work(const Buf& x, const int32_t* m_count, int32_t m_hint, const uint8_t* hub_row,
                            unsigned long long* acc, hipStream_t s);
// Row-local sum of the hub kernel's hit words into S (one wave per 64 edges;
// m_count: alive edges on the device, m_hint: an upper bound for the grid).
hipError_t launch_hit_sum(const Buf& x, const Scratch& sc, const int32_t* m_count, int32_t m_hint, const Ctl* ctl,
                          hipStream_t s);

// ---- cost model (k_mlp.hip, k_sched.hip)
int32_t mlp_grad_blocks(int32_t rows);
hipError_t launch_mlp_forward(const float* params, const float* X, int32_t rows, float* Y, hipStream_t s);
// rows read from device memory (upper bound rows_hint sizes the grid)
hipError_t launch_mlp_forward_dev(const float* params, const float* X, const int32_t* rows_dev, int32_t rows_hint,
                                  float* Y, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float* params, const float* X, const float* T, int32_t rows, float* partial,
                                float* loss_part, float* grad, float* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float b1,
                           float b2, float eps, hipStream_t s);
// Sum of in-neighbour out-degrees of every row (once per run), and the
// training-sample append after a timed pass.
hipError_t launch_in_outdeg_sum(const Buf& x, const Csc& c, int32_t n, int32_t m, Scratch& sc, hipStream_t s);
hipError_t launch_append_costs(Scratch& sc, int32_t n, int32_t capacity, float* out_x, float* out_y, Ctl* ctl,
                               hipStream_t s);

}  // namespace kt
