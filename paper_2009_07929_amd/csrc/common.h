// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ktruss.h"

namespace kt {

constexpr int kBlock = 256;          // threads per workgroup of the streaming kernels (4 wave64)
constexpr int kMaxScanBlocks = 4096; // workgroups of the compaction grid (one scan workgroup covers them)
constexpr int kScanThreads = 1024;

// workgroup-per-hub-row kernel
constexpr int kHubThreads = 256;     // 4 waves
constexpr int kHubChunk = 256;       // tasks (in-edges of one row kappa) per hub item
constexpr int kHubUnroll = 8;        // tail chunks whose loads a hub wave issues together
constexpr int kHubBatch = 8;         // consecutive hub items per ticket of the persistent hub kernel
// LDS of one hub workgroup: the rank bitmap (or the keys) and the accumulators
// of row kappa, about 24.6 KB, so that the six workgroups per CU that the
// kernel's register use allows all fit in the 160 KB of a CU.
constexpr int kSpanWords = 1536;
constexpr int kSpanCap = kSpanWords * 32;  // widest label span staged as a rank bitmap (49,152)
constexpr int kKeyCap = 2 * kSpanWords;    // longest row kappa staged in LDS as keys (3,072)
constexpr int kHubMaxGrid = 256 * 6;     // persistent hub grid: the 6 workgroups per CU that registers and LDS allow
constexpr int kStreamMaxGrid = 256 * 16; // grid-stride cap of the thread/wave task kernels
constexpr int kMlpGradMaxBlocks = 512;   // workgroups of the cost-model gradient kernel
constexpr int kRsTile = 4096;            // (column, edge) pairs per workgroup of the radix-sort transpose
constexpr int kHitWordsPerEdge = 8;      // hit-word capacity of the workspace per edge (see hit_words_upto)

// learned schedule: the cost model predicts, for a row kappa, log2 of its
// wave-cycles on the hub kernel minus log2 of its wave-cycles on the
// wavefront-per-edge kernel; the row goes to the hub kernel when the
// prediction is at most the threshold (default 0: the hub kernel is cheaper)
constexpr float kDefaultLearnedHubMax = 0.0f;
constexpr int32_t kDefaultPlainMaxWork = 32;
constexpr int kMinLearnedChunk = 16;     // fewest tasks per hub item
// incremental maintenance, mode 2: a prune removing more than this fraction of
// the edges it keeps is followed by a recomputation instead of a peel (measured
// on R-MAT scales 20 and 23 over 0.125 .. 2: 0.125 was the fastest or tied)
constexpr float kDefaultPeelRatio = 0.125f;
// internal schedule of cost sampling: every task on the wavefront kernel,
// through the binned path (in-edge lists, row features, per-row timing)
constexpr int kSchedSampleWave = 100;

// static degree heuristic defaults
constexpr int kDefaultHubMinIn = 8;    // in-edges for a row kappa to be a hub row
constexpr int kDefaultWaveMin = 192;   // merge length for wavefront-per-edge

// Per-pass statistics gathered while profiling (ktruss_profile_stats): alive
// edges, sum of their tail lengths, sum of their row-kappa lengths, sum of
// supports (3 x triangles); for the tasks the hub kernel ran: their count,
// tail sum and hit words, and the row-kappa elements it staged in LDS.
enum PassStat {
    kStatEdges = 0, kStatTail, kStatRowK, kStatSupport, kStatHubTasks, kStatHubTail, kStatHubWords,
    kStatHubStaged, kPassStats
};

// Device-resident control block of one run.  Buffer b of the double-buffered
// working graph holds m_buf[b] alive edges.
// Support value of an edge that an in-place round has removed (alive edges
// hold their support, >= 0); which round removed it is in the liveness words.
constexpr int32_t kDying = -2;

struct Ctl {
    int32_t m_buf[2];
    int32_t done;        // a pass removed nothing: later kernels of the run do no work
    int32_t final_buf;   // buffer holding the final alive set and supports
    int32_t rounds;      // support passes executed
    int32_t err;         // validation error bits
    int32_t kept;        // survivors of the last prune
    int32_t n_items;     // hub items of the current pass
    int32_t n_wave;      // wavefront-per-edge tasks of the current pass
    int32_t n_thread;    // thread-per-edge tasks of the current pass
    int32_t item_next;   // next hub item to take (persistent hub kernel)
    int32_t n_active;    // rows with support work in the current pass (learned schedule, sampling)
    int32_t n_samples;   // cost-model samples written so far
    int32_t csc_m;       // in-edge list entries (alive edges + tombstones of removed ones)
    int32_t csc_pack;    // the lists are being packed in this round (tombstones dominate)
    int32_t csc_next;    // entries after packing
    int32_t need_support; // incremental maintenance skipped its peel: the next round recomputes supports
    int32_t front_n;      // edges an in-place prune lists for the peel (removed with support > 0)
    int32_t removed_now;  // edges the in-place prune removes (the listed ones and those in no triangle)
    int32_t n_long;       // rows whose hit words are summed per row (k_hit_sum_long) in the current pass
    int64_t removed_total;
    unsigned long long merge_work;  // input's merge length summed over its edges (row tail + row kappa)
};

// One buffer of the working graph: the alive edges compacted in canonical
// order, with their row (src), column (col), canonical position (eid) and the
// support accumulator (S); rowptr indexes them by row.
struct Buf {
    int32_t* col;
    int32_t* src;
    int32_t* eid;
    int32_t* S;
    int32_t* rowptr;
};

// In-edge lists: for every row kappa, the positions of the edges whose column
// is kappa (edge[ptr[kappa] .. ptr[kappa+1])), their rows (src) and kappa
// itself (key).  Built once per run; after every prune the positions are
// remapped in place and the entries of removed edges become tombstones
// (edge = -1), so the lists keep their length (Ctl::csc_m) for the whole run.
struct Csc {
    int32_t* edge;
    int32_t* src;
    int32_t* key;
    int32_t* ptr;
};

// One hub item: row kappa (its first position rs, length d and last label)
// and the in-edge list entries [c0, c1) of the tasks that select it.
struct HubItem {
    int32_t k, c0, c1, rs, d, last, pad0, pad1;
};

// Keep flags of a compaction, 64 elements to a word, with the number of kept
// elements before the word: element e's new position is pref plus the kept
// bits below e's bit.  A 16-byte entry per 64 elements, so the scattered
// lookups of the in-edge list remap hit a table 1/16 the size of a
// per-element one.
struct alignas(16) KeepWord {
    unsigned long long bits;
    int32_t pref;
    int32_t pad;
};

// Liveness of an in-place round, 64 positions to a word: removed by an
// earlier round (dead) or by this one (dying).  Same size as a KeepWord, and
// kept in the same scratch (the two are never live at once).  Words of waves
// that lie in a finished graph (batched form) say nothing useful: no peel
// reaches those positions.
struct alignas(16) LiveWord {
    unsigned long long dead;
    unsigned long long dying;
};

// Per-run scratch arrays inside the workspace.
struct Scratch {
    int32_t* xscan;       // int32[m+1]: new CSR position of every old position
    KeepWord* keepw;      // KeepWord[m/64 + 1]: the same as keep bits and per-word counts
    int32_t* cxscan;      // int32[m+1]: same for in-edge list entries when the lists are packed
    int32_t* blockcnt;    // int32[kMaxScanBlocks]
    int32_t* blockoff;    // int32[kMaxScanBlocks]
    int32_t* blockcnt2;   // int32[2*kMaxScanBlocks]
    int32_t* blockoff2;   // int32[2*kMaxScanBlocks]
    int32_t* alive_in;    // int32[n+1]: alive in-edges per row kappa (the lists also hold tombstones)
    int32_t* itemoff;     // int32[n+1]
    HubItem* items;       // HubItem[item capacity]
    int32_t* ctail;       // int32[m]: tail length of the task of every in-edge list entry
    unsigned long long* insum;   // uint64[n]: sum of in-neighbour out-degrees
    unsigned long long* cycles;  // uint64[n]: measured hub cycles per row (sampling)
    int32_t* act_off;     // int32[n+1]
    int32_t* act_list;    // int32[n]
    float* feats;         // float[n*5]
    float* pred;          // float[n]
    int32_t* chunk_sz;    // int32[n]
    int32_t* rs_hist;     // int32[256 * ceil(m / kRsTile) + 1]: radix-sort digit histograms
    uint8_t* is_hub;      // uint8[n]
    uint8_t* hub_row;     // uint8[n]: row kappa has hub items in the current pass
    unsigned long long* hitw;  // uint64[hit_cap]: hub hit words, per row and task (hit_words_upto)
    int64_t* hwoff;            // int64[n+1]: first hit word of every row's tasks in the current pass
    int64_t hit_cap;           // words of hitw (kHitWordsPerEdge * m)
    int32_t* wave_tasks;  // int32[m]
    int32_t* thread_tasks;// int32[m]
    int32_t* long_off;    // int32[n+1]: scan of the rows whose hit words are summed per row
    int32_t* long_rows;   // int32[n]: those rows
};

// Rows whose length d lies in (kHitLongMin, kHitLongMax] have their hit words
// summed by one workgroup per row (every word read once, counts in LDS); the
// others by windows of 64 positions.
constexpr int32_t kHitLongMin = 192;
constexpr int32_t kHitLongMax = 4096;

// Batched form: per-vertex graph id and threshold, per-graph state, outputs.
// thrv == nullptr means a single graph (the scalar threshold applies).
struct BatchCtx {
    const int32_t* vert_off;  // int32[G+1]
    int32_t* gidv;            // int32[n]: vertex -> graph
    int32_t* thrv;            // int32[n]: K of the vertex's graph, minus 2
    uint8_t* graph_done;      // uint8[G]
    uint8_t* done_now;        // uint8[G]: finished in the current pass
    uint8_t* mask;            // outputs, canonical positions of the union
    int32_t* support;
    int32_t* low_cnt;         // int32[G]: edges an in-place round removes, per graph (zero between rounds)
    int32_t* rounds;          // int32[G]: the caller's per-graph pass counts
};

// Hit words of the hub kernel.  A task whose tail has L elements owns
// ceil(L / 64) consecutive 64-bit words, bit b of word c standing for tail
// offset 64 c + b.  The tasks of a row (tails d-1, d-2, ..., 0 for a row of
// d alive edges) own consecutive ranges, rows follow each other in label
// order: hwoff[i] is the first word of row i and hwoff[i+1] its end, so the
// task with tail L starts at hwoff[i+1] - hit_words_upto(L), where
// hit_words_upto(x) = sum over L = 0..x of ceil(L / 64) = (q+1)(32q + r) for
// x = 64q + r.  Words at or past the workspace's capacity do not exist: those
// chunks add their hits directly.
__host__ __device__ inline int64_t hit_words_upto(int32_t x) {
    if (x <= 0) return 0;
    const int64_t q = x >> 6, r = x & 63;
    return (q + 1) * (32 * q + r);
}

struct Layout {
    size_t col[2], src[2], eid[2], S[2], rowptr[2];
    size_t cedge, csrc, ckey, cptr;
    size_t xscan, keepw, cxscan, blockcnt, blockoff, blockcnt2, blockoff2, alive_in, itemoff, items, ctail,
        is_hub, hub_row, hitw, hwoff, wave_tasks, thread_tasks, insum, cycles, act_off, act_list, feats, pred, chunk_sz,
        rs_hist, long_off, long_rows;
    size_t ctl;        // Ctl
    size_t total;
};

// Upper bound on hub items: one per row plus one per kMinLearnedChunk edges
// (the smallest split the learned schedule makes).
inline int64_t item_capacity(int32_t n, int64_t m) { return (int64_t)n + m / kMinLearnedChunk + 1; }

Layout layout(int32_t n, int64_t m);

// Records `code` and a printf-style message as this thread's last error and
// returns `code`.
int32_t fail(int32_t code, const char* fmt, ...);
// Records a failed HIP call (status KTRUSS_E_HIP) and returns KTRUSS_E_HIP.
int32_t fail_hip(hipError_t e, const char* what);
void clear_error();

}  // namespace kt
