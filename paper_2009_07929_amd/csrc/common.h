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

// Device-resident control block of one run.  Buffer b of the double-buffered
// working graph holds m_buf[b] alive edges.
struct Ctl {
    int32_t m_buf[2];
    int32_t done;        // a pass removed nothing: later kernels of the run do no work
    int32_t final_buf;   // buffer holding the final alive set and supports
    int32_t rounds;      // support passes executed
    int32_t err;         // validation error bits
    int32_t kept;        // survivors of the last prune
    int32_t pad;
    int64_t removed_total;
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

struct Layout {
    size_t col[2], src[2], eid[2], S[2], rowptr[2];
    size_t xscan;      // int32[m+1]: new position of every old position
    size_t blockcnt;   // int32[kMaxScanBlocks]
    size_t blockoff;   // int32[kMaxScanBlocks]
    size_t ctl;        // Ctl
    size_t total;
};

Layout layout(int32_t n, int64_t m);

// Records `code` and a printf-style message as this thread's last error and
// returns `code`.
int32_t fail(int32_t code, const char* fmt, ...);
// Records a failed HIP call (status KTRUSS_E_HIP) and returns KTRUSS_E_HIP.
int32_t fail_hip(hipError_t e, const char* what);
void clear_error();

}  // namespace kt
