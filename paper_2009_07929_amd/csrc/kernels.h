// Launch wrappers of the device kernels (kernels.hip).  All are asynchronous on
// `s` and return the hipError_t of the launch.
#pragma once

#include "common.h"

namespace kt {

// ---- input validation and set-up
hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m,
                           int32_t* src_out, Ctl* ctl, hipStream_t s);
hipError_t launch_init_run(const Buf& b, const int32_t* rowptr, const int32_t* col, int32_t n, int32_t m,
                           Ctl* ctl, hipStream_t s);

// ---- one support pass over buffer p (S of that buffer must be zero)
hipError_t launch_support_thread_edge(const Buf& x, const Ctl* ctl, int p, int32_t m_hint, hipStream_t s);

// ---- prune + compaction of buffer p into buffer 1-p
// mode 0: keep = S[e] >= thr (a prune round); mode 1: keep = alive_can[eid[e]] != 0
// (initial restriction to a caller's alive set; never ends the run).
hipError_t launch_compact(const Buf& x, const Buf& y, int32_t n, int mode, int32_t thr,
                          const uint8_t* alive_can, int32_t* xscan, int32_t* blockcnt, int32_t* blockoff,
                          Ctl* ctl, int p, int32_t m_hint, hipStream_t s);

// ---- outputs
hipError_t launch_set_final(Ctl* ctl, int f, hipStream_t s);
hipError_t launch_scatter_out(const Buf& b0, const Buf& b1, const Ctl* ctl, uint8_t* mask, int32_t* support,
                              int32_t m_hint, hipStream_t s);
hipError_t launch_prune_canonical(const int32_t* support, uint8_t* alive, int32_t m, int32_t thr,
                                  unsigned long long* removed, hipStream_t s);

}  // namespace kt
