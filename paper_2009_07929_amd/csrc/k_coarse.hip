// Coarse-grained support computation: one thread per row i running the tasks
// of its edges one after the other, the one-task-per-row granularity of
// Algorithm 2 (Section III-A).  Each task is the merge of the fine-grained
// thread-per-edge kernel: the tail of row i after the edge (i, kappa) against
// row kappa, and every common column w adds to the supports of all three
// edges of the triangle (Algorithm 3's rule, so the result equals every other
// schedule's).  Kept as the ablation of the fine-grained kernels.
#include "common.h"
#include "device_util.h"
#include "kernels.h"

namespace kt {
namespace {

__global__ __launch_bounds__(kBlock) void k_support_row(Buf x, int32_t n, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int32_t* __restrict__ col = x.col;
    for (int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x); i < n; i += (int32_t)(gridDim.x * kBlock)) {
        const int32_t ae = x.rowptr[i + 1];
        for (int32_t e = x.rowptr[i]; e < ae; ++e) {
            const int32_t k = col[e];
            int32_t a = e + 1, b = x.rowptr[k];
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
    }
}

}  // namespace

hipError_t launch_support_row(const Buf& x, int32_t n, const Ctl* ctl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_support_row<<<min(grid_for(n), (unsigned)kStreamMaxGrid), kBlock, 0, s>>>(x, n, ctl);
    return hipGetLastError();
}

}  // namespace kt
