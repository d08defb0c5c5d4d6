// Cost-model network (5 -> 64 ReLU -> 64 ReLU -> 1, FP32) on plain VALU FMAs:
// forward, loss gradient and Adam.  It predicts the cost of a hub row's
// support work and only steers scheduling, never results.
//
// Parameter vector (kMlpParams floats): W1[64x5] (row j = weights into hidden
// unit j), b1[64], W2[64x64] (row k = weights into unit k of layer 2), b2[64],
// w3[64], b3[1].
#include "device_util.h"
#include "kernels.h"

namespace kt {

namespace {

constexpr int kIn = KTRUSS_MLP_IN, kHid = KTRUSS_MLP_HIDDEN;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
static_assert(oB3 + 1 == KTRUSS_MLP_PARAMS, "parameter layout");

constexpr int kTile = 64;           // rows per gradient tile
constexpr int kMlpThreads = 256;
constexpr int kPerThread = (KTRUSS_MLP_PARAMS + kMlpThreads - 1) / kMlpThreads;

__device__ __forceinline__ void stage_params(const float* __restrict__ params, float* s_p) {
    for (int i = threadIdx.x; i < KTRUSS_MLP_PARAMS; i += blockDim.x) s_p[i] = params[i];
    __syncthreads();
}

__device__ __forceinline__ float mlp_row(const float* s_p, const float* x) {
    float h1[kHid];
#pragma unroll
    for (int j = 0; j < kHid; ++j) {
        float z = s_p[oB1 + j];
#pragma unroll
        for (int i = 0; i < kIn; ++i) z = fmaf(s_p[oW1 + j * kIn + i], x[i], z);
        h1[j] = fmaxf(z, 0.f);
    }
    float y = s_p[oB3];
    for (int k = 0; k < kHid; ++k) {
        float z = s_p[oB2 + k];
#pragma unroll
        for (int j = 0; j < kHid; ++j) z = fmaf(s_p[oW2 + k * kHid + j], h1[j], z);
        y = fmaf(s_p[oW3 + k], fmaxf(z, 0.f), y);
    }
    return y;
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(const float* __restrict__ params,
                                                           const float* __restrict__ X, int32_t rows,
                                                           float* __restrict__ Y) {
    __shared__ float s_p[KTRUSS_MLP_PARAMS];
    stage_params(params, s_p);
    for (int32_t r = (int32_t)(blockIdx.x * kMlpThreads + threadIdx.x); r < rows;
         r += (int32_t)(gridDim.x * kMlpThreads)) {
        float x[kIn];
#pragma unroll
        for (int i = 0; i < kIn; ++i) x[i] = X[(int64_t)r * kIn + i];
        Y[r] = mlp_row(s_p, x);
    }
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward_dev(const float* __restrict__ params,
                                                               const float* __restrict__ X,
                                                               const int32_t* __restrict__ rows_dev,
                                                               float* __restrict__ Y) {
    __shared__ float s_p[KTRUSS_MLP_PARAMS];
    const int32_t rows = *rows_dev;
    if ((int32_t)(blockIdx.x * kMlpThreads) >= rows) return;
    stage_params(params, s_p);
    for (int32_t r = (int32_t)(blockIdx.x * kMlpThreads + threadIdx.x); r < rows;
         r += (int32_t)(gridDim.x * kMlpThreads)) {
        float x[kIn];
#pragma unroll
        for (int i = 0; i < kIn; ++i) x[i] = X[(int64_t)r * kIn + i];
        Y[r] = mlp_row(s_p, x);
    }
}

// Per workgroup: sum over its row tiles of d(mean (y-t)^2)/dtheta, written to
// partial[blockIdx][*], and its share of the loss.  Within a tile, 64 threads
// run one row each forward and backward (activations and layer gradients to
// LDS); then every thread accumulates its own parameters over the tile's rows.
__global__ __launch_bounds__(kMlpThreads) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                        const float* __restrict__ T, int32_t rows,
                                                        float* __restrict__ partial, float* __restrict__ loss_part) {
    __shared__ float s_p[KTRUSS_MLP_PARAMS];
    __shared__ float s_x[kTile][kIn];
    __shared__ float s_h1[kTile][kHid + 1];  // +1: rows start in different LDS banks
    __shared__ float s_h2[kTile][kHid + 1];
    __shared__ float s_d2[kTile][kHid + 1];  // dL/dz2
    __shared__ float s_d1[kTile][kHid + 1];  // dL/dz1
    __shared__ float s_dy[kTile];
    __shared__ float s_l[kTile];
    stage_params(params, s_p);
    const int t = threadIdx.x;
    const float inv_b = 2.f / (float)rows;
    float acc[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) acc[u] = 0.f;
    float lsum = 0.f;
    const int32_t ntiles = (rows + kTile - 1) / kTile;
    for (int32_t tile = (int32_t)blockIdx.x; tile < ntiles; tile += (int32_t)gridDim.x) {
        const int32_t r0 = tile * kTile;
        const int nr = min(kTile, rows - r0);
        if (t < kTile) {
            float x[kIn];
            float y = 0.f, dy = 0.f;
            if (t < nr) {
#pragma unroll
                for (int i = 0; i < kIn; ++i) x[i] = X[(int64_t)(r0 + t) * kIn + i];
            } else {
#pragma unroll
                for (int i = 0; i < kIn; ++i) x[i] = 0.f;
            }
#pragma unroll
            for (int i = 0; i < kIn; ++i) s_x[t][i] = x[i];
            float z1[kHid];
#pragma unroll
            for (int j = 0; j < kHid; ++j) {
                float z = s_p[oB1 + j];
#pragma unroll
                for (int i = 0; i < kIn; ++i) z = fmaf(s_p[oW1 + j * kIn + i], x[i], z);
                z1[j] = z;
                s_h1[t][j] = fmaxf(z, 0.f);
            }
            y = s_p[oB3];
            for (int k = 0; k < kHid; ++k) {
                float z = s_p[oB2 + k];
#pragma unroll
                for (int j = 0; j < kHid; ++j) z = fmaf(s_p[oW2 + k * kHid + j], fmaxf(z1[j], 0.f), z);
                const float h = fmaxf(z, 0.f);
                s_h2[t][k] = h;
                s_d2[t][k] = z;  // pre-activation, turned into dL/dz2 below
                y = fmaf(s_p[oW3 + k], h, y);
            }
            if (t < nr) {
                const float r = y - T[r0 + t];
                dy = inv_b * r;
                s_l[t] = r * r;
            } else {
                s_l[t] = 0.f;
            }
            s_dy[t] = dy;
            for (int k = 0; k < kHid; ++k) s_d2[t][k] = s_d2[t][k] > 0.f ? dy * s_p[oW3 + k] : 0.f;
#pragma unroll
            for (int j = 0; j < kHid; ++j) {
                float g = 0.f;
                for (int k = 0; k < kHid; ++k) g = fmaf(s_d2[t][k], s_p[oW2 + k * kHid + j], g);
                s_d1[t][j] = z1[j] > 0.f ? g : 0.f;
            }
        }
        __syncthreads();
        if (t == 0)
            for (int r = 0; r < kTile; ++r) lsum += s_l[r];
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            const int p = t + u * kMlpThreads;
            if (p >= KTRUSS_MLP_PARAMS) break;
            float a = 0.f;
            if (p < oB1) {
                const int j = (p - oW1) / kIn, i = (p - oW1) % kIn;
                for (int r = 0; r < kTile; ++r) a = fmaf(s_d1[r][j], s_x[r][i], a);
            } else if (p < oW2) {
                const int j = p - oB1;
                for (int r = 0; r < kTile; ++r) a += s_d1[r][j];
            } else if (p < oB2) {
                const int k = (p - oW2) / kHid, j = (p - oW2) % kHid;
                for (int r = 0; r < kTile; ++r) a = fmaf(s_d2[r][k], s_h1[r][j], a);
            } else if (p < oW3) {
                const int k = p - oB2;
                for (int r = 0; r < kTile; ++r) a += s_d2[r][k];
            } else if (p < oB3) {
                const int k = p - oW3;
                for (int r = 0; r < kTile; ++r) a = fmaf(s_dy[r], s_h2[r][k], a);
            } else {
                for (int r = 0; r < kTile; ++r) a += s_dy[r];
            }
            acc[u] += a;
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const int p = t + u * kMlpThreads;
        if (p < KTRUSS_MLP_PARAMS) partial[(int64_t)blockIdx.x * KTRUSS_MLP_PARAMS + p] = acc[u];
    }
    if (t == 0) loss_part[blockIdx.x] = lsum;
}

// Fixed-order sum of the per-workgroup partials (deterministic).
__global__ __launch_bounds__(kBlock) void k_mlp_reduce(const float* __restrict__ partial, int32_t nblk,
                                                     const float* __restrict__ loss_part, int32_t rows,
                                                     float* __restrict__ grad, float* __restrict__ loss) {
    const int p = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (p < KTRUSS_MLP_PARAMS) {
        float a = 0.f;
        for (int32_t b = 0; b < nblk; ++b) a += partial[(int64_t)b * KTRUSS_MLP_PARAMS + p];
        grad[p] = a;
    }
    if (p == 0 && loss) {
        float l = 0.f;
        for (int32_t b = 0; b < nblk; ++b) l += loss_part[b];
        *loss = l / (float)rows;
    }
}

__global__ __launch_bounds__(kBlock) void k_mlp_adam(float* __restrict__ params, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
    const int p = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (p >= KTRUSS_MLP_PARAMS) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace

int32_t mlp_grad_blocks(int32_t rows) {
    const int32_t tiles = (rows + kTile - 1) / kTile;
    return tiles < kMlpGradMaxBlocks ? (tiles < 1 ? 1 : tiles) : kMlpGradMaxBlocks;
}

hipError_t launch_mlp_forward(const float* params, const float* X, int32_t rows, float* Y, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int32_t g = (int32_t)min((int64_t)(rows + kMlpThreads - 1) / kMlpThreads, (int64_t)kStreamMaxGrid);
    k_mlp_forward<<<g, kMlpThreads, 0, s>>>(params, X, rows, Y);
    return hipGetLastError();
}

hipError_t launch_mlp_forward_dev(const float* params, const float* X, const int32_t* rows_dev, int32_t rows_hint,
                                  float* Y, hipStream_t s) {
    if (rows_hint <= 0) return hipSuccess;
    const int32_t g = (int32_t)min((int64_t)(rows_hint + kMlpThreads - 1) / kMlpThreads, (int64_t)kStreamMaxGrid);
    k_mlp_forward_dev<<<g, kMlpThreads, 0, s>>>(params, X, rows_dev, Y);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* params, const float* X, const float* T, int32_t rows, float* partial,
                                float* loss_part, float* grad, float* loss, hipStream_t s) {
    const int32_t nblk = mlp_grad_blocks(rows);
    k_mlp_grad<<<nblk, kMlpThreads, 0, s>>>(params, X, T, rows, partial, loss_part);
    k_mlp_reduce<<<grid_for(KTRUSS_MLP_PARAMS), kBlock, 0, s>>>(partial, nblk, loss_part, rows, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float b1,
                           float b2, float eps, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_mlp_adam<<<grid_for(KTRUSS_MLP_PARAMS), kBlock, 0, s>>>(params, grad, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace kt
