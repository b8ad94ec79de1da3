// Two-hidden-layer perceptron (ReLU, FP32) for the learned tree-shape
// choice: forward pass, loss gradient by back-propagation, and Adam, as
// hand-written HIP kernels over plain device pointers.
//
// Parameters, one device array (row-major, input index first):
//   W1[d_in x h], b1[h], W2[h x h], b2[h], W3[h x d_out], b3[d_out].
// Forward:  h1 = relu(x W1 + b1),  h2 = relu(h1 W2 + b2),  y = h2 W3 + b3.
// Loss:     L = (1/B) sum_b sum_o w_o (y_bo - t_bo)^2.
// Every reduction runs in a fixed order (no atomics), so results are
// reproducible run to run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tqs_internal.h"

namespace tqs {

constexpr int kTile = 16;

// C[M x N] = op(A) op(B) (+ bias[N]) (relu), op(A)[m][k] = A[m*sam + k*sak],
// op(B)[k][n] = B[k*sbk + n*sbn]: 16 x 16 output tiles, K staged in LDS.
__global__ __launch_bounds__(kTile *kTile) void gemm_kernel(const float *A, uint32_t sam, uint32_t sak,
                                                           const float *B, uint32_t sbk, uint32_t sbn,
                                                           float *C, uint32_t M, uint32_t N, uint32_t K,
                                                           const float *bias, int relu) {
    __shared__ float As[kTile][kTile + 1];
    __shared__ float Bs[kTile][kTile + 1];
    const uint32_t tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const uint32_t row = blockIdx.y * kTile + ty, col = blockIdx.x * kTile + tx;
    float acc = 0.0f;
    for (uint32_t k0 = 0; k0 < K; k0 += kTile) {
        const uint32_t ka = k0 + tx, kb = k0 + ty;
        As[ty][tx] = (row < M && ka < K) ? A[(uint64_t)row * sam + (uint64_t)ka * sak] : 0.0f;
        Bs[ty][tx] = (kb < K && col < N) ? B[(uint64_t)kb * sbk + (uint64_t)col * sbn] : 0.0f;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTile; k++) acc += As[ty][k] * Bs[k][tx];
        __syncthreads();
    }
    if (row < M && col < N) {
        if (bias) acc += bias[col];
        if (relu) acc = acc > 0.0f ? acc : 0.0f;
        C[(uint64_t)row * N + col] = acc;
    }
}

// out[n] = sum_m X[m][n] (column sums, one thread per column, rows in order).
__global__ __launch_bounds__(256) void colsum_kernel(const float *X, uint32_t M, uint32_t N, float *out) {
    const uint32_t n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (uint32_t m = 0; m < M; m++) s += X[(uint64_t)m * N + n];
    out[n] = s;
}

// dX = dX * (H > 0): the ReLU derivative, elementwise.
__global__ __launch_bounds__(256) void relu_back_kernel(float *dX, const float *H, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n && !(H[i] > 0.0f)) dX[i] = 0.0f;
}

// dy = (2/B) w_o (y - t); per-row partial losses sum_o w_o (y - t)^2.
__global__ __launch_bounds__(256) void loss_grad_kernel(const float *y, const float *t, const float *w,
                                                        uint32_t B, uint32_t D, float *dy, float *row_loss) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    float l = 0.0f;
    for (uint32_t o = 0; o < D; o++) {
        const float d = y[(uint64_t)b * D + o] - t[(uint64_t)b * D + o];
        l += w[o] * d * d;
        dy[(uint64_t)b * D + o] = 2.0f * w[o] * d / (float)B;
    }
    row_loss[b] = l;
}

// loss = (1/B) sum_b row_loss[b], one thread, rows in order.
__global__ __launch_bounds__(64) void loss_sum_kernel(const float *row_loss, uint32_t B, float *loss) {
    if (threadIdx.x != 0) return;
    float s = 0.0f;
    for (uint32_t b = 0; b < B; b++) s += row_loss[b];
    *loss = s / (float)B;
}

// Adam (Kingma and Ba 2015) with bias correction.
__global__ __launch_bounds__(256) void adam_kernel(float *p, const float *g, float *m, float *v, uint64_t n,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct MlpShape {
    uint32_t din, h, dout;
    uint64_t w1, b1, w2, b2, w3, b3, count;
};

static MlpShape mlp_shape(uint32_t din, uint32_t h, uint32_t dout) {
    MlpShape s;
    s.din = din;
    s.h = h;
    s.dout = dout;
    s.w1 = 0;
    s.b1 = s.w1 + (uint64_t)din * h;
    s.w2 = s.b1 + h;
    s.b2 = s.w2 + (uint64_t)h * h;
    s.w3 = s.b2 + h;
    s.b3 = s.w3 + (uint64_t)h * dout;
    s.count = s.b3 + dout;
    return s;
}

static void gemm(hipStream_t st, const float *A, uint32_t sam, uint32_t sak, const float *B, uint32_t sbk,
                 uint32_t sbn, float *C, uint32_t M, uint32_t N, uint32_t K, const float *bias, int relu) {
    const dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(kTile * kTile), 0, st, A, sam, sak, B, sbk, sbn, C, M, N, K,
                       bias, relu);
}

static tqs_status check_dims(uint32_t din, uint32_t h, uint32_t dout, uint32_t batch) {
    if (!din || !h || !dout || !batch) return fail(TQS_E_ARG, "perceptron sizes and batch must be positive");
    if (din > 4096 || h > 4096 || dout > 64 || batch > (1u << 20))
        return fail(TQS_E_ARG, "perceptron sizes out of range (d_in, h <= 4096, d_out <= 64, batch <= 2^20)");
    return TQS_OK;
}

// scratch: h1[B h], h2[B h], y[B dout], dy[B dout], dh2[B h], dh1[B h], row_loss[B]
static uint64_t scratch_floats(uint32_t h, uint32_t dout, uint32_t B) {
    return (uint64_t)B * (4ull * h + 2ull * dout + 1ull);
}

static void forward(hipStream_t st, const MlpShape &s, const float *P, const float *x, uint32_t B, float *h1,
                    float *h2, float *y) {
    gemm(st, x, s.din, 1, P + s.w1, s.h, 1, h1, B, s.h, s.din, P + s.b1, 1);
    gemm(st, h1, s.h, 1, P + s.w2, s.h, 1, h2, B, s.h, s.h, P + s.b2, 1);
    gemm(st, h2, s.h, 1, P + s.w3, s.dout, 1, y, B, s.dout, s.h, P + s.b3, 0);
}

}  // namespace tqs

using namespace tqs;

extern "C" uint64_t tqs_mlp_param_count(uint32_t d_in, uint32_t h, uint32_t d_out) {
    return mlp_shape(d_in, h, d_out).count;
}

extern "C" uint64_t tqs_mlp_scratch_floats(uint32_t d_in, uint32_t h, uint32_t d_out, uint32_t batch) {
    (void)d_in;
    return scratch_floats(h, d_out, batch);
}

extern "C" tqs_status tqs_mlp_forward(const float *params, uint32_t d_in, uint32_t h, uint32_t d_out,
                                      const float *x, uint32_t batch, float *y, float *scratch, void *stream) {
    tqs_status rc = check_dims(d_in, h, d_out, batch);
    if (rc) return rc;
    if (!params || !x || !y || !scratch) return fail(TQS_E_ARG, "NULL pointer");
    const MlpShape s = mlp_shape(d_in, h, d_out);
    hipStream_t st = (hipStream_t)stream;
    float *h1 = scratch, *h2 = h1 + (uint64_t)batch * h;
    forward(st, s, params, x, batch, h1, h2, y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TQS_E_HIP, "perceptron forward: %s", hipGetErrorString(e));
    return TQS_OK;
}

extern "C" tqs_status tqs_mlp_loss_grad(const float *params, uint32_t d_in, uint32_t h, uint32_t d_out,
                                        const float *x, const float *target, const float *out_weight,
                                        uint32_t batch, float *grad, float *loss, float *scratch,
                                        void *stream) {
    tqs_status rc = check_dims(d_in, h, d_out, batch);
    if (rc) return rc;
    if (!params || !x || !target || !out_weight || !grad || !loss || !scratch)
        return fail(TQS_E_ARG, "NULL pointer");
    const MlpShape s = mlp_shape(d_in, h, d_out);
    hipStream_t st = (hipStream_t)stream;
    const uint32_t B = batch;
    float *h1 = scratch, *h2 = h1 + (uint64_t)B * h, *y = h2 + (uint64_t)B * h;
    float *dy = y + (uint64_t)B * d_out, *dh2 = dy + (uint64_t)B * d_out, *dh1 = dh2 + (uint64_t)B * h;
    float *row_loss = dh1 + (uint64_t)B * h;
    forward(st, s, params, x, B, h1, h2, y);
    hipLaunchKernelGGL(loss_grad_kernel, dim3((B + 255) / 256), dim3(256), 0, st, y, target, out_weight, B,
                       d_out, dy, row_loss);
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, st, row_loss, B, loss);
    // layer 3: dW3 = h2^T dy, db3 = colsum(dy), dh2 = (dy W3^T) * (h2 > 0)
    gemm(st, h2, 1, h, dy, d_out, 1, grad + s.w3, h, d_out, B, nullptr, 0);
    hipLaunchKernelGGL(colsum_kernel, dim3((d_out + 255) / 256), dim3(256), 0, st, dy, B, d_out, grad + s.b3);
    gemm(st, dy, d_out, 1, params + s.w3, 1, d_out, dh2, B, h, d_out, nullptr, 0);
    hipLaunchKernelGGL(relu_back_kernel, dim3((uint32_t)(((uint64_t)B * h + 255) / 256)), dim3(256), 0, st, dh2,
                       h2, (uint64_t)B * h);
    // layer 2
    gemm(st, h1, 1, h, dh2, h, 1, grad + s.w2, h, h, B, nullptr, 0);
    hipLaunchKernelGGL(colsum_kernel, dim3((h + 255) / 256), dim3(256), 0, st, dh2, B, h, grad + s.b2);
    gemm(st, dh2, h, 1, params + s.w2, 1, h, dh1, B, h, h, nullptr, 0);
    hipLaunchKernelGGL(relu_back_kernel, dim3((uint32_t)(((uint64_t)B * h + 255) / 256)), dim3(256), 0, st, dh1,
                       h1, (uint64_t)B * h);
    // layer 1
    gemm(st, x, 1, d_in, dh1, h, 1, grad + s.w1, d_in, h, B, nullptr, 0);
    hipLaunchKernelGGL(colsum_kernel, dim3((h + 255) / 256), dim3(256), 0, st, dh1, B, h, grad + s.b1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TQS_E_HIP, "perceptron gradient: %s", hipGetErrorString(e));
    return TQS_OK;
}

extern "C" tqs_status tqs_mlp_adam(float *params, const float *grad, float *m, float *v, uint64_t count,
                                   float lr, float beta1, float beta2, float eps, uint32_t step, void *stream) {
    if (!params || !grad || !m || !v || !count) return fail(TQS_E_ARG, "NULL pointer or empty parameter array");
    if (step < 1) return fail(TQS_E_ARG, "Adam step counts from 1");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       params, grad, m, v, count, lr, beta1, beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TQS_E_HIP, "Adam update: %s", hipGetErrorString(e));
    return TQS_OK;
}
