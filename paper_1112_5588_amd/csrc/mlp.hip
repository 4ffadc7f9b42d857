// The learned configuration tuner's network on the GPU: a three-layer perceptron
// d_in -> 64 -> 64 -> d_out (ReLU after the two hidden layers), binary32.
//
//   Z1 = X W1 + b1, H1 = relu(Z1);  Z2 = H1 W2 + b2, H2 = relu(Z2);  P = H2 W3 + b3
//   loss = sum(M (P - T)^2) / sum(M)                              (masked mean squared error)
//
// Parameters are one packed array [W1 (d_in x 64) | b1 | W2 (64 x 64) | b2 | W3 (64 x d_out)
// | b3], weights stored (fan_in, fan_out) row-major.  Every kernel works on tiles of 64
// rows of the batch held in LDS (one workgroup of 256 threads per tile; thread t owns row
// t / 4 and 16 consecutive outputs).  The backward pass recomputes the forward of its tile,
// writes the tile's unnormalised gradient to a workspace, and a second kernel adds the
// tiles in tile order and divides by sum(M): the result does not depend on scheduling.
// The layers are tiny (at most 64 x 64), so plain FMA loops are used; these GEMMs are far
// too small to feed matrix cores.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace pjds {
namespace {

constexpr int kH = 64;         // hidden width
constexpr int kTile = 64;      // batch rows per workgroup
constexpr int kThreads = 256;
constexpr int kLd = 65;        // padded LDS row stride (no bank conflicts down a column)

struct Shapes {
    int d_in, d_out;
    int64_t o_w1, o_b1, o_w2, o_b2, o_w3, o_b3, n_params;
};

__host__ __device__ inline Shapes shapes(int d_in, int d_out) {
    Shapes s{};
    s.d_in = d_in;
    s.d_out = d_out;
    s.o_w1 = 0;
    s.o_b1 = s.o_w1 + int64_t(d_in) * kH;
    s.o_w2 = s.o_b1 + kH;
    s.o_b2 = s.o_w2 + int64_t(kH) * kH;
    s.o_w3 = s.o_b2 + kH;
    s.o_b3 = s.o_w3 + int64_t(kH) * d_out;
    s.n_params = s.o_b3 + d_out;
    return s;
}

// out[r][c] = act(sum_k in[r][k] * W[k][c] + b[c]) for the tile; in and out live in LDS
// with row stride kLd; W is (K x C) row-major in global memory.
template <bool RELU>
__device__ void dense(const float *in, int K, const float *__restrict__ W, const float *__restrict__ b,
                      int C, float *out) {
    const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    float acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = (c0 + q < C) ? b[c0 + q] : 0.f;
    for (int k = 0; k < K; ++k) {
        const float a = in[r * kLd + k];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (c0 + q < C) acc[q] = __builtin_fmaf(a, W[int64_t(k) * C + c0 + q], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
        if (c0 + q < C) out[r * kLd + c0 + q] = RELU ? (acc[q] > 0.f ? acc[q] : 0.f) : acc[q];
}

// Forward of one tile: X (rows beyond `rows` zero) -> H1, H2, P in LDS.
__device__ void tile_forward(const Shapes &s, const float *__restrict__ p, const float *__restrict__ X,
                             int64_t row0, int rows, float *sX, float *sH1, float *sH2, float *sP) {
    for (int e = threadIdx.x; e < kTile * s.d_in; e += kThreads) {
        const int r = e / s.d_in, k = e % s.d_in;
        sX[r * kLd + k] = r < rows ? X[(row0 + r) * s.d_in + k] : 0.f;
    }
    __syncthreads();
    dense<true>(sX, s.d_in, p + s.o_w1, p + s.o_b1, kH, sH1);
    __syncthreads();
    dense<true>(sH1, kH, p + s.o_w2, p + s.o_b2, kH, sH2);
    __syncthreads();
    dense<false>(sH2, kH, p + s.o_w3, p + s.o_b3, s.d_out, sP);
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(Shapes s, const float *__restrict__ p,
                                                               const float *__restrict__ X, int64_t batch,
                                                               float *__restrict__ P) {
    __shared__ float sX[kTile * kLd], sH1[kTile * kLd], sH2[kTile * kLd], sP[kTile * kLd];
    const int64_t row0 = int64_t(blockIdx.x) * kTile;
    const int rows = int(min<int64_t>(kTile, batch - row0));
    tile_forward(s, p, X, row0, rows, sX, sH1, sH2, sP);
    for (int e = threadIdx.x; e < rows * s.d_out; e += kThreads) {
        const int r = e / s.d_out, c = e % s.d_out;
        P[(row0 + r) * s.d_out + c] = sP[r * kLd + c];
    }
}

// Inference: forward, then per row the output with the smallest value after the affine map
// v = P * scale + shift (outputs with valid == 0 are skipped), and the gap to the runner-up.
__global__ __launch_bounds__(kThreads) void mlp_infer_kernel(Shapes s, const float *__restrict__ p,
                                                             const float *__restrict__ X, int64_t batch,
                                                             const float *__restrict__ scale,
                                                             const float *__restrict__ shift,
                                                             const float *__restrict__ valid,
                                                             int32_t *__restrict__ idx, float *__restrict__ margin) {
    __shared__ float sX[kTile * kLd], sH1[kTile * kLd], sH2[kTile * kLd], sP[kTile * kLd];
    const int64_t row0 = int64_t(blockIdx.x) * kTile;
    const int rows = int(min<int64_t>(kTile, batch - row0));
    tile_forward(s, p, X, row0, rows, sX, sH1, sH2, sP);
    if (threadIdx.x < rows) {
        const int r = threadIdx.x;
        float best = 3.4e38f, second = 3.4e38f;
        int bi = -1;
        for (int c = 0; c < s.d_out; ++c) {
            if (valid && valid[c] == 0.f) continue;
            const float v = sP[r * kLd + c] * (scale ? scale[c] : 1.f) + (shift ? shift[c] : 0.f);
            if (v < best) { second = best; best = v; bi = c; }
            else if (v < second) second = v;
        }
        idx[row0 + r] = bi;
        margin[row0 + r] = second - best;
    }
}

// Forward + backward of one tile; writes the tile's unnormalised gradient of
// sum(M (P - T)^2), its partial loss numerator and its mask count to part[tile][...].
__global__ __launch_bounds__(kThreads) void mlp_backward_tile_kernel(Shapes s, const float *__restrict__ p,
                                                                     const float *__restrict__ X,
                                                                     const float *__restrict__ T,
                                                                     const float *__restrict__ M, int64_t batch,
                                                                     float *__restrict__ part) {
    __shared__ float sX[kTile * kLd], sH1[kTile * kLd], sH2[kTile * kLd], sP[kTile * kLd], sD[kTile * kLd];
    __shared__ float red[kThreads], redm[kThreads];
    const int64_t row0 = int64_t(blockIdx.x) * kTile;
    const int rows = int(min<int64_t>(kTile, batch - row0));
    tile_forward(s, p, X, row0, rows, sX, sH1, sH2, sP);
    float* g = part + int64_t(blockIdx.x) * (s.n_params + 2);
    // dP = 2 M (P - T) in sP (rows past the batch contribute nothing)
    float lsum = 0.f, msum = 0.f;
    for (int e = threadIdx.x; e < kTile * s.d_out; e += kThreads) {
        const int r = e / s.d_out, c = e % s.d_out;
        float d = 0.f;
        if (r < rows) {
            const int64_t at = (row0 + r) * s.d_out + c;
            const float m = M[at], diff = sP[r * kLd + c] - T[at];
            lsum = __builtin_fmaf(m * diff, diff, lsum);
            msum += m;
            d = 2.f * m * diff;
        }
        sP[r * kLd + c] = d;
    }
    red[threadIdx.x] = lsum;
    redm[threadIdx.x] = msum;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            red[threadIdx.x] += red[threadIdx.x + st];
            redm[threadIdx.x] += redm[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        g[s.n_params] = red[0];
        g[s.n_params + 1] = redm[0];
    }
    // layer 3: dW3 = H2^T dP, db3 = column sums of dP, dH2 = dP W3^T masked by H2 > 0
    const int tr = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    {
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
        for (int r = 0; r < kTile; ++r) {
            const float h = sH2[r * kLd + tr];
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (c0 + q < s.d_out) acc[q] = __builtin_fmaf(h, sP[r * kLd + c0 + q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (c0 + q < s.d_out) g[s.o_w3 + int64_t(tr) * s.d_out + c0 + q] = acc[q];
        if (threadIdx.x < s.d_out) {
            float b = 0.f;
            for (int r = 0; r < kTile; ++r) b += sP[r * kLd + threadIdx.x];
            g[s.o_b3 + threadIdx.x] = b;
        }
        float d[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) d[q] = 0.f;
        const float *W3 = p + s.o_w3;
        for (int c = 0; c < s.d_out; ++c) {
            const float dp = sP[tr * kLd + c];
#pragma unroll
            for (int q = 0; q < 16; ++q) d[q] = __builtin_fmaf(dp, W3[int64_t(c0 + q) * s.d_out + c], d[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) sD[tr * kLd + c0 + q] = sH2[tr * kLd + c0 + q] > 0.f ? d[q] : 0.f;
    }
    __syncthreads();
    // layer 2: dW2 = H1^T dZ2, db2, dH1 = dZ2 W2^T masked by H1 > 0 (written over sH2)
    {
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
        for (int r = 0; r < kTile; ++r) {
            const float h = sH1[r * kLd + tr];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = __builtin_fmaf(h, sD[r * kLd + c0 + q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) g[s.o_w2 + int64_t(tr) * kH + c0 + q] = acc[q];
        if (threadIdx.x < kH) {
            float b = 0.f;
            for (int r = 0; r < kTile; ++r) b += sD[r * kLd + threadIdx.x];
            g[s.o_b2 + threadIdx.x] = b;
        }
        float d[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) d[q] = 0.f;
        const float *W2 = p + s.o_w2;
        for (int c = 0; c < kH; ++c) {
            const float dz = sD[tr * kLd + c];
#pragma unroll
            for (int q = 0; q < 16; ++q) d[q] = __builtin_fmaf(dz, W2[int64_t(c0 + q) * kH + c], d[q]);
        }
        __syncthreads();   // everyone has read sD and sH2 of this layer
#pragma unroll
        for (int q = 0; q < 16; ++q) sH2[tr * kLd + c0 + q] = sH1[tr * kLd + c0 + q] > 0.f ? d[q] : 0.f;
    }
    __syncthreads();
    // layer 1: dW1 = X^T dZ1, db1
    {
        if (tr < s.d_in) {
            float acc[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = 0.f;
            for (int r = 0; r < kTile; ++r) {
                const float xv = sX[r * kLd + tr];
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[q] = __builtin_fmaf(xv, sH2[r * kLd + c0 + q], acc[q]);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) g[s.o_w1 + int64_t(tr) * kH + c0 + q] = acc[q];
        }
        if (threadIdx.x < kH) {
            float b = 0.f;
            for (int r = 0; r < kTile; ++r) b += sH2[r * kLd + threadIdx.x];
            g[s.o_b1 + threadIdx.x] = b;
        }
    }
}

// grad[q] = (sum over tiles in tile order of part[t][q]) / sum(M); loss likewise.
__global__ void mlp_reduce_kernel(int64_t n_params, int32_t tiles, const float *__restrict__ part,
                                  float *__restrict__ grad, float *__restrict__ loss) {
    const int64_t stride = n_params + 2;
    float msum = 0.f;
    for (int t = 0; t < tiles; ++t) msum += part[t * stride + n_params + 1];
    const float inv = msum > 0.f ? 1.f / msum : 0.f;
    for (int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; q <= n_params; q += int64_t(gridDim.x) * blockDim.x) {
        float acc = 0.f;
        for (int t = 0; t < tiles; ++t) acc += part[t * stride + q];
        if (q < n_params) grad[q] = acc * inv;
        else if (loss) *loss = acc * inv;
    }
}

__global__ void mlp_adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                                float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
    for (int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + (1.f - b1) * gq;
        const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
    }
}

int check_dims(int32_t d_in, int32_t d_out, int64_t batch) {
    if (d_in < 1 || d_in > kH || d_out < 1 || d_out > kH)
        return fail(PJDS_ERR_ARG, "d_in and d_out must lie in [1, 64] (got %d, %d)", d_in, d_out);
    if (batch < 0) return fail(PJDS_ERR_ARG, "negative batch");
    if ((batch + kTile - 1) / kTile > INT32_MAX) return fail(PJDS_ERR_OVERFLOW, "batch too large");
    return PJDS_OK;
}

int status(const char *what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PJDS_OK : fail(PJDS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace
}  // namespace pjds

using namespace pjds;

extern "C" {

int mlp_param_count(int32_t d_in, int32_t d_out, int64_t *n) {
    if (int rc = check_dims(d_in, d_out, 0)) return rc;
    if (!n) return fail(PJDS_ERR_ARG, "n is NULL");
    *n = shapes(d_in, d_out).n_params;
    return PJDS_OK;
}

int mlp_workspace_size(int32_t d_in, int32_t d_out, int64_t batch, int64_t *bytes) {
    if (int rc = check_dims(d_in, d_out, batch)) return rc;
    if (!bytes) return fail(PJDS_ERR_ARG, "bytes is NULL");
    *bytes = ((batch + kTile - 1) / kTile) * (shapes(d_in, d_out).n_params + 2) * int64_t(sizeof(float));
    return PJDS_OK;
}

int mlp_forward(const float *d_params, int32_t d_in, int32_t d_out, int64_t batch, const float *d_X,
                float *d_P, void *stream) {
    if (int rc = check_dims(d_in, d_out, batch)) return rc;
    if (batch == 0) return PJDS_OK;
    if (!d_params || !d_X || !d_P) return fail(PJDS_ERR_ARG, "NULL device array");
    const Shapes s = shapes(d_in, d_out);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(unsigned((batch + kTile - 1) / kTile)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), s, d_params, d_X, batch, d_P);
    return status("mlp_forward");
}

int mlp_backward(const float *d_params, int32_t d_in, int32_t d_out, int64_t batch, const float *d_X,
                 const float *d_T, const float *d_M, float *d_grad, float *d_loss, void *d_work, void *stream) {
    if (int rc = check_dims(d_in, d_out, batch)) return rc;
    if (batch == 0) return fail(PJDS_ERR_ARG, "empty batch");
    if (!d_params || !d_X || !d_T || !d_M || !d_grad || !d_work) return fail(PJDS_ERR_ARG, "NULL device array");
    const Shapes s = shapes(d_in, d_out);
    const int32_t tiles = int32_t((batch + kTile - 1) / kTile);
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *part = static_cast<float *>(d_work);
    hipLaunchKernelGGL(mlp_backward_tile_kernel, dim3(unsigned(tiles)), dim3(kThreads), 0, st, s, d_params, d_X,
                       d_T, d_M, batch, part);
    const unsigned g = unsigned(std::min<int64_t>((s.n_params + 1 + 255) / 256, 1024));
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(g), dim3(256), 0, st, s.n_params, tiles, part, d_grad, d_loss);
    return status("mlp_backward");
}

int mlp_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t n, int32_t step,
                  float lr, float beta1, float beta2, float eps, void *stream) {
    if (n < 0 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(PJDS_ERR_ARG, "bad Adam arguments");
    if (n == 0) return PJDS_OK;
    if (!d_params || !d_grad || !d_m || !d_v) return fail(PJDS_ERR_ARG, "NULL device array");
    // bias corrections 1 - beta^step, evaluated on the host in binary64
    double p1 = 1.0, p2 = 1.0;
    for (int32_t q = 0; q < step; ++q) { p1 *= beta1; p2 *= beta2; }
    const float c1 = float(1.0 - p1), c2 = float(1.0 - p2);
    const unsigned g = unsigned(std::min<int64_t>((n + 255) / 256, 1024));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(g), dim3(256), 0, static_cast<hipStream_t>(stream), d_params, d_grad,
                       d_m, d_v, n, lr, beta1, beta2, eps, c1, c2);
    return status("mlp_adam_step");
}

int mlp_infer(const float *d_params, int32_t d_in, int32_t d_out, int64_t batch, const float *d_X,
              const float *d_scale, const float *d_shift, const float *d_valid, int32_t *d_idx,
              float *d_margin, void *stream) {
    if (int rc = check_dims(d_in, d_out, batch)) return rc;
    if (batch == 0) return PJDS_OK;
    if (!d_params || !d_X || !d_idx || !d_margin) return fail(PJDS_ERR_ARG, "NULL device array");
    const Shapes s = shapes(d_in, d_out);
    hipLaunchKernelGGL(mlp_infer_kernel, dim3(unsigned((batch + kTile - 1) / kTile)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), s, d_params, d_X, batch, d_scale, d_shift, d_valid, d_idx,
                       d_margin);
    return status("mlp_infer");
}

}  // extern "C"
