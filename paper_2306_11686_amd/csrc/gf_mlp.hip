// gf_mlp.hip -- the launch-config predictor: a 3-layer FP32 MLP
// (8 -> 64 -> ReLU -> 64 -> ReLU -> 32) with hand-written forward, backward,
// masked-MSE loss and Adam kernels, plus a host forward pass for inference
// at launch time. FP32 VALU arithmetic: the network is tiny and latency-bound,
// nothing here is worth a matrix core.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "gf_internal.h"

namespace gf {

constexpr int kIn = GF_MLP_IN;
constexpr int kH = GF_MLP_HIDDEN;
constexpr int kOut = GF_MLP_OUT;
// parameter layout: W1[kH][kIn] b1[kH] W2[kH][kH] b2[kH] W3[kOut][kH] b3[kOut]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kIn;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kOut * kH;
constexpr int kNParams = kOffB3 + kOut;
static_assert(kNParams == GF_MLP_NPARAMS, "parameter count");

constexpr int kMlpThreads = 64;   // one wavefront: thread j owns hidden unit j
constexpr int kSamplesPerBlock = 16;

// Forward pass. Block b handles samples [b*S, b*S+S); thread j computes hidden
// unit j of both layers and (j < kOut) output j, sample by sample, the
// activations of a sample shared through LDS.
__global__ void __launch_bounds__(kMlpThreads) k_mlp_forward(const float *__restrict__ P,
                                                             const float *__restrict__ feats, int32_t batch,
                                                             float *__restrict__ y, float *__restrict__ z1o,
                                                             float *__restrict__ z2o)
{
    __shared__ float s_f[kIn];
    __shared__ float s_a1[kH];
    __shared__ float s_a2[kH];
    const int j = threadIdx.x;
    float w1[kIn], w2[kH];
#pragma unroll
    for (int k = 0; k < kIn; ++k)
        w1[k] = P[kOffW1 + j * kIn + k];
#pragma unroll
    for (int k = 0; k < kH; ++k)
        w2[k] = P[kOffW2 + j * kH + k];
    const float b1 = P[kOffB1 + j], b2 = P[kOffB2 + j];
    const int s0 = blockIdx.x * kSamplesPerBlock;
    for (int s = s0; s < s0 + kSamplesPerBlock && s < batch; ++s) {
        if (j < kIn)
            s_f[j] = feats[(int64_t)s * kIn + j];
        __syncthreads();
        float z1 = b1;
#pragma unroll
        for (int k = 0; k < kIn; ++k)
            z1 += w1[k] * s_f[k];
        if (z1o)
            z1o[(int64_t)s * kH + j] = z1;
        s_a1[j] = z1 > 0.0f ? z1 : 0.0f;
        __syncthreads();
        float z2 = b2;
#pragma unroll
        for (int k = 0; k < kH; ++k)
            z2 += w2[k] * s_a1[k];
        if (z2o)
            z2o[(int64_t)s * kH + j] = z2;
        s_a2[j] = z2 > 0.0f ? z2 : 0.0f;
        __syncthreads();
        if (j < kOut) {
            float o = P[kOffB3 + j];
            for (int k = 0; k < kH; ++k)
                o += P[kOffW3 + j * kH + k] * s_a2[k];
            y[(int64_t)s * kOut + j] = o;
        }
        __syncthreads();
    }
}

// Backward pass of the masked MSE L = sum m (y - t)^2 * inv_norm. Block b
// accumulates the gradients of its samples into its own partial row
// part[b][kNParams] (fixed sample order); k_mlp_sum_grads then sums rows in
// block order, so gradients are deterministic.
__global__ void __launch_bounds__(kMlpThreads) k_mlp_backward(
    const float *__restrict__ P, const float *__restrict__ feats, const float *__restrict__ z1,
    const float *__restrict__ z2, const float *__restrict__ y, const float *__restrict__ tgt,
    const float *__restrict__ mask, int32_t batch, float inv_norm, float *__restrict__ part)
{
    __shared__ float s_f[kIn], s_a1[kH], s_a2[kH], s_dy[kOut], s_dz2[kH], s_dz1[kH];
    const int j = threadIdx.x;
    // per-thread gradient accumulators: row j of W1, W2 and (j < kOut) W3
    float gw1[kIn], gw2[kH], gw3[kH];
#pragma unroll
    for (int k = 0; k < kIn; ++k)
        gw1[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        gw2[k] = 0.0f;
        gw3[k] = 0.0f;
    }
    float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f;
    const int s0 = blockIdx.x * kSamplesPerBlock;
    for (int s = s0; s < s0 + kSamplesPerBlock && s < batch; ++s) {
        const float zz1 = z1[(int64_t)s * kH + j];
        const float zz2 = z2[(int64_t)s * kH + j];
        if (j < kIn)
            s_f[j] = feats[(int64_t)s * kIn + j];
        s_a1[j] = zz1 > 0.0f ? zz1 : 0.0f;
        s_a2[j] = zz2 > 0.0f ? zz2 : 0.0f;
        if (j < kOut) {
            const int64_t o = (int64_t)s * kOut + j;
            s_dy[j] = 2.0f * mask[o] * (y[o] - tgt[o]) * inv_norm;
        }
        __syncthreads();
        // dz2_j = relu'(z2_j) * sum_c W3[c][j] dy_c
        float da2 = 0.0f;
        for (int c = 0; c < kOut; ++c)
            da2 += P[kOffW3 + c * kH + j] * s_dy[c];
        const float dz2 = zz2 > 0.0f ? da2 : 0.0f;
        s_dz2[j] = dz2;
        __syncthreads();
        float da1 = 0.0f;
        for (int i = 0; i < kH; ++i)
            da1 += P[kOffW2 + i * kH + j] * s_dz2[i];
        const float dz1 = zz1 > 0.0f ? da1 : 0.0f;
        s_dz1[j] = dz1;
        // accumulate this sample's gradients
#pragma unroll
        for (int k = 0; k < kIn; ++k)
            gw1[k] += dz1 * s_f[k];
        gb1 += dz1;
#pragma unroll
        for (int k = 0; k < kH; ++k)
            gw2[k] += dz2 * s_a1[k];
        gb2 += dz2;
        if (j < kOut) {
            const float dy = s_dy[j];
#pragma unroll
            for (int k = 0; k < kH; ++k)
                gw3[k] += dy * s_a2[k];
            gb3 += dy;
        }
        __syncthreads();
    }
    float *row = part + (int64_t)blockIdx.x * kNParams;
#pragma unroll
    for (int k = 0; k < kIn; ++k)
        row[kOffW1 + j * kIn + k] = gw1[k];
    row[kOffB1 + j] = gb1;
#pragma unroll
    for (int k = 0; k < kH; ++k)
        row[kOffW2 + j * kH + k] = gw2[k];
    row[kOffB2 + j] = gb2;
    if (j < kOut) {
#pragma unroll
        for (int k = 0; k < kH; ++k)
            row[kOffW3 + j * kH + k] = gw3[k];
        row[kOffB3 + j] = gb3;
    }
}

__global__ void k_mlp_sum_grads(const float *__restrict__ part, int32_t nblocks, float *__restrict__ g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) {
        float acc = 0.0f;
        for (int b = 0; b < nblocks; ++b)
            acc += part[(int64_t)b * kNParams + p];
        g[p] = acc;
    }
}

// Masked MSE: per-block partial sums of m (y - t)^2, summed in block order by
// one thread of the last launch (tiny sizes).
__global__ void __launch_bounds__(256) k_mlp_loss_part(const float *__restrict__ y, const float *__restrict__ tgt,
                                                       const float *__restrict__ mask, int64_t count,
                                                       float *__restrict__ part)
{
    __shared__ float s[256];
    float acc = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = y[i] - tgt[i];
        acc += mask[i] * d * d;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = s[0];
}

__global__ void k_mlp_loss_final(const float *__restrict__ part, int32_t n, float inv_norm, float *__restrict__ loss)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float acc = 0.0f;
        for (int i = 0; i < n; ++i)
            acc += part[i];
        *loss = acc * inv_norm;
    }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int32_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

int mlp_blocks(int32_t batch) { return (batch + kSamplesPerBlock - 1) / kSamplesPerBlock; }

hipError_t launch_mlp_forward(const float *P, const float *feats, int32_t batch, float *y, float *z1, float *z2,
                              hipStream_t s)
{
    if (batch <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_blocks(batch)), dim3(kMlpThreads), 0, s, P, feats, batch, y, z1, z2);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *P, const float *feats, const float *z1, const float *z2, const float *y,
                               const float *tgt, const float *mask, int32_t batch, float inv_norm, float *part,
                               float *grads, hipStream_t s)
{
    const int nb = mlp_blocks(batch);
    hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(kMlpThreads), 0, s, P, feats, z1, z2, y, tgt, mask, batch,
                       inv_norm, part);
    hipLaunchKernelGGL(k_mlp_sum_grads, dim3((kNParams + 255) / 256), dim3(256), 0, s, part, nb, grads);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float *y, const float *tgt, const float *mask, int64_t count, float inv_norm,
                           float *part, float *loss, hipStream_t s)
{
    const int nb = 32;
    hipLaunchKernelGGL(k_mlp_loss_part, dim3(nb), dim3(256), 0, s, y, tgt, mask, count, part);
    hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(64), 0, s, part, nb, inv_norm, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int32_t n, float lr, float b1, float b2, float eps,
                       int32_t t, hipStream_t s)
{
    const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// Host forward pass (FP32, same layer order as the kernel) for single
// launch-time predictions without a device round trip.
void mlp_forward_host(const float *P, const float *f, float *out)
{
    float a1[kH], a2[kH];
    for (int j = 0; j < kH; ++j) {
        float z = P[kOffB1 + j];
        for (int k = 0; k < kIn; ++k)
            z += P[kOffW1 + j * kIn + k] * f[k];
        a1[j] = z > 0.0f ? z : 0.0f;
    }
    for (int j = 0; j < kH; ++j) {
        float z = P[kOffB2 + j];
        for (int k = 0; k < kH; ++k)
            z += P[kOffW2 + j * kH + k] * a1[k];
        a2[j] = z > 0.0f ? z : 0.0f;
    }
    for (int c = 0; c < kOut; ++c) {
        float o = P[kOffB3 + c];
        for (int k = 0; k < kH; ++k)
            o += P[kOffW3 + c * kH + k] * a2[k];
        out[c] = o;
    }
}

}  // namespace gf
