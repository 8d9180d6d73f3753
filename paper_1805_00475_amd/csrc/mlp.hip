// Training and inference kernels of the order-scoring perceptron (fp32):
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3
// over rows x of pair features. The loss is listwise: the rows of a group
// are the candidate pairs of one state of a teacher's order, some of them
// marked as merges the teacher makes next; per group
//   L = log sum_all exp(y) - log sum_pos exp(y),
// averaged over groups. Gradients go through the three layers by hand;
// parameter gradients are summed over rows with float atomics. Adam updates
// the packed parameters in place. Every buffer belongs to the caller.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"
#include "learned.hpp"

namespace tn {

namespace {

constexpr int F = kFeatures, H = kHidden;

__global__ __launch_bounds__(256) void k_fill(float* p, int64_t n, float v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// layer 1: one thread per (row, unit)
__global__ __launch_bounds__(256) void k_fwd1(const float* P, const float* X, int64_t n, float* H1) {
    __shared__ float w[H * F + H];
    for (int t = threadIdx.x; t < H * F + H; t += blockDim.x) w[t] = P[kOffW1 + t];  // W1 then b1
    __syncthreads();
    const int64_t total = n * H;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = e / H;
        const int j = int(e % H);
        float a = w[H * F + j];
#pragma unroll
        for (int k = 0; k < F; ++k) a += w[j * F + k] * X[i * F + k];
        H1[e] = a > 0.0f ? a : 0.0f;
    }
}

// out[i][j] = relu?(sum_k In[i][k] M[j][k] + bias[j]) with M = W2 (transpose
// = false: forward) or out[i][k] = sum_j In[i][j] W2[j][k] masked by
// Mask[i][k] > 0 (backward through layer 2). 32 rows per block, the weight
// matrix staged in LDS in the orientation that keeps reads conflict-free.
template <bool FORWARD>
__global__ __launch_bounds__(256) void k_dense(const float* P, const float* In, const float* Mask, int64_t n,
                                               float* Out) {
    __shared__ float wt[H * H];  // wt[k][j]: contribution of input k to output j
    __shared__ float rows[32][H];
    const float* W2 = P + kOffW2;
    for (int t = threadIdx.x; t < H * H; t += blockDim.x) {
        const int a = t / H, b = t % H;
        // forward: out j = sum_k W2[j][k] in k  -> wt[k][j] = W2[j][k]
        // backward: out k = sum_j W2[j][k] in j -> wt[j][k] = W2[j][k]
        if (FORWARD)
            wt[b * H + a] = W2[a * H + b];
        else
            wt[a * H + b] = W2[a * H + b];
    }
    const int j = threadIdx.x & (H - 1);
    const int r0 = threadIdx.x >> 7;  // 0 or 1
    for (int64_t base = int64_t(blockIdx.x) * 32; base < n; base += int64_t(gridDim.x) * 32) {
        __syncthreads();
        for (int t = threadIdx.x; t < 32 * H; t += blockDim.x) {
            const int64_t i = base + t / H;
            rows[t / H][t % H] = i < n ? In[i * H + t % H] : 0.0f;
        }
        __syncthreads();
        for (int r = r0; r < 32; r += 2) {
            const int64_t i = base + r;
            if (i >= n) break;
            float a = FORWARD ? P[kOffB2 + j] : 0.0f;
#pragma unroll 8
            for (int k = 0; k < H; ++k) a += rows[r][k] * wt[k * H + j];
            if (FORWARD) {
                Out[i * H + j] = a > 0.0f ? a : 0.0f;
            } else {
                Out[i * H + j] = Mask[i * H + j] > 0.0f ? a : 0.0f;
            }
        }
    }
}

// layer 3: one wavefront per row
__global__ __launch_bounds__(256) void k_fwd3(const float* P, const float* H2, int64_t n, float* y) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); i < n; i += int64_t(gridDim.x) * 4) {
        float a = P[kOffW3 + lane] * H2[i * H + lane] + P[kOffW3 + lane + 64] * H2[i * H + lane + 64];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if (lane == 0) y[i] = a + P[kOffB3];
    }
}

// listwise loss per group: dy = (softmax_all - softmax_pos) / G
__global__ __launch_bounds__(256) void k_loss(const float* y, const uint8_t* lab, const int32_t* groups, int32_t G,
                                              float* dy, float* loss) {
    __shared__ float red[3][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int32_t g = blockIdx.x; g < G; g += gridDim.x) {
        const int64_t b = groups[g], e = groups[g + 1];
        float mx = -INFINITY;
        for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) mx = fmaxf(mx, y[i]);
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        if (lane == 0) red[0][wv] = mx;
        __syncthreads();
        mx = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
        float sa = 0.0f, sp = 0.0f;
        for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
            const float ex = expf(y[i] - mx);
            sa += ex;
            if (lab[i]) sp += ex;
        }
        for (int o = 32; o > 0; o >>= 1) {
            sa += __shfl_xor(sa, o);
            sp += __shfl_xor(sp, o);
        }
        __syncthreads();
        if (lane == 0) {
            red[1][wv] = sa;
            red[2][wv] = sp;
        }
        __syncthreads();
        sa = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        sp = red[2][0] + red[2][1] + red[2][2] + red[2][3];
        const float inv_g = 1.0f / float(G);
        for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
            const float ex = expf(y[i] - mx);
            const float d = ex / sa - (lab[i] && sp > 0.0f ? ex / sp : 0.0f);
            dy[i] = sp > 0.0f ? d * inv_g : 0.0f;
        }
        if (threadIdx.x == 0 && sp > 0.0f) atomicAdd(loss, (logf(sa) - logf(sp)) * inv_g);
        __syncthreads();
    }
}

// dZ2[i][j] = dy[i] w3[j] [h2 > 0]; gradients of w3 and b3
__global__ __launch_bounds__(256) void k_bwd3(const float* P, const float* H2, const float* dy, int64_t n, float* dZ2,
                                              float* grad) {
    const int j = threadIdx.x & (H - 1);
    const int r0 = threadIdx.x >> 7;
    float gw = 0.0f, gb = 0.0f;
    for (int64_t i = int64_t(blockIdx.x) * 2 + r0; i < n; i += int64_t(gridDim.x) * 2) {
        const float h = H2[i * H + j];
        const float d = dy[i];
        dZ2[i * H + j] = h > 0.0f ? d * P[kOffW3 + j] : 0.0f;
        gw += d * h;
        if (j == 0) gb += d;
    }
    atomicAdd(&grad[kOffW3 + j], gw);
    if (j == 0) atomicAdd(&grad[kOffB3], gb);
}

// parameter gradient of a dense layer: G[j][k] += sum_i D[i][j] In[i][k],
// Gb[j] += sum_i D[i][j]; K inputs per row (H or F), 64 rows per block
template <int K>
__global__ __launch_bounds__(256) void k_wgrad(const float* D, const float* In, int64_t n, float* Gw, float* Gb) {
    __shared__ float sd[64][H];
    __shared__ float si[64][K];
    constexpr int OUT = H * (K + 1);  // weights and bias
    float acc[(OUT + 255) / 256];
#pragma unroll
    for (int q = 0; q < (OUT + 255) / 256; ++q) acc[q] = 0.0f;
    for (int64_t base = int64_t(blockIdx.x) * 64; base < n; base += int64_t(gridDim.x) * 64) {
        __syncthreads();
        for (int t = threadIdx.x; t < 64 * H; t += blockDim.x) {
            const int64_t i = base + t / H;
            sd[t / H][t % H] = i < n ? D[i * H + t % H] : 0.0f;
        }
        for (int t = threadIdx.x; t < 64 * K; t += blockDim.x) {
            const int64_t i = base + t / K;
            si[t / K][t % K] = i < n ? In[i * K + t % K] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (OUT + 255) / 256; ++q) {
            const int o = threadIdx.x + 256 * q;
            if (o >= OUT) break;
            const int j = o / (K + 1), k = o % (K + 1);
            float a = 0.0f;
            if (k < K) {
                for (int r = 0; r < 64; ++r) a += sd[r][j] * si[r][k];
            } else {
                for (int r = 0; r < 64; ++r) a += sd[r][j];
            }
            acc[q] += a;
        }
    }
#pragma unroll
    for (int q = 0; q < (OUT + 255) / 256; ++q) {
        const int o = threadIdx.x + 256 * q;
        if (o >= OUT) break;
        const int j = o / (K + 1), k = o % (K + 1);
        if (k < K)
            atomicAdd(&Gw[j * K + k], acc[q]);
        else
            atomicAdd(&Gb[j], acc[q]);
    }
}

__global__ __launch_bounds__(256) void k_adam(float* P, const float* g, float* m, float* v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

uint32_t blocks_for(int64_t work, int64_t per, uint32_t cap) {
    return uint32_t(std::max<int64_t>(1, std::min<int64_t>((work + per - 1) / per, cap)));
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_mlp_forward(const float* P, const float* X, int64_t n, float* H1, float* H2, float* y, void* stream_) {
    if (!P || n < 0 || (n > 0 && (!X || !H1 || !H2 || !y))) return TN_EINVAL;
    if (n == 0) return TN_OK;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    hipLaunchKernelGGL(k_fwd1, dim3(blocks_for(n * H, 256, 65535)), dim3(256), 0, s, P, X, n, H1);
    hipLaunchKernelGGL(k_dense<true>, dim3(blocks_for(n, 32, 4096)), dim3(256), 0, s, P, H1, nullptr, n, H2);
    hipLaunchKernelGGL(k_fwd3, dim3(blocks_for(n, 4, 65535)), dim3(256), 0, s, P, H2, n, y);
    return hipGetLastError() == hipSuccess ? TN_OK : TN_EHIP;
}

tn_status tn_mlp_backward(const float* P, const float* X, const float* H1, const float* H2, const float* y,
                          const uint8_t* labels, const int32_t* groups, int32_t n_groups, int64_t n, float* grad,
                          float* dZ2, float* dZ1, float* dy, float* loss, void* stream_) {
    if (!P || !grad || !loss || n < 0 || n_groups < 0) return TN_EINVAL;
    if (n > 0 && (!X || !H1 || !H2 || !y || !labels || !groups || !dZ2 || !dZ1 || !dy)) return TN_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(kParams, 256, 1024)), dim3(256), 0, s, grad, int64_t(kParams), 0.0f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, s, loss, int64_t(1), 0.0f);
    if (n == 0 || n_groups == 0) return hipGetLastError() == hipSuccess ? TN_OK : TN_EHIP;
    hipLaunchKernelGGL(k_loss, dim3(uint32_t(std::min<int32_t>(n_groups, 65535))), dim3(256), 0, s, y, labels, groups,
                       n_groups, dy, loss);
    hipLaunchKernelGGL(k_bwd3, dim3(blocks_for(n, 2, 8192)), dim3(256), 0, s, P, H2, dy, n, dZ2, grad);
    hipLaunchKernelGGL(k_wgrad<H>, dim3(blocks_for(n, 64, 1024)), dim3(256), 0, s, dZ2, H1, n, grad + kOffW2,
                       grad + kOffB2);
    hipLaunchKernelGGL(k_dense<false>, dim3(blocks_for(n, 32, 4096)), dim3(256), 0, s, P, dZ2, H1, n, dZ1);
    hipLaunchKernelGGL(k_wgrad<F>, dim3(blocks_for(n, 64, 1024)), dim3(256), 0, s, dZ1, X, n, grad + kOffW1,
                       grad + kOffB1);
    return hipGetLastError() == hipSuccess ? TN_OK : TN_EHIP;
}

tn_status tn_mlp_adam(float* P, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                      float beta2, float eps, void* stream_) {
    if (!P || !grad || !m || !v || step < 1) return TN_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    const float c1 = 1.0f - std::pow(beta1, float(step)), c2 = 1.0f - std::pow(beta2, float(step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(kParams, 256, 1024)), dim3(256), 0, s, P, grad, m, v, int64_t(kParams),
                       lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? TN_OK : TN_EHIP;
}

}  // extern "C"
