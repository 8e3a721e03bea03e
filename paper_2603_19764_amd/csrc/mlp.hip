// Small multilayer perceptron 4 -> 64 -> 64 -> 1 (tanh, tanh, logistic) that
// maps an impact (log total mass, impact speed over escape speed, mass
// ratio, strength flag; standardised) to the largest-remnant mass fraction.
// Forward, backward (mean squared error) and Adam update as gfx950 kernels,
// all in float.  Parameters live in one flat array:
//   W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3[1]  (4545 values).
// The layers are far too small for matrix cores (a batch of a few hundred
// samples is a few million multiply-adds); one thread per sample with the
// weights broadcast from LDS, and one thread per parameter for the batch
// reductions (fixed sample order, deterministic).
#include "sph_internal.h"

namespace sph {

constexpr int kIn = 4, kHid = 64;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid,
              kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid,
              kNumParams = kOffB3 + 1;
static_assert(kNumParams == 4545, "parameter count");

__device__ __forceinline__ float logistic(float z) { return 1.0f / (1.0f + expf(-z)); }

// out[s] = sigma(W3 tanh(W2 tanh(W1 x_s + b1) + b2) + b3); keeps h1, h2 for
// the backward pass when they are given.
__global__ __launch_bounds__(256) void k_mlp_forward(int32_t B, const float *__restrict__ X,
                                                     const float *__restrict__ P,
                                                     float *__restrict__ out,
                                                     float *__restrict__ H1,
                                                     float *__restrict__ H2) {
    __shared__ float w[kNumParams];
    for (int k = threadIdx.x; k < kNumParams; k += blockDim.x) w[k] = P[k];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float x[kIn];
    for (int c = 0; c < kIn; ++c) x[c] = X[s * kIn + c];
    float h1[kHid];
#pragma unroll
    for (int k = 0; k < kHid; ++k) {
        float z = w[kOffB1 + k];
        for (int c = 0; c < kIn; ++c) z += w[kOffW1 + k * kIn + c] * x[c];
        h1[k] = tanhf(z);
        if (H1) H1[s * kHid + k] = h1[k];
    }
    float z3 = w[kOffB3];
    for (int j = 0; j < kHid; ++j) {
        float z = w[kOffB2 + j];
#pragma unroll
        for (int k = 0; k < kHid; ++k) z += w[kOffW2 + j * kHid + k] * h1[k];
        const float h2 = tanhf(z);
        if (H2) H2[s * kHid + j] = h2;
        z3 += w[kOffW3 + j] * h2;
    }
    out[s] = logistic(z3);
}

// Per-sample error signals of L = (1/B) sum_s (out_s - y_s)^2:
//   d3 = 2/B (out - y) out (1 - out)
//   d2_j = d3 W3_j (1 - h2_j^2)
//   d1_k = (sum_j d2_j W2_jk) (1 - h1_k^2)
__global__ __launch_bounds__(256) void k_mlp_deltas(int32_t B, const float *__restrict__ Y,
                                                    const float *__restrict__ P,
                                                    const float *__restrict__ out,
                                                    const float *__restrict__ H1,
                                                    const float *__restrict__ H2,
                                                    float *__restrict__ D1,
                                                    float *__restrict__ D2,
                                                    float *__restrict__ D3) {
    __shared__ float w[kNumParams];
    for (int k = threadIdx.x; k < kNumParams; k += blockDim.x) w[k] = P[k];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const float o = out[s];
    const float d3 = 2.0f / (float)B * (o - Y[s]) * o * (1.0f - o);
    D3[s] = d3;
    float d2[kHid];
#pragma unroll
    for (int j = 0; j < kHid; ++j) {
        const float h2 = H2[s * kHid + j];
        d2[j] = d3 * w[kOffW3 + j] * (1.0f - h2 * h2);
        D2[s * kHid + j] = d2[j];
    }
    for (int k = 0; k < kHid; ++k) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < kHid; ++j) a += d2[j] * w[kOffW2 + j * kHid + k];
        const float h1 = H1[s * kHid + k];
        D1[s * kHid + k] = a * (1.0f - h1 * h1);
    }
}

// Gradient of every parameter as a sum over samples in sample order.
__global__ void k_mlp_grads(int32_t B, const float *__restrict__ X, const float *__restrict__ H1,
                            const float *__restrict__ H2, const float *__restrict__ D1,
                            const float *__restrict__ D2, const float *__restrict__ D3,
                            float *__restrict__ G) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNumParams) return;
    float g = 0.0f;
    if (p < kOffB1) {  // W1[k][c]
        const int k = p / kIn, c = p % kIn;
        for (int s = 0; s < B; ++s) g += D1[s * kHid + k] * X[s * kIn + c];
    } else if (p < kOffW2) {  // b1[k]
        const int k = p - kOffB1;
        for (int s = 0; s < B; ++s) g += D1[s * kHid + k];
    } else if (p < kOffB2) {  // W2[j][k]
        const int q = p - kOffW2, j = q / kHid, k = q % kHid;
        for (int s = 0; s < B; ++s) g += D2[s * kHid + j] * H1[s * kHid + k];
    } else if (p < kOffW3) {  // b2[j]
        const int j = p - kOffB2;
        for (int s = 0; s < B; ++s) g += D2[s * kHid + j];
    } else if (p < kOffB3) {  // W3[j]
        const int j = p - kOffW3;
        for (int s = 0; s < B; ++s) g += D3[s] * H2[s * kHid + j];
    } else {  // b3
        for (int s = 0; s < B; ++s) g += D3[s];
    }
    G[p] = g;
}

// Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
__global__ void k_mlp_adam(int32_t n, float *__restrict__ P, const float *__restrict__ G,
                           float *__restrict__ M, float *__restrict__ V, int32_t t, float lr,
                           float b1, float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    const float mh = m / (1.0f - powf(b1, (float)t));
    const float vh = v / (1.0f - powf(b2, (float)t));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// loss = (1/B) sum_s (out_s - y_s)^2: one work-group, each thread sums a
// fixed stride of samples, then a fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void k_mlp_loss(int32_t B, const float *__restrict__ out,
                                                  const float *__restrict__ Y,
                                                  float *__restrict__ loss) {
    __shared__ float part[256];
    float a = 0.0f;
    for (int s = threadIdx.x; s < B; s += blockDim.x) {
        const float d = out[s] - Y[s];
        a += d * d;
    }
    part[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = B > 0 ? part[0] / (float)B : 0.0f;
}

}  // namespace sph

using namespace sph;

extern "C" {

int32_t sph_mlp_num_params(void) { return kNumParams; }

sph_status sph_mlp_forward(int32_t batch, const float *X, const float *params, float *out,
                           float *h1, float *h2, sph_stream stream) {
    if (batch < 0 || (batch > 0 && (!X || !params || !out))) return SPH_EINVAL;
    if (batch == 0) return SPH_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((batch + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, batch, X, params, out, h1, h2);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_backward(int32_t batch, const float *X, const float *Y, const float *params,
                            const float *out, const float *h1, const float *h2, float *work,
                            float *grads, sph_stream stream) {
    if (batch < 0 ||
        (batch > 0 && (!X || !Y || !params || !out || !h1 || !h2 || !work || !grads)))
        return SPH_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    float *D1 = work, *D2 = work + (size_t)batch * kHid, *D3 = work + (size_t)2 * batch * kHid;
    if (batch > 0)
        hipLaunchKernelGGL(k_mlp_deltas, dim3((batch + 255) / 256), dim3(256), 0, s, batch, Y,
                           params, out, h1, h2, D1, D2, D3);
    hipLaunchKernelGGL(k_mlp_grads, dim3((kNumParams + 255) / 256), dim3(256), 0, s, batch, X, h1,
                       h2, D1, D2, D3, grads);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_loss(int32_t batch, const float *out, const float *Y, float *loss,
                        sph_stream stream) {
    if (batch < 0 || !loss || (batch > 0 && (!out || !Y))) return SPH_EINVAL;
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, (hipStream_t)stream, batch, out, Y,
                       loss);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_adam(float *params, const float *grads, float *m, float *v, int32_t step,
                        float lr, float beta1, float beta2, float eps, sph_stream stream) {
    if (!params || !grads || !m || !v || step < 1) return SPH_EINVAL;
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNumParams + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, kNumParams, params, grads, m, v, step, lr, beta1,
                       beta2, eps);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}

}  // extern "C"
