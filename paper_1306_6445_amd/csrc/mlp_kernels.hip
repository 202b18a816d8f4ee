// Training and inference kernels of the 3-64-64-3 tanh surrogate network
// (declared in include/lbm_mlp.h).
//
// A workgroup of 256 threads (four wave64s) owns a chunk of 32 samples: the
// parameters, the chunk's inputs and both hidden layers sit in LDS, so one
// launch runs the whole forward pass and backpropagation for the chunk and
// writes the chunk's gradient (plus its share of the loss) to a per-chunk
// slot.  A second kernel sums the chunk gradients in a fixed order and applies
// the Adam update, so results do not depend on scheduling.
//
// Thread mapping: for [sample][unit] arrays a wave takes one sample row at a
// time and its 64 lanes take the 64 units, so the sample's activations are
// broadcast.  W2 and the row-major activations use a padded row stride of 65
// floats: lanes that walk a column (unit j of W2[j][k], sample s of h2[s][j])
// then hit 64 different banks, and lanes that walk a row stay contiguous.
// The whole working set (about 54 KB) fits the default LDS allocation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_kernels.hpp"

namespace lbm {
namespace mlp {

constexpr int CH = 32;      // samples per workgroup
constexpr int LDP = H + 1;  // padded row stride of W2 and the activation arrays
constexpr int NT = 256;     // threads per workgroup

struct Smem {
    float W1[H * IN], b1[H], W2[H * LDP], b2[H], W3[OUT * H], b3[4];
    float x[CH * IN];
    float h1[CH * LDP], h2[CH * LDP], dz2[CH * LDP], dz1[CH * LDP];
    float dy[OUT * CH];  // [k][s]
    float red[NT];
};

__device__ __forceinline__ void load_params(Smem &S, const float *__restrict__ th)
{
    const int t = threadIdx.x;
    for (int i = t; i < H * IN; i += NT) S.W1[i] = th[OFF_W1 + i];
    for (int i = t; i < H; i += NT) {
        S.b1[i] = th[OFF_B1 + i];
        S.b2[i] = th[OFF_B2 + i];
    }
    for (int i = t; i < H * H; i += NT) S.W2[(i / H) * LDP + i % H] = th[OFF_W2 + i];
    for (int i = t; i < OUT * H; i += NT) S.W3[i] = th[OFF_W3 + i];
    if (t < OUT) S.b3[t] = th[OFF_B3 + t];
}

// Inputs of the chunk starting at sample s0 (rows past n are zero).
__device__ __forceinline__ void load_inputs(Smem &S, const float *__restrict__ x, int s0, int n)
{
    for (int i = threadIdx.x; i < CH * IN; i += NT) {
        const int s = s0 + i / IN;
        S.x[i] = s < n ? x[(int64_t)s0 * IN + i] : 0.0f;
    }
}

// Both hidden layers of the chunk into S.h1 and S.h2.
__device__ __forceinline__ void hidden_layers(Smem &S)
{
    const int j = threadIdx.x & (H - 1), w = threadIdx.x >> 6;
    for (int s = w; s < CH; s += NT / H) {
        float z = S.b1[j];
#pragma unroll
        for (int i = 0; i < IN; ++i) z += S.W1[j * IN + i] * S.x[s * IN + i];
        S.h1[s * LDP + j] = tanhf(z);
    }
    __syncthreads();
    for (int s = w; s < CH; s += NT / H) {
        float z = S.b2[j];
#pragma unroll 16
        for (int k = 0; k < H; ++k) z += S.W2[j * LDP + k] * S.h1[s * LDP + k];
        S.h2[s * LDP + j] = tanhf(z);
    }
    __syncthreads();
}

// Output k of sample s (threads 0..95: k = t / 32, s = t % 32).
__device__ __forceinline__ float output_unit(const Smem &S, int k, int s)
{
    float y = S.b3[k];
#pragma unroll 16
    for (int j = 0; j < H; ++j) y += S.W3[k * H + j] * S.h2[s * LDP + j];
    return y;
}

__global__ void __launch_bounds__(NT) forward_kernel(const float *__restrict__ th, const float *__restrict__ x, int n,
                                                     float *__restrict__ y)
{
    extern __shared__ float smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const int s0 = blockIdx.x * CH;
    load_params(S, th);
    load_inputs(S, x, s0, n);
    __syncthreads();
    hidden_layers(S);
    const int t = threadIdx.x;
    if (t < OUT * CH) {
        const int k = t / CH, s = t % CH;
        if (s0 + s < n) y[(int64_t)(s0 + s) * OUT + k] = output_unit(S, k, s);
    }
}

// Sum of the weights m over all entries -> inv[0] = 1 / sum (0 when the sum is 0).
__global__ void __launch_bounds__(NT) weight_sum_kernel(const float *__restrict__ m, int n, float *__restrict__ inv)
{
    __shared__ double red[NT];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)n * OUT; i += NT) acc += (double)m[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (unsigned o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) inv[0] = red[0] > 0.0 ? (float)(1.0 / red[0]) : 0.0f;
}

// Loss share and gradient of one chunk: partial[blockIdx.x][P], ploss[blockIdx.x].
__global__ void __launch_bounds__(NT) grad_kernel(const float *__restrict__ th, const float *__restrict__ x,
                                                  const float *__restrict__ tg, const float *__restrict__ mw, int n,
                                                  const float *__restrict__ inv_wsum, float *__restrict__ partial,
                                                  float *__restrict__ ploss)
{
    extern __shared__ float smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const int t = threadIdx.x;
    const int s0 = blockIdx.x * CH;
    float *g = partial + (int64_t)blockIdx.x * P;
    load_params(S, th);
    load_inputs(S, x, s0, n);
    __syncthreads();
    hidden_layers(S);

    // dL/dy = m (y - t) / sum(m); loss share m (y - t)^2 / (2 sum(m))
    const float iw = inv_wsum[0];
    float lsum = 0.0f;
    if (t < OUT * CH) {
        const int k = t / CH, s = t % CH;
        float d = 0.0f;
        if (s0 + s < n) {
            const int64_t e = (int64_t)(s0 + s) * OUT + k;
            const float r = output_unit(S, k, s) - tg[e];
            const float mr = mw[e] * r;
            d = mr * iw;
            lsum = 0.5f * iw * (mr * r);
        }
        S.dy[k * CH + s] = d;
    }
    S.red[t] = lsum;
    __syncthreads();

    // output layer: dW3[k][j] = sum_s dy[k][s] h2[s][j], db3[k] = sum_s dy[k][s]
    if (t < OUT * H) {
        const int k = t >> 6, j = t & (H - 1);
        float acc = 0.0f;
        for (int s = 0; s < CH; ++s) acc += S.dy[k * CH + s] * S.h2[s * LDP + j];
        g[OFF_W3 + k * H + j] = acc;
    } else if (t < OUT * H + OUT) {
        const int k = t - OUT * H;
        float acc = 0.0f;
        for (int s = 0; s < CH; ++s) acc += S.dy[k * CH + s];
        g[OFF_B3 + k] = acc;
    }
    // through tanh: dz2[s][j] = (sum_k W3[k][j] dy[k][s]) (1 - h2[s][j]^2)
    {
        const int j = t & (H - 1), w = t >> 6;
        for (int s = w; s < CH; s += NT / H) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < OUT; ++k) a += S.W3[k * H + j] * S.dy[k * CH + s];
            const float h = S.h2[s * LDP + j];
            S.dz2[s * LDP + j] = a * (1.0f - h * h);
        }
    }
    __syncthreads();

    // hidden layer 2: dW2[j][k] = sum_s dz2[s][j] h1[s][k], db2[j] = sum_s dz2[s][j]
    {
        const int k = t & (H - 1), w = t >> 6;
        for (int j = w; j < H; j += NT / H) {
            float acc = 0.0f;
#pragma unroll 8
            for (int s = 0; s < CH; ++s) acc += S.dz2[s * LDP + j] * S.h1[s * LDP + k];
            g[OFF_W2 + j * H + k] = acc;
        }
        if (t < H) {
            float acc = 0.0f;
            for (int s = 0; s < CH; ++s) acc += S.dz2[s * LDP + t];
            g[OFF_B2 + t] = acc;
        }
        // dz1[s][k] = (sum_j W2[j][k] dz2[s][j]) (1 - h1[s][k]^2)
        for (int s = w; s < CH; s += NT / H) {
            float a = 0.0f;
#pragma unroll 16
            for (int j = 0; j < H; ++j) a += S.W2[j * LDP + k] * S.dz2[s * LDP + j];
            const float h = S.h1[s * LDP + k];
            S.dz1[s * LDP + k] = a * (1.0f - h * h);
        }
    }
    __syncthreads();

    // hidden layer 1: dW1[j][i] = sum_s dz1[s][j] x[s][i], db1[j] = sum_s dz1[s][j]
    if (t < IN * H) {
        const int i = t >> 6, j = t & (H - 1);
        float acc = 0.0f;
        for (int s = 0; s < CH; ++s) acc += S.dz1[s * LDP + j] * S.x[s * IN + i];
        g[OFF_W1 + j * IN + i] = acc;
    } else if (t < IN * H + H) {
        const int j = t - IN * H;
        float acc = 0.0f;
        for (int s = 0; s < CH; ++s) acc += S.dz1[s * LDP + j];
        g[OFF_B1 + j] = acc;
    }
    // the chunk's loss share
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (t < o) S.red[t] += S.red[t + o];
        __syncthreads();
    }
    if (t == 0) ploss[blockIdx.x] = S.red[0];
}

// Sum of the chunk gradients (fixed order); optionally the Adam update
//   m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
//   theta <- theta - lr (c1 m) / (sqrt(c2 v) + eps),  c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void __launch_bounds__(NT) adam_kernel(float *__restrict__ th, float *__restrict__ m1,
                                                  float *__restrict__ m2, const float *__restrict__ partial, int nch,
                                                  float *__restrict__ grad, AdamArgs a)
{
    const int p = blockIdx.x * NT + threadIdx.x;
    if (p >= P) return;
    float g = 0.0f;
    for (int c = 0; c < nch; ++c) g += partial[(int64_t)c * P + p];
    if (grad) grad[p] = g;
    if (!a.update) return;
    const float m = a.beta1 * m1[p] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * m2[p] + (1.0f - a.beta2) * (g * g);
    m1[p] = m;
    m2[p] = v;
    th[p] -= a.lr * (a.c1 * m) / (sqrtf(a.c2 * v) + a.eps);
}

int chunks(int n) { return (n + CH - 1) / CH; }

hipError_t launch_forward(const float *th, const float *x, int n, float *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(forward_kernel, dim3(chunks(n)), dim3(NT), sizeof(Smem), st, th, x, n, y);
    return hipGetLastError();
}

hipError_t launch_weight_sum(const float *m, int n, float *inv, hipStream_t st)
{
    hipLaunchKernelGGL(weight_sum_kernel, dim3(1), dim3(NT), 0, st, m, n, inv);
    return hipGetLastError();
}

hipError_t launch_grad(const float *th, const float *x, const float *tg, const float *mw, int n, const float *inv,
                       float *partial, float *ploss, hipStream_t st)
{
    hipLaunchKernelGGL(grad_kernel, dim3(chunks(n)), dim3(NT), sizeof(Smem), st, th, x, tg, mw, n, inv, partial,
                       ploss);
    return hipGetLastError();
}

hipError_t launch_adam(float *th, float *m1, float *m2, const float *partial, int nch, float *grad, const AdamArgs &a,
                       hipStream_t st)
{
    hipLaunchKernelGGL(adam_kernel, dim3((P + NT - 1) / NT), dim3(NT), 0, st, th, m1, m2, partial, nch, grad, a);
    return hipGetLastError();
}

size_t smem_bytes() { return sizeof(Smem); }
static_assert(sizeof(Smem) <= 64 * 1024, "surrogate kernels fit the default LDS allocation");

} // namespace mlp
} // namespace lbm
