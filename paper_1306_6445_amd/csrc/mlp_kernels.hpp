// Launch interface of the surrogate-network kernels (mlp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace lbm {
namespace mlp {

constexpr int IN = 3, H = 64, OUT = 3;
// offsets of the parameter blocks in the flat vector (row-major, out x in)
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * IN;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + OUT * H;
constexpr int P = OFF_B3 + OUT;
static_assert(P == 4611, "parameter count");

struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2; // c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
    int update;                          // 0: only reduce the gradient
};

int chunks(int n); // workgroups (chunks of samples) for a batch of n
size_t smem_bytes();
hipError_t launch_forward(const float *th, const float *x, int n, float *y, hipStream_t st);
hipError_t launch_weight_sum(const float *m, int n, float *inv, hipStream_t st);
hipError_t launch_grad(const float *th, const float *x, const float *tg, const float *mw, int n, const float *inv,
                       float *partial, float *ploss, hipStream_t st);
hipError_t launch_adam(float *th, float *m1, float *m2, const float *partial, int nch, float *grad, const AdamArgs &a,
                       hipStream_t st);

} // namespace mlp
} // namespace lbm
