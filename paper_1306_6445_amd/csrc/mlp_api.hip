// Host side of the surrogate-network C ABI (include/lbm_mlp.h): workspace
// layout, argument checks and the training loop (one gradient launch and one
// reduction/Adam launch per step on the caller's stream).
#include "../../include/lbm_mlp.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "lbm_error.hpp"
#include "mlp_kernels.hpp"

namespace {

using lbm::set_last_error;
namespace M = lbm::mlp;

lbm_status fail(lbm_status s, const std::string &msg)
{
    set_last_error(msg);
    return s;
}

#define MLP_HIP(call)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t theta, m1, m2, grad, partial, ploss, inv, total;
};

Layout layout(int max_batch)
{
    const int nch = M::chunks(max_batch);
    const size_t pb = sizeof(float) * M::P;
    Layout L;
    size_t o = 0;
    L.theta = o, o += align256(pb);
    L.m1 = o, o += align256(pb);
    L.m2 = o, o += align256(pb);
    L.grad = o, o += align256(pb);
    L.partial = o, o += align256(pb * nch);
    L.ploss = o, o += align256(sizeof(float) * nch);
    L.inv = o, o += align256(sizeof(float));
    L.total = o;
    return L;
}

bool finite_params(const float *p)
{
    for (int i = 0; i < M::P; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

} // namespace

struct lbm_mlp {
    int max_batch = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    uint8_t *ws = nullptr;
    Layout L{};
    int64_t t = 0; // Adam steps taken

    float *f(size_t off) { return reinterpret_cast<float *>(ws + off); }
};

namespace {

lbm_status check_batch(const lbm_mlp *net, int32_t n, bool allow_empty)
{
    if (!net) return fail(LBM_EINVAL, "null network");
    if (n < (allow_empty ? 0 : 1) || n > net->max_batch)
        return fail(LBM_EINVAL, "batch size " + std::to_string(n) + " outside [" + (allow_empty ? "0" : "1") +
                                    ", " + std::to_string(net->max_batch) + "]");
    return LBM_OK;
}

// 1 / sum(m) on the device; EINVAL when every weight is zero.
lbm_status weight_sum(lbm_mlp *net, const float *m, int32_t n)
{
    float inv = 0.0f;
    MLP_HIP(M::launch_weight_sum(m, n, net->f(net->L.inv), net->stream));
    MLP_HIP(hipMemcpyAsync(&inv, net->f(net->L.inv), sizeof(float), hipMemcpyDeviceToHost, net->stream));
    MLP_HIP(hipStreamSynchronize(net->stream));
    if (!(inv > 0.0f) || !std::isfinite(inv)) return fail(LBM_EINVAL, "loss weights sum to zero (or are not finite)");
    return LBM_OK;
}

lbm_status read_loss(lbm_mlp *net, int nch, double *loss)
{
    std::vector<float> pl(nch);
    MLP_HIP(hipMemcpyAsync(pl.data(), net->f(net->L.ploss), sizeof(float) * nch, hipMemcpyDeviceToHost,
                           net->stream));
    MLP_HIP(hipStreamSynchronize(net->stream));
    double s = 0.0;
    for (float v : pl) s += v;
    *loss = s;
    return LBM_OK;
}

} // namespace

extern "C" {

size_t lbm_mlp_workspace_bytes(int32_t max_batch)
{
    if (max_batch < 1 || max_batch > LBM_MLP_MAX_BATCH) return 0;
    return layout(max_batch).total;
}

lbm_status lbm_mlp_create(int32_t max_batch, const float *params, void *workspace, size_t workspace_bytes,
                          void *stream, lbm_mlp **out)
{
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    if (max_batch < 1 || max_batch > LBM_MLP_MAX_BATCH) return fail(LBM_EINVAL, "max_batch out of range");
    if (!params) return fail(LBM_EINVAL, "initial parameters are required");
    if (!finite_params(params)) return fail(LBM_EINVAL, "initial parameters are not finite");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(LBM_EINVAL, "workspace must be a 256-byte aligned device pointer");
    const Layout L = layout(max_batch);
    if (workspace_bytes < L.total)
        return fail(LBM_EINVAL, "workspace too small: need " + std::to_string(L.total) + " bytes");
    lbm_mlp *net = new (std::nothrow) lbm_mlp;
    if (!net) return fail(LBM_ENOMEM, "host allocation failed");
    net->max_batch = max_batch;
    net->ws = static_cast<uint8_t *>(workspace);
    net->L = L;
    net->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&net->device) != hipSuccess) {
        delete net;
        return fail(LBM_EDEVICE, "hipGetDevice failed");
    }
    lbm_status s = lbm_mlp_set_params(net, params);
    if (s != LBM_OK) {
        delete net;
        return s;
    }
    *out = net;
    return LBM_OK;
}

lbm_status lbm_mlp_set_params(lbm_mlp *net, const float *params)
{
    if (!net || !params) return fail(LBM_EINVAL, "null argument");
    if (!finite_params(params)) return fail(LBM_EINVAL, "parameters are not finite");
    MLP_HIP(hipSetDevice(net->device));
    const size_t pb = sizeof(float) * M::P;
    MLP_HIP(hipMemcpyAsync(net->f(net->L.theta), params, pb, hipMemcpyHostToDevice, net->stream));
    MLP_HIP(hipMemsetAsync(net->f(net->L.m1), 0, pb, net->stream));
    MLP_HIP(hipMemsetAsync(net->f(net->L.m2), 0, pb, net->stream));
    MLP_HIP(hipStreamSynchronize(net->stream));
    net->t = 0;
    return LBM_OK;
}

lbm_status lbm_mlp_get_params(lbm_mlp *net, float *params)
{
    if (!net || !params) return fail(LBM_EINVAL, "null argument");
    MLP_HIP(hipSetDevice(net->device));
    MLP_HIP(hipMemcpyAsync(params, net->f(net->L.theta), sizeof(float) * M::P, hipMemcpyDeviceToHost, net->stream));
    MLP_HIP(hipStreamSynchronize(net->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_mlp *net, const float *x, int32_t n, float *y)
{
    lbm_status s = check_batch(net, n, true);
    if (s != LBM_OK) return s;
    if (n == 0) return LBM_OK;
    if (!x || !y) return fail(LBM_EINVAL, "null input or output");
    MLP_HIP(hipSetDevice(net->device));
    MLP_HIP(M::launch_forward(net->f(net->L.theta), x, n, y, net->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_loss_grad(lbm_mlp *net, const float *x, const float *t, const float *m, int32_t n, double *loss,
                             float *grad)
{
    lbm_status s = check_batch(net, n, false);
    if (s != LBM_OK) return s;
    if (!x || !t || !m || !loss) return fail(LBM_EINVAL, "null argument");
    MLP_HIP(hipSetDevice(net->device));
    if ((s = weight_sum(net, m, n)) != LBM_OK) return s;
    const int nch = M::chunks(n);
    MLP_HIP(M::launch_grad(net->f(net->L.theta), x, t, m, n, net->f(net->L.inv), net->f(net->L.partial),
                           net->f(net->L.ploss), net->stream));
    M::AdamArgs a{};
    a.update = 0;
    MLP_HIP(M::launch_adam(net->f(net->L.theta), net->f(net->L.m1), net->f(net->L.m2), net->f(net->L.partial), nch,
                           net->f(net->L.grad), a, net->stream));
    if (grad)
        MLP_HIP(hipMemcpyAsync(grad, net->f(net->L.grad), sizeof(float) * M::P, hipMemcpyDeviceToHost,
                               net->stream));
    return read_loss(net, nch, loss);
}

lbm_status lbm_mlp_train(lbm_mlp *net, const float *x, const float *t, const float *m, int32_t n, int32_t steps,
                         float lr, float beta1, float beta2, float eps, double *last_loss)
{
    lbm_status s = check_batch(net, n, false);
    if (s != LBM_OK) return s;
    if (!x || !t || !m) return fail(LBM_EINVAL, "null argument");
    if (steps < 0) return fail(LBM_EINVAL, "negative step count");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(LBM_EINVAL, "learning rate must be positive");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(LBM_EINVAL, "Adam decay rates must lie in [0, 1)");
    if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(LBM_EINVAL, "Adam eps must be positive");
    MLP_HIP(hipSetDevice(net->device));
    if ((s = weight_sum(net, m, n)) != LBM_OK) return s;
    const int nch = M::chunks(n);
    for (int32_t k = 0; k < steps; ++k) {
        const int64_t tt = net->t + 1;
        M::AdamArgs a;
        a.lr = lr;
        a.beta1 = beta1;
        a.beta2 = beta2;
        a.eps = eps;
        a.c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)tt)));
        a.c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)tt)));
        a.update = 1;
        MLP_HIP(M::launch_grad(net->f(net->L.theta), x, t, m, n, net->f(net->L.inv), net->f(net->L.partial),
                               net->f(net->L.ploss), net->stream));
        MLP_HIP(M::launch_adam(net->f(net->L.theta), net->f(net->L.m1), net->f(net->L.m2), net->f(net->L.partial),
                               nch, nullptr, a, net->stream));
        net->t = tt;
    }
    if (last_loss) {
        if (steps == 0) return fail(LBM_EINVAL, "no step taken, no loss to report");
        return read_loss(net, nch, last_loss);
    }
    MLP_HIP(hipStreamSynchronize(net->stream));
    return LBM_OK;
}

int64_t lbm_mlp_steps_taken(const lbm_mlp *net) { return net ? net->t : -1; }

void lbm_mlp_destroy(lbm_mlp *net) { delete net; }

} // extern "C"
