// proposal.hip -- C ABI of the learned proposal network (mppi_mlp_*):
// buffers, argument checks and launch sequencing; the arithmetic is in
// mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "mlp.hpp"
#include "mppi.h"

using namespace mppi;

struct mppi_mlp {
    MlpDev d{};
    void* base = nullptr;
    int max_batch = 0;
    long long step = 0;   // Adam steps taken since the parameters were set
};

namespace {

// the Adam arguments of the next step (step count m->step + 1)
int adam_args(const mppi_mlp* m, const mppi_adam_params* p, MlpAdam& a)
{
    if (!p || !(p->lr > 0) || !(p->beta1 >= 0 && p->beta1 < 1) || !(p->beta2 >= 0 && p->beta2 < 1) ||
        !(p->eps > 0))
        return MPPI_EINVAL;
    const long long t = m->step + 1;
    const double c1 = 1.0 / (1.0 - std::pow(p->beta1, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow(p->beta2, (double)t));
    a = MlpAdam{1, (float)p->lr, (float)p->beta1, (float)p->beta2, (float)p->eps, (float)c1, (float)c2};
    return MPPI_OK;
}

int adam_enqueue(mppi_mlp* m, const mppi_adam_params* p, hipStream_t s)
{
    MlpAdam a;
    const int st = adam_args(m, p, a);
    if (st) return st;
    if (launch_mlp_adam(m->d, a, s) != hipSuccess) return MPPI_EDEVICE;
    m->step += 1;
    return MPPI_OK;
}

int grad_enqueue(mppi_mlp* m, const float* x, const float* y_target, int B, float* loss, hipStream_t s)
{
    if (!x || !y_target || B < 1 || B > m->max_batch) return MPPI_EINVAL;
    if (launch_mlp_forward(m->d, x, B, y_target, nullptr, nullptr, 0, s) != hipSuccess ||
        launch_mlp_wgrad(m->d, B, loss, s) != hipSuccess)
        return MPPI_EDEVICE;
    return MPPI_OK;
}

}  // namespace

extern "C" {

int mppi_mlp_create(const mppi_robot_params* robot, int max_batch, mppi_mlp_t* out)
{
    if (!out) return MPPI_EINVAL;
    *out = nullptr;
    if (!robot || robot->n_joints != MPPI_NJ || max_batch < 1 || max_batch > 65536) return MPPI_EINVAL;
    double scale[21];
    for (int j = 0; j < MPPI_NJ; ++j) {
        const mppi_link_params& L = robot->link[j];
        scale[j] = L.q_max;
        scale[7 + j] = L.qd_max;
        scale[14 + j] = L.tau_max;
        for (int c = 0; c < 3; ++c)
            if (!(std::isfinite(scale[7 * c + j]) && scale[7 * c + j] > 0)) return MPPI_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MPPI_EDEVICE;
    mppi_mlp* m = new (std::nothrow) mppi_mlp;
    if (!m) return MPPI_ENOMEM;
    m->max_batch = max_batch;
    const int Bp = (max_batch + kMlpRows - 1) / kMlpRows * kMlpRows;
    const size_t bytes = mlp_scratch_bytes(Bp);
    if (hipMalloc(&m->base, bytes) != hipSuccess) {
        delete m;
        return MPPI_ENOMEM;
    }
    mlp_carve(m->d, m->base, Bp);
    // zero everything (padding rows/columns of the BF16 copies stay zero)
    if (hipMemset(m->base, 0, bytes) != hipSuccess ||
        hipMemcpy((void*)m->d.scale, scale, sizeof scale, hipMemcpyHostToDevice) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(m->base);
        delete m;
        return MPPI_EDEVICE;
    }
    *out = m;
    return MPPI_OK;
}

int mppi_mlp_destroy(mppi_mlp_t m)
{
    if (m) {
        (void)hipDeviceSynchronize();
        (void)hipFree(m->base);
        delete m;
    }
    return MPPI_OK;
}

int mppi_mlp_set_params(mppi_mlp_t m, const float* params, size_t n)
{
    if (!m || !params || n != (size_t)kMlpParams) return MPPI_EINVAL;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return MPPI_EINVAL;
    const size_t b = n * sizeof(float);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(m->d.theta, params, b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->d.m, 0, b) != hipSuccess || hipMemset(m->d.v, 0, b) != hipSuccess ||
        launch_mlp_adam(m->d, MlpAdam{0, 0.f, 0.f, 0.f, 1.f, 1.f, 1.f}, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return MPPI_EDEVICE;
    m->step = 0;
    return MPPI_OK;
}

int mppi_mlp_get_params(mppi_mlp_t m, float* params, size_t n)
{
    if (!m || !params || n != (size_t)kMlpParams) return MPPI_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(params, m->d.theta, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return MPPI_EDEVICE;
    return MPPI_OK;
}

int mppi_mlp_forward_async(mppi_mlp_t m, const float* x, int B, float* y, void* stream)
{
    if (!m || !x || !y || B < 1 || B > m->max_batch) return MPPI_EINVAL;
    return launch_mlp_forward(m->d, x, B, nullptr, y, nullptr, 0, (hipStream_t)stream) == hipSuccess ? MPPI_OK
                                                                                                     : MPPI_EDEVICE;
}

int mppi_mlp_grad_async(mppi_mlp_t m, const float* x, const float* y_target, int B, float* grad, float* loss,
                        void* stream)
{
    if (!m) return MPPI_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    int st = grad_enqueue(m, x, y_target, B, loss, s);
    if (st) return st;
    if (grad &&
        hipMemcpyAsync(grad, m->d.grad, (size_t)kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MPPI_EDEVICE;
    return MPPI_OK;
}

int mppi_mlp_adam_async(mppi_mlp_t m, const mppi_adam_params* p, void* stream)
{
    if (!m) return MPPI_EINVAL;
    return adam_enqueue(m, p, (hipStream_t)stream);
}

int mppi_mlp_train_step_async(mppi_mlp_t m, const float* x, const float* y_target, int B,
                              const mppi_adam_params* p, float* loss, void* stream)
{
    if (!m || !p) return MPPI_EINVAL;
    if (!x || !y_target || B < 1 || B > m->max_batch) return MPPI_EINVAL;
    MlpAdam a;
    const int st = adam_args(m, p, a);
    if (st) return st;
    // two launches: the forward/backward pass, then the weight gradients
    // with the Adam step applied as each gradient tile completes
    const hipStream_t s = (hipStream_t)stream;
    if (launch_mlp_forward(m->d, x, B, y_target, nullptr, nullptr, 0, s) != hipSuccess ||
        launch_mlp_wgrad(m->d, B, loss, s, &a) != hipSuccess)
        return MPPI_EDEVICE;
    m->step += 1;
    return MPPI_OK;
}

int mppi_mlp_propose_async(mppi_mlp_t m, int n, const double* q, const double* qd, const double* target,
                           double* U, int u_stride, void* stream)
{
    if (!m || !q || !qd || !target || !U || n < 1 || n > m->max_batch || u_stride < kMlpOut) return MPPI_EINVAL;
    // one launch: the features are encoded in the forward kernel's input load
    return launch_mlp_forward(m->d, nullptr, n, nullptr, nullptr, U, u_stride, (hipStream_t)stream, q, qd, target) ==
                   hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

int mppi_mlp_encode_async(mppi_mlp_t m, int n, const double* q, const double* qd, const double* target,
                          const double* U, int u_stride, float* x, float* y, void* stream)
{
    if (!m || !q || !qd || !target || !x || n < 1 || (y && (!U || u_stride < kMlpOut))) return MPPI_EINVAL;
    return launch_mlp_features(m->d, n, q, qd, target, x, y ? U : nullptr, u_stride, y, (hipStream_t)stream) ==
                   hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

}  // extern "C"
