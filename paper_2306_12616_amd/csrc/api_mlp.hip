// C ABI of the learned chemical potential network (forward, backward, Adam).
#include <cmath>
#include <string>

#include "ctx.h"
#include "internal.h"

using namespace chebdm;

namespace {

int ensure_mlp_work(chebdm_handle h, int64_t floats) {
    if (h->mlp_work && floats <= h->mlp_work_floats) return 0;
    if (h->mlp_work) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(hipFree(h->mlp_work));
        h->mlp_work = nullptr;
    }
    if (hipMalloc((void**)&h->mlp_work, sizeof(float) * (size_t)floats) != hipSuccess) {
        h->mlp_work = nullptr;
        (void)hipGetLastError();
        return fail(CHEBDM_ERR_OOM, "cannot allocate the network workspace");
    }
    h->mlp_work_floats = floats;
    return 0;
}

}  // namespace

extern "C" {

int chebdm_mlp_num_params(void) { return (int)mlp_nparams(); }

int chebdm_mlp_forward(chebdm_handle h, const float* dW, const float* dX, int32_t batch, float* dY) {
    if (!h || !dW || !dX || !dY) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (batch < 1) return fail(CHEBDM_ERR_ARG, "batch must be >= 1");
    HIP_TRY(hipSetDevice(h->device));
    CHECK(ensure_mlp_work(h, 2 * (int64_t)batch * 256));
    HIP_TRY(launch_mlp_forward(dW, dX, batch, dY, h->mlp_work, h->stream));
    return CHEBDM_OK;
}

int chebdm_mlp_backward(chebdm_handle h, const float* dW, const float* dX, const float* dT, int32_t batch,
                        float* dGrad, float* loss_out) {
    if (!h || !dW || !dX || !dT || !dGrad) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (batch < 1) return fail(CHEBDM_ERR_ARG, "batch must be >= 1");
    HIP_TRY(hipSetDevice(h->device));
    const int64_t floats = 4 * (int64_t)batch * 256 + 2 * (int64_t)batch + 1;
    CHECK(ensure_mlp_work(h, floats));
    float* loss = h->mlp_work + floats - 1;
    HIP_TRY(launch_mlp_backward(dW, dX, dT, batch, dGrad, h->mlp_work, loss, h->stream));
    if (loss_out) {
        HIP_TRY(hipMemcpyAsync(loss_out, loss, sizeof(float), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return CHEBDM_OK;
}

int chebdm_mlp_adam(chebdm_handle h, float* dW, const float* dGrad, float* dM, float* dV, int32_t step, float lr,
                    float beta1, float beta2, float eps) {
    if (!h || !dW || !dGrad || !dM || !dV) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f))
        return fail(CHEBDM_ERR_ARG, "bad Adam hyper-parameters");
    HIP_TRY(hipSetDevice(h->device));
    const float bc1 = (float)(1.0 - std::pow((double)beta1, step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, step));
    HIP_TRY(launch_mlp_adam(dW, dGrad, dM, dV, mlp_nparams(), lr, beta1, beta2, eps, bc1, bc2, h->stream));
    return CHEBDM_OK;
}

}  // extern "C"
