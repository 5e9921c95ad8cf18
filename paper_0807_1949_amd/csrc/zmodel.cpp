// Trainer of the learned impedance model (C ABI part): device-resident
// training data, minibatch gradients from the BF16 MFMA kernels, Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "mlp.hpp"
#include "vtm.h"

namespace vtm {
std::string &last_error_ref();
}

namespace {

vtm_status tfail(vtm_status code, const std::string &m) {
    vtm::last_error_ref() = m;
    return code;
}

#define TRY(expr)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return tfail(e_ == hipErrorOutOfMemory ? VTM_ERR_OOM : VTM_ERR_HIP,                    \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                       \
    } while (0)

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace

struct vtm_trainer_ctx {
    int32_t device = 0;
    hipStream_t st = nullptr;
    float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *part = nullptr;
    float *X = nullptr, *Y = nullptr, *losses = nullptr;
    int64_t *idx = nullptr;
    int64_t n = 0, cap = 0, step = 0;
    int nparts = 0;
    ~vtm_trainer_ctx() {
        (void)hipSetDevice(device);
        for (void *p : {(void *)P, (void *)m, (void *)v, (void *)g, (void *)part, (void *)X, (void *)Y,
                        (void *)losses, (void *)idx})
            if (p) (void)hipFree(p);
        if (st) (void)hipStreamDestroy(st);
    }
};

extern "C" {

vtm_status vtm_trainer_create(int32_t device, const float *params, vtm_trainer *out) {
    if (!params || !out) return tfail(VTM_ERR_INVALID, "null argument");
    *out = nullptr;
    auto *t = new (std::nothrow) vtm_trainer_ctx();
    if (!t) return tfail(VTM_ERR_OOM, "trainer allocation failed");
    t->device = device;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { delete t; return tfail(VTM_ERR_HIP, hipGetErrorString(e)); }
    t->nparts = 1024;
    if ((e = hipStreamCreateWithFlags(&t->st, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipMalloc(&t->P, sizeof(float) * vtm::kParams)) != hipSuccess ||
        (e = hipMalloc(&t->m, sizeof(float) * vtm::kTrain)) != hipSuccess ||
        (e = hipMalloc(&t->v, sizeof(float) * vtm::kTrain)) != hipSuccess ||
        (e = hipMalloc(&t->g, sizeof(float) * (vtm::kTrain + 1))) != hipSuccess ||
        (e = hipMalloc(&t->part, sizeof(float) * (vtm::kTrain + 1) * t->nparts)) != hipSuccess) {
        delete t;
        return tfail(VTM_ERR_OOM, hipGetErrorString(e));
    }
    for (int i = 0; i < vtm::kNumFeatures; ++i)
        if (!(params[vtm::kNumFeatures + i] > 0.f)) {
            delete t;
            return tfail(VTM_ERR_INVALID, "feature standard deviations must be > 0");
        }
    (void)hipMemcpy(t->P, params, sizeof(float) * vtm::kParams, hipMemcpyHostToDevice);
    (void)hipMemset(t->m, 0, sizeof(float) * vtm::kTrain);
    (void)hipMemset(t->v, 0, sizeof(float) * vtm::kTrain);
    *out = t;
    return VTM_OK;
}

vtm_status vtm_trainer_destroy(vtm_trainer t) {
    delete t;
    return VTM_OK;
}

vtm_status vtm_trainer_set_data(vtm_trainer t, const float *feats, const float *labels, int64_t n) {
    if (!t || !feats || !labels || n < 1) return tfail(VTM_ERR_INVALID, "bad argument");
    TRY(hipSetDevice(t->device));
    if (n > t->cap) {
        if (t->X) (void)hipFree(t->X);
        if (t->Y) (void)hipFree(t->Y);
        if (t->idx) (void)hipFree(t->idx);
        t->X = t->Y = nullptr;
        t->idx = nullptr;
        TRY(hipMalloc(&t->X, sizeof(float) * vtm::kNumFeatures * n));
        TRY(hipMalloc(&t->Y, sizeof(float) * n));
        TRY(hipMalloc(&t->idx, sizeof(int64_t) * n));
        t->cap = n;
    }
    TRY(hipMemcpy(t->X, feats, sizeof(float) * vtm::kNumFeatures * n, hipMemcpyHostToDevice));
    TRY(hipMemcpy(t->Y, labels, sizeof(float) * n, hipMemcpyHostToDevice));
    t->n = n;
    return VTM_OK;
}

vtm_status vtm_trainer_grad(vtm_trainer t, int64_t row0, int64_t nrows, float *grad, float *loss) {
    if (!t || nrows < 1 || row0 < 0 || row0 + nrows > t->n) return tfail(VTM_ERR_INVALID, "bad row range");
    TRY(hipSetDevice(t->device));
    const int np = std::min(t->nparts, vtm::mlp_grid(nrows));
    vtm::launch_mlp_grad(t->P, t->X, t->Y, nullptr, row0, nrows, 1.f / (float)nrows, t->part, np, t->g, t->st);
    std::vector<float> h(vtm::kTrain + 1);
    TRY(hipMemcpyAsync(h.data(), t->g, sizeof(float) * (vtm::kTrain + 1), hipMemcpyDeviceToHost, t->st));
    TRY(hipStreamSynchronize(t->st));
    if (grad) std::copy(h.begin(), h.begin() + vtm::kTrain, grad);
    if (loss) *loss = h[vtm::kTrain] / (float)nrows;
    return VTM_OK;
}

vtm_status vtm_trainer_epoch(vtm_trainer t, int64_t batch, float lr, uint64_t seed, float *loss) {
    if (!t || batch < 1 || !(lr > 0.f) || t->n < 1) return tfail(VTM_ERR_INVALID, "bad argument or no data");
    TRY(hipSetDevice(t->device));
    // Fisher-Yates shuffle driven by splitmix64
    std::vector<int64_t> perm(t->n);
    for (int64_t i = 0; i < t->n; ++i) perm[i] = i;
    uint64_t s = seed;
    for (int64_t i = t->n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(splitmix(s) % (uint64_t)(i + 1))]);
    TRY(hipMemcpyAsync(t->idx, perm.data(), sizeof(int64_t) * t->n, hipMemcpyHostToDevice, t->st));
    const int64_t nb = (t->n + batch - 1) / batch;
    if (t->losses) (void)hipFree(t->losses);
    t->losses = nullptr;
    TRY(hipMalloc(&t->losses, sizeof(float) * nb));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t q = 0; q < nb; ++q) {
        const int64_t r0 = q * batch, cnt = std::min(batch, t->n - r0);
        const int np = std::min(t->nparts, vtm::mlp_grid(cnt));
        vtm::launch_mlp_grad(t->P, t->X, t->Y, t->idx + r0, 0, cnt, 1.f / (float)cnt, t->part, np, t->g, t->st);
        ++t->step;
        const float c1 = 1.f - std::pow(b1, (float)t->step), c2 = 1.f - std::pow(b2, (float)t->step);
        vtm::launch_adam(t->P, t->g, t->m, t->v, lr, b1, b2, eps, c1, c2, t->st);
        TRY(hipMemcpyAsync(t->losses + q, t->g + vtm::kTrain, sizeof(float), hipMemcpyDeviceToDevice, t->st));
    }
    std::vector<float> h(nb);
    TRY(hipMemcpyAsync(h.data(), t->losses, sizeof(float) * nb, hipMemcpyDeviceToHost, t->st));
    TRY(hipStreamSynchronize(t->st));
    double tot = 0.0;
    for (float x : h) tot += x;
    if (loss) *loss = (float)(tot / (double)t->n);
    return VTM_OK;
}

vtm_status vtm_trainer_predict(vtm_trainer t, const float *feats, int64_t n, float *out) {
    if (!t || !feats || !out || n < 1) return tfail(VTM_ERR_INVALID, "bad argument");
    TRY(hipSetDevice(t->device));
    float *X = nullptr, *y = nullptr;
    TRY(hipMalloc(&X, sizeof(float) * vtm::kNumFeatures * n));
    hipError_t e = hipMalloc(&y, sizeof(float) * n);
    if (e != hipSuccess) { (void)hipFree(X); return tfail(VTM_ERR_OOM, "predict buffer"); }
    (void)hipMemcpyAsync(X, feats, sizeof(float) * vtm::kNumFeatures * n, hipMemcpyHostToDevice, t->st);
    vtm::launch_mlp_predict(t->P, X, n, y, t->st);
    (void)hipMemcpyAsync(out, y, sizeof(float) * n, hipMemcpyDeviceToHost, t->st);
    e = hipStreamSynchronize(t->st);
    (void)hipFree(X);
    (void)hipFree(y);
    if (e != hipSuccess) return tfail(VTM_ERR_HIP, hipGetErrorString(e));
    return VTM_OK;
}

vtm_status vtm_trainer_get_params(vtm_trainer t, float *params) {
    if (!t || !params) return tfail(VTM_ERR_INVALID, "bad argument");
    TRY(hipSetDevice(t->device));
    TRY(hipMemcpy(params, t->P, sizeof(float) * vtm::kParams, hipMemcpyDeviceToHost));
    return VTM_OK;
}

}  // extern "C"
