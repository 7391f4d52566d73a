// C-ABI of the learned warm start: patch extraction, network forward,
// subspace loss with back-propagation, and the Adam update.  Buffer sizing
// and launch sequencing only; the arithmetic runs in k_cnn.hip.
#include <cmath>
#include <string>

#include "common.hpp"
#include "../../include/specmg.h"

using namespace specmg;

namespace specmg {
int fail_message(int code, const char* msg);   // sets the thread's last error, returns code
}

namespace {

#define CNNCHK(x)                                                  \
    do {                                                           \
        hipError_t _e = (x);                                       \
        if (_e != hipSuccess) throw HipError{_e, #x};              \
    } while (0)

bool fine_geom(const specmg_grid* G, FineGeom& fg) {
    if (!G || G->nx <= 0 || G->ny <= 0 || G->nz <= 0 || G->nx % 8 || G->ny % 8 || G->nz % 8) return false;
    fg = FineGeom{};
    fg.nx = G->nx;
    fg.ny = G->ny;
    fg.nz = G->nz;
    fg.mx = G->nx / 8;
    fg.my = G->ny / 8;
    fg.mz = G->nz / 8;
    return true;
}

template <class F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const HipError& e) {
        return fail_message(SPECMG_EDEVICE, (std::string(e.what) + ": " + hipGetErrorString(e.e)).c_str());
    }
}

}  // namespace

struct specmg_cnn {
    int k = 0, kp = 0, max_batch = 0, nblk = 0;
    void* packs = nullptr;
    float *a1 = nullptr, *a2 = nullptr, *g1 = nullptr, *g2 = nullptr, *gX = nullptr, *part = nullptr;
    double* loss_part = nullptr;
    double* loss_host = nullptr;   // pinned
    int last_count = -1;
    const float* last_patches = nullptr;
    ~specmg_cnn() {
        for (void* p : {(void*)packs, (void*)a1, (void*)a2, (void*)g1, (void*)g2, (void*)gX, (void*)part,
                        (void*)loss_part})
            if (p) (void)hipFree(p);
        if (loss_host) (void)hipHostFree(loss_host);
    }
};

extern "C" int64_t specmg_cnn_param_count(int32_t k) {
    if (k < 2 || k > 8 || (k & 1)) return -1;
    return cnn_param_count(k);
}

extern "C" int specmg_cnn_create(int32_t k, int32_t max_batch, specmg_cnn** out) {
    if (!out) return fail_message(SPECMG_EINVAL, "null argument");
    *out = nullptr;
    if (k < 2 || k > 8 || (k & 1)) return fail_message(SPECMG_EINVAL, "k must be 2, 4, 6 or 8");
    if (max_batch < 1 || max_batch > (1 << 20)) return fail_message(SPECMG_EINVAL, "max_batch out of range");
    return guarded([&] {
        specmg_cnn* n = new specmg_cnn();
        n->k = k;
        n->kp = k + (k & 1);
        n->max_batch = max_batch;
        n->nblk = max_batch < 256 ? max_batch : 256;
        try {
            const size_t act = (size_t)max_batch * 32 * 512 * sizeof(float);
            CNNCHK(hipMalloc(&n->packs, cnn_pack_words(n->kp) * sizeof(uint32_t)));
            CNNCHK(hipMalloc((void**)&n->a1, act));
            CNNCHK(hipMalloc((void**)&n->a2, act));
            CNNCHK(hipMalloc((void**)&n->g1, act));
            CNNCHK(hipMalloc((void**)&n->g2, act));
            CNNCHK(hipMalloc((void**)&n->gX, (size_t)max_batch * n->kp * 512 * sizeof(float)));
            CNNCHK(hipMalloc((void**)&n->part, (size_t)n->nblk * (32 * 32 * 27 + 32) * sizeof(float)));
            CNNCHK(hipMalloc((void**)&n->loss_part, (size_t)max_batch * sizeof(double)));
            CNNCHK(hipHostMalloc((void**)&n->loss_host, (size_t)max_batch * sizeof(double), hipHostMallocDefault));
        } catch (...) {
            delete n;
            throw;
        }
        *out = n;
        return SPECMG_OK;
    });
}

extern "C" void specmg_cnn_destroy(specmg_cnn* n) {
    if (!n) return;
    (void)hipDeviceSynchronize();
    delete n;
}

extern "C" int specmg_cnn_load(specmg_cnn* n, const float* theta32, const uint16_t* theta16, void* stream) {
    if (!n || (!theta32 == !theta16)) return fail_message(SPECMG_EINVAL, "give exactly one parameter vector");
    return guarded([&] {
        launch_cnn_pack(theta32, theta16, n->k, n->kp, n->packs, (hipStream_t)stream);
        CNNCHK(hipGetLastError());
        return SPECMG_OK;
    });
}

extern "C" int specmg_cnn_patches(const double* perm_dev, const specmg_grid* grid, int32_t e0, int32_t count,
                                  float* patches_dev, double* s_dev, void* stream) {
    FineGeom fg;
    if (!perm_dev || !patches_dev || !fine_geom(grid, fg) || !(grid->hx > 0))
        return fail_message(SPECMG_EINVAL, "bad arguments");
    const int64_t m = (int64_t)fg.mx * fg.my * fg.mz;
    if (e0 < 0 || count < 0 || e0 + (int64_t)count > m) return fail_message(SPECMG_EINVAL, "element range");
    if (count == 0) return SPECMG_OK;
    return guarded([&] {
        launch_cnn_patches(fg, perm_dev, e0, count, 3.0 / (grid->hx * grid->hx), patches_dev, s_dev,
                           (hipStream_t)stream);
        CNNCHK(hipGetLastError());
        return SPECMG_OK;
    });
}

extern "C" int specmg_cnn_forward(specmg_cnn* n, const float* patches_dev, int32_t count, float* X_dev,
                                  void* stream) {
    if (!n || !patches_dev || !X_dev) return fail_message(SPECMG_EINVAL, "null argument");
    if (count < 1 || count > n->max_batch) return fail_message(SPECMG_EINVAL, "count out of range");
    return guarded([&] {
        launch_cnn_forward(n->packs, n->kp, patches_dev, count, n->a1, n->a2, X_dev, (hipStream_t)stream);
        CNNCHK(hipGetLastError());
        n->last_count = count;
        n->last_patches = patches_dev;
        return SPECMG_OK;
    });
}

extern "C" int specmg_cnn_loss_backward(specmg_cnn* n, const float* patches_dev, const float* X_dev,
                                        const double* phi_dev, int32_t ldphi, const double* s_dev, int32_t count,
                                        double* loss, float* grad_dev, void* stream) {
    if (!n || !patches_dev || !X_dev || !phi_dev || !s_dev || !grad_dev)
        return fail_message(SPECMG_EINVAL, "null argument");
    if (ldphi < n->k) return fail_message(SPECMG_EINVAL, "ldphi < k");
    if (count != n->last_count || patches_dev != n->last_patches)
        return fail_message(SPECMG_EINVAL, "loss_backward must follow forward on the same batch");
    return guarded([&] {
        hipStream_t s = (hipStream_t)stream;
        launch_cnn_loss(X_dev, phi_dev, ldphi, s_dev, n->k, n->kp, count, 1.0 / count, n->loss_part, n->gX, s);
        const int nblk = count < n->nblk ? count : n->nblk;
        launch_cnn_backward(n->packs, n->k, n->kp, patches_dev, n->a1, n->a2, n->gX, count, n->g2, n->g1, n->part,
                            nblk, grad_dev, s);
        CNNCHK(hipGetLastError());
        if (loss) {
            CNNCHK(hipMemcpyAsync(n->loss_host, n->loss_part, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s));
            CNNCHK(hipStreamSynchronize(s));
            double t = 0.0;
            for (int i = 0; i < count; ++i) t += n->loss_host[i];
            *loss = t;
        }
        return SPECMG_OK;
    });
}

extern "C" int specmg_cnn_adam(float* theta_dev, const float* grad_dev, float* m1_dev, float* m2_dev, int64_t n,
                               double lr, double beta1, double beta2, double eps, int32_t step,
                               uint16_t* theta16_dev, void* stream) {
    if (!theta_dev || !grad_dev || !m1_dev || !m2_dev || n < 1 || step < 1)
        return fail_message(SPECMG_EINVAL, "bad arguments");
    const double c1 = 1.0 / (1.0 - std::pow(beta1, step)), c2 = 1.0 / (1.0 - std::pow(beta2, step));
    return guarded([&] {
        launch_cnn_adam(theta_dev, grad_dev, m1_dev, m2_dev, n, (float)lr, (float)beta1, (float)beta2, (float)eps,
                        (float)c1, (float)c2, theta16_dev, (hipStream_t)stream);
        CNNCHK(hipGetLastError());
        return SPECMG_OK;
    });
}
