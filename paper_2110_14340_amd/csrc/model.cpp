// C ABI of the learned cost model: a small FP32 network trained and
// evaluated on the GPU by the kernels of k_mlp.hip.  The host side only
// moves arrays, shuffles sample order and loops over minibatches.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "ctx_internal.h"
#include "jacc.h"
#include "kernels.h"

struct jacc_model {
    jacc_ctx *ctx = nullptr;
    jk::MlpBufs B;
    int step = 0;  // Adam steps taken
    std::vector<void *> owned;
    int64_t loss_cap = 0;
};

namespace {

#define MCHK(m, expr, what)                                              \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) return jr::device_error((m)->ctx, e_, what); \
    } while (0)

int alloc_f(jacc_model *m, size_t count, float **out) {
    void *p = nullptr;
    int rc = jr::alloc(m->ctx, count * sizeof(float) + 64, &p);
    if (rc) return rc;
    m->owned.push_back(p);
    *out = (float *)p;
    return JACC_OK;
}

int ensure_capacity(jacc_model *m, int n) {
    if (n <= m->B.cap) return JACC_OK;
    const int F = m->B.F, H = jk::kMlpHidden;
    jk::MlpBufs &B = m->B;
    int rc = alloc_f(m, (size_t)n * F, &B.xs);
    if (!rc) rc = alloc_f(m, (size_t)n * H, &B.h1);
    if (!rc) rc = alloc_f(m, (size_t)n * H, &B.h2);
    if (!rc) rc = alloc_f(m, (size_t)n * H, &B.h3);
    if (!rc) rc = alloc_f(m, (size_t)n, &B.yhat);
    if (!rc) rc = alloc_f(m, (size_t)n, &B.g);
    if (!rc) rc = alloc_f(m, (size_t)n * H, &B.d1);
    if (!rc) rc = alloc_f(m, (size_t)n * H, &B.d2);
    if (!rc) rc = alloc_f(m, (size_t)n * H, &B.d3);
    if (!rc) rc = alloc_f(m, (size_t)n, &B.sqerr);
    if (!rc) B.cap = n;
    return rc;
}

int ensure_loss(jacc_model *m, int64_t steps) {
    if (steps <= m->loss_cap) return JACC_OK;
    int rc = alloc_f(m, (size_t)steps, &m->B.loss);
    if (!rc) m->loss_cap = steps;
    return rc;
}

// splitmix64 (Steele, Lea, Flood 2014) for the sample order of each epoch.
uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

bool bad(const jacc_model *m) { return !m || !m->ctx || jr::failed(m->ctx) || jr::dry(m->ctx); }

}  // namespace

extern "C" {

int jacc_model_nparams(int nfeat) {
    if (nfeat < 1 || nfeat > jk::kMlpMaxFeatures) return JACC_ERR_INVALID;
    return jk::mlp_nparams(nfeat);
}

int jacc_model_create(jacc_ctx *ctx, int nfeat, jacc_model **out) {
    if (!ctx || !out) return JACC_ERR_INVALID;
    *out = nullptr;
    if (jr::failed(ctx)) return JACC_ERR_DEVICE;
    if (jr::dry(ctx)) return jr::error(ctx, JACC_ERR_UNSUPPORTED, "the cost model needs the device");
    if (nfeat < 1 || nfeat > jk::kMlpMaxFeatures) return jr::error(ctx, JACC_ERR_INVALID, "1..16 features");
    jacc_model *m = new (std::nothrow) jacc_model();
    if (!m) return JACC_ERR_ALLOC;
    m->ctx = ctx;
    m->B.F = nfeat;
    const int P = jk::mlp_nparams(nfeat);
    jk::MlpBufs &B = m->B;
    int rc = alloc_f(m, P, &B.params);
    if (!rc) rc = alloc_f(m, P, &B.m);
    if (!rc) rc = alloc_f(m, P, &B.v);
    if (!rc) rc = alloc_f(m, P, &B.grad);
    if (!rc) rc = alloc_f(m, nfeat, &B.mu);
    if (!rc) rc = alloc_f(m, nfeat, &B.sd);
    if (!rc) rc = ensure_loss(m, 1);
    if (!rc) {
        std::vector<float> zero(P, 0.f), one(nfeat, 1.f);
        hipError_t e = hipMemcpy(B.params, zero.data(), P * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(B.m, zero.data(), P * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(B.v, zero.data(), P * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(B.mu, zero.data(), nfeat * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(B.sd, one.data(), nfeat * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = jr::device_error(ctx, e, "hipMemcpy");
    }
    if (rc) {
        jacc_model_destroy(m);
        return rc;
    }
    *out = m;
    return JACC_OK;
}

int jacc_model_destroy(jacc_model *m) {
    if (!m) return JACC_ERR_INVALID;
    if (m->ctx && !jr::dry(m->ctx)) (void)hipStreamSynchronize(jr::stream0(m->ctx));
    for (void *p : m->owned) jr::release(m->ctx, p);
    delete m;
    return JACC_OK;
}

int jacc_model_set_params(jacc_model *m, const float *params, int nparams) {
    if (bad(m) || !params) return JACC_ERR_INVALID;
    const int P = jk::mlp_nparams(m->B.F);
    if (nparams != P) return jr::error(m->ctx, JACC_ERR_INVALID, "wrong parameter count");
    std::vector<float> zero(P, 0.f);
    MCHK(m, hipMemcpy(m->B.params, params, P * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    MCHK(m, hipMemcpy(m->B.m, zero.data(), P * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    MCHK(m, hipMemcpy(m->B.v, zero.data(), P * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    m->step = 0;
    return JACC_OK;
}

int jacc_model_get_params(jacc_model *m, float *params, int nparams) {
    if (bad(m) || !params) return JACC_ERR_INVALID;
    const int P = jk::mlp_nparams(m->B.F);
    if (nparams != P) return jr::error(m->ctx, JACC_ERR_INVALID, "wrong parameter count");
    MCHK(m, hipStreamSynchronize(jr::stream0(m->ctx)), "hipStreamSynchronize");
    MCHK(m, hipMemcpy(params, m->B.params, P * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    return JACC_OK;
}

int jacc_model_set_scaler(jacc_model *m, const float *mean, const float *stdev) {
    if (bad(m) || !mean || !stdev) return JACC_ERR_INVALID;
    for (int f = 0; f < m->B.F; ++f)
        if (!(stdev[f] > 0.f)) return jr::error(m->ctx, JACC_ERR_INVALID, "standard deviations must be > 0");
    MCHK(m, hipMemcpy(m->B.mu, mean, m->B.F * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    MCHK(m, hipMemcpy(m->B.sd, stdev, m->B.F * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    return JACC_OK;
}

int jacc_model_predict(jacc_model *m, const float *X, int n, float *yhat) {
    if (bad(m) || !X || !yhat || n < 0) return JACC_ERR_INVALID;
    if (n == 0) return JACC_OK;
    int rc = ensure_capacity(m, n);
    if (rc) return rc;
    float *dX = nullptr;
    rc = alloc_f(m, (size_t)n * m->B.F, &dX);
    if (rc) return rc;
    hipStream_t s = jr::stream0(m->ctx);
    MCHK(m, hipMemcpyAsync(dX, X, (size_t)n * m->B.F * sizeof(float), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    MCHK(m, jk::mlp_forward(m->B, dX, nullptr, n, m->B.yhat, false, s), "mlp forward");
    MCHK(m, hipMemcpyAsync(yhat, m->B.yhat, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    MCHK(m, hipStreamSynchronize(s), "hipStreamSynchronize");
    jr::release(m->ctx, dX);
    m->owned.pop_back();
    return JACC_OK;
}

int jacc_model_gradients(jacc_model *m, const float *X, const float *y, int n, float *grad, float *loss) {
    if (bad(m) || !X || !y || n < 1) return JACC_ERR_INVALID;
    int rc = ensure_capacity(m, n);
    if (rc) return rc;
    float *dX = nullptr, *dy = nullptr;
    rc = alloc_f(m, (size_t)n * m->B.F, &dX);
    if (!rc) rc = alloc_f(m, (size_t)n, &dy);
    if (rc) return rc;
    hipStream_t s = jr::stream0(m->ctx);
    MCHK(m, hipMemcpyAsync(dX, X, (size_t)n * m->B.F * sizeof(float), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    MCHK(m, hipMemcpyAsync(dy, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    m->B.loss_at = 0;
    MCHK(m, jk::mlp_forward(m->B, dX, nullptr, n, m->B.yhat, true, s), "mlp forward");
    MCHK(m, jk::mlp_backward(m->B, dy, nullptr, n, s), "mlp backward");
    const int P = jk::mlp_nparams(m->B.F);
    if (grad) MCHK(m, hipMemcpyAsync(grad, m->B.grad, P * sizeof(float), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    if (loss) MCHK(m, hipMemcpyAsync(loss, m->B.loss, sizeof(float), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    MCHK(m, hipStreamSynchronize(s), "hipStreamSynchronize");
    jr::release(m->ctx, dy);
    jr::release(m->ctx, dX);
    m->owned.pop_back();
    m->owned.pop_back();
    return JACC_OK;
}

int jacc_model_adam_step(jacc_model *m, float lr) {
    if (bad(m)) return JACC_ERR_INVALID;
    m->step++;
    MCHK(m, jk::mlp_adam(m->B, m->step, lr, jr::stream0(m->ctx)), "mlp adam");
    return JACC_OK;
}

int jacc_model_fit(jacc_model *m, const float *X, const float *y, int n, int epochs, int batch, float lr,
                   uint64_t seed, float *epoch_loss) {
    if (bad(m) || !X || !y || n < 1 || epochs < 0 || batch < 1) return JACC_ERR_INVALID;
    const int bsz = batch < n ? batch : n;
    const int nb = (n + bsz - 1) / bsz;
    int rc = ensure_capacity(m, bsz);
    if (!rc) rc = ensure_loss(m, (int64_t)epochs * nb + 1);
    if (rc) return rc;
    float *dX = nullptr, *dy = nullptr, *didx = nullptr;
    rc = alloc_f(m, (size_t)n * m->B.F, &dX);
    if (!rc) rc = alloc_f(m, (size_t)n, &dy);
    if (!rc) rc = alloc_f(m, (size_t)n, &didx);
    if (rc) return rc;
    int *dperm = (int *)didx;
    hipStream_t s = jr::stream0(m->ctx);
    MCHK(m, hipMemcpyAsync(dX, X, (size_t)n * m->B.F * sizeof(float), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    MCHK(m, hipMemcpyAsync(dy, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    std::vector<int> perm(n);
    std::vector<int> staged(n);
    uint64_t st = seed;
    for (int e = 0; e < epochs; ++e) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {  // Fisher-Yates
            const int j = (int)(splitmix64(st) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        MCHK(m, hipStreamSynchronize(s), "hipStreamSynchronize");  // the previous epoch has read dperm
        staged = perm;
        MCHK(m, hipMemcpyAsync(dperm, staged.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, s),
             "hipMemcpyAsync");
        for (int k = 0; k < nb; ++k) {
            const int off = k * bsz;
            const int cnt = (off + bsz <= n) ? bsz : n - off;
            m->B.loss_at = (int64_t)e * nb + k;
            MCHK(m, jk::mlp_forward(m->B, dX, dperm + off, cnt, m->B.yhat, true, s), "mlp forward");
            MCHK(m, jk::mlp_backward(m->B, dy, dperm + off, cnt, s), "mlp backward");
            m->step++;
            MCHK(m, jk::mlp_adam(m->B, m->step, lr, s), "mlp adam");
        }
    }
    if (epoch_loss && epochs > 0) {
        std::vector<float> losses((size_t)epochs * nb);
        MCHK(m, hipMemcpyAsync(losses.data(), m->B.loss, losses.size() * sizeof(float), hipMemcpyDeviceToHost, s),
             "hipMemcpyAsync");
        MCHK(m, hipStreamSynchronize(s), "hipStreamSynchronize");
        for (int e = 0; e < epochs; ++e) {
            double acc = 0.0, cnt = 0.0;  // minibatch losses weighted by their sizes
            for (int k = 0; k < nb; ++k) {
                const int c = (k * bsz + bsz <= n) ? bsz : n - k * bsz;
                acc += (double)losses[(size_t)e * nb + k] * c;
                cnt += c;
            }
            epoch_loss[e] = (float)(acc / cnt);
        }
    }
    MCHK(m, hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int i = 0; i < 3; ++i) {
        jr::release(m->ctx, m->owned.back());
        m->owned.pop_back();
    }
    return JACC_OK;
}

}  // extern "C"
