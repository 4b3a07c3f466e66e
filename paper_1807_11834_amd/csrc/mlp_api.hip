// mlp_api.hip -- C ABI of the learned velocity surrogate (see include/couple_mlp.h).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "couple_mlp.h"
#include "launch.hpp"
#include "mlp.hpp"
#include "mlp_state.hpp"

using namespace cpl;
using namespace cpl::mlp;

static thread_local std::string g_mlp_init_err;
static constexpr double kStdRelFloor = 1e-4;

static int mfail(couple_mlp *m, int code, const std::string &msg) {
    if (m) m->err = msg;
    else g_mlp_init_err = msg;
    return code;
}

template <typename X> static bool alloc0(X **p, size_t bytes) {
    void *q = nullptr;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&q, bytes) != hipSuccess || hipMemset(q, 0, bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (q) (void)hipFree(q);
        *p = nullptr;
        return false;
    }
    *p = static_cast<X *>(q);
    return true;
}

static void mlp_release(couple_mlp *m) {
    std::vector<void *> ptrs = {m->net.params, m->net.m, m->net.v, m->net.mean_inv, m->tb.x0, m->tb.tr,
                                m->tb.y, m->tb.loss_part, m->tb.grads, m->stats};
    for (int l = 0; l < 4; ++l) {
        ptrs.push_back(m->net.wt[l]);
        ptrs.push_back(m->net.wn[l]);
        ptrs.push_back(m->net.wtp[l]);
        ptrs.push_back(m->net.wnp[l]);
        ptrs.push_back(m->tb.part_w[l]);
        ptrs.push_back(m->tb.part_b[l]);
    }
    for (int l = 0; l < 3; ++l) {
        ptrs.push_back(m->tb.h[l]);
    }
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    m->net = NetBufs{};
    m->tb = TrainBufs{};
    m->stats = nullptr;
}

// Standardisation tables as the kernels read them: mean, then 1/std, FP32 [2][224].
static int upload_norm(couple_mlp *m) {
    std::vector<float> mi(2 * kK1, 0.f);
    for (int k = 0; k < kFeat; ++k) {
        mi[k] = (float)m->mean[k];
        mi[kK1 + k] = (float)(1.0 / m->std[k]);
    }
    if (hipMemcpy(m->net.mean_inv, mi.data(), sizeof(float) * 2 * kK1, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(m, COUPLE_EHIP, "couple_mlp: copy of the standardisation failed");
    }
    return COUPLE_OK;
}

extern "C" int couple_mlp_init(const couple_mlp_config *cfg, couple_mlp **out) {
    if (!cfg || !out) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_init: NULL argument");
    *out = nullptr;
    if (cfg->max_batch < 32 || cfg->max_batch >= (int64_t(1) << 26))
        return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_init: max_batch must be in [32, 2^26)");
    if (!(std::isfinite(cfg->lr) && cfg->lr > 0.0)) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_init: lr must be > 0");
    if (!(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0 && cfg->beta2 >= 0.0 && cfg->beta2 < 1.0))
        return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_init: beta1 and beta2 must be in [0, 1)");
    if (!(std::isfinite(cfg->eps) && cfg->eps > 0.0)) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_init: eps must be > 0");
    couple_mlp *m = new (std::nothrow) couple_mlp();
    if (!m) return mfail(nullptr, COUPLE_ENOMEM, "couple_mlp_init: host allocation failed");
    m->cfg = *cfg;
    for (int k = 0; k < kFeat; ++k) {
        m->mean[k] = 0.0;
        m->std[k] = 1.0;
    }
    for (int a = 0; a < 3; ++a) m->scale[a] = 1.0;
    const int64_t B = (cfg->max_batch + 31) / 32 * 32;
    const int64_t nc = n_chunks(B), ng = n_train_groups(B);
    TrainBufs &tb = m->tb;
    tb.max_batch = cfg->max_batch;
    bool ok = alloc0(&m->net.params, sizeof(float) * kNParam) && alloc0(&m->net.m, sizeof(float) * kNParam) &&
              alloc0(&m->net.v, sizeof(float) * kNParam) && alloc0(&m->net.mean_inv, sizeof(float) * 2 * kK1);
    for (int l = 0; l < 4 && ok; ++l) {
        ok = alloc0(&m->net.wt[l], sizeof(uint16_t) * mpad(l) * kpad(l)) &&
             (l == 0 || (alloc0(&m->net.wn[l], sizeof(uint16_t) * kpad(l) * cpad(l)) &&
                         alloc0(&m->net.wtp[l], sizeof(uint16_t) * mpad(l) * kpad(l)) &&
                         alloc0(&m->net.wnp[l], sizeof(uint16_t) * kpad(l) * cpad(l)))) &&
             alloc0(&tb.part_w[l], sizeof(float) * nc * mpad(l) * kpad(l)) &&
             alloc0(&tb.part_b[l], sizeof(double) * ng * mpad(l));
    }
    for (int l = 0; l < 3 && ok; ++l)
        ok = alloc0(&tb.h[l], sizeof(uint16_t) * B * kHid);
    m->stats_chunks = 256;
    ok = ok && alloc0(&tb.x0, sizeof(uint16_t) * B * kK1) && alloc0(&tb.tr, sizeof(uint16_t) * B * kTrRows) &&
         alloc0(&tb.y, sizeof(float) * B * 16) &&
         alloc0(&tb.loss_part, sizeof(double) * ((B + 15) / 16)) && alloc0(&tb.grads, sizeof(float) * kNParam) &&
         alloc0(&m->stats, sizeof(double) * (m->stats_chunks * 256 + 4 * 256));
    if (!ok) {
        mlp_release(m);
        delete m;
        return mfail(nullptr, COUPLE_ENOMEM, "couple_mlp_init: device allocation failed");
    }
    if (upload_norm(m) != COUPLE_OK) {
        mlp_release(m);
        delete m;
        return mfail(nullptr, COUPLE_EHIP, "couple_mlp_init: copy of the standardisation failed");
    }
    *out = m;
    return COUPLE_OK;
}

extern "C" int couple_mlp_free(couple_mlp *m) {
    if (!m) return COUPLE_OK;
    (void)hipDeviceSynchronize();
    mlp_release(m);
    delete m;
    return COUPLE_OK;
}

extern "C" const char *couple_mlp_last_error(const couple_mlp *m) { return m ? m->err.c_str() : g_mlp_init_err.c_str(); }

static int sync_or_fail(couple_mlp *m, const char *what) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return mfail(m, COUPLE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    }
    return COUPLE_OK;
}

extern "C" int couple_mlp_set_params(couple_mlp *m, const float *params) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_set_params: NULL handle");
    if (!params) return mfail(m, COUPLE_EINVAL, "couple_mlp_set_params: NULL params");
    if (sync_or_fail(m, "couple_mlp_set_params") != COUPLE_OK) return COUPLE_EHIP;
    if (hipMemcpy(m->net.params, params, sizeof(float) * kNParam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->net.m, 0, sizeof(float) * kNParam) != hipSuccess ||
        hipMemset(m->net.v, 0, sizeof(float) * kNParam) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(m, COUPLE_EHIP, "couple_mlp_set_params: copy failed");
    }
    m->t = 0;
    if (launch_cast(m->net, nullptr) != hipSuccess) return mfail(m, COUPLE_EHIP, "couple_mlp_set_params: launch failed");
    return sync_or_fail(m, "couple_mlp_set_params");
}

static bool check_norm(const double *mean, const double *std, const double *scale, std::string &why) {
    for (int k = 0; k < kFeat; ++k)
        if (!std::isfinite(mean[k]) || !(std::isfinite(std[k]) && std[k] > 0.0)) {
            why = "feature mean must be finite and std finite and > 0";
            return false;
        }
    for (int a = 0; a < 3; ++a)
        if (!(std::isfinite(scale[a]) && scale[a] > 0.0)) {
            why = "scale must be finite and > 0";
            return false;
        }
    return true;
}

extern "C" int couple_mlp_set_norm(couple_mlp *m, const double *mean, const double *std, const double *scale) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_set_norm: NULL handle");
    if (!mean || !std || !scale) return mfail(m, COUPLE_EINVAL, "couple_mlp_set_norm: NULL argument");
    std::string why;
    if (!check_norm(mean, std, scale, why)) return mfail(m, COUPLE_EINVAL, "couple_mlp_set_norm: " + why);
    if (sync_or_fail(m, "couple_mlp_set_norm") != COUPLE_OK) return COUPLE_EHIP;
    std::memcpy(m->mean, mean, sizeof(m->mean));
    std::memcpy(m->std, std, sizeof(m->std));
    std::memcpy(m->scale, scale, sizeof(m->scale));
    return upload_norm(m);
}

extern "C" int couple_mlp_fit_norm(couple_mlp *m, const float *feat, const float *resid, int64_t n, void *stream) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_fit_norm: NULL handle");
    if (!feat || !resid) return mfail(m, COUPLE_EINVAL, "couple_mlp_fit_norm: NULL argument");
    if (n < 1) return mfail(m, COUPLE_EINVAL, "couple_mlp_fit_norm: n must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nc = (n < m->stats_chunks) ? n : m->stats_chunks;
    double *part = m->stats, *res = m->stats + m->stats_chunks * 256;   // res: fmean, fstd, rmean, rstd (256 each)
    (void)hipGetLastError();
    if (launch_column_stats(feat, n, kFeat, part, nc, res, res + 256, st) != hipSuccess ||
        launch_column_stats(resid, n, 3, part, nc, res + 512, res + 768, st) != hipSuccess)
        return mfail(m, COUPLE_EHIP, "couple_mlp_fit_norm: launch failed");
    std::vector<double> h(1024);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(h.data(), res, sizeof(double) * 1024, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(m, COUPLE_EHIP, "couple_mlp_fit_norm: copy failed");
    }
    double mean[kFeat], sd[kFeat], sc[3];
    for (int k = 0; k < kFeat; ++k) {
        mean[k] = h[k];
        sd[k] = h[256 + k];
    }
    // a neighbour difference's std is at least kStdRelFloor times the std of the
    // centre cell's value of the same channel (differences of a field that does
    // not vary in that direction are FP32 rounding only); then std < 1e-12 -> 1
    for (int u = 0; u < 27; ++u)
        if (u != 13)
            for (int ch = 0; ch < 7; ++ch)
                sd[7 * u + ch] = std::fmax(sd[7 * u + ch], kStdRelFloor * h[256 + 7 * 13 + ch]);
    for (int k = 0; k < kFeat; ++k)
        if (sd[k] < 1e-12) sd[k] = 1.0;
    double big = 0.0;
    for (int a = 0; a < 3; ++a) big = std::fmax(big, h[768 + a]);
    for (int a = 0; a < 3; ++a) {
        sc[a] = h[768 + a];
        if (big == 0.0) sc[a] = 1.0;
        else if (sc[a] < 1e-12 * big) sc[a] = big;
    }
    std::string why;
    if (!check_norm(mean, sd, sc, why)) return mfail(m, COUPLE_EINVAL, "couple_mlp_fit_norm: non-finite statistics");
    std::memcpy(m->mean, mean, sizeof(m->mean));
    std::memcpy(m->std, sd, sizeof(m->std));
    std::memcpy(m->scale, sc, sizeof(m->scale));
    return upload_norm(m);
}

extern "C" int couple_mlp_get_state(couple_mlp *m, float *params, float *adam_m, float *adam_v, int64_t *step,
                                    double *mean, double *std, double *scale) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_get_state: NULL handle");
    if (sync_or_fail(m, "couple_mlp_get_state") != COUPLE_OK) return COUPLE_EHIP;
    const size_t bytes = sizeof(float) * kNParam;
    if ((params && hipMemcpy(params, m->net.params, bytes, hipMemcpyDeviceToHost) != hipSuccess) ||
        (adam_m && hipMemcpy(adam_m, m->net.m, bytes, hipMemcpyDeviceToHost) != hipSuccess) ||
        (adam_v && hipMemcpy(adam_v, m->net.v, bytes, hipMemcpyDeviceToHost) != hipSuccess)) {
        (void)hipGetLastError();
        return mfail(m, COUPLE_EHIP, "couple_mlp_get_state: copy failed");
    }
    if (step) *step = m->t;
    if (mean) std::memcpy(mean, m->mean, sizeof(m->mean));
    if (std) std::memcpy(std, m->std, sizeof(m->std));
    if (scale) std::memcpy(scale, m->scale, sizeof(m->scale));
    return COUPLE_OK;
}

extern "C" int couple_mlp_set_state(couple_mlp *m, const float *params, const float *adam_m, const float *adam_v,
                                    int64_t step, const double *mean, const double *std, const double *scale) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_set_state: NULL handle");
    if (!params || !adam_m || !adam_v || !mean || !std || !scale)
        return mfail(m, COUPLE_EINVAL, "couple_mlp_set_state: NULL argument");
    if (step < 0) return mfail(m, COUPLE_EINVAL, "couple_mlp_set_state: step < 0");
    std::string why;
    if (!check_norm(mean, std, scale, why)) return mfail(m, COUPLE_EINVAL, "couple_mlp_set_state: " + why);
    if (sync_or_fail(m, "couple_mlp_set_state") != COUPLE_OK) return COUPLE_EHIP;
    const size_t bytes = sizeof(float) * kNParam;
    if (hipMemcpy(m->net.params, params, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->net.m, adam_m, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->net.v, adam_v, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(m, COUPLE_EHIP, "couple_mlp_set_state: copy failed");
    }
    m->t = step;
    std::memcpy(m->mean, mean, sizeof(m->mean));
    std::memcpy(m->std, std, sizeof(m->std));
    std::memcpy(m->scale, scale, sizeof(m->scale));
    if (upload_norm(m) != COUPLE_OK) return COUPLE_EHIP;
    if (launch_cast(m->net, nullptr) != hipSuccess) return mfail(m, COUPLE_EHIP, "couple_mlp_set_state: launch failed");
    return sync_or_fail(m, "couple_mlp_set_state");
}

static void inv_scale(const couple_mlp *m, float out[3]) {
    for (int a = 0; a < 3; ++a) out[a] = (float)(1.0 / m->scale[a]);
}

extern "C" int couple_mlp_forward(couple_mlp *m, const float *feat, int64_t n, float *y, void *stream) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_forward: NULL handle");
    if (n < 0 || n > m->tb.max_batch) return mfail(m, COUPLE_EINVAL, "couple_mlp_forward: n out of [0, max_batch]");
    if (n > 0 && (!feat || !y)) return mfail(m, COUPLE_EINVAL, "couple_mlp_forward: NULL argument");
    if (n == 0) return COUPLE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (launch_standardise(feat, n, m->net.mean_inv, m->tb.x0, st) != hipSuccess ||
        launch_forward(m->net, m->tb, n, st) != hipSuccess || launch_output(m->tb, n, y, st) != hipSuccess)
        return mfail(m, COUPLE_EHIP, "couple_mlp_forward: launch failed");
    return COUPLE_OK;
}

static int grads_impl(couple_mlp *m, const char *who, const float *feat, const float *resid, int64_t nrows,
                      const int32_t *idx, int64_t B, float *grads, float *loss, hipStream_t st) {
    if (!feat || !resid || !grads) return mfail(m, COUPLE_EINVAL, std::string(who) + ": NULL argument");
    if (B < 32 || B % 32 != 0 || B > m->tb.max_batch)
        return mfail(m, COUPLE_EINVAL, std::string(who) + ": B must be a multiple of 32 in [32, max_batch]");
    if (nrows < 1 || (!idx && nrows < B)) return mfail(m, COUPLE_EINVAL, std::string(who) + ": nrows too small");
    float is[3];
    inv_scale(m, is);
    (void)hipGetLastError();
    if (launch_gradients(m->net, m->tb, feat, resid, idx, nrows, B, is, grads, loss, st) != hipSuccess)
        return mfail(m, COUPLE_EHIP, std::string(who) + ": launch failed");
    return COUPLE_OK;
}

extern "C" int couple_mlp_grads(couple_mlp *m, const float *feat, const float *resid, int64_t nrows, const int32_t *idx,
                                int64_t B, float *grads, float *loss, void *stream) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_grads: NULL handle");
    return grads_impl(m, "couple_mlp_grads", feat, resid, nrows, idx, B, grads, loss, static_cast<hipStream_t>(stream));
}

static int adam_impl(couple_mlp *m, const float *grads, hipStream_t st) {
    const int64_t t = m->t + 1;
    const double c1 = 1.0 - std::pow(m->cfg.beta1, (double)t), c2 = 1.0 - std::pow(m->cfg.beta2, (double)t);
    (void)hipGetLastError();
    if (launch_adam(m->net, grads, (float)m->cfg.lr, (float)m->cfg.beta1, (float)(1.0 - m->cfg.beta1),
                    (float)m->cfg.beta2, (float)(1.0 - m->cfg.beta2), (float)m->cfg.eps, (float)c1, (float)c2,
                    st) != hipSuccess)
        return mfail(m, COUPLE_EHIP, "couple_mlp: Adam launch failed");
    m->t = t;
    return COUPLE_OK;
}

extern "C" int couple_mlp_adam(couple_mlp *m, const float *grads, void *stream) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_adam: NULL handle");
    if (!grads) return mfail(m, COUPLE_EINVAL, "couple_mlp_adam: NULL grads");
    return adam_impl(m, grads, static_cast<hipStream_t>(stream));
}

extern "C" int couple_mlp_train_step(couple_mlp *m, const float *feat, const float *resid, int64_t nrows,
                                     const int32_t *idx, int64_t B, float *loss, void *stream) {
    if (!m) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_train_step: NULL handle");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = grads_impl(m, "couple_mlp_train_step", feat, resid, nrows, idx, B, m->tb.grads, loss, st);
    if (rc != COUPLE_OK) return rc;
    return adam_impl(m, m->tb.grads, st);
}

extern "C" int couple_mlp_features(const couple_config *cfg, int64_t n, const float *pos, const float *diam,
                                   const float *bulk_phi, const float *bulk_U, const float *bulk_G, const float *u_fine,
                                   const int32_t *sel, int64_t nsel, float *feat, float *u_bulk, float *resid,
                                   void *stream) {
    if (!cfg) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: NULL config");
    for (int a = 0; a < 3; ++a)
        if (!(std::isfinite(cfg->box[a]) && cfg->box[a] > 0.0) || cfg->nb[a] < 1)
            return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: invalid grid");
    if ((int64_t)cfg->nb[0] * cfg->nb[1] * cfg->nb[2] >= (int64_t(1) << 31) - 1)
        return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: too many bulk cells");
    if (cfg->precision == COUPLE_FP64) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: FP32 fields only");
    if (n < 0 || nsel < 0 || (!sel && nsel > n)) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: bad n or nsel");
    if (nsel > 0 && (!pos || !diam || !bulk_phi || !bulk_U || !bulk_G || !feat || n < 1))
        return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: NULL argument");
    if (resid && !u_fine) return mfail(nullptr, COUPLE_EINVAL, "couple_mlp_features: resid needs u_fine");
    (void)hipGetLastError();
    if (launch_features(cfg->nb, cfg->box, n, pos, diam, bulk_phi, bulk_U, bulk_G, u_fine, sel, nsel, feat, u_bulk, resid,
                        static_cast<hipStream_t>(stream)) != hipSuccess)
        return mfail(nullptr, COUPLE_EHIP, "couple_mlp_features: launch failed");
    return COUPLE_OK;
}
