// surrogate_api.cpp -- C ABI of the MLP surrogate (host runtime).
//
// Parameter vector layout (FP32): W1[256*3] (unit-major), b1[256],
// W2[256*256] (out-major), b2[256], W3[256], b3[1]; followed, in the
// get/set entry points only, by the input normalisation mu[3], sigma[3].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "smc.h"
#include "smc_internal.h"

namespace smc {
std::vector<double> convex_hull_planes(const float *pts, size_t n);
hipError_t sg_gemm(hipStream_t s, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk,
                   long sbn, float *C, long ldc, int M, int N, int K, int accumulate);
hipError_t sg_layer1_forward(hipStream_t s, const float *x, int n, const float *mu, const float *sigma,
                             const uint16_t *W1b, const float *b1, uint16_t *xb, float *pre1, uint16_t *h1b);
hipError_t sg_layer2_epilogue(hipStream_t s, float *pre2, int n, const float *b2, uint16_t *h2b);
hipError_t sg_layer3_forward_loss(hipStream_t s, const uint16_t *h2b, int n, const uint16_t *W3b,
                                  const float *b3, const float *y, const float *w, float inv_wsum,
                                  float *p_out, float *loss_row, float *dz);
hipError_t sg_layer3_backward(hipStream_t s, const uint16_t *h2b, const float *pre2, int n,
                              const uint16_t *W3b, const float *dz, float *dW3, float *db3, float *db2,
                              uint16_t *d2b);
hipError_t sg_layer1_backward(hipStream_t s, const float *dh1, const float *pre1, const uint16_t *xb, int n,
                              float *dW1, float *db1);
hipError_t sg_loss_sum(hipStream_t s, const float *loss_row, int n, float *out);
hipError_t sg_adam(hipStream_t s, float *w, const float *g, float *m, float *v, uint16_t *wb, long count,
                   float lr, float beta1, float beta2, float eps, float bc1, float bc2);
hipError_t sg_round(hipStream_t s, const float *w, uint16_t *wb, long count);
hipError_t sg_expand_neighbours(hipStream_t s, const float *x, long n, float delta, float *x6);
hipError_t sg_confirm(hipStream_t s, const float *p, const unsigned long long *succ, const unsigned long long *trials,
                      long n, float threshold, uint8_t *use);
hipError_t sg_neighbour_gate(hipStream_t s, const float *p, const float *p6, long n, float threshold, float margin,
                             uint8_t *use);
hipError_t sg_query(hipStream_t s, const float *x, long n, const float *mu, const float *sigma,
                    const uint16_t *W1b, const float *b1, const uint16_t *W2b, const float *b2,
                    const uint16_t *W3b, const float *b3, const float *planes, int n_planes, float hull_tol,
                    float threshold, float margin, float *p_out, uint8_t *use);
}  // namespace smc

using namespace smc;

namespace {
constexpr int H = 256;
constexpr long OFF_W1 = 0, OFF_B1 = OFF_W1 + H * 3, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
               OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, N_PARAMS = OFF_B3 + 1;
}  // namespace

struct smc_surrogate {
    smc_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // [N_PARAMS] each
    uint16_t *wb = nullptr;                                          // BF16 copies [N_PARAMS]
    float *norm = nullptr;                                           // mu[3], sigma[3]
    float host_norm[6] = {0, 0, 0, 1, 1, 1};
    float *planes = nullptr;
    int n_planes = 0;
    std::vector<float> host_planes;
    long step = 0;
    // activations for a training batch of up to cap rows
    int cap = 0;
    float *x = nullptr, *y = nullptr, *wt = nullptr, *pre1 = nullptr, *pre2 = nullptr,
          *dh1 = nullptr, *p = nullptr, *loss_row = nullptr, *dz = nullptr;
    uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr, *d2b = nullptr;
    // query buffers
    long qcap = 0;
    float *qx = nullptr, *qp = nullptr;
    uint8_t *quse = nullptr;
    // gate calibrated on held-out estimates (smc_surrogate_calibrate): the
    // smallest margin at which no held-out answer was off; refuse: none was
    bool calibrated = false;
    bool refuse = false;
    float cal_margin = 0.0f;
    float cal_threshold = 0.5f;
    // neighbourhood of the calibrated gate (0: none): an answer also needs
    // the six points x +- delta e_k on the same side, `margin` away
    float cal_delta = 0.0f;
    long nbcap = 0;
    float *nbx = nullptr, *nbp = nullptr;
};

extern "C" const char *smc_last_error(const smc_ctx *ctx);

namespace {

int sfail(smc_surrogate *s, int code, const std::string &msg);

#define SG_TRY(s, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return sfail(s, e_ == hipErrorOutOfMemory ? SMC_E_NOMEM : SMC_E_HIP, \
                                           std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

}  // namespace

// error reporting goes through the context's message (smc_api.cpp)
namespace smc {
int set_ctx_error(smc_ctx *ctx, int code, const std::string &msg);
hipStream_t ctx_stream(smc_ctx *ctx);
int ctx_device(smc_ctx *ctx);
}  // namespace smc

namespace {
int sfail(smc_surrogate *s, int code, const std::string &msg)
{
    return set_ctx_error(s ? s->ctx : nullptr, code, msg);
}

template <typename T>
hipError_t dalloc(T *&p, size_t n)
{
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T));
}

int ensure_batch(smc_surrogate *s, int n)
{
    if (n <= s->cap) return SMC_OK;
    const int c = ((n + 31) / 32) * 32;
    SG_TRY(s, dalloc(s->x, (size_t)c * 3));
    SG_TRY(s, dalloc(s->y, c));
    SG_TRY(s, dalloc(s->wt, c));
    SG_TRY(s, dalloc(s->p, c));
    SG_TRY(s, dalloc(s->loss_row, c));
    SG_TRY(s, dalloc(s->dz, c));
    SG_TRY(s, dalloc(s->xb, (size_t)c * 3));
    SG_TRY(s, dalloc(s->pre1, (size_t)c * H));
    SG_TRY(s, dalloc(s->pre2, (size_t)c * H));
    SG_TRY(s, dalloc(s->dh1, (size_t)c * H));
    SG_TRY(s, dalloc(s->h1b, (size_t)c * H));
    SG_TRY(s, dalloc(s->h2b, (size_t)c * H));
    SG_TRY(s, dalloc(s->d2b, (size_t)c * H));
    s->cap = c;
    return SMC_OK;
}

// Upload a batch padded to a multiple of 32 rows (padding rows weigh 0).
int upload_batch(smc_surrogate *s, const float *x, const float *y, const float *w, size_t n, int *n_pad,
                 float *inv_wsum)
{
    const int np = (int)(((n + 31) / 32) * 32);
    int rc = ensure_batch(s, np);
    if (rc != SMC_OK) return rc;
    std::vector<float> hx((size_t)np * 3, 0.0f), hy(np, 0.0f), hw(np, 0.0f);
    double wsum = 0.0;
    for (size_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) hx[3 * i + k] = x[3 * i + k];
        hy[i] = y ? y[i] : 0.0f;
        hw[i] = w ? w[i] : 1.0f;
        wsum += hw[i];
    }
    for (size_t i = n; i < (size_t)np; ++i)
        for (int k = 0; k < 3; ++k) hx[3 * i + k] = s->host_norm[k];
    SG_TRY(s, hipMemcpyAsync(s->x, hx.data(), hx.size() * 4, hipMemcpyHostToDevice, s->stream));
    SG_TRY(s, hipMemcpyAsync(s->y, hy.data(), hy.size() * 4, hipMemcpyHostToDevice, s->stream));
    SG_TRY(s, hipMemcpyAsync(s->wt, hw.data(), hw.size() * 4, hipMemcpyHostToDevice, s->stream));
    *n_pad = np;
    *inv_wsum = wsum > 0.0 ? (float)(1.0 / wsum) : 0.0f;
    return SMC_OK;
}

// Forward and backward over the uploaded batch; gradients in s->g.
int forward_backward(smc_surrogate *s, int n, float inv_wsum)
{
    hipStream_t st = s->stream;
    const float *mu = s->norm, *sigma = s->norm + 3;
    float *w = s->w, *g = s->g;
    uint16_t *wb = s->wb;
    SG_TRY(s, sg_layer1_forward(st, s->x, n, mu, sigma, wb + OFF_W1, w + OFF_B1, s->xb, s->pre1, s->h1b));
    SG_TRY(s, sg_gemm(st, s->h1b, H, 1, wb + OFF_W2, 1, H, s->pre2, H, n, H, H, 0));
    SG_TRY(s, sg_layer2_epilogue(st, s->pre2, n, w + OFF_B2, s->h2b));
    SG_TRY(s, sg_layer3_forward_loss(st, s->h2b, n, wb + OFF_W3, w + OFF_B3, s->y, s->wt, inv_wsum, s->p,
                                     s->loss_row, s->dz));
    SG_TRY(s, sg_layer3_backward(st, s->h2b, s->pre2, n, wb + OFF_W3, s->dz, g + OFF_W3, g + OFF_B3,
                                 g + OFF_B2, s->d2b));
    // dW2[j][i] = sum_b d2b[b][j] h1b[b][i]
    SG_TRY(s, sg_gemm(st, s->d2b, 1, H, s->h1b, H, 1, g + OFF_W2, H, H, H, n, 0));
    // dh1[b][i] = sum_j d2b[b][j] W2b[j][i]
    SG_TRY(s, sg_gemm(st, s->d2b, H, 1, wb + OFF_W2, H, 1, s->dh1, H, n, H, H, 0));
    SG_TRY(s, sg_layer1_backward(st, s->dh1, s->pre1, s->xb, n, g + OFF_W1, g + OFF_B1));
    return SMC_OK;
}

int sum_loss(smc_surrogate *s, int n, float *loss)
{
    std::vector<float> lr(n);
    SG_TRY(s, hipMemcpyAsync(lr.data(), s->loss_row, n * 4, hipMemcpyDeviceToHost, s->stream));
    SG_TRY(s, hipStreamSynchronize(s->stream));
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += lr[i];
    *loss = (float)acc;
    return SMC_OK;
}

}  // namespace

extern "C" {

int smc_surrogate_create(smc_ctx *ctx, uint64_t seed, smc_surrogate **out)
{
    if (!ctx || !out) return set_ctx_error(ctx, SMC_E_INVALID, "null argument");
    *out = nullptr;
    auto *s = new smc_surrogate();
    s->ctx = ctx;
    s->stream = ctx_stream(ctx);
    (void)hipSetDevice(ctx_device(ctx));
    hipError_t e = hipSuccess;
    if ((e = dalloc(s->w, N_PARAMS)) != hipSuccess || (e = dalloc(s->g, N_PARAMS)) != hipSuccess ||
        (e = dalloc(s->m, N_PARAMS)) != hipSuccess || (e = dalloc(s->v, N_PARAMS)) != hipSuccess ||
        (e = dalloc(s->wb, N_PARAMS)) != hipSuccess || (e = dalloc(s->norm, 6)) != hipSuccess) {
        smc_surrogate_destroy(s);
        return set_ctx_error(ctx, SMC_E_NOMEM, hipGetErrorString(e));
    }
    // Glorot-uniform weights, zero biases, identity normalisation.
    std::vector<float> h(N_PARAMS, 0.0f);
    std::mt19937_64 rng(seed);
    auto fill = [&](long off, long count, int fan_in, int fan_out) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        std::uniform_real_distribution<double> U(-a, a);
        for (long i = 0; i < count; ++i) h[off + i] = (float)U(rng);
    };
    fill(OFF_W1, H * 3, 3, H);
    fill(OFF_W2, (long)H * H, H, H);
    fill(OFF_W3, H, H, 1);
    std::vector<float> p(N_PARAMS + 6);
    std::copy(h.begin(), h.end(), p.begin());
    for (int k = 0; k < 3; ++k) {
        p[N_PARAMS + k] = 0.0f;
        p[N_PARAMS + 3 + k] = 1.0f;
    }
    const int rc = smc_surrogate_set_params(s, p.data(), p.size());
    if (rc != SMC_OK) {
        smc_surrogate_destroy(s);
        return rc;
    }
    *out = s;
    return SMC_OK;
}

size_t smc_surrogate_param_count(void) { return (size_t)N_PARAMS + 6; }

int smc_surrogate_set_params(smc_surrogate *s, const float *params, size_t count)
{
    if (!s || !params || count != (size_t)N_PARAMS + 6) return sfail(s, SMC_E_INVALID, "need param_count values");
    for (int k = 0; k < 3; ++k)
        if (!(params[N_PARAMS + 3 + k] > 0.0f)) return sfail(s, SMC_E_INVALID, "sigma must be > 0");
    SG_TRY(s, hipMemcpyAsync(s->w, params, N_PARAMS * 4, hipMemcpyHostToDevice, s->stream));
    SG_TRY(s, hipMemcpyAsync(s->norm, params + N_PARAMS, 6 * 4, hipMemcpyHostToDevice, s->stream));
    std::copy(params + N_PARAMS, params + N_PARAMS + 6, s->host_norm);
    SG_TRY(s, sg_round(s->stream, s->w, s->wb, N_PARAMS));
    SG_TRY(s, hipMemsetAsync(s->m, 0, N_PARAMS * 4, s->stream));
    SG_TRY(s, hipMemsetAsync(s->v, 0, N_PARAMS * 4, s->stream));
    SG_TRY(s, hipStreamSynchronize(s->stream));
    s->step = 0;
    s->calibrated = false;
    return SMC_OK;
}

int smc_surrogate_get_params(const smc_surrogate *s, float *params, size_t count)
{
    if (!s || !params || count != (size_t)N_PARAMS + 6) return SMC_E_INVALID;
    auto *ms = const_cast<smc_surrogate *>(s);
    SG_TRY(ms, hipMemcpyAsync(params, s->w, N_PARAMS * 4, hipMemcpyDeviceToHost, s->stream));
    SG_TRY(ms, hipStreamSynchronize(s->stream));
    std::copy(s->host_norm, s->host_norm + 6, params + N_PARAMS);
    return SMC_OK;
}

int smc_surrogate_gradients(smc_surrogate *s, const float *x, const float *y, const float *w, size_t n,
                            float *loss, float *grads)
{
    if (!s || !x || !y || n == 0 || n > (1u << 20)) return sfail(s, SMC_E_INVALID, "bad batch");
    int np = 0;
    float inv = 0.0f;
    int rc = upload_batch(s, x, y, w, n, &np, &inv);
    if (rc == SMC_OK) rc = forward_backward(s, np, inv);
    if (rc == SMC_OK && loss) rc = sum_loss(s, np, loss);
    if (rc != SMC_OK) return rc;
    if (grads) {
        SG_TRY(s, hipMemcpyAsync(grads, s->g, N_PARAMS * 4, hipMemcpyDeviceToHost, s->stream));
        SG_TRY(s, hipStreamSynchronize(s->stream));
    }
    return SMC_OK;
}

int smc_surrogate_train(smc_surrogate *s, const float *x, const float *y, const float *w, size_t n,
                        const smc_train_opts *opts, float *loss_out)
{
    if (!s || !x || !y || !opts || n < 4 || n > (1u << 20)) return sfail(s, SMC_E_INVALID, "bad training set");
    if (!(opts->lr > 0.0f) || opts->steps == 0) return sfail(s, SMC_E_INVALID, "need lr > 0 and steps > 0");
    s->calibrated = false;   // a retrained network needs a new calibration
    // input normalisation from the training points
    double mu[3] = {0, 0, 0}, var[3] = {0, 0, 0};
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) mu[k] += x[3 * i + k];
    for (int k = 0; k < 3; ++k) mu[k] /= (double)n;
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) var[k] += (x[3 * i + k] - mu[k]) * (x[3 * i + k] - mu[k]);
    for (int k = 0; k < 3; ++k) {
        s->host_norm[k] = (float)mu[k];
        s->host_norm[3 + k] = (float)std::sqrt(std::max(var[k] / (double)n, 1e-12));
    }
    SG_TRY(s, hipMemcpyAsync(s->norm, s->host_norm, 24, hipMemcpyHostToDevice, s->stream));
    // training hull in raw log10-rate space
    std::vector<double> pl = convex_hull_planes(x, n);
    s->host_planes.assign(pl.begin(), pl.end());
    s->n_planes = (int)(pl.size() / 4);
    SG_TRY(s, dalloc(s->planes, std::max<size_t>(pl.size(), 4)));
    if (!pl.empty())
        SG_TRY(s, hipMemcpyAsync(s->planes, s->host_planes.data(), pl.size() * 4, hipMemcpyHostToDevice, s->stream));
    int np = 0;
    float inv = 0.0f;
    int rc = upload_batch(s, x, y, w, n, &np, &inv);
    if (rc != SMC_OK) return rc;
    const float b1 = opts->beta1 > 0.0f ? opts->beta1 : 0.9f;
    const float b2 = opts->beta2 > 0.0f ? opts->beta2 : 0.999f;
    const float eps = opts->adam_eps > 0.0f ? opts->adam_eps : 1e-8f;
    // per-step losses are summed on the device and copied back once
    float *hist = nullptr;
    if (loss_out) SG_TRY(s, hipMalloc((void **)&hist, (size_t)opts->steps * sizeof(float)));
    struct Free {
        float *p;
        ~Free() { if (p) (void)hipFree(p); }
    } free_hist{hist};
    for (uint32_t it = 0; it < opts->steps; ++it) {
        rc = forward_backward(s, np, inv);
        if (rc != SMC_OK) return rc;
        if (hist) SG_TRY(s, sg_loss_sum(s->stream, s->loss_row, np, hist + it));
        s->step += 1;
        const float bc1 = 1.0f - std::pow(b1, (float)s->step);
        const float bc2 = 1.0f - std::pow(b2, (float)s->step);
        SG_TRY(s, sg_adam(s->stream, s->w, s->g, s->m, s->v, s->wb, N_PARAMS, opts->lr, b1, b2, eps, bc1, bc2));
    }
    if (hist)
        SG_TRY(s, hipMemcpyAsync(loss_out, hist, (size_t)opts->steps * sizeof(float), hipMemcpyDeviceToHost,
                                 s->stream));
    SG_TRY(s, hipStreamSynchronize(s->stream));
    return SMC_OK;
}

int smc_surrogate_query(smc_surrogate *s, const float *x, size_t n, float threshold, float margin, uint32_t flags,
                        float *p_out, uint8_t *use_surrogate)
{
    if (!s || (n && (!x || !p_out))) return sfail(s, SMC_E_INVALID, "null argument");
    if (flags & ~SMC_DEVICE_PTRS) return sfail(s, SMC_E_INVALID, "unknown flags");
    if (n == 0) return SMC_OK;
    const bool on_device = (flags & SMC_DEVICE_PTRS) != 0;
    if (on_device && ((uintptr_t)x % 4 || (uintptr_t)p_out % 4))
        return sfail(s, SMC_E_INVALID, "x and p_out must be 4-byte aligned");
    if (!on_device && (long)n > s->qcap) {
        SG_TRY(s, dalloc(s->qx, n * 3));
        SG_TRY(s, dalloc(s->qp, n));
        SG_TRY(s, dalloc(s->quse, n));
        s->qcap = (long)n;
    }
    if (!s->planes) {
        SG_TRY(s, dalloc(s->planes, 4));
        s->n_planes = 0;
    }
    const float *d_x = on_device ? x : s->qx;
    float *d_p = on_device ? p_out : s->qp;
    uint8_t *d_use = use_surrogate ? (on_device ? use_surrogate : s->quse) : nullptr;
    if (!on_device) SG_TRY(s, hipMemcpyAsync(s->qx, x, n * 12, hipMemcpyHostToDevice, s->stream));
    // a calibrated gate never answers closer to its threshold than the
    // calibrated margin, and answers nothing when calibration refused it
    float m = margin;
    if (s->calibrated && threshold == s->cal_threshold) m = std::max(m, s->cal_margin);
    if (s->calibrated && (s->refuse || threshold != s->cal_threshold)) m = 2.0f;   // |p - t| < 2 always
    SG_TRY(s, sg_query(s->stream, d_x, (long)n, s->norm, s->norm + 3, s->wb + OFF_W1, s->w + OFF_B1,
                       s->wb + OFF_W2, s->w + OFF_B2, s->wb + OFF_W3, s->w + OFF_B3, s->planes, s->n_planes,
                       1e-6f, threshold, m, d_p, d_use));
    if (d_use && s->calibrated && !s->refuse && s->cal_delta > 0.0f && threshold == s->cal_threshold) {
        // the neighbourhood gate: the network at x +- delta e_k
        if ((long)n > s->nbcap) {
            SG_TRY(s, dalloc(s->nbx, n * 18));
            SG_TRY(s, dalloc(s->nbp, n * 6));
            s->nbcap = (long)n;
        }
        SG_TRY(s, sg_expand_neighbours(s->stream, d_x, (long)n, s->cal_delta, s->nbx));
        SG_TRY(s, sg_query(s->stream, s->nbx, 6L * (long)n, s->norm, s->norm + 3, s->wb + OFF_W1, s->w + OFF_B1,
                           s->wb + OFF_W2, s->w + OFF_B2, s->wb + OFF_W3, s->w + OFF_B3, s->planes, 0, 1e-6f,
                           threshold, 0.0f, s->nbp, nullptr));
        SG_TRY(s, sg_neighbour_gate(s->stream, d_p, s->nbp, (long)n, threshold, m, d_use));
    }
    if (!on_device) {
        SG_TRY(s, hipMemcpyAsync(p_out, s->qp, n * 4, hipMemcpyDeviceToHost, s->stream));
        if (use_surrogate) SG_TRY(s, hipMemcpyAsync(use_surrogate, s->quse, n, hipMemcpyDeviceToHost, s->stream));
    }
    SG_TRY(s, hipStreamSynchronize(s->stream));
    return SMC_OK;
}

int smc_surrogate_calibrate(smc_surrogate *s, const float *x, const double *lo, const double *hi, size_t n,
                            float threshold, float bound, float min_margin, float *margin_out, float *share_out)
{
    if (!s || (n && (!x || !lo || !hi))) return sfail(s, SMC_E_INVALID, "null argument");
    if (!(bound >= 0.0f) || !(min_margin >= 0.0f) || !(threshold >= 0.0f && threshold <= 1.0f))
        return sfail(s, SMC_E_INVALID, "need bound >= 0, min_margin >= 0, threshold in [0, 1]");
    for (size_t i = 0; i < n; ++i)
        if (!(lo[i] <= hi[i])) return sfail(s, SMC_E_INVALID, "need lo <= hi");
    s->calibrated = false;
    std::vector<float> p(n);
    std::vector<uint8_t> in_hull(n);
    if (n) {
        // network outputs and hull membership (margin 0: every point in the hull)
        const int rc = smc_surrogate_query(s, x, n, threshold, 0.0f, 0, p.data(), in_hull.data());
        if (rc != SMC_OK) return rc;
    }
    // For each neighbourhood size delta (log10 units, 0 = the point alone),
    // the stability of each held-out point: the least signed distance from
    // the threshold, on the point's side, of the outputs at x and at x +-
    // delta e_k.  The margin must exceed the stability of every held-out point
    // in the hull whose answer lies more than `bound` outside its interval;
    // the delta that leaves the largest share answered is kept.
    static const float kDeltas[] = {0.0f, 0.01f, 0.02f, 0.05f, 0.1f, 0.2f};
    std::vector<float> x6(n * 18), p6(n * 6);
    double best_m = 2.0, best_share = -1.0;
    float best_delta = 0.0f;
    size_t inside = 0;
    for (size_t i = 0; i < n; ++i) inside += in_hull[i] ? 1 : 0;
    for (float delta : kDeltas) {
        std::vector<double> stab(n);
        for (size_t i = 0; i < n; ++i) stab[i] = std::fabs((double)p[i] - threshold);
        if (delta > 0.0f && n) {
            for (size_t i = 0; i < n; ++i)
                for (int k = 0; k < 6; ++k)
                    for (int a = 0; a < 3; ++a)
                        x6[18 * i + 3 * k + a] = x[3 * i + a] + (a == (k >> 1) ? ((k & 1) ? -delta : delta) : 0.0f);
            const int rc = smc_surrogate_query(s, x6.data(), 6 * n, threshold, 0.0f, 0, p6.data(), nullptr);
            if (rc != SMC_OK) return rc;
            for (size_t i = 0; i < n; ++i) {
                const double side = p[i] >= threshold ? 1.0 : -1.0;
                for (int k = 0; k < 6; ++k) stab[i] = std::min(stab[i], ((double)p6[6 * i + k] - threshold) * side);
            }
        }
        double need = min_margin;
        for (size_t i = 0; i < n; ++i) {
            if (!in_hull[i]) continue;
            const bool off = p[i] < lo[i] - bound || p[i] > hi[i] + bound;
            if (off) need = std::max(need, (double)std::nextafter((float)stab[i], 2.0f));
        }
        if (need > 0.5) continue;
        size_t answered = 0;
        for (size_t i = 0; i < n; ++i)
            if (in_hull[i] && stab[i] >= (double)(float)need) ++answered;
        const double share = n ? (double)answered / (double)n : 0.0;
        if (share > best_share) {
            best_share = share;
            best_m = need;
            best_delta = delta;
        }
    }
    const bool refuse = inside == 0 || best_share < 0.0;
    s->calibrated = true;
    s->refuse = refuse;
    s->cal_margin = refuse ? 2.0f : (float)best_m;
    s->cal_delta = refuse ? 0.0f : best_delta;
    s->cal_threshold = threshold;
    if (margin_out) *margin_out = refuse ? -1.0f : (float)best_m;
    if (share_out) *share_out = refuse ? 0.0f : (float)best_share;
    return SMC_OK;
}

int smc_surrogate_confirm(smc_surrogate *s, const float *p, const uint64_t *successes, const uint64_t *trials,
                          size_t n, float threshold, uint32_t flags, uint8_t *use_surrogate)
{
    if (!s || (n && (!p || !successes || !trials || !use_surrogate))) return sfail(s, SMC_E_INVALID, "null argument");
    if (flags & ~SMC_DEVICE_PTRS) return sfail(s, SMC_E_INVALID, "unknown flags");
    if (!(threshold >= 0.0f && threshold <= 1.0f)) return sfail(s, SMC_E_INVALID, "threshold must lie in [0, 1]");
    if (n == 0) return SMC_OK;
    if (flags & SMC_DEVICE_PTRS) {
        if ((uintptr_t)p % 4 || (uintptr_t)successes % 8 || (uintptr_t)trials % 8)
            return sfail(s, SMC_E_INVALID, "p must be 4-byte and the counts 8-byte aligned");
        SG_TRY(s, hipSetDevice(ctx_device(s->ctx)));
        SG_TRY(s, sg_confirm(s->stream, p, reinterpret_cast<const unsigned long long *>(successes),
                             reinterpret_cast<const unsigned long long *>(trials), (long)n, threshold,
                             use_surrogate));
        SG_TRY(s, hipStreamSynchronize(s->stream));
        return SMC_OK;
    }
    for (size_t i = 0; i < n; ++i)
        if (successes[i] > trials[i]) return sfail(s, SMC_E_INVALID, "more successes than trials");
    for (size_t i = 0; i < n; ++i) {
        if (!use_surrogate[i]) continue;
        const bool stands = trials[i] > 0 && (p[i] >= threshold ? successes[i] == trials[i] : successes[i] == 0);
        use_surrogate[i] = stands ? 1 : 0;
    }
    return SMC_OK;
}

float smc_surrogate_neighbourhood(const smc_surrogate *s)
{
    return (s && s->calibrated && !s->refuse) ? s->cal_delta : 0.0f;
}

int smc_surrogate_hull(const smc_surrogate *s, float *planes, size_t cap)
{
    if (!s) return SMC_E_INVALID;
    const int n = s->n_planes;
    if (planes)
        for (int f = 0; f < n && (size_t)f < cap; ++f)
            for (int q = 0; q < 4; ++q) planes[4 * f + q] = s->host_planes[4 * f + q];
    return n;
}

int smc_convex_hull(const float *pts, size_t n, float *planes, size_t cap)
{
    if (!pts && n) return SMC_E_INVALID;
    const std::vector<double> pl = convex_hull_planes(pts, n);
    const int nf = (int)(pl.size() / 4);
    if (planes)
        for (int f = 0; f < nf && (size_t)f < cap; ++f)
            for (int q = 0; q < 4; ++q) planes[4 * f + q] = (float)pl[4 * f + q];
    return nf;
}

void smc_surrogate_destroy(smc_surrogate *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (float *p : {s->w, s->g, s->m, s->v, s->norm, s->planes, s->x, s->y, s->wt, s->pre1, s->pre2,
                     s->dh1, s->p, s->loss_row, s->dz, s->qx, s->qp, s->nbx, s->nbp})
        if (p) (void)hipFree(p);
    for (uint16_t *p : {s->wb, s->xb, s->h1b, s->h2b, s->d2b})
        if (p) (void)hipFree(p);
    if (s->quse) (void)hipFree(s->quse);
    delete s;
}

}  // extern "C"
