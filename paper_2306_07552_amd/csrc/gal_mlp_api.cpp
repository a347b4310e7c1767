// Host runtime of the collision-surrogate MLP (declared in include/gal.h):
// parameters, training step (forward, logistic loss, backward, Adam) and
// inference, all on the device with the MFMA kernels of k_mlp.hip.
#include "gal.h"
#include "gal_mlp.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

namespace gal {
int api_fail(int code, const char *fmt, ...);
}

namespace {

#define MLP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return gal::api_fail(GAL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kDims[6] = {gal::kMlpIn, gal::kMlpHidden, gal::kMlpHidden, gal::kMlpHidden,
                          gal::kMlpHidden, 1};

}  // namespace

struct gal_mlp {
    std::vector<void *> allocs;
    int32_t max_rows = 0;
    int64_t off_w[5], off_b[5], n_params = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *wb = nullptr;
    uint16_t *wi = nullptr;     // inference copy of the matrix layers (fragment order)
    uint16_t *h[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // h[1..4]
    uint16_t *dp[2] = {nullptr, nullptr};
    float *z = nullptr, *dz = nullptr, *loss = nullptr;
    float *part = nullptr;      // inference: the first layer's partial sums
    float *dw_part = nullptr;   // split-K partial sums of the weight gradients
    size_t dw_part_floats = 0;
    int64_t t = 0;
    ~gal_mlp()
    {
        for (void *p : allocs) (void)hipFree(p);
    }
    template <class T>
    int alloc(T **out, size_t count)
    {
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
        if (hipMalloc(&p, bytes) != hipSuccess)
            return gal::api_fail(GAL_ENOMEM, "hipMalloc(%zu bytes) failed", bytes);
        allocs.push_back(p);
        *out = static_cast<T *>(p);
        return GAL_OK;
    }
};

extern "C" {

int gal_mlp_num_params(int64_t *n)
{
    if (!n) return gal::api_fail(GAL_EINVAL, "null argument");
    int64_t c = 0;
    for (int l = 0; l < 5; ++l) c += (int64_t)kDims[l + 1] * kDims[l] + kDims[l + 1];
    *n = c;
    return GAL_OK;
}

int gal_mlp_create(int32_t max_rows, uint64_t seed, gal_mlp **out)
{
    if (!out || max_rows < 1 || max_rows > (1 << 22)) return gal::api_fail(GAL_EINVAL, "bad arguments");
    *out = nullptr;
    gal_mlp *m = new gal_mlp();
    m->max_rows = max_rows;
    int64_t off = 0;
    for (int l = 0; l < 5; ++l) {
        m->off_w[l] = off;
        off += (int64_t)kDims[l + 1] * kDims[l];
        m->off_b[l] = off;
        off += kDims[l + 1];
    }
    m->n_params = off;
    int rc;
    if ((rc = m->alloc(&m->w, off)) || (rc = m->alloc(&m->m, off)) || (rc = m->alloc(&m->v, off)) ||
        (rc = m->alloc(&m->g, off)) || (rc = m->alloc(&m->wb, off)) ||
        (rc = m->alloc(&m->wi, gal::sur_infer_layout_elems())) ||
        (rc = m->alloc(&m->dp[0], (size_t)max_rows * gal::kMlpHidden)) ||
        (rc = m->alloc(&m->dp[1], (size_t)max_rows * gal::kMlpHidden)) ||
        (rc = m->alloc(&m->z, max_rows)) || (rc = m->alloc(&m->dz, max_rows)) ||
        (rc = m->alloc(&m->part, gal::sur_infer_part_floats_max(max_rows))) ||
        (rc = m->alloc(&m->dw_part, (m->dw_part_floats = (size_t)gal::kMaxDwSplits * kDims[1] * kDims[0]))) ||
        (rc = m->alloc(&m->loss, 1))) {
        delete m;
        return rc;
    }
    for (int l = 1; l <= 4; ++l)
        if ((rc = m->alloc(&m->h[l], (size_t)max_rows * gal::kMlpHidden))) {
            delete m;
            return rc;
        }
    // He-uniform initialisation of the weights, zero biases
    std::vector<float> host(off, 0.0f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < 5; ++l) {
        const float lim = std::sqrt(6.0f / (float)kDims[l]);
        std::uniform_real_distribution<float> U(-lim, lim);
        for (int64_t i = 0; i < (int64_t)kDims[l + 1] * kDims[l]; ++i) host[m->off_w[l] + i] = U(rng);
    }
    int rc2 = gal_mlp_set_weights(m, host.data(), (size_t)off);
    if (rc2) {
        delete m;
        return rc2;
    }
    *out = m;
    return GAL_OK;
}

int gal_mlp_set_weights(gal_mlp *m, const float *host, size_t count)
{
    if (!m || !host) return gal::api_fail(GAL_EINVAL, "null argument");
    if ((int64_t)count != m->n_params) return gal::api_fail(GAL_EINVAL, "need %lld parameters", (long long)m->n_params);
    MLP_TRY(hipMemcpy(m->w, host, sizeof(float) * count, hipMemcpyHostToDevice));
    MLP_TRY(hipMemset(m->m, 0, sizeof(float) * count));
    MLP_TRY(hipMemset(m->v, 0, sizeof(float) * count));
    MLP_TRY(gal::mlp_to_bf16(m->w, (int64_t)count, m->wb, nullptr));
    MLP_TRY(gal::mlp_refresh_inference(m, nullptr));
    MLP_TRY(hipDeviceSynchronize());
    m->t = 0;
    return GAL_OK;
}

int gal_mlp_get_weights(gal_mlp *m, float *host, size_t count)
{
    if (!m || !host) return gal::api_fail(GAL_EINVAL, "null argument");
    if ((int64_t)count != m->n_params) return gal::api_fail(GAL_EINVAL, "need %lld parameters", (long long)m->n_params);
    MLP_TRY(hipDeviceSynchronize());
    MLP_TRY(hipMemcpy(host, m->w, sizeof(float) * count, hipMemcpyDeviceToHost));
    return GAL_OK;
}

}  // extern "C"

namespace gal {

int mlp_max_rows(const gal_mlp *m) { return m->max_rows; }

// the inference copy of the matrix layers, after the BF16 weights changed
hipError_t mlp_refresh_inference(gal_mlp *m, hipStream_t s)
{
    return sur_infer_layout(m->wb + m->off_w[0], m->wb + m->off_w[1], m->wb + m->off_w[2],
                            m->wb + m->off_w[3], m->wi, s);
}

// forward pass of rows inputs (BF16 [rows][2112]) into m->h[1..4] and m->z
int mlp_forward_rows(gal_mlp *m, const uint16_t *x, int rows, hipStream_t s)
{
    const uint16_t *in = x;
    for (int l = 0; l < 4; ++l) {
        MLP_TRY(mlp_gemm(kGemmFwd, in, m->wb + m->off_w[l], rows, kDims[l + 1], kDims[l], kDims[l],
                         kDims[l], m->w + m->off_b[l], nullptr, 0, nullptr, m->h[l + 1], kDims[l + 1],
                         s));
        in = m->h[l + 1];
    }
    MLP_TRY(mlp_head_fwd(m->h[4], m->wb + m->off_w[4], m->w + m->off_b[4], rows, kMlpHidden, m->z, s));
    return GAL_OK;
}

// inference: the inputs x, or (x null) the features of the batch envs
// described by `src` computed on the fly; logits into z (may be null),
// routing flags and counts with route
int mlp_infer_rows(gal_mlp *m, const uint16_t *x, const SurInferArgs *src, int rows, float *z,
                   const RouteArgs *route, hipStream_t s, float *part)
{
    SurInferArgs a = src ? *src : SurInferArgs{};
    a.t.w0 = m->wi;
    a.t.b0 = m->w + m->off_b[0];
    for (int l = 0; l < 4; ++l) {
        a.t.w[l] = l < 3 ? m->wi + (size_t)kMlpIn * kMlpHidden + (size_t)l * kMlpHidden * kMlpHidden
                         : m->wb + m->off_w[4];
        a.t.b[l] = m->w + m->off_b[l + 1];
    }
    a.x = x;
    a.rows = rows;
    a.part = part ? part : m->part;
    a.z = z;
    a.route = route ? 1 : 0;
    if (route) a.ra = *route;
    MLP_TRY(sur_infer(a, s));
    return GAL_OK;
}

int mlp_gradients_rows(gal_mlp *m, const uint16_t *x, const float *y, int rows, float pos_w,
                       hipStream_t s)
{
    int rc = mlp_forward_rows(m, x, rows, s);
    if (rc) return rc;
    MLP_TRY(hipMemsetAsync(m->loss, 0, sizeof(float), s));
    MLP_TRY(mlp_loss(m->z, y, rows, pos_w, m->dz, m->loss, s));
    MLP_TRY(mlp_head_bwd(m->h[4], m->wb + m->off_w[4], m->dz, rows, kMlpHidden, m->dp[0],
                         m->g + m->off_w[4], m->g + m->off_b[4], s));
    int cur = 0;
    for (int l = 3; l >= 0; --l) {
        const int din = kDims[l], dout = kDims[l + 1];
        const uint16_t *hin = l == 0 ? x : m->h[l];
        // dW_l [dout][din] = dpre^T h_{l-1}
        MLP_TRY(mlp_gemm(kGemmDw, m->dp[cur], hin, dout, din, rows, dout, din, nullptr, nullptr, 0,
                         m->g + m->off_w[l], nullptr, din, s, m->dw_part, m->dw_part_floats));
        MLP_TRY(mlp_colsum(m->dp[cur], rows, dout, m->g + m->off_b[l], s));
        if (l > 0) {
            // dpre_{l-1} = bf16((dpre W_l) * [h_{l-1} > 0])
            MLP_TRY(mlp_gemm(kGemmDx, m->dp[cur], m->wb + m->off_w[l], rows, din, dout, dout, din,
                             nullptr, m->h[l], din, nullptr, m->dp[cur ^ 1], din, s));
            cur ^= 1;
        }
    }
    return GAL_OK;
}

}  // namespace gal

extern "C" {

int gal_mlp_forward(gal_mlp *m, const uint16_t *x_dev, int32_t rows, float *logits_dev, void *stream)
{
    if (!m || !x_dev || rows < 0 || rows > m->max_rows) return gal::api_fail(GAL_EINVAL, "bad arguments");
    if ((uintptr_t)x_dev % 16) return gal::api_fail(GAL_EINVAL, "x_dev must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    return gal::mlp_infer_rows(m, x_dev, nullptr, rows, logits_dev ? logits_dev : m->z, nullptr, s);
}

int gal_mlp_gradients(gal_mlp *m, const uint16_t *x_dev, const float *labels_dev, int32_t rows,
                      float pos_weight, float *grads_dev, float *loss_dev, void *stream)
{
    if (!m || !x_dev || !labels_dev || rows < 1 || rows > m->max_rows)
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = gal::mlp_gradients_rows(m, x_dev, labels_dev, rows, pos_weight, s);
    if (rc) return rc;
    if (grads_dev)
        MLP_TRY(hipMemcpyAsync(grads_dev, m->g, sizeof(float) * m->n_params, hipMemcpyDeviceToDevice, s));
    if (loss_dev) MLP_TRY(hipMemcpyAsync(loss_dev, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return GAL_OK;
}

int gal_mlp_train_step(gal_mlp *m, const uint16_t *x_dev, const float *labels_dev, int32_t rows,
                       float pos_weight, float lr, float *loss_dev, void *stream)
{
    if (!m || !x_dev || !labels_dev || rows < 1 || rows > m->max_rows || !(lr > 0.0f))
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = gal::mlp_gradients_rows(m, x_dev, labels_dev, rows, pos_weight, s);
    if (rc) return rc;
    m->t += 1;
    MLP_TRY(gal::mlp_adam(m->w, m->m, m->v, m->g, m->n_params, lr, 0.9f, 0.999f, 1e-8f, m->t, m->wb, s));
    MLP_TRY(gal::mlp_refresh_inference(m, s));
    if (loss_dev) MLP_TRY(hipMemcpyAsync(loss_dev, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return GAL_OK;
}

int gal_mlp_gemm_test(int32_t variant, const uint16_t *a_dev, const uint16_t *b_dev, int32_t M,
                      int32_t N, int32_t K, int32_t lda, int32_t ldb, float *c_dev, int32_t ldc,
                      void *stream)
{
    if (variant < gal::kGemmNtF32 || variant > gal::kGemmTnF32 || !a_dev || !b_dev || !c_dev)
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    MLP_TRY(gal::mlp_gemm(variant, a_dev, b_dev, M, N, K, lda, ldb, nullptr, nullptr, 0, c_dev,
                          nullptr, ldc, (hipStream_t)stream));
    return GAL_OK;
}

void gal_mlp_destroy(gal_mlp *m) { delete m; }

}  // extern "C"
