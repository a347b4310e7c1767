// Host runtime of the policy network that consumes the depth stack (declared
// in include/gal.h): parameters and batched inference, on the device with the
// implicit-GEMM convolutions and heads of k_policy.hip and the fully connected
// layer on the surrogate's MFMA GEMM.
#include "gal.h"
#include "gal_mlp.h"
#include "gal_policy.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

namespace gal {
int api_fail(int code, const char *fmt, ...);
}

namespace {

#define POL_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return gal::api_fail(GAL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// the encoder: three convolutions (out channels, kernel, stride, in channels)
constexpr int kConv[3][4] = {{32, 8, 4, 1}, {64, 4, 2, 32}, {32, 3, 1, 64}};

int out_size(int n, int k, int s) { return (n - k) / s + 1; }

}  // namespace

struct gal_policy {
    std::vector<void *> allocs;
    int32_t max_envs = 0, A = 0;
    int side[4] = {gal::kPolicyRes, 0, 0, 0};   // input edge of each layer's map
    int64_t off_w[4], off_b[4];                  // conv1..3, fc
    int64_t off_aw, off_ab, off_vw, off_vb, off_ls, n_params = 0;
    float *w = nullptr;        // FP32 parameters
    uint16_t *wb = nullptr;    // BF16 copy (the convolutions' and the fc layer's weights are read from it)
    uint16_t *h[4] = {nullptr, nullptr, nullptr, nullptr};   // activations of conv1..3, fc
    float *fc_ws = nullptr;    // split-K partial products of the fc layer
    size_t fc_ws_floats = 0;
    int32_t last_envs = 0;
    // training (allocated on the first update)
    float *g = nullptr, *m = nullptr, *v = nullptr;          // gradient, Adam moments
    uint16_t *d[4] = {nullptr, nullptr, nullptr, nullptr};   // gradients of the pre-activations of conv1..3, fc
    uint16_t *wt = nullptr;                                  // adjoint weights
    float *gm = nullptr, *gls = nullptr, *gv = nullptr, *terms = nullptr;
    float *part = nullptr;
    size_t part_floats = 0;
    int64_t t = 0;
    ~gal_policy()
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
    size_t act_count(int l, int n) const
    {
        if (l < 3) {
            const int s = side[l + 1];
            return (size_t)n * s * s * kConv[l][0];
        }
        return (size_t)n * gal::kPolicyFeat;
    }
};

extern "C" {

int gal_policy_create(int32_t max_envs, int32_t act_dim, uint64_t seed, gal_policy **out)
{
    if (!out || max_envs < 1 || max_envs > (1 << 16) || act_dim < 1 || act_dim > 32)
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    *out = nullptr;
    gal_policy *p = new gal_policy();
    p->max_envs = max_envs;
    p->A = act_dim;
    for (int l = 0; l < 3; ++l) p->side[l + 1] = out_size(p->side[l], kConv[l][1], kConv[l][2]);
    const int flat = p->side[3] * p->side[3] * kConv[2][0];
    int64_t off = 0;
    for (int l = 0; l < 3; ++l) {
        p->off_w[l] = off;
        off += (int64_t)kConv[l][0] * kConv[l][1] * kConv[l][1] * kConv[l][3];
        p->off_b[l] = off;
        off += kConv[l][0];
    }
    p->off_w[3] = off;
    off += (int64_t)gal::kPolicyFeat * flat;
    p->off_b[3] = off;
    off += gal::kPolicyFeat;
    const int F = gal::kPolicyFeat + gal::kPolicyProprio;
    p->off_aw = off;
    off += (int64_t)act_dim * F;
    p->off_ab = off;
    off += act_dim;
    p->off_vw = off;
    off += F;
    p->off_vb = off;
    off += 1;
    p->off_ls = off;
    off += act_dim;
    p->n_params = off;
    int rc;
    if ((rc = p->alloc(&p->w, off)) || (rc = p->alloc(&p->wb, off))) {
        delete p;
        return rc;
    }
    for (int l = 0; l < 4; ++l)
        if ((rc = p->alloc(&p->h[l], p->act_count(l, max_envs)))) {
            delete p;
            return rc;
        }
    {
        // the fc layer's split-K workspace: the most any batch size up to max_envs needs
        const int flat = p->side[3] * p->side[3] * kConv[2][0];
        size_t need = 0;
        for (int n = 1; n <= max_envs; n = n < 64 ? n + 1 : n + 64) {
            const int m = std::min(n, (int)max_envs);
            need = std::max(need, (size_t)gal::fc_splits(m, gal::kPolicyFeat, flat) * m * gal::kPolicyFeat);
        }
        need = std::max(need, (size_t)gal::fc_splits(max_envs, gal::kPolicyFeat, flat) * max_envs * gal::kPolicyFeat);
        p->fc_ws_floats = need;
        if ((rc = p->alloc(&p->fc_ws, need))) {
            delete p;
            return rc;
        }
    }
    // He-uniform weights of the encoder, small heads, zero biases, log_std -0.5
    std::vector<float> host(off, 0.0f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int64_t o, int64_t n, float lim) {
        std::uniform_real_distribution<float> U(-lim, lim);
        for (int64_t i = 0; i < n; ++i) host[o + i] = U(rng);
    };
    for (int l = 0; l < 3; ++l) {
        const int fan = kConv[l][1] * kConv[l][1] * kConv[l][3];
        fill(p->off_w[l], (int64_t)kConv[l][0] * fan, std::sqrt(6.0f / (float)fan));
    }
    fill(p->off_w[3], (int64_t)gal::kPolicyFeat * flat, std::sqrt(6.0f / (float)flat));
    fill(p->off_aw, (int64_t)act_dim * F, 0.01f);
    fill(p->off_vw, F, 0.01f);
    for (int a = 0; a < act_dim; ++a) host[p->off_ls + a] = -0.5f;
    rc = gal_policy_set_weights(p, host.data(), (size_t)off);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return GAL_OK;
}

int gal_policy_num_params(const gal_policy *p, int64_t *n)
{
    if (!p || !n) return gal::api_fail(GAL_EINVAL, "null argument");
    *n = p->n_params;
    return GAL_OK;
}

int gal_policy_set_weights(gal_policy *p, const float *host, size_t count)
{
    if (!p || !host) return gal::api_fail(GAL_EINVAL, "null argument");
    if ((int64_t)count != p->n_params)
        return gal::api_fail(GAL_EINVAL, "need %lld parameters", (long long)p->n_params);
    POL_TRY(hipMemcpy(p->w, host, sizeof(float) * count, hipMemcpyHostToDevice));
    POL_TRY(gal::mlp_to_bf16(p->w, (int64_t)count, p->wb, nullptr));
    POL_TRY(hipDeviceSynchronize());
    return GAL_OK;
}

int gal_policy_get_weights(gal_policy *p, float *host, size_t count)
{
    if (!p || !host) return gal::api_fail(GAL_EINVAL, "null argument");
    if ((int64_t)count != p->n_params)
        return gal::api_fail(GAL_EINVAL, "need %lld parameters", (long long)p->n_params);
    POL_TRY(hipDeviceSynchronize());
    POL_TRY(hipMemcpy(host, p->w, sizeof(float) * count, hipMemcpyDeviceToHost));
    return GAL_OK;
}

}  // extern "C"

namespace {

gal::ConvGeom geom(const gal_policy *p, int l, int n)
{
    gal::ConvGeom g;
    g.ih = g.iw = p->side[l];
    g.in_c = kConv[l][3];
    g.kw = kConv[l][1];
    g.stride = kConv[l][2];
    g.oh = g.ow = p->side[l + 1];
    g.out_c = kConv[l][0];
    g.k = g.kw * g.kw * g.in_c;
    g.rows = n * g.oh * g.ow;
    return g;
}

// the encoder on n images: h[0..3]
int encode(gal_policy *p, const uint32_t *depth_dev, int n, hipStream_t s)
{
    const void *in = depth_dev;
    for (int l = 0; l < 3; ++l) {
        POL_TRY(gal::conv_gemm(l == 0, in, p->wb + p->off_w[l], p->w + p->off_b[l], geom(p, l, n), p->h[l], s));
        in = p->h[l];
    }
    const int flat = p->side[3] * p->side[3] * kConv[2][0];
    POL_TRY(gal::fc_forward(p->h[2], p->wb + p->off_w[3], p->w + p->off_b[3], n, gal::kPolicyFeat, flat, p->fc_ws,
                            p->fc_ws_floats, p->h[3], s));
    return GAL_OK;
}

int train_buffers(gal_policy *p)
{
    if (p->g) return GAL_OK;
    const int n = p->max_envs, A = p->A;
    const int flat = p->side[3] * p->side[3] * kConv[2][0];
    // split-K workspace: the fc weight gradient's (<= 16 splits) or a convolution's (<= 256 splits)
    p->part_floats = std::max<size_t>((size_t)16 * gal::kPolicyFeat * flat, (size_t)256 * 64 * 16 * 32);
    int rc;
    if ((rc = p->alloc(&p->g, p->n_params)) || (rc = p->alloc(&p->m, p->n_params)) ||
        (rc = p->alloc(&p->v, p->n_params)) || (rc = p->alloc(&p->wt, (size_t)64 * 16 * 32)) ||
        (rc = p->alloc(&p->gm, (size_t)n * A)) || (rc = p->alloc(&p->gls, (size_t)n * A)) ||
        (rc = p->alloc(&p->gv, (size_t)n)) || (rc = p->alloc(&p->terms, (size_t)n * 3)) ||
        (rc = p->alloc(&p->part, p->part_floats)))
        return rc;
    for (int l = 0; l < 4; ++l)
        if ((rc = p->alloc(&p->d[l], p->act_count(l, n)))) return rc;
    POL_TRY(hipMemset(p->m, 0, sizeof(float) * p->n_params));
    POL_TRY(hipMemset(p->v, 0, sizeof(float) * p->n_params));
    return GAL_OK;
}

}  // namespace

extern "C" {

int gal_policy_act(gal_policy *p, const uint32_t *depth_dev, const float *state_dev, int32_t n_envs,
                   const float *noise_dev, float *actions_dev, float *value_dev, float *logp_dev, void *stream)
{
    if (!p || !depth_dev || !state_dev || !actions_dev || n_envs < 0 || n_envs > p->max_envs)
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    if ((uintptr_t)depth_dev % 16) return gal::api_fail(GAL_EINVAL, "depth_dev must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (n_envs == 0) return GAL_OK;
    int rc = encode(p, depth_dev, n_envs, s);
    if (rc) return rc;
    POL_TRY(gal::policy_heads(p->h[3], state_dev, p->w + p->off_aw, p->w + p->off_ab, p->w + p->off_vw,
                              p->w + p->off_vb, p->w + p->off_ls, p->A, n_envs, noise_dev, actions_dev, value_dev,
                              logp_dev, s));
    p->last_envs = n_envs;
    return GAL_OK;
}

int gal_policy_ppo_gradients(gal_policy *p, const uint32_t *depth_dev, const float *state_dev,
                             const float *actions_dev, const float *old_logp_dev, const float *adv_dev,
                             const float *ret_dev, int32_t samples, const gal_ppo_params *hp, float *grads_dev,
                             float *stats_dev, void *stream)
{
    if (!p || !depth_dev || !state_dev || !actions_dev || !old_logp_dev || !adv_dev || !ret_dev || !hp ||
        samples < 1 || samples > p->max_envs)
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    if ((uintptr_t)depth_dev % 16) return gal::api_fail(GAL_EINVAL, "depth_dev must be 16-byte aligned");
    if (!(hp->clip >= 0.0f) || !(hp->value_coef >= 0.0f) || !(hp->entropy_coef >= 0.0f))
        return gal::api_fail(GAL_EINVAL, "clip and coefficients must be >= 0");
    int rc = train_buffers(p);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int S = samples, A = p->A;
    if ((rc = encode(p, depth_dev, S, s))) return rc;
    p->last_envs = S;
    const int F = gal::kPolicyFeat + gal::kPolicyProprio;
    (void)F;
    float *g = p->g;
    // heads: per-sample loss gradients, the features' gradient, then the
    // heads' own parameter gradients and the statistics
    POL_TRY(gal::ppo_heads(p->h[3], state_dev, p->w + p->off_aw, p->w + p->off_ab, p->w + p->off_vw,
                           p->w + p->off_vb, p->w + p->off_ls, A, S, actions_dev, old_logp_dev, adv_dev, ret_dev,
                           hp->clip, hp->value_coef, p->gm, p->gls, p->gv, p->terms, p->d[3], s));
    POL_TRY(gal::ppo_head_grads(p->h[3], state_dev, p->gm, p->gls, p->gv, p->terms, p->w + p->off_ls, A, S,
                                hp->entropy_coef, g + p->off_aw, g + p->off_ab, g + p->off_vw, g + p->off_vb,
                                g + p->off_ls, stats_dev, p->part, p->part_floats, s));
    // fully connected layer
    const int flat = p->side[3] * p->side[3] * kConv[2][0];
    POL_TRY(gal::mlp_gemm(gal::kGemmDw, p->d[3], p->h[2], gal::kPolicyFeat, flat, S, gal::kPolicyFeat, flat, nullptr,
                          nullptr, 0, g + p->off_w[3], nullptr, flat, s, p->part, p->part_floats));
    POL_TRY(gal::colsum(p->d[3], S, gal::kPolicyFeat, p->part, p->part_floats, g + p->off_b[3], s));
    POL_TRY(gal::mlp_gemm(gal::kGemmDx, p->d[3], p->wb + p->off_w[3], S, flat, gal::kPolicyFeat, gal::kPolicyFeat,
                          flat, nullptr, p->h[2], flat, nullptr, p->d[2], flat, s));
    // convolutions 3, 2, 1
    for (int l = 2; l >= 0; --l) {
        const gal::ConvGeom gg = geom(p, l, S);
        const void *in = l == 0 ? (const void *)depth_dev : (const void *)p->h[l - 1];
        POL_TRY(gal::conv_dw(l == 0, in, p->d[l], gg, p->part, p->part_floats, g + p->off_w[l], g + p->off_b[l], s));
        if (l > 0)
            POL_TRY(gal::conv_dx(p->d[l], p->wb + p->off_w[l], p->wt, p->h[l - 1], gg, p->d[l - 1], s));
    }
    if (grads_dev)
        POL_TRY(hipMemcpyAsync(grads_dev, g, sizeof(float) * p->n_params, hipMemcpyDeviceToDevice, s));
    return GAL_OK;
}

int gal_policy_adam_step(gal_policy *p, float lr, void *stream)
{
    if (!p || !(lr >= 0.0f)) return gal::api_fail(GAL_EINVAL, "bad arguments");
    if (!p->g) return gal::api_fail(GAL_ESTATE, "no gradient computed yet");
    p->t += 1;
    POL_TRY(gal::mlp_adam(p->w, p->m, p->v, p->g, p->n_params, lr, 0.9f, 0.999f, 1e-5f, p->t, p->wb,
                          (hipStream_t)stream));
    return GAL_OK;
}

int gal_gae(const float *rewards_dev, const float *values_dev, const uint8_t *dones_dev, const float *last_value_dev,
            int32_t T, int32_t N, float gamma, float lam, float *adv_dev, float *ret_dev, void *stream)
{
    if (!rewards_dev || !values_dev || !dones_dev || !last_value_dev || !adv_dev || !ret_dev || T < 0 || N < 0)
        return gal::api_fail(GAL_EINVAL, "bad arguments");
    POL_TRY(gal::gae(rewards_dev, values_dev, dones_dev, last_value_dev, T, N, gamma, lam, adv_dev, ret_dev,
                     (hipStream_t)stream));
    return GAL_OK;
}

int gal_policy_activations(gal_policy *p, int32_t layer, uint16_t *host, size_t count)
{
    if (!p || !host || layer < 1 || layer > 4) return gal::api_fail(GAL_EINVAL, "bad arguments");
    const size_t need = p->act_count(layer - 1, p->last_envs);
    if (count != need) return gal::api_fail(GAL_EINVAL, "layer %d holds %zu values", layer, need);
    POL_TRY(hipDeviceSynchronize());
    POL_TRY(hipMemcpy(host, p->h[layer - 1], sizeof(uint16_t) * count, hipMemcpyDeviceToHost));
    return GAL_OK;
}

void gal_policy_destroy(gal_policy *p) { delete p; }

}  // extern "C"
