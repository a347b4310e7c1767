// Internal definitions of the policy network that consumes the depth stack
// (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

constexpr int kPolicyRes = 128;      // depth image edge the encoder takes
constexpr int kPolicyFeat = 512;     // encoder features
constexpr int kPolicyProprio = 7;    // joint angles fed to the heads beside the features
constexpr int kPolicyMaxAct = 32;    // action dimensions

// One convolution as an implicit GEMM over NHWC input: `rows` = envs x oh x
// ow output pixels, `k` = kw x kw x in_c, `out_c` output channels.
struct ConvGeom {
    int rows, out_c, k;
    int ih, iw, in_c;
    int oh, ow, kw, stride;
};

hipError_t conv_gemm(bool depth_input, const void *in, const uint16_t *W, const float *bias, const ConvGeom &g,
                     uint16_t *out, hipStream_t s);
hipError_t policy_heads(const uint16_t *h, const float *state, const float *aw, const float *ab, const float *vw,
                        const float *vb, const float *log_std, int A, int n_envs, const float *noise,
                        float *actions, float *value, float *logp, hipStream_t s);

// The fully connected layer Y = bf16(relu(X W^T + b)) (X [rows][K], W [N][K]):
// split over K into ws when the tiles alone leave the chip idle (the splits
// are added in order), else one pass with the bias and ReLU fused.  The
// workspace needed: at most fc_splits(rows, N, K) * rows * N floats.
int fc_splits(int rows, int N, int K);
hipError_t fc_forward(const uint16_t *x, const uint16_t *W, const float *bias, int rows, int N, int K, float *ws,
                      size_t ws_floats, uint16_t *out, hipStream_t s);

// Backward: weight gradient of a convolution into out [out_c][k] and its
// bias gradient into bias_out [out_c] (FP32, split over the output pixels
// into `part`, then summed in split order); the input gradient (adjoint)
// masked by the ReLU of h (the layer's input activation), through
// Wt [in_c][taps x out_c] (scratch, rebuilt here).
hipError_t conv_dw(bool depth_input, const void *in, const uint16_t *dy, const ConvGeom &g, float *part,
                   size_t part_floats, float *out, float *bias_out, hipStream_t s);
// Column sums of a BF16 [rows][D] matrix (bias gradients), chunked through
// part and summed in chunk order (deterministic).
hipError_t colsum(const uint16_t *g, int rows, int D, float *part, size_t part_floats, float *out, hipStream_t s);
hipError_t conv_dx(const uint16_t *dy, const uint16_t *W, uint16_t *Wt, const uint16_t *h, const ConvGeom &g,
                   uint16_t *dx, hipStream_t s);
hipError_t ppo_heads(const uint16_t *h, const float *state, const float *aw, const float *ab, const float *vw,
                     const float *vb, const float *log_std, int A, int S, const float *actions, const float *old_logp,
                     const float *adv, const float *ret, float clip, float vcoef, float *gm, float *gls, float *gv,
                     float *terms, uint16_t *d4, hipStream_t s);
// The heads' parameter gradients and the loss statistics, summed over the
// samples in chunks through part (then in chunk order: deterministic).
hipError_t ppo_head_grads(const uint16_t *h, const float *state, const float *gm, const float *gls, const float *gv,
                          const float *terms, const float *log_std, int A, int S, float ecoef, float *g_aw,
                          float *g_ab, float *g_vw, float *g_vb, float *g_ls, float *stats, float *part,
                          size_t part_floats, hipStream_t s);
hipError_t gae(const float *rew, const float *val, const uint8_t *done, const float *last, int T, int N, float gamma,
               float lam, float *adv, float *ret, hipStream_t s);

}  // namespace gal
