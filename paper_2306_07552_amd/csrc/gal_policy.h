// Internal definitions of the policy network that consumes the depth stack
// (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

constexpr int kPolicyRes = 128;      // depth image edge the encoder takes
constexpr int kPolicyFeat = 512;     // encoder features
constexpr int kPolicyProprio = 7;    // joint angles fed to the heads beside the features

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

}  // namespace gal
