// The policy that consumes the depth stack in place (Section 4.2 "Approach:
// End-to-End RL"; the SimpleCNN visual encoder of the appendix on model
// sizes: three convolutions without padding or dilation, 8x8 stride 4, 4x4
// stride 2, 3x3 stride 1, each with ReLU, then a fully connected layer), with
// a Gaussian actor and a critic linear in the 512 features and the 7 joint
// angles.  BF16 weights and activations, FP32 accumulation on the matrix
// cores, FP32 heads.
//
// A convolution is one GEMM whose A operand is gathered on the fly from the
// layer's NHWC input (implicit GEMM: no im2col matrix in memory): row m =
// (env, oy, ox), column k = (ky * kw + kx) * C + c.  With C a multiple of 8,
// the 8 consecutive k a lane loads are 8 consecutive channels of one input
// pixel (one 16-byte load).  The first layer reads the batch's depth image
// directly: 8 consecutive k are 8 consecutive pixels of one image row, each
// scaled to D / (2^24 - 1) and rounded to BF16 as it is loaded.
#include "gal_internal.h"
#include "gal_policy.h"

namespace gal {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t depth_bf16(uint32_t D)
{
    const uint32_t d = D < 16777215u ? D : 16777215u;
    return f2bf((float)d / 16777215.0f);
}

// Y[m][n] = relu(sum_k A(m, k) W[n][k] + b[n]) in BF16, A gathered from the
// layer input (DEPTH: the u32 depth images, one channel).  One workgroup (4
// waves) per 64 x 64 tile, as the surrogate's GEMM.
template <bool DEPTH>
__global__ __launch_bounds__(256) void k_conv_gemm(const void *__restrict__ in, const uint16_t *__restrict__ W,
                                                   const float *__restrict__ bias, ConvGeom g,
                                                   uint16_t *__restrict__ out)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kBK + kPad];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int M = g.rows, N = g.out_c, K = g.k;
    const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;   // M tiles on x (up to 2^31 - 1)
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    // this thread's A row, decomposed once: env, output pixel
    const int r = t >> 2, kk = (t & 3) * 8;
    const int m = m0 + r;
    const bool mrow = m < M;
    size_t base = 0;
    {
        const int per = g.oh * g.ow;
        const int e = mrow ? m / per : 0, rem = mrow ? m - e * per : 0;
        const int oy = rem / g.ow, ox = rem - oy * g.ow;
        base = (((size_t)e * g.ih + (size_t)(g.stride * oy)) * g.iw + (size_t)(g.stride * ox)) * g.in_c;
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += kBK) {
        // ---- A tile: 8 consecutive k of row m
        {
            const int k = k0 + kk;
            uint16_t v[8];
            if (mrow && k < K) {
                if (DEPTH) {
                    // k = ky * kw + kx, 8 | kw: pixels (ky, kx .. kx + 7) of the window
                    const int ky = k / g.kw, kx = k - ky * g.kw;
                    const uint32_t *p = static_cast<const uint32_t *>(in) + base + (size_t)ky * g.iw + kx;
                    const uint4 q0 = *reinterpret_cast<const uint4 *>(p);
                    const uint4 q1 = *reinterpret_cast<const uint4 *>(p + 4);
                    v[0] = depth_bf16(q0.x); v[1] = depth_bf16(q0.y); v[2] = depth_bf16(q0.z); v[3] = depth_bf16(q0.w);
                    v[4] = depth_bf16(q1.x); v[5] = depth_bf16(q1.y); v[6] = depth_bf16(q1.z); v[7] = depth_bf16(q1.w);
                } else {
                    // k = (ky * kw + kx) * C + c, 8 | C: channels c .. c + 7 of one pixel
                    const int tap = k / g.in_c, c = k - tap * g.in_c;
                    const int ky = tap / g.kw, kx = tap - ky * g.kw;
                    const uint16_t *p = static_cast<const uint16_t *>(in) + base +
                                        ((size_t)ky * g.iw + (size_t)kx) * g.in_c + c;
                    const uint4 q = *reinterpret_cast<const uint4 *>(p);
                    memcpy(v, &q, 16);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = 0;
            }
            memcpy(&As[r][kk], v, 16);
        }
        // ---- B tile: W [N][K] rows
        {
            const int n = n0 + r, k = k0 + kk;
            uint16_t v[8];
            if (n < N && k + 8 <= K) {
                const uint4 q = *reinterpret_cast<const uint4 *>(W + (size_t)n * K + k);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (n < N && k + j < K) ? W[(size_t)n * K + k + j] : 0;
            }
            memcpy(&Bs[r][kk], v, 16);
        }
        __syncthreads();
        const int r16 = lane & 15, kq = (lane >> 4) * 8;
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + i * 16 + r16][kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + j * 16 + r16][kq]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int mm = m0 + wm + i * 16 + (lane >> 4) * 4 + q;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (mm >= M || n >= N) continue;
                float v = acc[i][j][q] + bias[n];
                v = v > 0.f ? v : 0.f;
                out[(size_t)mm * N + n] = f2bf(v);
            }
}

// The heads of env e (one wave): f = [h (BF16 features), q (joint angles)];
// mean_a = b_a + sum_k W_a[k] f_k, value = b_v + sum_k w_v[k] f_k (FP32,
// lane-strided partial sums combined by a fixed butterfly); the action
// mean + std * noise and its Gaussian log-density sum_a (-noise_a^2 / 2 -
// log_std_a) - A log(2 pi) / 2 (noise null: the mean, no log-density).
__global__ __launch_bounds__(256) void k_policy_heads(const uint16_t *__restrict__ h, const float *__restrict__ state,
                                                      const float *__restrict__ aw, const float *__restrict__ ab,
                                                      const float *__restrict__ vw, const float *__restrict__ vb,
                                                      const float *__restrict__ log_std, int A, int n_envs,
                                                      const float *__restrict__ noise, float *__restrict__ actions,
                                                      float *__restrict__ value, float *__restrict__ logp)
{
    const int lane = threadIdx.x & 63;
    const int e = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)threadIdx.x / 64);
    if (e >= n_envs) return;
    constexpr int F = kPolicyFeat + kPolicyProprio;
    float f[(F + 63) / 64];
#pragma unroll
    for (int i = 0; i < (F + 63) / 64; ++i) {
        const int k = lane + 64 * i;
        f[i] = k < kPolicyFeat ? bf2f(h[(size_t)e * kPolicyFeat + k])
                               : (k < F ? state[(size_t)e * 10 + 3 + (k - kPolicyFeat)] : 0.0f);
    }
    float lp = 0.0f;
    for (int a = 0; a <= A; ++a) {
        const float *w = a < A ? aw + (size_t)a * F : vw;
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < (F + 63) / 64; ++i) {
            const int k = lane + 64 * i;
            if (k < F) s += w[k] * f[i];
        }
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        if (a < A) {
            const float mean = s + ab[a];
            float act = mean;
            if (noise) {
                const float z = noise[(size_t)e * A + a];
                act = mean + expf(log_std[a]) * z;
                lp += -0.5f * z * z - log_std[a];
            }
            if (lane == 0) actions[(size_t)e * A + a] = act;
        } else if (lane == 0 && value) {
            value[e] = s + vb[0];
        }
    }
    if (lane == 0 && noise && logp) logp[e] = lp - 0.9189385332046727f * (float)A;
}

}  // namespace

hipError_t conv_gemm(bool depth_input, const void *in, const uint16_t *W, const float *bias, const ConvGeom &g,
                     uint16_t *out, hipStream_t s)
{
    if (g.rows <= 0) return hipSuccess;
    const dim3 grid((g.rows + kBM - 1) / kBM, (g.out_c + kBN - 1) / kBN);
    if (depth_input)
        hipLaunchKernelGGL(k_conv_gemm<true>, grid, dim3(256), 0, s, in, W, bias, g, out);
    else
        hipLaunchKernelGGL(k_conv_gemm<false>, grid, dim3(256), 0, s, in, W, bias, g, out);
    return hipGetLastError();
}

hipError_t policy_heads(const uint16_t *h, const float *state, const float *aw, const float *ab, const float *vw,
                        const float *vb, const float *log_std, int A, int n_envs, const float *noise,
                        float *actions, float *value, float *logp, hipStream_t s)
{
    if (n_envs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_policy_heads, dim3((n_envs + 3) / 4), dim3(256), 0, s, h, state, aw, ab, vw, vb, log_std,
                       A, n_envs, noise, actions, value, logp);
    return hipGetLastError();
}

}  // namespace gal
