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
#include "gal_mlp.h"
#include "gal_policy.h"

#include <algorithm>

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

// x = d / (2^24 - 1) correctly rounded to FP32, without a division: for
// 1 <= d < 2^24, d / (2^24 - 1) = d 2^-24 (1 + 2^-24 + 2^-48 + ...), and the
// exact value d 2^-24 = m 2^k (m a 24-bit significand) is followed by a
// fraction m / (2^24 - 1) of one unit in the last place that always lies in
// (1/2, 1], so the rounded quotient is d 2^-24 plus one ulp (checked for
// every d against the IEEE division).  Then rounded to BF16.
__device__ __forceinline__ uint16_t depth_bf16(uint32_t D)
{
    const uint32_t d = D < 16777215u ? D : 16777215u;
    const uint32_t x = __float_as_uint((float)d * 0x1p-24f) + (d != 0u ? 1u : 0u);
    return f2bf(__uint_as_float(x));
}

// Y[m][n] = relu(sum_k A(m, k) W[n][k] + b[n]) in BF16, A gathered from the
// layer input (DEPTH: the u32 depth images, one channel).  One workgroup (4
// waves, each 32 x 32 outputs) per TM x TN tile: 64 x 64 (waves 2 x 2), or
// 128 x 32 for the layers with 32 output channels (waves stacked in M), so
// that no matrix-core work is spent on columns that do not exist.
template <int TN>
struct ConvTile {
    static constexpr int TM = TN == 64 ? 64 : 128;
    static constexpr int kALoads = TM / 64;   // 16-byte A loads per thread and K-step
    __device__ static int wm(int wave) { return TN == 64 ? (wave >> 1) * 32 : wave * 32; }
    __device__ static int wn(int wave) { return TN == 64 ? (wave & 1) * 32 : 0; }
};

template <bool DEPTH, int TN>
__global__ __launch_bounds__(256) void k_conv_gemm(const void *__restrict__ in, const uint16_t *__restrict__ W,
                                                   const float *__restrict__ bias, ConvGeom g,
                                                   uint16_t *__restrict__ out)
{
    using T = ConvTile<TN>;
    constexpr int TM = T::TM;
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][kBK + kPad];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int M = g.rows, N = g.out_c, K = g.k;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;   // M tiles on x (up to 2^31 - 1)
    const int wm = T::wm(wave), wn = T::wn(wave);
    // this thread's A rows (t / 4 and t / 4 + 64), decomposed once: env, output pixel
    const int kk = (t & 3) * 8;
    int ar[T::kALoads];
    bool mrow[T::kALoads];
    size_t base[T::kALoads];
#pragma unroll
    for (int h = 0; h < T::kALoads; ++h) {
        ar[h] = (t >> 2) + 64 * h;
        const int m = m0 + ar[h];
        mrow[h] = m < M;
        const int per = g.oh * g.ow;
        const int e = mrow[h] ? m / per : 0, rem = mrow[h] ? m - e * per : 0;
        const int oy = rem / g.ow, ox = rem - oy * g.ow;
        base[h] = (((size_t)e * g.ih + (size_t)(g.stride * oy)) * g.iw + (size_t)(g.stride * ox)) * g.in_c;
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += kBK) {
        // ---- A tile: 8 consecutive k of rows ar[h]
        const int k = k0 + kk;
        size_t koff = 0;
        if (k < K) {
            if (DEPTH) {
                // k = ky * kw + kx, 8 | kw: pixels (ky, kx .. kx + 7) of the window
                const int ky = k / g.kw, kx = k - ky * g.kw;
                koff = (size_t)ky * g.iw + kx;
            } else {
                // k = (ky * kw + kx) * C + c, 8 | C: channels c .. c + 7 of one pixel
                const int tap = k / g.in_c, c = k - tap * g.in_c;
                const int ky = tap / g.kw, kx = tap - ky * g.kw;
                koff = ((size_t)ky * g.iw + (size_t)kx) * g.in_c + c;
            }
        }
#pragma unroll
        for (int h = 0; h < T::kALoads; ++h) {
            uint16_t v[8];
            if (mrow[h] && k < K) {
                if (DEPTH) {
                    const uint32_t *p = static_cast<const uint32_t *>(in) + base[h] + koff;
                    const uint4 q0 = *reinterpret_cast<const uint4 *>(p);
                    const uint4 q1 = *reinterpret_cast<const uint4 *>(p + 4);
                    v[0] = depth_bf16(q0.x); v[1] = depth_bf16(q0.y); v[2] = depth_bf16(q0.z); v[3] = depth_bf16(q0.w);
                    v[4] = depth_bf16(q1.x); v[5] = depth_bf16(q1.y); v[6] = depth_bf16(q1.z); v[7] = depth_bf16(q1.w);
                } else {
                    const uint4 q = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(in) + base[h] + koff);
                    memcpy(v, &q, 16);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = 0;
            }
            memcpy(&As[ar[h]][kk], v, 16);
        }
        // ---- B tile: W [N][K] rows
        if (t < TN * 4) {
            const int r = t >> 2;
            const int n = n0 + r;
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

// The first convolution (8x8 stride 4 over the 128x128 depth image, one
// input channel, at most 32 output channels) with its input staged in LDS:
// one workgroup per (env, 4 output rows) converts the 20 image rows their
// windows cover to BF16 once (the windows overlap: each pixel is in up to 4
// of them) and then runs the same 16x16x32 MFMA tiles as k_conv_gemm, its A
// fragments (8 consecutive pixels of one window row) read from LDS.  Output
// rows m = (oy - oy0) * ow + ox of the block, 128 per workgroup (4 x 31
// used).
constexpr int kC1Rows = 4;                                  // output rows per workgroup
constexpr int kC1InRows = (kC1Rows - 1) * 4 + 8;            // image rows they cover
constexpr int kC1Pitch = kPolicyRes + 8;                    // LDS row pitch (BF16 values)
__global__ __launch_bounds__(256) void k_conv1_depth(const uint32_t *__restrict__ depth,
                                                     const uint16_t *__restrict__ W,
                                                     const float *__restrict__ bias, ConvGeom g,
                                                     uint16_t *__restrict__ out)
{
    __shared__ __attribute__((aligned(16))) uint16_t img[kC1InRows][kC1Pitch];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[32][64 + kPad];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nblk = (g.oh + kC1Rows - 1) / kC1Rows;
    const int env = blockIdx.x / nblk, oy0 = (blockIdx.x - env * nblk) * kC1Rows;
    const int rows_out = min(kC1Rows, g.oh - oy0);
    const int rows_in = (rows_out - 1) * 4 + 8;
    // the image rows, four pixels per thread and pass (16-byte loads)
    const uint32_t *src = depth + ((size_t)env * g.ih + (size_t)(4 * oy0)) * g.iw;
    for (int i = t; i < rows_in * (kPolicyRes / 4); i += 256) {
        const int r = i / (kPolicyRes / 4), c4 = (i - r * (kPolicyRes / 4)) * 4;
        const uint4 q = *reinterpret_cast<const uint4 *>(src + (size_t)r * g.iw + c4);
        img[r][c4 + 0] = depth_bf16(q.x);
        img[r][c4 + 1] = depth_bf16(q.y);
        img[r][c4 + 2] = depth_bf16(q.z);
        img[r][c4 + 3] = depth_bf16(q.w);
    }
    // the weights W [out_c][64], 8 per thread
    {
        const int o = t >> 3, k8 = (t & 7) * 8;
        uint4 q = make_uint4(0u, 0u, 0u, 0u);
        if (o < g.out_c) q = *reinterpret_cast<const uint4 *>(W + (size_t)o * 64 + k8);
        memcpy(&Bs[o][k8], &q, 16);
    }
    __syncthreads();
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const int wm = wave * 32;
    // this lane's two A rows: output pixel (oy0 + m / ow, m % ow), or none
    int arow[2], acol[2];
    bool alive[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = wm + 16 * i + r16;
        alive[i] = m < rows_out * g.ow;
        const int oy = alive[i] ? m / g.ow : 0;
        arow[i] = 4 * oy;
        acol[i] = 4 * (alive[i] ? m - oy * g.ow : 0);
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        // K = 32 ks + kq .. + 7: window row ky = 4 ks + kq / 8, pixels 0..7
        const int ky = 4 * ks + (lane >> 4);
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            uint2 lo = make_uint2(0u, 0u), hi = make_uint2(0u, 0u);
            if (alive[i]) {
                const uint16_t *p = &img[arow[i] + ky][acol[i]];
                lo = *reinterpret_cast<const uint2 *>(p);
                hi = *reinterpret_cast<const uint2 *>(p + 4);
            }
            const uint4 q = make_uint4(lo.x, lo.y, hi.x, hi.y);
            memcpy(&a[i], &q, 16);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[16 * j + r16][32 * ks + kq]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    const size_t obase = ((size_t)env * g.oh + (size_t)oy0) * g.ow;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int mm = wm + i * 16 + (lane >> 4) * 4 + q;
                const int n = j * 16 + (lane & 15);
                if (mm >= rows_out * g.ow || n >= g.out_c) continue;
                float v = acc[i][j][q] + bias[n];
                v = v > 0.f ? v : 0.f;
                out[(obase + (size_t)mm) * g.out_c + n] = f2bf(v);
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

// ---------------------------------------------------------------- backward

// The gathered input operand of a convolution (8 consecutive k of row m), as
// in the forward: the depth image for the first layer, NHWC BF16 otherwise.
template <bool DEPTH>
__device__ __forceinline__ void gather8(const void *in, const ConvGeom &g, int m, int k, uint16_t (&v)[8])
{
    if (m >= g.rows || k >= g.k) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = 0;
        return;
    }
    const int per = g.oh * g.ow;
    const int e = m / per, rem = m - e * per;
    const int oy = rem / g.ow, ox = rem - oy * g.ow;
    const size_t base = (((size_t)e * g.ih + (size_t)(g.stride * oy)) * g.iw + (size_t)(g.stride * ox)) * g.in_c;
    if (DEPTH) {
        const int ky = k / g.kw, kx = k - ky * g.kw;
        const uint32_t *p = static_cast<const uint32_t *>(in) + base + (size_t)ky * g.iw + kx;
        const uint4 q0 = *reinterpret_cast<const uint4 *>(p);
        const uint4 q1 = *reinterpret_cast<const uint4 *>(p + 4);
        v[0] = depth_bf16(q0.x); v[1] = depth_bf16(q0.y); v[2] = depth_bf16(q0.z); v[3] = depth_bf16(q0.w);
        v[4] = depth_bf16(q1.x); v[5] = depth_bf16(q1.y); v[6] = depth_bf16(q1.z); v[7] = depth_bf16(q1.w);
    } else {
        const int tap = k / g.in_c, c = k - tap * g.in_c;
        const int ky = tap / g.kw, kx = tap - ky * g.kw;
        const uint16_t *p = static_cast<const uint16_t *>(in) + base + ((size_t)ky * g.iw + (size_t)kx) * g.in_c + c;
        const uint4 q = *reinterpret_cast<const uint4 *>(p);
        memcpy(v, &q, 16);
    }
}

// Weight gradient of a convolution, split over the output pixels:
// part[z][o][k] = sum over rows m of split z of dY[m][o] A(m, k), A gathered
// as in the forward, dY BF16 [rows][out_c].  Workgroup (64 o x 64 k tile, one
// split), 64 rows per stage: lane = row, wave = 8-column group (and the group
// 32 columns on), so that the transposed stores into LDS (the matrix cores
// take K = rows) fall on consecutive addresses; each thread follows its row's
// (sample, oy, ox) by increments instead of divisions.  The first column
// tile's workgroups also sum the dY values they load (the bias gradient):
// bpart[z][o], each thread over its rows in order, then over the 64 lanes by
// a fixed butterfly.
constexpr int kDwRows = 64;
template <bool DEPTH>
__global__ __launch_bounds__(256) void k_conv_dw(const void *__restrict__ in, const uint16_t *__restrict__ dy,
                                                 ConvGeom g, int rows_per_split, float *__restrict__ part,
                                                 float *__restrict__ bpart)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kDwRows + kPad];   // [o][row]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kDwRows + kPad];   // [k][row]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int O = g.out_c, K = g.k;
    const int k0 = blockIdx.x * kBN;
    const int rbeg = blockIdx.y * rows_per_split, rend = min(g.rows, rbeg + rows_per_split);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool bias = bpart && blockIdx.x == 0;
    float bs[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 8; ++j) bs[h][j] = 0.f;
    // this thread's two column groups and their offsets inside the window
    int cg[2];
    size_t koff[2];
    bool kin[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cg[h] = 8 * wave + 32 * h;
        const int k = k0 + cg[h];
        kin[h] = k < K;
        koff[h] = 0;
        if (kin[h]) {
            if (DEPTH) {
                const int ky = k / g.kw, kx = k - ky * g.kw;
                koff[h] = (size_t)ky * g.iw + kx;
            } else {
                const int tap = k / g.in_c, c = k - tap * g.in_c;
                const int ky = tap / g.kw, kx = tap - ky * g.kw;
                koff[h] = ((size_t)ky * g.iw + kx) * g.in_c + c;
            }
        }
    }
    // this thread's row: m = r0 + lane, as (sample e, oy, ox)
    int e = 0, oy = 0, ox = 0;
    {
        const int m = rbeg + lane;
        const int per = g.oh * g.ow;
        e = m / per;
        const int rem = m - e * per;
        oy = rem / g.ow;
        ox = rem - oy * g.ow;
    }
    // Raw global data of one stage, loaded a stage ahead: the next stage's
    // loads are in flight during this stage's MFMAs.
    uint4 qy[2], qa[2][2];
    auto fetch = [&](int r0) {
        const int m = r0 + lane;
        const bool live = m < rend;
        const size_t base = (((size_t)e * g.ih + (size_t)(g.stride * oy)) * g.iw + (size_t)(g.stride * ox)) * g.in_c;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            qy[h] = make_uint4(0u, 0u, 0u, 0u);
            qa[h][0] = qa[h][1] = make_uint4(0u, 0u, 0u, 0u);
            if (live && cg[h] < O) qy[h] = *reinterpret_cast<const uint4 *>(dy + (size_t)m * O + cg[h]);
            if (live && kin[h]) {
                if (DEPTH) {
                    const uint32_t *p = static_cast<const uint32_t *>(in) + base + koff[h];
                    qa[h][0] = *reinterpret_cast<const uint4 *>(p);
                    qa[h][1] = *reinterpret_cast<const uint4 *>(p + 4);
                } else {
                    qa[h][0] = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(in) + base + koff[h]);
                }
            }
        }
        // the next stage's row: 64 pixels on (64 < oh * ow for every layer)
        ox += kDwRows;
        while (ox >= g.ow) {
            ox -= g.ow;
            ++oy;
        }
        if (oy >= g.oh) {
            oy -= g.oh;
            ++e;
        }
    };
    if (rbeg < rend) fetch(rbeg);
    for (int r0 = rbeg; r0 < rend; r0 += kDwRows) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // dY[m][cg .. cg + 7] -> As[o][lane]
            uint16_t v[8];
            memcpy(v, &qy[h], 16);
            if (bias) {
#pragma unroll
                for (int j = 0; j < 8; ++j) bs[h][j] += bf2f(v[j]);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) As[cg[h] + j][lane] = v[j];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // A(m, k0 + cg .. + 7) -> Bs[k][lane]
            uint16_t v[8];
            if (DEPTH) {
                const uint4 q0 = qa[h][0], q1 = qa[h][1];
                v[0] = depth_bf16(q0.x); v[1] = depth_bf16(q0.y); v[2] = depth_bf16(q0.z); v[3] = depth_bf16(q0.w);
                v[4] = depth_bf16(q1.x); v[5] = depth_bf16(q1.y); v[6] = depth_bf16(q1.z); v[7] = depth_bf16(q1.w);
            } else {
                memcpy(v, &qa[h][0], 16);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[cg[h] + j][lane] = v[j];
        }
        __syncthreads();
        if (r0 + kDwRows < rend) fetch(r0 + kDwRows);
        const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
        for (int ks = 0; ks < kDwRows; ks += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + i * 16 + r16][ks + kq]);
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + j * 16 + r16][ks + kq]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    float *dst = part + (size_t)blockIdx.y * O * K;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = wm + i * 16 + (lane >> 4) * 4 + q;
                const int k = k0 + wn + j * 16 + (lane & 15);
                if (o < O && k < K) dst[(size_t)o * K + k] = acc[i][j][q];
            }
    if (bias) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float v = bs[h][j];
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
                if (lane == 0 && cg[h] + j < O) bpart[(size_t)blockIdx.y * O + cg[h] + j] = v;
            }
    }
}

// out[i] = sum over splits of part[z][i], in split order
__global__ void k_sum_parts(const float *__restrict__ part, int splits, int64_t n, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = part[i];
    for (int z = 1; z < splits; ++z) v += part[(size_t)z * n + i];
    out[i] = v;
}

// Input gradient of a convolution (the adjoint), masked by the ReLU of the
// layer that produced the input: dX[m][c] = bf16([h[m][c] > 0] sum over
// taps (ky, kx) and o of dY[n][oy][ox][o] W[o][ky][kx][c]), where
// (oy, ox) s + (ky, kx) = (iy, ix) is an output pixel.  With stride s the
// input pixels fall into s x s classes by (iy mod s, ix mod s), and a class
// receives only the taps with (ky, kx) = (iy, ix) mod s: (kw / s)^2 of them.
// Each class (blockIdx.z) is a GEMM whose rows are its input pixels,
// K = its taps x out_c (8 consecutive o of one tap per load, zero where the
// tap reaches no output pixel) and B = Wt [in_c][taps x out_c] at its taps.
template <int TN>
__global__ __launch_bounds__(256) void k_conv_dx(const uint16_t *__restrict__ dy, const uint16_t *__restrict__ Wt,
                                                 const uint16_t *__restrict__ h, ConvGeom g,
                                                 uint16_t *__restrict__ dx)
{
    using T = ConvTile<TN>;
    constexpr int TM = T::TM;
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][kBK + kPad];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int st = g.stride, ts = g.kw / st;
    const int py = blockIdx.z / st, px = blockIdx.z - py * st;
    const int qh = (g.ih - py + st - 1) / st, qw = (g.iw - px + st - 1) / st;
    const int M = (g.rows / (g.oh * g.ow)) * qh * qw;   // input pixels of the class
    const int N = g.in_c, K = ts * ts * g.out_c, Kall = g.kw * g.kw * g.out_c;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    if (m0 >= M) return;
    const int wm = T::wm(wave), wn = T::wn(wave);
    const int kk = (t & 3) * 8;
    // this thread's A rows (t / 4 and t / 4 + 64): sample and class pixel, once
    int ar[T::kALoads], ae[T::kALoads], aqy[T::kALoads], aqx[T::kALoads];
    bool arow[T::kALoads];
#pragma unroll
    for (int hh = 0; hh < T::kALoads; ++hh) {
        ar[hh] = (t >> 2) + 64 * hh;
        const int m = m0 + ar[hh];
        arow[hh] = m < M;
        ae[hh] = aqy[hh] = aqx[hh] = 0;
        if (arow[hh]) {
            const int per = qh * qw;
            ae[hh] = m / per;
            const int rem = m - ae[hh] * per;
            aqy[hh] = rem / qw;
            aqx[hh] = rem - aqy[hh] * qw;
        }
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kBK) {
        const int k = k0 + kk;
        // the K column's tap (within the class) and output channel
        int jy = 0, jx = 0, o = 0;
        if (k < K) {
            const int tap = k / g.out_c;
            o = k - tap * g.out_c;
            jy = tap / ts;
            jx = tap - jy * ts;
        }
#pragma unroll
        for (int hh = 0; hh < T::kALoads; ++hh) {
            uint16_t v[8];
            const int oy = aqy[hh] - jy, ox = aqx[hh] - jx;
            const bool ok = arow[hh] && k < K && oy >= 0 && ox >= 0 && oy < g.oh && ox < g.ow;
            if (ok) {
                const size_t src = (((size_t)ae[hh] * g.oh + (size_t)oy) * g.ow + (size_t)ox) * g.out_c + o;
                const uint4 q = *reinterpret_cast<const uint4 *>(dy + src);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = 0;
            }
            memcpy(&As[ar[hh]][kk], v, 16);
        }
        if (t < TN * 4) {
            const int r = t >> 2;
            const int n = n0 + r;
            uint16_t v[8];
            if (n < N && k < K) {
                // 8 | out_c: the 8 values share one tap
                const int ky = py + st * jy, kx = px + st * jx;
                const uint4 q = *reinterpret_cast<const uint4 *>(Wt + (size_t)n * Kall + (size_t)(ky * g.kw + kx) * g.out_c + o);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = 0;
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
        for (int q = 0; q < 4; ++q) {
            const int mm = m0 + wm + i * 16 + (lane >> 4) * 4 + q;
            if (mm >= M) continue;
            const int per = qh * qw;
            const int ee = mm / per, rem = mm - ee * per;
            const int yy = rem / qw, xx = rem - yy * qw;
            const size_t row = ((size_t)ee * g.ih + (size_t)(py + st * yy)) * g.iw + (size_t)(px + st * xx);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (n >= N) continue;
                const uint16_t hv = h[row * N + n];
                const bool on = (hv & 0x8000u) == 0 && (hv & 0x7FFFu) != 0;
                dx[row * N + n] = f2bf(on ? acc[i][j][q] : 0.f);
            }
        }
}

// Wt[c][tap * O + o] = W[o][tap][c] (the adjoint's B operand)
__global__ void k_conv_wt(const uint16_t *__restrict__ W, int O, int taps, int C, uint16_t *__restrict__ Wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= O * taps * C) return;
    const int o = i / (taps * C), rem = i - o * taps * C, tap = rem / C, c = rem - tap * C;
    Wt[((size_t)c * taps + tap) * O + o] = W[i];
}

// The PPO loss of sample s (one wave): the heads from h4 and the joint angles,
// logp of the taken action, the ratio to the behaviour policy's, the clipped
// surrogate and the value error.  Writes per sample: gm [A] = dL/dmean,
// gls [A] = dL/dlog_std (without the entropy term), gv = dL/dV, the loss terms
// [3] (policy, value, 0), and d4 = bf16([h4 > 0] (gm W_a + gv w_v)) over the
// 512 features.  L is the mean over S samples.
__global__ __launch_bounds__(256) void k_ppo_heads(const uint16_t *__restrict__ h, const float *__restrict__ state,
                                                   const float *__restrict__ aw, const float *__restrict__ ab,
                                                   const float *__restrict__ vw, const float *__restrict__ vb,
                                                   const float *__restrict__ log_std, int A, int S,
                                                   const float *__restrict__ actions, const float *__restrict__ old_logp,
                                                   const float *__restrict__ adv, const float *__restrict__ ret,
                                                   float clip, float vcoef, float *__restrict__ gm,
                                                   float *__restrict__ gls, float *__restrict__ gv,
                                                   float *__restrict__ terms, uint16_t *__restrict__ d4)
{
    const int lane = threadIdx.x & 63;
    const int e = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)threadIdx.x / 64);
    if (e >= S) return;
    constexpr int F = kPolicyFeat + kPolicyProprio;
    constexpr int NF = (F + 63) / 64;
    float f[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const int k = lane + 64 * i;
        f[i] = k < kPolicyFeat ? bf2f(h[(size_t)e * kPolicyFeat + k])
                               : (k < F ? state[(size_t)e * 10 + 3 + (k - kPolicyFeat)] : 0.0f);
    }
    float zs[kPolicyMaxAct];
    float logp = 0.0f, V = 0.0f;
    for (int a = 0; a <= A; ++a) {
        const float *w = a < A ? aw + (size_t)a * F : vw;
        float sum = 0.0f;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int k = lane + 64 * i;
            if (k < F) sum += w[k] * f[i];
        }
        for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
        if (a < A) {
            const float mean = sum + ab[a];
            const float z = (actions[(size_t)e * A + a] - mean) / expf(log_std[a]);
            zs[a] = z;
            logp += -0.5f * z * z - log_std[a];
        } else {
            V = sum + vb[0];
        }
    }
    logp -= 0.9189385332046727f * (float)A;
    const float r = expf(logp - old_logp[e]);
    const float Ad = adv[e];
    const float rc = fminf(fmaxf(r, 1.0f - clip), 1.0f + clip);
    const float s1 = r * Ad, s2 = rc * Ad;
    const bool use1 = s1 <= s2;
    const float invS = 1.0f / (float)S;
    const float dlogp = use1 ? -Ad * r * invS : 0.0f;
    const float dv = vcoef * 2.0f * (V - ret[e]) * invS;
    float g_mean[kPolicyMaxAct];
    for (int a = 0; a < A; ++a) {
        g_mean[a] = dlogp * zs[a] / expf(log_std[a]);
        if (lane == 0) {
            gm[(size_t)e * A + a] = g_mean[a];
            gls[(size_t)e * A + a] = dlogp * (zs[a] * zs[a] - 1.0f);
        }
    }
    if (lane == 0) {
        gv[e] = dv;
        terms[(size_t)e * 3 + 0] = -(use1 ? s1 : s2);
        terms[(size_t)e * 3 + 1] = (V - ret[e]) * (V - ret[e]);
        terms[(size_t)e * 3 + 2] = r;
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const int k = lane + 64 * i;
        if (k < kPolicyFeat) {
            float df = dv * vw[k];
            for (int a = 0; a < A; ++a) df += g_mean[a] * aw[(size_t)a * F + k];
            d4[(size_t)e * kPolicyFeat + k] = f2bf(f[i] > 0.0f ? df : 0.0f);
        }
    }
}

// Gradients of the heads as sums over the samples, in chunks of kHeadChunk
// samples (one thread per output and chunk, the chunks then added in chunk
// order: deterministic).  Output i of a chunk: i < (A + 1) F the actor's
// W [A][F] then the critic's w [F] (gradient of the output times the
// feature), then the actor bias [A], log_std [A] (without the entropy term),
// the critic bias, and the three loss terms (policy, value, ratio).
constexpr int kHeadChunk = 512;
__global__ void k_ppo_head_part(const uint16_t *__restrict__ h, const float *__restrict__ state,
                                const float *__restrict__ gm, const float *__restrict__ gls,
                                const float *__restrict__ gv, const float *__restrict__ terms, int A, int S,
                                int nout, float *__restrict__ part)
{
    constexpr int F = kPolicyFeat + kPolicyProprio;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nout) return;
    const int e0 = blockIdx.y * kHeadChunk, e1 = min(S, e0 + kHeadChunk);
    const int nw = (A + 1) * F;
    float acc = 0.0f;
    if (i < nw) {
        const int a = i / F, k = i - a * F;
        for (int e = e0; e < e1; ++e) {
            const float fk = k < kPolicyFeat ? bf2f(h[(size_t)e * kPolicyFeat + k])
                                             : state[(size_t)e * 10 + 3 + (k - kPolicyFeat)];
            acc += (a < A ? gm[(size_t)e * A + a] : gv[e]) * fk;
        }
    } else if (i < nw + A) {
        const int a = i - nw;
        for (int e = e0; e < e1; ++e) acc += gm[(size_t)e * A + a];
    } else if (i < nw + 2 * A) {
        const int a = i - nw - A;
        for (int e = e0; e < e1; ++e) acc += gls[(size_t)e * A + a];
    } else if (i == nw + 2 * A) {
        for (int e = e0; e < e1; ++e) acc += gv[e];
    } else {
        const int t = i - nw - 2 * A - 1;
        for (int e = e0; e < e1; ++e) acc += terms[(size_t)e * 3 + t];
    }
    part[(size_t)blockIdx.y * nout + i] = acc;
}

// The summed head outputs into the gradient vector and the statistics [4] =
// mean policy loss, mean value error, entropy, mean ratio.
__global__ void k_ppo_head_finish(const float *__restrict__ sum, const float *__restrict__ log_std, int A, int S,
                                  float ecoef, float *__restrict__ g_aw, float *__restrict__ g_ab,
                                  float *__restrict__ g_vw, float *__restrict__ g_vb, float *__restrict__ g_ls,
                                  float *__restrict__ stats)
{
    constexpr int F = kPolicyFeat + kPolicyProprio;
    const int nw = (A + 1) * F;
    for (int i = threadIdx.x; i < nw + 2 * A + 1; i += blockDim.x) {
        const float v = sum[i];
        if (i < A * F) g_aw[i] = v;
        else if (i < nw) g_vw[i - A * F] = v;
        else if (i < nw + A) g_ab[i - nw] = v;
        else if (i < nw + 2 * A) g_ls[i - nw - A] = v - ecoef;
        else g_vb[0] = v;
    }
    if (threadIdx.x == 0 && stats) {
        float ent = 0.0f;
        for (int a = 0; a < A; ++a) ent += log_std[a] + 1.4189385332046727f;
        const float *t = sum + nw + 2 * A + 1;
        stats[0] = t[0] / (float)S;
        stats[1] = t[1] / (float)S;
        stats[2] = ent;
        stats[3] = t[2] / (float)S;
    }
}

// Column sums of a BF16 [rows][D] matrix in chunks of `per` rows: part
// [chunk][D] (one thread per column; the chunks are summed in order after).
__global__ void k_colsum_chunks(const uint16_t *__restrict__ g, int rows, int D, int per, float *__restrict__ part)
{
    const int c = threadIdx.x, chunk = blockIdx.x;
    if (c >= D) return;
    const int r0 = chunk * per, r1 = min(rows, r0 + per);
    float acc = 0.0f;
    for (int r = r0; r < r1; ++r) acc += bf2f(g[(size_t)r * D + c]);
    part[(size_t)chunk * D + c] = acc;
}

// The fully connected layer from split-K partial products: out[m][n] =
// bf16(relu(sum over splits in order of part[z][m][n] + b[n])).
__global__ void k_fc_finish(const float *__restrict__ part, int splits, int M, int N, const float *__restrict__ bias,
                            uint16_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_all = (int64_t)M * N;
    if (i >= n_all) return;
    float v = part[i];
    for (int z = 1; z < splits; ++z) v += part[(size_t)z * n_all + i];
    v += bias[i % N];
    out[i] = f2bf(v > 0.f ? v : 0.f);
}

// Generalised advantage estimation, one thread per env, backwards in time.
__global__ void k_gae(const float *__restrict__ rew, const float *__restrict__ val, const uint8_t *__restrict__ done,
                      const float *__restrict__ last, int T, int N, float gamma, float lam, float *__restrict__ adv,
                      float *__restrict__ ret)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float nv = last[n], na = 0.0f;
    for (int t = T - 1; t >= 0; --t) {
        const size_t i = (size_t)t * N + n;
        const float live = done[i] ? 0.0f : 1.0f;
        const float delta = (rew[i] + gamma * nv * live) - val[i];
        na = delta + gamma * lam * live * na;
        adv[i] = na;
        ret[i] = na + val[i];
        nv = val[i];
    }
}

}  // namespace

hipError_t conv_dw(bool depth_input, const void *in, const uint16_t *dy, const ConvGeom &g, float *part,
                   size_t part_floats, float *out, float *bias_out, hipStream_t s)
{
    if (g.rows <= 0) {
        hipError_t e = hipMemsetAsync(out, 0, sizeof(float) * g.out_c * g.k, s);
        if (e == hipSuccess) e = hipMemsetAsync(bias_out, 0, sizeof(float) * g.out_c, s);
        return e;
    }
    if (g.out_c > kBM) return hipErrorInvalidValue;
    const size_t slab = (size_t)g.out_c * g.k;
    int splits = (int)std::min<size_t>(part_floats / (slab + g.out_c), (size_t)256);
    splits = std::max(1, std::min(splits, (g.rows + 4095) / 4096));
    int per = (g.rows + splits - 1) / splits;
    per = (per + kDwRows - 1) / kDwRows * kDwRows;
    splits = (g.rows + per - 1) / per;
    const dim3 grid((g.k + kBN - 1) / kBN, splits);
    float *bpart = part + (size_t)splits * slab;
    if (depth_input)
        hipLaunchKernelGGL(k_conv_dw<true>, grid, dim3(256), 0, s, in, dy, g, per, part, bpart);
    else
        hipLaunchKernelGGL(k_conv_dw<false>, grid, dim3(256), 0, s, in, dy, g, per, part, bpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)slab;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, splits, n, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((g.out_c + 255) / 256)), dim3(256), 0, s, bpart, splits,
                       (int64_t)g.out_c, bias_out);
    return hipGetLastError();
}

hipError_t colsum(const uint16_t *g, int rows, int D, float *part, size_t part_floats, float *out, hipStream_t s)
{
    if (rows <= 0) return hipMemsetAsync(out, 0, sizeof(float) * D, s);
    // about 256 chunks of at least 64 rows
    const int per = std::max(64, (rows + 255) / 256);
    const int chunks = (rows + per - 1) / per;
    if ((size_t)chunks * D > part_floats || D > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colsum_chunks, dim3(chunks), dim3((D + 63) / 64 * 64), 0, s, g, rows, D, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3((D + 255) / 256), dim3(256), 0, s, part, chunks, (int64_t)D, out);
    return hipGetLastError();
}

hipError_t conv_dx(const uint16_t *dy, const uint16_t *W, uint16_t *Wt, const uint16_t *h, const ConvGeom &g,
                   uint16_t *dx, hipStream_t s)
{
    const int taps = g.kw * g.kw;
    const int nw = g.out_c * taps * g.in_c;
    hipLaunchKernelGGL(k_conv_wt, dim3((nw + 255) / 256), dim3(256), 0, s, W, g.out_c, taps, g.in_c, Wt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.kw % g.stride || g.out_c % 8) return hipErrorInvalidValue;
    // the largest parity class: ceil(ih / s) x ceil(iw / s) input pixels per sample
    const int M = (g.rows / (g.oh * g.ow)) * ((g.ih + g.stride - 1) / g.stride) * ((g.iw + g.stride - 1) / g.stride);
    if (M <= 0) return hipSuccess;
    const dim3 grid((M + kBM - 1) / kBM, (g.in_c + kBN - 1) / kBN, g.stride * g.stride);
    if (g.in_c <= 32) {
        const dim3 grid32((M + 127) / 128, 1, g.stride * g.stride);
        hipLaunchKernelGGL(k_conv_dx<32>, grid32, dim3(256), 0, s, dy, Wt, h, g, dx);
    } else {
        hipLaunchKernelGGL(k_conv_dx<64>, grid, dim3(256), 0, s, dy, Wt, h, g, dx);
    }
    return hipGetLastError();
}

hipError_t ppo_heads(const uint16_t *h, const float *state, const float *aw, const float *ab, const float *vw,
                     const float *vb, const float *log_std, int A, int S, const float *actions, const float *old_logp,
                     const float *adv, const float *ret, float clip, float vcoef, float *gm, float *gls, float *gv,
                     float *terms, uint16_t *d4, hipStream_t s)
{
    if (S <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ppo_heads, dim3((S + 3) / 4), dim3(256), 0, s, h, state, aw, ab, vw, vb, log_std, A, S,
                       actions, old_logp, adv, ret, clip, vcoef, gm, gls, gv, terms, d4);
    return hipGetLastError();
}

hipError_t ppo_head_grads(const uint16_t *h, const float *state, const float *gm, const float *gls, const float *gv,
                          const float *terms, const float *log_std, int A, int S, float ecoef, float *g_aw,
                          float *g_ab, float *g_vw, float *g_vb, float *g_ls, float *stats, float *part,
                          size_t part_floats, hipStream_t s)
{
    if (S <= 0) return hipErrorInvalidValue;
    const int nout = (A + 1) * (kPolicyFeat + kPolicyProprio) + 2 * A + 1 + 3;
    const int chunks = (S + kHeadChunk - 1) / kHeadChunk;
    if ((size_t)(chunks + 1) * nout > part_floats) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ppo_head_part, dim3((nout + 255) / 256, chunks), dim3(256), 0, s, h, state, gm, gls, gv,
                       terms, A, S, nout, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    float *sum = part + (size_t)chunks * nout;
    hipLaunchKernelGGL(k_sum_parts, dim3((nout + 255) / 256), dim3(256), 0, s, part, chunks, (int64_t)nout, sum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ppo_head_finish, dim3(1), dim3(256), 0, s, sum, log_std, A, S, ecoef, g_aw, g_ab, g_vw,
                       g_vb, g_ls, stats);
    return hipGetLastError();
}

hipError_t gae(const float *rew, const float *val, const uint8_t *done, const float *last, int T, int N, float gamma,
               float lam, float *adv, float *ret, hipStream_t s)
{
    if (N <= 0 || T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gae, dim3((N + 255) / 256), dim3(256), 0, s, rew, val, done, last, T, N, gamma, lam, adv, ret);
    return hipGetLastError();
}

hipError_t conv_gemm(bool depth_input, const void *in, const uint16_t *W, const float *bias, const ConvGeom &g,
                     uint16_t *out, hipStream_t s)
{
    if (g.rows <= 0) return hipSuccess;
    if (depth_input && g.ih == kPolicyRes && g.iw == kPolicyRes && g.kw == 8 && g.stride == 4 && g.in_c == 1 &&
        g.k == 64 && g.out_c <= 32 && kC1Rows * g.ow <= 128 && (g.oh - 1) * 4 + 8 <= g.ih) {
        const int envs = g.rows / (g.oh * g.ow);
        const dim3 grid((unsigned)(envs * ((g.oh + kC1Rows - 1) / kC1Rows)));
        hipLaunchKernelGGL(k_conv1_depth, grid, dim3(256), 0, s, static_cast<const uint32_t *>(in), W, bias, g, out);
        return hipGetLastError();
    }
    if (g.out_c <= 32) {
        const dim3 grid((g.rows + 127) / 128, 1);
        if (depth_input)
            hipLaunchKernelGGL((k_conv_gemm<true, 32>), grid, dim3(256), 0, s, in, W, bias, g, out);
        else
            hipLaunchKernelGGL((k_conv_gemm<false, 32>), grid, dim3(256), 0, s, in, W, bias, g, out);
        return hipGetLastError();
    }
    const dim3 grid((g.rows + 63) / 64, (g.out_c + 63) / 64);
    if (depth_input)
        hipLaunchKernelGGL((k_conv_gemm<true, 64>), grid, dim3(256), 0, s, in, W, bias, g, out);
    else
        hipLaunchKernelGGL((k_conv_gemm<false, 64>), grid, dim3(256), 0, s, in, W, bias, g, out);
    return hipGetLastError();
}

int fc_splits(int rows, int N, int K)
{
    const int tiles = ((rows + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    int splits = 512 / std::max(tiles, 1);              // about 512 workgroups
    splits = std::min(splits, K / 512);                 // at least 512 columns of K each
    return std::max(splits, 1);
}

hipError_t fc_forward(const uint16_t *x, const uint16_t *W, const float *bias, int rows, int N, int K, float *ws,
                      size_t ws_floats, uint16_t *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int splits = fc_splits(rows, N, K);
    if (splits == 1 || !ws || (size_t)splits * rows * N > ws_floats)
        return mlp_gemm(kGemmFwd, x, W, rows, N, K, K, K, bias, nullptr, 0, nullptr, out, N, s);
    hipError_t e = mlp_gemm_parts(x, W, rows, N, K, K, K, splits, ws, s);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)rows * N;
    hipLaunchKernelGGL(k_fc_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ws, splits, rows, N, bias, out);
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
