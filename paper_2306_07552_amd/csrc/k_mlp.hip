// Collision-surrogate MLP on the matrix cores (gfx950 v_mfma_f32_16x16x32_bf16).
//
// The surrogate is this build's learned pre-filter for the static-scene
// overlap test of the kinematic step (Section 3.2 of the paper describes the
// exact test it stands in front of).  Network: 2112 inputs -> 4 x 256 ReLU ->
// 1 logit.  Weights and activations are BF16 (round to nearest even after
// bias + ReLU), accumulation FP32, biases and master weights FP32.
//
// GEMM: C[M][N] = sum_k opA[m][k] * opB[k][n] with
//   opA[m][k] = TA ? A[k*lda + m] : A[m*lda + k]
//   opB[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n]
// One workgroup (4 waves) computes a 64x64 tile; each wave a 32x32 quarter as
// 2x2 MFMA 16x16 blocks; K advances 32 at a time through LDS, operands laid
// out so each lane reads its 8 consecutive K values with one 16-byte load.
#include "gal_internal.h"
#include "gal_mlp.h"

namespace gal {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float relu(float v) { return v > 0.f ? v : 0.f; }

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                              int M, int N, int K, int lda, int ldb,
                                              const float *__restrict__ bias,
                                              const uint16_t *__restrict__ mask, int ldm,
                                              float *__restrict__ Cf, uint16_t *__restrict__ Cb,
                                              int ldc)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kBK + kPad];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    // split-K: workgroup z reduces K range [kbeg, kend) into its own output slab
    const int kchunk = ((K + (int)gridDim.z - 1) / (int)gridDim.z + kBK - 1) / kBK * kBK;
    const int kbeg = (int)blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    if (gridDim.z > 1 && Cf) Cf += (size_t)blockIdx.z * M * ldc;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        // ---- A tile (64 x 32) -> As[m][k]
        if (!TA) {
            const int r = t >> 2, kk = (t & 3) * 8;
            const int m = m0 + r, k = k0 + kk;
            uint16_t v[8];
            if (m < M && k + 8 <= kend && ((((size_t)m * lda + k) & 7) == 0)) {
                const uint4 q = *reinterpret_cast<const uint4 *>(A + (size_t)m * lda + k);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (m < M && k + j < kend) ? A[(size_t)m * lda + k + j] : 0;
            }
            memcpy(&As[r][kk], v, 16);
        } else {
            // lane = K row, so that the transposed LDS stores of a wave fall
            // on consecutive addresses (32 K rows x 8 column groups)
            const int kk = t & 31, mm = (t >> 5) * 8;
            const int k = k0 + kk, m = m0 + mm;
            uint16_t v[8];
            if (k < kend && m + 8 <= M && ((((size_t)k * lda + m) & 7) == 0)) {
                const uint4 q = *reinterpret_cast<const uint4 *>(A + (size_t)k * lda + m);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (k < kend && m + j < M) ? A[(size_t)k * lda + m + j] : 0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) As[mm + j][kk] = v[j];
        }
        // ---- B tile (32 x 64) -> Bs[n][k]
        if (TB) {
            const int r = t >> 2, kk = (t & 3) * 8;
            const int n = n0 + r, k = k0 + kk;
            uint16_t v[8];
            if (n < N && k + 8 <= kend && ((((size_t)n * ldb + k) & 7) == 0)) {
                const uint4 q = *reinterpret_cast<const uint4 *>(B + (size_t)n * ldb + k);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (n < N && k + j < kend) ? B[(size_t)n * ldb + k + j] : 0;
            }
            memcpy(&Bs[r][kk], v, 16);
        } else {
            const int kk = t >> 3, nn = (t & 7) * 8;
            const int k = k0 + kk, n = n0 + nn;
            uint16_t v[8];
            if (k < kend && n + 8 <= N && ((((size_t)k * ldb + n) & 7) == 0)) {
                const uint4 q = *reinterpret_cast<const uint4 *>(B + (size_t)k * ldb + n);
                memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (k < kend && n + j < N) ? B[(size_t)k * ldb + n + j] : 0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[nn + j][kk] = v[j];
        }
        __syncthreads();
        // ---- 2x2 MFMA 16x16x32 per wave; lane: row/col = lane % 16, K slice = 8*(lane/16)
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
    // ---- epilogue: lane holds column n = lane % 16 and rows 4*(lane/16) + 0..3
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= M || n >= N) continue;
                float v = acc[i][j][r];
                if (EPI == kEpiF32) {
                    if (bias) v += bias[n];
                    Cf[(size_t)m * ldc + n] = v;
                } else if (EPI == kEpiBiasReluBf16) {
                    v += bias[n];
                    v = v > 0.f ? v : 0.f;
                    Cb[(size_t)m * ldc + n] = f2bf(v);
                } else {   // kEpiMaskBf16: gradient through ReLU
                    const uint16_t h = mask[(size_t)m * ldm + n];
                    const bool on = (h & 0x8000u) == 0 && (h & 0x7FFFu) != 0;
                    Cb[(size_t)m * ldc + n] = f2bf(on ? v : 0.f);
                }
            }
}

// logit head: z[i] = sum_j h[i][j] * w[j] + b  (one wave per row)
__global__ void k_head_fwd(const uint16_t *__restrict__ h, const uint16_t *__restrict__ w,
                           const float *__restrict__ b, int rows, int D, float *__restrict__ z)
{
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    float acc = 0.f;
    for (int j = lane; j < D; j += 64) acc += bf2f(h[(size_t)row * D + j]) * bf2f(w[j]);
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) z[row] = acc + b[0];
}

// weighted logistic loss and dz = w (sigmoid(z) - y) / rows
__global__ void k_loss(const float *__restrict__ z, const float *__restrict__ y, int rows, float pos_w,
                       float *__restrict__ dz, float *__restrict__ loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < rows) {
        const float zi = z[i], yi = y[i];
        const float w = yi > 0.5f ? pos_w : 1.f;
        const float p = 1.f / (1.f + expf(-zi));
        dz[i] = w * (p - yi) / (float)rows;
        l = w * ((zi > 0.f ? zi : 0.f) - zi * yi + log1pf(expf(-fabsf(zi)))) / (float)rows;
    }
    for (int d = 32; d >= 1; d >>= 1) l += __shfl_xor(l, d, 64);
    if (loss && (threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// head backward: dpre[i][j] = bf16(dz_i * w_j * [h > 0]); dw[j] += sum_i dz_i h[i][j];
// db += sum_i dz_i.  Block = 64 rows x D columns (thread = column); partial
// sums are added atomically (dw, db zeroed by the caller).
__global__ void k_head_bwd(const uint16_t *__restrict__ h, const uint16_t *__restrict__ w,
                           const float *__restrict__ dz, int rows, int D,
                           uint16_t *__restrict__ dpre, float *__restrict__ dw, float *__restrict__ db)
{
    const int j = threadIdx.x;
    const int i0 = blockIdx.x * 64, i1 = min(rows, i0 + 64);
    if (j < D) {
        const float wj = bf2f(w[j]);
        float acc = 0.f;
        for (int i = i0; i < i1; ++i) {
            const uint16_t hv = h[(size_t)i * D + j];
            const float d = dz[i];
            acc += d * bf2f(hv);
            const bool on = (hv & 0x8000u) == 0 && (hv & 0x7FFFu) != 0;
            dpre[(size_t)i * D + j] = f2bf(on ? d * wj : 0.f);
        }
        atomicAdd(&dw[j], acc);
    }
    if (j == 0) {
        float acc = 0.f;
        for (int i = i0; i < i1; ++i) acc += dz[i];
        atomicAdd(db, acc);
    }
}

// bias gradient: column sums of a BF16 [rows][D] matrix, 64 rows per block
// (out zeroed by the caller)
__global__ void k_colsum(const uint16_t *__restrict__ g, int rows, int D, float *__restrict__ out)
{
    const int j = threadIdx.x;
    const int i0 = blockIdx.x * 64, i1 = min(rows, i0 + 64);
    if (j >= D) return;
    float acc = 0.f;
    for (int i = i0; i < i1; ++i) acc += bf2f(g[(size_t)i * D + j]);
    atomicAdd(&out[j], acc);
}

// Adam on the FP32 master parameters, then their BF16 copy (weights only)
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t *__restrict__ wb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float *__restrict__ a, int64_t n, uint16_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(a[i]);
}

// out[i] = sum over splits of part[sp][i], in split order (deterministic)
__global__ void k_sum_splits(const float *__restrict__ part, int splits, int64_t n, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = part[i];
    for (int sp = 1; sp < splits; ++sp) v += part[(size_t)sp * n + i];
    out[i] = v;
}

template <bool TA, bool TB, int EPI>
hipError_t gemm(const uint16_t *A, const uint16_t *B, int M, int N, int K, int lda, int ldb,
                const float *bias, const uint16_t *mask, int ldm, float *Cf, uint16_t *Cb, int ldc,
                hipStream_t s, int splits = 1, float *part = nullptr)
{
    dim3 grid((N + kBN - 1) / kBN, (M + kBM - 1) / kBM, splits > 1 ? splits : 1);
    if (splits > 1) {
        // each split into its own [M][N] slab of part, then their ordered sum into Cf
        hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, A, B, M, N, K, lda, ldb, bias,
                           mask, ldm, part, Cb, N);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t n = (int64_t)M * N;
        if (ldc != N) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, splits, n, Cf);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, A, B, M, N, K, lda, ldb, bias,
                       mask, ldm, Cf, Cb, ldc);
    return hipGetLastError();
}

}  // namespace

hipError_t mlp_gemm(int variant, const uint16_t *A, const uint16_t *B, int M, int N, int K, int lda,
                    int ldb, const float *bias, const uint16_t *mask, int ldm, float *Cf,
                    uint16_t *Cb, int ldc, hipStream_t s, float *ws, size_t ws_floats)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    switch (variant) {
    case kGemmFwd:    // Y = X W^T (+ b, ReLU, BF16)
        return gemm<false, true, kEpiBiasReluBf16>(A, B, M, N, K, lda, ldb, bias, mask, ldm, Cf, Cb, ldc, s);
    case kGemmDx:     // dpre_prev = mask(dY W)
        return gemm<false, false, kEpiMaskBf16>(A, B, M, N, K, lda, ldb, bias, mask, ldm, Cf, Cb, ldc, s);
    case kGemmDw: {   // dW = dY^T X, split over the rows (K) into the workspace when given
        const int tiles = ((N + kBN - 1) / kBN) * ((M + kBM - 1) / kBM);
        int splits = 1;
        if (ws && ldc == N) {
            splits = (int)(512 / tiles);                          // aim at >= 512 workgroups
            splits = splits > K / 256 ? K / 256 : splits;         // >= 256 rows per split
            const int64_t cap = (int64_t)(ws_floats / ((size_t)M * N));
            splits = splits > cap ? (int)cap : splits;
            splits = splits > kMaxDwSplits ? kMaxDwSplits : splits;
            if (splits < 1) splits = 1;
        }
        return gemm<true, false, kEpiF32>(A, B, M, N, K, lda, ldb, bias, mask, ldm, Cf, Cb, ldc, s,
                                          splits, ws);
    }
    case kGemmNtF32:  // plain C = A B^T in FP32 (tests)
        return gemm<false, true, kEpiF32>(A, B, M, N, K, lda, ldb, bias, mask, ldm, Cf, Cb, ldc, s);
    case kGemmNnF32:
        return gemm<false, false, kEpiF32>(A, B, M, N, K, lda, ldb, bias, mask, ldm, Cf, Cb, ldc, s);
    case kGemmTnF32:
        return gemm<true, false, kEpiF32>(A, B, M, N, K, lda, ldb, bias, mask, ldm, Cf, Cb, ldc, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t mlp_gemm_parts(const uint16_t *A, const uint16_t *B, int M, int N, int K, int lda, int ldb, int splits,
                          float *part, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (splits < 1 || !part) return hipErrorInvalidValue;
    const dim3 grid((N + kBN - 1) / kBN, (M + kBM - 1) / kBM, splits);
    hipLaunchKernelGGL((k_gemm<false, true, kEpiF32>), grid, dim3(256), 0, s, A, B, M, N, K, lda, ldb, nullptr,
                       nullptr, 0, part, nullptr, N);
    return hipGetLastError();
}

hipError_t mlp_head_fwd(const uint16_t *h, const uint16_t *w, const float *b, int rows, int D,
                        float *z, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_head_fwd, dim3((rows + 3) / 4), dim3(256), 0, s, h, w, b, rows, D, z);
    return hipGetLastError();
}

hipError_t mlp_loss(const float *z, const float *y, int rows, float pos_w, float *dz, float *loss,
                    hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss, dim3((rows + 255) / 256), dim3(256), 0, s, z, y, rows, pos_w, dz, loss);
    return hipGetLastError();
}

hipError_t mlp_head_bwd(const uint16_t *h, const uint16_t *w, const float *dz, int rows, int D,
                        uint16_t *dpre, float *dw, float *db, hipStream_t s)
{
    if (D > 1024) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(dw, 0, sizeof(float) * D, s);
    if (e == hipSuccess) e = hipMemsetAsync(db, 0, sizeof(float), s);
    if (e != hipSuccess || rows <= 0) return e;
    const int threads = ((D + 63) / 64) * 64;
    hipLaunchKernelGGL(k_head_bwd, dim3((rows + 63) / 64), dim3(threads), 0, s, h, w, dz, rows, D,
                       dpre, dw, db);
    return hipGetLastError();
}

hipError_t mlp_colsum(const uint16_t *g, int rows, int D, float *out, hipStream_t s)
{
    if (D > 1024) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(out, 0, sizeof(float) * D, s);
    if (e != hipSuccess || rows <= 0) return e;
    const int threads = ((D + 63) / 64) * 64;
    hipLaunchKernelGGL(k_colsum, dim3((rows + 63) / 64), dim3(threads), 0, s, g, rows, D, out);
    return hipGetLastError();
}

hipError_t mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                    float b2, float eps, int64_t t, uint16_t *wb, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, n, lr,
                       b1, b2, eps, c1, c2, wb);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *a, int64_t n, uint16_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n, out);
    return hipGetLastError();
}

}  // namespace gal
