// Collision-surrogate inference: inputs -> 2112 x 256 first layer -> three
// 256 x 256 layers -> logit -> routing flags.  The surrogate is this build's
// learned pre-filter in front of the static-scene overlap test of the
// kinematic step (Section 3.2 of the paper describes the exact test).
//
// A tile of 32 rows (two 16-row MFMA tiles) is served by `splits` workgroups
// (1, 2, 4 or 8) that share the first layer's K = 2112 inputs, cut into 8
// chunks: chunk 0 = the 64 scalar inputs and patch columns 0..31 (10 K-steps
// of 32), chunk c >= 1 = patch columns 32c..32c+31 (8 K-steps).  A workgroup
// builds its chunks' inputs in LDS (computed from the batch's state, actions
// and occupancy lattice, or copied from an input array) while its waves load
// their weight fragments straight into registers, then runs the chunk on the
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation): wave w owns
// output columns 32w..32w+31 of all 32 rows.  With one split (large batches)
// the workgroup goes on to the hidden layers itself.  With more, each writes
// its FP32 partial sums and a second launch, one workgroup per tile, adds the
// splits in split order and runs the hidden layers.  (A single launch whose
// last-arriving workgroup finishes the tile needs device-scope fences, which
// write back and invalidate the XCD's L2 on every workgroup: several times
// slower here.)  Layers 2..4 keep the activations in LDS and load the next
// layer's weights while the current one runs; then the head and the routing.
// No input rows are written to memory.
#include "gal_features.h"

namespace gal {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kR = 32;                      // rows per tile
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kColsW = kMlpHidden / kWaves; // output columns per wave (two 16-column tiles)
constexpr int kChunk0 = 10;                 // K-steps of chunk 0
constexpr int kChunkN = 8;                  // K-steps of chunks 1..7
constexpr int kChunks = 8;
constexpr int kAPitch = kChunk0 * 32 + 8;   // LDS row pitch of a chunk (BF16 values)
constexpr int kHPitch = kMlpHidden + 8;     // LDS row pitch of a hidden layer
static_assert(kChunk0 * 32 + (kChunks - 1) * kChunkN * 32 == kMlpIn, "chunks cover the input");
static_assert(kChunk0 * 32 - kFeatPatchBase == 32 * kPatchZ, "chunk 0 holds 32 patch columns");
static_assert(kColsW == 32, "two 16-column MFMA tiles per wave");

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float relu(float v) { return v > 0.f ? v : 0.f; }


// Layers 2..4, the head and the routing of the tile's 32 rows, from the first
// hidden layer in H[0]; fa holds this wave's fragments of layer 2.
__device__ __forceinline__ void tail_layers(const SurInferArgs &p, int row0,
                                            uint16_t (*H)[kR][kHPitch], float *zs,
                                            bf16x8 (&fa)[kMlpHidden / 32][2])
{
    constexpr int D = kMlpHidden;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    auto load_w = [&](const uint16_t *W, bf16x8(&f)[D / 32][2]) {
#pragma unroll
        for (int st = 0; st < D / 32; ++st)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                f[st][j] = *reinterpret_cast<const bf16x8 *>(W + (size_t)(kColsW * wave + 16 * j + r16) * D + 32 * st + kq);
    };
    bf16x8 fb[D / 32][2];
    float bias[3][2];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int j = 0; j < 2; ++j) bias[l][j] = p.t.b[l][kColsW * wave + 16 * j + r16];
    uint16_t hw[D / 64];
#pragma unroll
    for (int k = 0; k < D / 64; ++k) hw[k] = p.t.w[3][lane + 64 * k];
    auto layer = [&](const bf16x8(&f)[D / 32][2], const float(&bl)[2], int cur) {
        floatx4 ac[2][2];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j) ac[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < D / 32; ++st)
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&H[cur][16 * m + r16][32 * st + kq]);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    ac[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, f[st][j], ac[m][j], 0, 0, 0);
            }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = kColsW * wave + 16 * j + r16;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    H[cur ^ 1][16 * m + 4 * (lane >> 4) + i][n] = to_bf16(relu(ac[m][j][i] + bl[j]));
        }
        __syncthreads();
    };
    load_w(p.t.w[1], fb);
    layer(fa, bias[0], 0);
    load_w(p.t.w[2], fa);
    layer(fb, bias[1], 1);
    layer(fa, bias[2], 0);
    // head (summed in the training head's order): wave w takes rows 4w .. 4w + 3
#pragma unroll
    for (int rr = 0; rr < kR / kWaves; ++rr) {
        const int r = (kR / kWaves) * wave + rr;
        float h = 0.f;
#pragma unroll
        for (int k = 0; k < D / 64; ++k) h += bf16_to_f(H[1][r][lane + 64 * k]) * bf16_to_f(hw[k]);
        for (int d = 32; d >= 1; d >>= 1) h += __shfl_xor(h, d, 64);
        if (lane == 0) zs[r] = h + p.t.b[3][0];
    }
    __syncthreads();
    if (wave == 0) {
        const int e = row0 + lane;
        const bool live = lane < kR && e < p.rows;
        int flag = 0;
        if (live) {
            if (p.z) p.z[e] = zs[lane];
            if (p.route) {
                flag = route_flag(p.ra, p.ra.base + e, zs[lane]);
                p.ra.flags[p.ra.base + e] = (uint8_t)flag;
            }
        }
        if (p.route) {
            const uint64_t mq = __ballot(live), ms = __ballot(flag != 0), ma = __ballot(flag == 2);
            if (lane == 0) {
                atomicAdd(&p.ra.stats[0], (unsigned long long)__popcll(mq));
                if (ms) atomicAdd(&p.ra.stats[1], (unsigned long long)__popcll(ms));
                if (ma) atomicAdd(&p.ra.stats[2], (unsigned long long)__popcll(ma));
            }
        }
    }
}

// this wave's fragments of a 256 x 256 layer: column 32 wave + 16 j + r16
__device__ __forceinline__ void load_layer(const uint16_t *W, bf16x8 (&f)[kMlpHidden / 32][2])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int st = 0; st < kMlpHidden / 32; ++st)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            f[st][j] = *reinterpret_cast<const bf16x8 *>(W + (size_t)(kColsW * wave + 16 * j + r16) * kMlpHidden +
                                                        32 * st + kq);
}

template <int FEAT>
__global__ __launch_bounds__(kThreads) void k_sur_l1(SurInferArgs p)
{
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kR * kHPitch];
    __shared__ float arm[kR][24];
    __shared__ float zs[kR];
    static_assert(kR * kAPitch <= 2 * kR * kHPitch, "chunk fits the activation buffer");
    uint16_t(*A)[kAPitch] = reinterpret_cast<uint16_t(*)[kAPitch]>(lds);
    uint16_t(*H)[kR][kHPitch] = reinterpret_cast<uint16_t(*)[kR][kHPitch]>(lds);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int S = p.splits;
    const int tile = blockIdx.x / S, split = blockIdx.x - tile * S;
    const int row0 = tile * kR;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const int cpb = kChunks / S;
    const int cbeg = split * cpb;

    floatx4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int c = cbeg; c < cbeg + cpb; ++c) {
        const int s0 = c == 0 ? 0 : kChunk0 + kChunkN * (c - 1);
        const int ns = c == 0 ? kChunk0 : kChunkN;
        // this wave's weight fragments: column 32 wave + 16 j + r16, K = 32 (s0 + st) + kq
        bf16x8 w[kChunk0][2];
#pragma unroll
        for (int st = 0; st < kChunk0; ++st)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                w[st][j] = st < ns ? *reinterpret_cast<const bf16x8 *>(
                                         p.t.w0 + (size_t)(kColsW * wave + 16 * j + r16) * kMlpIn +
                                         32 * (s0 + st) + kq)
                                   : bf16x8{};
        if (FEAT == 0) {
            // the chunk's columns of the input rows, 16 bytes per thread and pass
            const int per_row = ns * 4;
            for (int i = tid; i < kR * per_row; i += kThreads) {
                const int r = i / per_row, q = i - r * per_row;
                const int e = row0 + r;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (e < p.rows) v = *reinterpret_cast<const uint4 *>(p.x + (size_t)e * kMlpIn + 32 * s0 + 8 * q);
                *reinterpret_cast<uint4 *>(&A[r][8 * q]) = v;
            }
        } else {
            // chunk 0: wave 1 evaluates the arm frames of the 32 rows (one lane
            // each) while the other waves build the patch columns
            const bool fk_wave = c == 0 && wave == 1;
            if (fk_wave && lane < kR) {
                const int e = row0 + lane;
                float f[24];
                if (e < p.rows)
                    arm_frame_features(p.rp, p.sb.state + (size_t)e * 10, p.actions + (size_t)e * 9, f);
                else
#pragma unroll
                    for (int k = 0; k < 24; ++k) f[k] = 0.f;
#pragma unroll
                for (int k = 0; k < 24; ++k) arm[lane][k] = f[k];
            }
            // patch columns 32c .. 32c + 31 of every row
            const int pbase = c == 0 ? kFeatPatchBase : 0;
            const int t0 = c == 0 ? (tid < 64 ? tid : tid - 64) : tid;
            const int nt = c == 0 ? kThreads - 64 : kThreads;
            if (!fk_wave)
                for (int i = t0; i < kR * 32; i += nt) {
                    const int r = i >> 5, pc = i & 31;
                    const int e = row0 + r;
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (e < p.rows) {
                        const CandBase cb = cand_base(p.rp, p.sb.state + (size_t)e * 10, p.actions + (size_t)e * 9);
                        v = patch_words(patch_bits(p.og, p.sb.grid_meta[e], e, cb, 32 * c + pc));
                    }
                    *reinterpret_cast<uint4 *>(&A[r][pbase + 8 * pc]) = v;
                }
            if (c == 0) {
                __syncthreads();
                for (int i = tid; i < kR * 64; i += kThreads) {
                    const int r = i >> 6, t = i & 63;
                    const int e = row0 + r;
                    float v = 0.f;
                    if (e < p.rows)
                        v = scalar_feature(p.rp, p.sb, p.sb.grid_meta[e], e, p.sb.state + (size_t)e * 10,
                                           p.actions + (size_t)e * 9, t, arm[r]);
                    A[r][t] = feat_bf16(v);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kChunk0; ++st) {
            if (st < ns) {
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&A[16 * m + r16][32 * st + kq]);
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w[st][j], acc[m][j], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // lane holds rows 16 m + 4 (lane / 16) + i, column 32 wave + 16 j + r16
    if (S > 1) {
        float *mine = p.part + (size_t)blockIdx.x * kR * kMlpHidden;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    mine[(16 * m + 4 * (lane >> 4) + i) * kMlpHidden + kColsW * wave + 16 * j + r16] = acc[m][j][i];
        return;
    }
    // one split: the first hidden layer (bias, ReLU, BF16), then the rest
    bf16x8 fa[kMlpHidden / 32][2];
    load_layer(p.t.w[0], fa);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int n = kColsW * wave + 16 * j + r16;
        const float bn = p.t.b0[n];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) H[0][16 * m + 4 * (lane >> 4) + i][n] = to_bf16(relu(acc[m][j][i] + bn));
    }
    __syncthreads();
    tail_layers(p, row0, H, zs, fa);
}

// Second launch with several splits: one workgroup per tile adds the tile's
// partial sums in split order (bias, ReLU, BF16) and runs the hidden layers.
__global__ __launch_bounds__(kThreads) void k_sur_tail(SurInferArgs p)
{
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kR * kHPitch];
    __shared__ float zs[kR];
    uint16_t(*H)[kR][kHPitch] = reinterpret_cast<uint16_t(*)[kR][kHPitch]>(lds);
    const int S = p.splits;
    const int tile = blockIdx.x, row0 = tile * kR;
    bf16x8 fa[kMlpHidden / 32][2];
    load_layer(p.t.w[0], fa);
    // thread: 4 adjacent columns of rows r, r + 8, r + 16, r + 24
    const int c = (threadIdx.x % (kMlpHidden / 4)) * 4, r0 = threadIdx.x / (kMlpHidden / 4);
    constexpr int kRowStep = kThreads / (kMlpHidden / 4);   // 8
    const float4 bb = *reinterpret_cast<const float4 *>(p.t.b0 + c);
    const float *tp = p.part + (size_t)tile * S * kR * kMlpHidden;
#pragma unroll
    for (int h = 0; h < kR / kRowStep; h += 2) {
        float4 v[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = r0 + kRowStep * (h + k);
            const float *q = tp + (size_t)r * kMlpHidden + c;
            float4 a = *reinterpret_cast<const float4 *>(q);
            for (int sp = 1; sp < S; ++sp) {
                const float4 b = *reinterpret_cast<const float4 *>(q + (size_t)sp * kR * kMlpHidden);
                a.x += b.x;
                a.y += b.y;
                a.z += b.z;
                a.w += b.w;
            }
            v[k] = a;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = r0 + kRowStep * (h + k);
            H[0][r][c + 0] = to_bf16(relu(v[k].x + bb.x));
            H[0][r][c + 1] = to_bf16(relu(v[k].y + bb.y));
            H[0][r][c + 2] = to_bf16(relu(v[k].z + bb.z));
            H[0][r][c + 3] = to_bf16(relu(v[k].w + bb.w));
        }
    }
    __syncthreads();
    tail_layers(p, row0, H, zs, fa);
}

}  // namespace

int sur_infer_splits(int rows)
{
    const int tiles = (rows + kR - 1) / kR;
    // aim at about 512 workgroups; every split needs its own partial-sum slab
    if (tiles <= 64) return 8;
    if (tiles <= 128) return 4;
    if (tiles <= 256) return 2;
    return 1;
}

size_t sur_infer_part_floats(int rows)
{
    const int s = sur_infer_splits(rows);
    const size_t tiles = (size_t)(rows + kR - 1) / kR;
    return s > 1 ? tiles * s * kR * kMlpHidden : 0;
}

size_t sur_infer_part_floats_max(int max_rows)
{
    const size_t tiles = (size_t)(max_rows + kR - 1) / kR;
    const size_t slabs = tiles * 8 < 512 ? tiles * 8 : 512;
    return slabs * kR * kMlpHidden;
}

hipError_t sur_infer(const SurInferArgs &args, hipStream_t s)
{
    if (args.rows <= 0) return hipSuccess;
    SurInferArgs p = args;
    p.splits = sur_infer_splits(p.rows);
    const int tiles = (p.rows + kR - 1) / kR;
    const dim3 grid((unsigned)(tiles * p.splits));
    if (p.x)
        hipLaunchKernelGGL(k_sur_l1<0>, grid, dim3(kThreads), 0, s, p);
    else
        hipLaunchKernelGGL(k_sur_l1<1>, grid, dim3(kThreads), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.splits == 1) return e;
    hipLaunchKernelGGL(k_sur_tail, dim3((unsigned)tiles), dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace gal
