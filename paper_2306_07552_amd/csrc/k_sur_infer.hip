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
//
// The weights of the four matrix layers are read from a copy in fragment
// order (sur_infer_layout): the 16 bytes a lane needs for one MFMA operand
// sit at lane * 16 within a 1 KiB block per (wave, K-step, column tile), so
// every weight load of a wave reads whole cache lines once, where the
// row-major matrix would have it gather 16 half-lines 4 KiB apart.  Weight
// streaming into each workgroup is what bounds both launches at small
// batches.
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


// Layers 2..4, the head and the routing of R rows (16 or 32) from row0 on,
// from the first hidden layer in H[0]; f2, f3, f4 hold this wave's fragments
// of the three layers, all loaded before the first of them runs (a chain of
// per-layer loads waits on memory three times over).
template <int R>
__device__ __forceinline__ void tail_layers(const SurInferArgs &p, int row0,
                                            uint16_t (*H)[R][kHPitch], float *zs,
                                            const bf16x8 (&f2)[kMlpHidden / 32][2],
                                            const bf16x8 (&f3)[kMlpHidden / 32][2],
                                            const bf16x8 (&f4)[kMlpHidden / 32][2])
{
    constexpr int D = kMlpHidden, M = R / 16;
    static_assert(R % 16 == 0 && R % kWaves == 0 && R <= 64, "whole MFMA row tiles");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    float bias[3][2];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int j = 0; j < 2; ++j) bias[l][j] = p.t.b[l][kColsW * wave + 16 * j + r16];
    uint16_t hw[D / 64];
#pragma unroll
    for (int k = 0; k < D / 64; ++k) hw[k] = p.t.w[3][lane + 64 * k];
    auto layer = [&](const bf16x8(&f)[D / 32][2], const float(&bl)[2], int cur) {
        floatx4 ac[M][2];
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j) ac[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < D / 32; ++st)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&H[cur][16 * m + r16][32 * st + kq]);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    ac[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, f[st][j], ac[m][j], 0, 0, 0);
            }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = kColsW * wave + 16 * j + r16;
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    H[cur ^ 1][16 * m + 4 * (lane >> 4) + i][n] = to_bf16(relu(ac[m][j][i] + bl[j]));
        }
        __syncthreads();
    };
    layer(f2, bias[0], 0);
    layer(f3, bias[1], 1);
    layer(f4, bias[2], 0);
    // head (summed in the training head's order): wave w takes rows 4w .. 4w + 3
#pragma unroll
    for (int rr = 0; rr < R / kWaves; ++rr) {
        const int r = (R / kWaves) * wave + rr;
        float h = 0.f;
#pragma unroll
        for (int k = 0; k < D / 64; ++k) h += bf16_to_f(H[1][r][lane + 64 * k]) * bf16_to_f(hw[k]);
        for (int d = 32; d >= 1; d >>= 1) h += __shfl_xor(h, d, 64);
        if (lane == 0) zs[r] = h + p.t.b[3][0];
    }
    __syncthreads();
    if (wave == 0) {
        const int e = row0 + lane;
        const bool live = lane < R && e < p.rows;
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

// Element offset, in the fragment-ordered copy of a layer, of the block that
// holds K-steps s0 .. s0 + ns - 1: fragment (wave, st, j) of that block is
// 64 lanes x 8 BF16 values, lane = 16 (K group) + (column within the tile).
__device__ __forceinline__ size_t frag_offset(int s0, int ns, int wave, int st, int j, int lane)
{
    return (size_t)32 * s0 * kMlpHidden + ((size_t)((wave * ns + st) * 2 + j) * 64 + lane) * 8;
}

// this wave's fragments of a 256 x 256 layer (fragment order): column
// 32 wave + 16 j + r16, K = 32 st + kq
__device__ __forceinline__ void load_layer(const uint16_t *W, bf16x8 (&f)[kMlpHidden / 32][2])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int st = 0; st < kMlpHidden / 32; ++st)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            f[st][j] = *reinterpret_cast<const bf16x8 *>(W + frag_offset(0, kMlpHidden / 32, wave, st, j, lane));
}

// What the patch columns of one row need: the candidate base pose and where
// the env's lattice lies.
struct RowInfo {
    CandBase cb;
    float x0, y0;
    int ox, oy;
    uint64_t occ_off;
    bool live;
};

template <int FEAT>
__global__ __launch_bounds__(kThreads) void k_sur_l1(SurInferArgs p)
{
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kR * kHPitch];
    __shared__ RowInfo rows[kR];
    __shared__ float zs[kR];
    static_assert(kR * kAPitch <= 2 * kR * kHPitch, "chunk fits the activation buffer");
    uint16_t(*A)[kAPitch] = reinterpret_cast<uint16_t(*)[kAPitch]>(lds);
    uint16_t(*H)[kR][kHPitch] = reinterpret_cast<uint16_t(*)[kR][kHPitch]>(lds);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int S = p.splits;
    // Workgroups are handed to the 8 XCDs in turn (blockIdx mod 8).  When the
    // tile count allows, all splits of tile t go to XCD t mod 8, where the
    // second launch's workgroup t runs: its partial sums are then read from
    // the same L2 they were written to.
    const int tiles_all = gridDim.x / S;
    int tile, split;
    if (S > 1 && tiles_all % 8 == 0) {
        const int slot = blockIdx.x >> 3;
        tile = (blockIdx.x & 7) + 8 * (slot / S);
        split = slot - (slot / S) * S;
    } else {
        tile = blockIdx.x / S;
        split = blockIdx.x - tile * S;
    }
    const int row0 = tile * kR;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const int cpb = kChunks / S;
    const int cbeg = split * cpb;

    floatx4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // this wave's weight fragments of chunk c: column 32 wave + 16 j + r16,
    // K = 32 (first step + st) + kq; the first chunk's are issued before
    // anything else, each later chunk's as soon as the previous one's MFMAs
    // have been issued
    bf16x8 w[kChunk0][2];
    auto load_chunk = [&](int c) {
        const int s0 = c == 0 ? 0 : kChunk0 + kChunkN * (c - 1);
        const int ns = c == 0 ? kChunk0 : kChunkN;
#pragma unroll
        for (int st = 0; st < kChunk0; ++st)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                w[st][j] = st < ns ? *reinterpret_cast<const bf16x8 *>(p.t.w0 + frag_offset(s0, ns, wave, st, j, lane))
                                   : bf16x8{};
    };
    // per row: the candidate base pose and the lattice placement, once.  The
    // row's loads are issued before the weight fragments: loads complete in
    // order, and behind the fragments they would wait for all of them.
    const bool rlive = FEAT && tid < kR && row0 + tid < p.rows;
    float rst[3] = {0.f, 0.f, 0.f}, ract[2] = {0.f, 0.f}, rx0 = 0.f, ry0 = 0.f;
    int rox = 1, roy = 1;
    uint64_t roff = 0;
    if (rlive) {
        const int e = row0 + tid;
#pragma unroll
        for (int k = 0; k < 3; ++k) rst[k] = p.sb.state[(size_t)e * 10 + k];
#pragma unroll
        for (int k = 0; k < 2; ++k) ract[k] = p.actions[(size_t)e * 9 + k];
        rx0 = p.sb.grid_meta[e].x0;
        ry0 = p.sb.grid_meta[e].y0;
        rox = p.og.occ_dims[2 * e];
        roy = p.og.occ_dims[2 * e + 1];
        roff = p.og.occ_off[e];
    }
    load_chunk(cbeg);
    if (FEAT) {
        if (tid < kR) {
            RowInfo ri{};
            ri.live = rlive;
            if (rlive) {
                ri.cb = cand_base(p.rp, rst, ract);
                ri.x0 = rx0;
                ri.y0 = ry0;
                ri.ox = rox;
                ri.oy = roy;
                ri.occ_off = roff;
            }
            rows[tid] = ri;
        }
        __syncthreads();
    }

    for (int c = cbeg; c < cbeg + cpb; ++c) {
        const int s0 = c == 0 ? 0 : kChunk0 + kChunkN * (c - 1);
        const int ns = c == 0 ? kChunk0 : kChunkN;
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
            // chunk 0: wave 1 builds the 64 scalars of the 32 rows (one lane
            // each, with the arm frames) while the other waves build the patch
            // columns
            const bool fk_wave = c == 0 && wave == 1;
            if (fk_wave && lane < kR) {
                const int e = row0 + lane;
                if (e < p.rows) {
                    float st[10], a[9];
#pragma unroll
                    for (int k = 0; k < 10; ++k) st[k] = p.sb.state[(size_t)e * 10 + k];
#pragma unroll
                    for (int k = 0; k < 9; ++k) a[k] = p.actions[(size_t)e * 9 + k];
                    const GridMeta gm = p.sb.grid_meta[e];
                    float arm[24];
                    arm_frame_features(p.rp, st, a, arm);
#pragma unroll
                    for (int t = 0; t < 64; ++t)
                        A[lane][t] = feat_bf16(scalar_feature(p.rp, p.sb, gm, e, st, a, t, arm));
                } else {
#pragma unroll
                    for (int t = 0; t < 64; ++t) A[lane][t] = 0;
                }
            }
            // patch columns 32c .. 32c + 31 of every row: two per thread (three
            // in chunk 0, where wave 1 is busy), every lattice load of a
            // thread's columns in flight together
            const int pbase = c == 0 ? kFeatPatchBase : 0;
            const int t0 = c == 0 ? (tid < 64 ? tid : tid - 64) : tid;
            const int nt = c == 0 ? kThreads - 64 : kThreads;
            constexpr int kTasks = 3;
            if (!fk_wave) {
                int ti[kTasks], i0[kTasks], i1[kTasks], j0[kTasks], j1[kTasks], oxs[kTasks], oys[kTasks];
                bool in[kTasks];
                const uint8_t *occ[kTasks];
#pragma unroll
                for (int k = 0; k < kTasks; ++k) {
                    ti[k] = t0 + k * nt;
                    in[k] = false;
                    occ[k] = p.og.occ;
                    oxs[k] = oys[k] = 1;
                    i0[k] = i1[k] = j0[k] = j1[k] = 0;
                    if (ti[k] < kR * 32) {
                        const RowInfo &ri = rows[ti[k] >> 5];
                        if (ri.live) {
                            oxs[k] = ri.ox;
                            oys[k] = ri.oy;
                            occ[k] = p.og.occ + ri.occ_off;
                            in[k] = patch_box(ri.cb, ri.x0, ri.y0, p.og.occ_cell, ri.ox, ri.oy,
                                              32 * c + (ti[k] & 31), i0[k], i1[k], j0[k], j1[k]);
                        }
                    }
                }
                uint32_t bits[kTasks];
#pragma unroll
                for (int k = 0; k < kTasks; ++k)
                    bits[k] = patch_or(occ[k], oxs[k], oys[k], in[k], i0[k], i1[k], j0[k], j1[k]);
#pragma unroll
                for (int k = 0; k < kTasks; ++k)
                    if (ti[k] < kR * 32) {
                        const int r = ti[k] >> 5, pc = ti[k] & 31;
                        *reinterpret_cast<uint4 *>(&A[r][pbase + 8 * pc]) =
                            rows[r].live ? patch_words(bits[k]) : make_uint4(0u, 0u, 0u, 0u);
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
        if (c + 1 < cbeg + cpb) load_chunk(c + 1);
        __syncthreads();
    }

    // lane holds rows 16 m + 4 (lane / 16) + i, column 32 wave + 16 j + r16
    if (S > 1) {
        float *mine = p.part + (size_t)(tile * S + split) * kR * kMlpHidden;
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
    bf16x8 f2[kMlpHidden / 32][2], f3[kMlpHidden / 32][2], f4[kMlpHidden / 32][2];
    load_layer(p.t.w[0], f2);
    load_layer(p.t.w[1], f3);
    load_layer(p.t.w[2], f4);
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
    tail_layers<kR>(p, row0, H, zs, f2, f3, f4);
}

// Second launch with several splits: a workgroup per half tile (16 rows)
// adds the partial sums of its rows in split order (bias, ReLU, BF16) and
// runs the hidden layers.  The partial sums (up to 8 x 16 KB) go straight
// from memory into LDS (global_load_lds), so the registers hold the three
// hidden layers' weights, and all of it is requested at once: the workgroup
// waits on memory one time.
constexpr int kTR = 16;                     // rows per tail workgroup
constexpr int kMaxSplits = 8;

__global__ __launch_bounds__(kThreads) void k_sur_tail(SurInferArgs p)
{
    __shared__ __attribute__((aligned(16))) float part[kMaxSplits][kTR][kMlpHidden];
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kTR * kHPitch];
    __shared__ float zs[kTR];
    uint16_t(*H)[kTR][kHPitch] = reinterpret_cast<uint16_t(*)[kTR][kHPitch]>(lds);
    const int S = p.splits;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the first launch sends tile t to XCD t mod 8 when the tile count is a
    // multiple of 8; keep both halves of tile t there too
    const int tiles_all = gridDim.x / 2;
    int tile, half;
    if (tiles_all % 8 == 0) {
        tile = (blockIdx.x & 7) + 8 * (blockIdx.x >> 4);
        half = (blockIdx.x >> 3) & 1;
    } else {
        tile = blockIdx.x >> 1;
        half = blockIdx.x & 1;
    }
    const int row0 = tile * kR + kTR * half;
    // one wave-wide copy = one row of one split (256 floats, 16 bytes a lane)
    const float *tp = p.part + (size_t)tile * S * kR * kMlpHidden + (size_t)kTR * half * kMlpHidden;
    for (int i = wave; i < S * kTR; i += kWaves) {
        const int sp = i / kTR, r = i - sp * kTR;
        __builtin_amdgcn_global_load_lds(
            (const void *)(tp + (size_t)sp * kR * kMlpHidden + (size_t)r * kMlpHidden + 4 * lane),
            (__attribute__((address_space(3))) void *)&part[sp][r][0], 16, 0, 0);
    }
    bf16x8 f2[kMlpHidden / 32][2], f3[kMlpHidden / 32][2], f4[kMlpHidden / 32][2];
    load_layer(p.t.w[0], f2);
    load_layer(p.t.w[1], f3);
    load_layer(p.t.w[2], f4);
    __syncthreads();
    {
        // thread: 8 adjacent columns of one row
        const int r = tid >> 5, c = (tid & 31) * 8;
        float a[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float4 v = *reinterpret_cast<const float4 *>(&part[0][r][c + 4 * h]);
            a[4 * h + 0] = v.x;
            a[4 * h + 1] = v.y;
            a[4 * h + 2] = v.z;
            a[4 * h + 3] = v.w;
        }
        for (int sp = 1; sp < S; ++sp)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 v = *reinterpret_cast<const float4 *>(&part[sp][r][c + 4 * h]);
                a[4 * h + 0] += v.x;
                a[4 * h + 1] += v.y;
                a[4 * h + 2] += v.z;
                a[4 * h + 3] += v.w;
            }
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = (uint32_t)to_bf16(relu(a[2 * k] + p.t.b0[c + 2 * k])) |
                   ((uint32_t)to_bf16(relu(a[2 * k + 1] + p.t.b0[c + 2 * k + 1])) << 16);
        *reinterpret_cast<uint4 *>(&H[0][r][c]) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    __syncthreads();
    tail_layers<kTR>(p, row0, H, zs, f2, f3, f4);
}

// One thread per 8 consecutive K values of one output column of one layer:
// copies them from the row-major BF16 matrix to their fragment-order slot.
__global__ void k_infer_layout(const uint16_t *w0, const uint16_t *w1, const uint16_t *w2,
                               const uint16_t *w3, uint16_t *wi)
{
    constexpr int g0 = kMlpHidden * (kMlpIn / 8), gh = kMlpHidden * (kMlpHidden / 8);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g0 + 3 * gh) return;
    int layer, g;
    if (i < g0) {
        layer = 0;
        g = i;
    } else {
        layer = 1 + (i - g0) / gh;
        g = (i - g0) % gh;
    }
    const int K = layer == 0 ? kMlpIn : kMlpHidden;
    const int n = g / (K / 8), k = (g % (K / 8)) * 8;
    const uint16_t *src = layer == 0 ? w0 : layer == 1 ? w1 : layer == 2 ? w2 : w3;
    const int S = k / 32, kq = (k % 32) / 8;
    int s0 = 0, ns = kMlpHidden / 32;
    if (layer == 0) {
        if (S < kChunk0) {
            ns = kChunk0;
        } else {
            s0 = kChunk0 + kChunkN * ((S - kChunk0) / kChunkN);
            ns = kChunkN;
        }
    }
    const size_t base = layer == 0 ? 0 : (size_t)kMlpIn * kMlpHidden + (size_t)(layer - 1) * kMlpHidden * kMlpHidden;
    const int lane = kq * 16 + (n & 15);
    *reinterpret_cast<uint4 *>(wi + base + frag_offset(s0, ns, n / 32, S - s0, (n / 16) & 1, lane)) =
        *reinterpret_cast<const uint4 *>(src + (size_t)n * K + k);
}

}  // namespace

size_t sur_infer_layout_elems() { return (size_t)kMlpIn * kMlpHidden + 3 * (size_t)kMlpHidden * kMlpHidden; }

hipError_t sur_infer_layout(const uint16_t *w0, const uint16_t *w1, const uint16_t *w2, const uint16_t *w3,
                            uint16_t *wi, hipStream_t s)
{
    const int n = kMlpHidden * (kMlpIn / 8) + 3 * kMlpHidden * (kMlpHidden / 8);
    hipLaunchKernelGGL(k_infer_layout, dim3((n + 255) / 256), dim3(256), 0, s, w0, w1, w2, w3, wi);
    return hipGetLastError();
}

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
    hipLaunchKernelGGL(k_sur_tail, dim3((unsigned)(2 * tiles)), dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace gal
