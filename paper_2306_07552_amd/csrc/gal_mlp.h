// Internal definitions of the collision-surrogate MLP (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gal_internal.h"

struct gal_mlp;

namespace gal {

constexpr int kMlpIn = 2112;       // 44 scalars, 20 zeros, 16 x 16 x 8 occupancy patch
constexpr int kMlpHidden = 256;
constexpr int kMlpLayers = 5;      // 4 hidden + logit head
constexpr int kPatch = 16;         // patch edge in occupancy cells
constexpr int kPatchZ = 8;         // occupancy layers of 0.25 m from the floor
constexpr int kFeatPatchBase = 64; // first patch feature

enum { kEpiF32 = 0, kEpiBiasReluBf16 = 1, kEpiMaskBf16 = 2 };
enum { kGemmFwd = 0, kGemmDx, kGemmDw, kGemmNtF32, kGemmNnF32, kGemmTnF32 };

// C = op(A) op(B) on the matrix cores (variants above).  The weight-gradient
// variant splits its reduction over the rows into the FP32 workspace ws
// (ws_floats values; NULL = no split) and sums the splits in a fixed order.
constexpr int kMaxDwSplits = 16;
// Split-K partial products of A B^T (A [M][K], B [N][K], BF16): split z of
// K (in 32-column steps) into part + z M N, FP32 [M][N]; no reduction.
hipError_t mlp_gemm_parts(const uint16_t *A, const uint16_t *B, int M, int N, int K, int lda, int ldb, int splits,
                          float *part, hipStream_t s);
hipError_t mlp_gemm(int variant, const uint16_t *A, const uint16_t *B, int M, int N, int K, int lda,
                    int ldb, const float *bias, const uint16_t *mask, int ldm, float *Cf,
                    uint16_t *Cb, int ldc, hipStream_t s, float *ws = nullptr, size_t ws_floats = 0);
hipError_t mlp_head_fwd(const uint16_t *h, const uint16_t *w, const float *b, int rows, int D,
                        float *z, hipStream_t s);
hipError_t mlp_loss(const float *z, const float *y, int rows, float pos_w, float *dz, float *loss,
                    hipStream_t s);
hipError_t mlp_head_bwd(const uint16_t *h, const uint16_t *w, const float *dz, int rows, int D,
                        uint16_t *dpre, float *dw, float *db, hipStream_t s);
hipError_t mlp_colsum(const uint16_t *g, int rows, int D, float *out, hipStream_t s);
hipError_t mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                    float b2, float eps, int64_t t, uint16_t *wb, hipStream_t s);
hipError_t mlp_to_bf16(const float *a, int64_t n, uint16_t *out, hipStream_t s);

// Surrogate plumbing of a batch.
struct OccGrid {
    uint8_t *occ;              // per env [ny][nx]: bit k = layer k blocked (the last class's grid)
    const uint64_t *occ_off;   // [N] base of each env's block
    const int32_t *occ_dims;   // [N][2] nx, ny (the column grid's)
    float occ_cell;            // lateral cell (the column grid's)
};

hipError_t launch_occ_build(const SimBuffers &sb, const OccGrid &og, int num_envs, int num_classes,
                            int max_cells, hipStream_t s);
hipError_t launch_features(const RobotParams &rp, const SimBuffers &sb, const OccGrid &og,
                           const float *actions, uint16_t *x, hipStream_t s);
// Routing of the step's static checks by the surrogate's logits: env e is
// skipped when z_e <= thr (NaN never is), and a skipped env is audited (its
// exact check still runs and a disagreement is counted) when a hash of
// (env, episode, step) is 0 mod period.  Flag 0 = exact, 1 = skip, 2 = audit.
struct RouteArgs {
    const int32_t *counters;    // [N][2] step in episode, episode
    float thr;                  // logit threshold
    uint32_t period;            // audit 1 in period skipped envs (0 = never)
    uint8_t *flags;             // [N] out
    unsigned long long *stats;  // [0] queries [1] skipped [2] audited (accumulated)
    int base;                   // env index of the first row
};

__device__ __forceinline__ uint32_t route_hash(uint32_t a, uint32_t b, uint32_t c)
{
    uint64_t x = ((uint64_t)a << 40) ^ ((uint64_t)b << 20) ^ (uint64_t)c;
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return (uint32_t)x;
}

// flag of env e (batch index) whose logit is z
__device__ __forceinline__ int route_flag(const RouteArgs &ra, int e, float z)
{
    if (!(z <= ra.thr)) return 0;
    const bool audit = ra.period > 0 &&
                       route_hash((uint32_t)e, (uint32_t)ra.counters[2 * e + 1],
                                  (uint32_t)ra.counters[2 * e]) % ra.period == 0;
    return audit ? 2 : 1;
}

// Weights of inference: layer 1 (w0, b0), layers 2..4 (w[0..2], b[0..2]),
// all four matrices in the fragment order sur_infer_layout writes, and the
// head (w[3] BF16 [256], b[3]).
struct MlpTail {
    const uint16_t *w0;
    const float *b0;
    const uint16_t *w[4];
    const float *b[4];
};
// Inference (inputs -> logits -> routing; one launch for large batches, two
// otherwise).  The inputs are x (BF16 [rows][2112]) or, with x null,
// computed on the fly for envs 0 .. rows - 1 of the batch (rp, sb, og,
// actions) exactly as k_features would write them.  Scratch: part
// (sur_infer_part_floats(rows) FP32 values, the first layer's partial sums);
// launches that share it must not overlap.
struct SurInferArgs {
    MlpTail t;
    const uint16_t *x;
    RobotParams rp;
    SimBuffers sb;
    OccGrid og;
    const float *actions;
    int rows;
    int splits;            // chosen by sur_infer
    float *part;
    float *z;              // [rows] logits, or null
    RouteArgs ra;
    int route;             // 1 = write routing flags and counts (ra)
};
int sur_infer_splits(int rows);
size_t sur_infer_part_floats(int rows);
// The scratch that covers every row count up to max_rows (splits are chosen
// so that tiles x splits <= 512 whenever partial sums are used, so never more
// than 512 slabs of 32 x 256 FP32 values = 16 MiB).
size_t sur_infer_part_floats_max(int max_rows);
hipError_t sur_infer(const SurInferArgs &args, hipStream_t s);
// The copy of the four matrix layers that inference reads (BF16,
// sur_infer_layout_elems() values: layer 1 then layers 2..4), rewritten from
// the row-major BF16 matrices w0 [256][2112] and w1..w3 [256][256] whenever
// they change.
size_t sur_infer_layout_elems();
hipError_t sur_infer_layout(const uint16_t *w0, const uint16_t *w1, const uint16_t *w2, const uint16_t *w3,
                            uint16_t *wi, hipStream_t s);

// Rewrites m's inference copy of the weights (call after they change).
hipError_t mlp_refresh_inference(gal_mlp *m, hipStream_t s);
// Inference of the MLP m (gal_mlp_api.cpp); part null = the MLP's own scratch.
int mlp_infer_rows(gal_mlp *m, const uint16_t *x, const SurInferArgs *src, int rows, float *z,
                   const RouteArgs *route, hipStream_t s, float *part = nullptr);


}  // namespace gal
