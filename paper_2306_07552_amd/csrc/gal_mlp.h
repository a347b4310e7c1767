// Internal definitions of the collision-surrogate MLP (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gal_internal.h"

namespace gal {

constexpr int kMlpIn = 2112;       // 44 scalars, 20 zeros, 16 x 16 x 8 occupancy patch
constexpr int kMlpHidden = 256;
constexpr int kMlpLayers = 5;      // 4 hidden + logit head
constexpr int kPatch = 16;         // patch edge in occupancy cells
constexpr int kPatchZ = 8;         // occupancy layers of 0.25 m from the floor
constexpr int kFeatPatchBase = 64; // first patch feature

enum { kEpiF32 = 0, kEpiBiasReluBf16 = 1, kEpiMaskBf16 = 2 };
enum { kGemmFwd = 0, kGemmDx, kGemmDw, kGemmNtF32, kGemmNnF32, kGemmTnF32 };

hipError_t mlp_gemm(int variant, const uint16_t *A, const uint16_t *B, int M, int N, int K, int lda,
                    int ldb, const float *bias, const uint16_t *mask, int ldm, float *Cf,
                    uint16_t *Cb, int ldc, hipStream_t s);
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
    uint8_t *occ;              // per env [ny][nx][8] blocked flags of the class-0 grid
    const uint64_t *occ_off;   // [N] base of each env's block
    const int32_t *occ_dims;   // [N][2] nx, ny (the column grid's)
    float occ_cell;            // lateral cell (the column grid's)
};

hipError_t launch_occ_build(const SimBuffers &sb, const OccGrid &og, int num_envs, int num_classes,
                            int max_cells, hipStream_t s);
hipError_t launch_features(const RobotParams &rp, const SimBuffers &sb, const OccGrid &og,
                           const float *actions, uint16_t *x, hipStream_t s);
hipError_t launch_route(const float *z, const int32_t *counters, int num_envs, float thr_logit,
                        uint32_t audit_period, uint8_t *flags, unsigned long long *stats,
                        hipStream_t s);

}  // namespace gal
