// Surrogate inputs and routing on the device.
//
// Occupancy: per column of the grid and per layer of 0.25 m from the floor
// (8 layers), blocked when the column holds no free layer of the batch's
// last radius class (its largest in a plain batch) at any of four heights
// inside the layer (0.0625 m apart, none below 0.125 m so that the floor
// alone blocks nothing).  Every smaller class's blocked set lies inside the
// largest class's, so a sphere in contact sits in a blocked column
// (Appendix G's structure, summarised).  One byte per column, bit k = layer k.
// Features of one env's next move: the candidate joint angles, normalised
// joint and base offsets, normalised base pose, the held-object flag, the
// origins of the seven joint frames and the end-effector z axis of the
// candidate arm pose in the base frame (the step's own kinematics), and a
// 16 x 16 x 8 patch in the frame of the candidate base pose (0.1 m cells
// centred on the base, so it covers the arm's reach); a patch cell is
// blocked when any column under its rotated footprint's bounding box is, or
// when that box leaves the grid.
#include "gal_features.h"

namespace gal {

namespace {

// free-space test of one column of an env's class-0 grid at height z
__device__ __forceinline__ bool column_free(const SimBuffers &sb, const GridMeta &gm, size_t ek,
                                            int ci, int cj, float z)
{
    if (ci >= gm.nx || cj >= gm.ny) return false;
    const uint32_t *off = sb.grid_offsets + sb.grid_off_base[ek] + (size_t)cj * gm.nx + ci;
    const float2 *lay = sb.grid_layers + sb.grid_layer_base[ek];
    for (uint32_t l = off[0]; l < off[1]; ++l) {
        const float2 L = lay[l];
        if (L.x <= z && z <= L.y) return true;
    }
    return false;
}

// One thread per column: bit k of the column's byte = layer k blocked.
__global__ void k_occ_build(SimBuffers sb, OccGrid og, int num_envs, int max_cells, int num_classes)
{
    const int env = blockIdx.y;
    const int ij = blockIdx.x * blockDim.x + threadIdx.x;   // j * nx + i
    if (env >= num_envs) return;
    const int ox = og.occ_dims[2 * env], oy = og.occ_dims[2 * env + 1];
    if (ij >= ox * oy) return;
    const int i = ij % ox, j = ij / ox;
    const GridMeta gm = sb.grid_meta[env];
    const size_t ek = (size_t)env * num_classes + (num_classes - 1);
    uint32_t bits = 0;
    for (int k = 0; k < kPatchZ; ++k) {
        bool blocked = false;
        for (int m = 0; m < 4 && !blocked; ++m) {
            const float z = fmaxf((float)k * 0.25f + 0.0625f * (float)(m + 1), 0.125f);
            blocked = !column_free(sb, gm, ek, i, j, z);
        }
        if (blocked) bits |= 1u << k;
    }
    og.occ[og.occ_off[env] + ij] = (uint8_t)bits;
}

// one workgroup of 256 threads per env: wave 0 writes the 64 scalars, every
// thread one of the 256 patch columns (8 layers)
__global__ __launch_bounds__(256) void k_features(RobotParams rp, SimBuffers sb, OccGrid og,
                                                  const float *__restrict__ actions,
                                                  uint16_t *__restrict__ x)
{
    const int env = blockIdx.x;
    const int t = threadIdx.x;
    if (env >= sb.num_envs) return;
    const float *st = sb.state + (size_t)env * 10;
    const float *a = actions + (size_t)env * 9;
    uint16_t *row = x + (size_t)env * kMlpIn;
    const GridMeta gm = sb.grid_meta[env];
    if (t < 64) {
        float arm[24];
        if (t >= 20 && t < 44) arm_frame_features(rp, st, a, arm);
        row[t] = feat_bf16(scalar_feature(rp, sb, gm, env, st, a, t, arm));
    }
    const CandBase cb = cand_base(rp, st, a);
    *reinterpret_cast<uint4 *>(row + kFeatPatchBase + t * kPatchZ) = patch_words(patch_bits(og, gm, env, cb, t));
}

}  // namespace

hipError_t launch_occ_build(const SimBuffers &sb, const OccGrid &og, int num_envs, int num_classes,
                            int max_cells, hipStream_t s)
{
    dim3 grid((max_cells + 255) / 256, num_envs);   // max_cells: columns of the largest grid
    hipLaunchKernelGGL(k_occ_build, grid, dim3(256), 0, s, sb, og, num_envs, max_cells, num_classes);
    return hipGetLastError();
}

hipError_t launch_features(const RobotParams &rp, const SimBuffers &sb, const OccGrid &og,
                           const float *actions, uint16_t *x, hipStream_t s)
{
    static_assert(kPatch * kPatch == 256 && kFeatPatchBase == 64, "one thread per patch column");
    if (sb.num_envs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(sb.num_envs), dim3(256), 0, s, rp, sb, og, actions, x);
    return hipGetLastError();
}

}  // namespace gal
