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
#include "gal_fk.h"
#include "gal_math.h"
#include "gal_mlp.h"

namespace gal {

namespace {

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ float sanitize(float a, float lim)
{
    if (a != a) a = 0.0f;
    return clampf(a, -lim, lim);
}

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

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
    const float a0 = sanitize(a[0], rp.act_lim[0]), a1 = sanitize(a[1], rp.act_lim[1]);
    if (t < 64) {
        float v = 0.f;
        if (t < 7)
            v = clampf(st[3 + t] + sanitize(a[2 + t], rp.act_lim[2]), rp.qlim[t][0], rp.qlim[t][1]);
        else if (t < 14) v = sanitize(a[2 + t - 7], rp.act_lim[2]) / rp.act_lim[2];
        else if (t == 14) v = a0 / rp.act_lim[0];
        else if (t == 15) v = a1 / rp.act_lim[1];
        else if (t == 16) v = (st[0] - gm.x0) / ((float)gm.nx * sb.cell);
        else if (t == 17) v = (st[1] - gm.y0) / ((float)gm.ny * sb.cell);
        else if (t == 18) v = st[2] * 0.31830988618f;
        else if (t == 19) v = sb.held[env] ? 1.0f : 0.0f;
        else {
            // arm frames of the candidate joint angles with the base at the origin:
            // t = 20..40 origin of frame 1 + (t - 20) / 3, t = 41..43 z axis of frame 7
            float q[10] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < 7; ++j)
                q[3 + j] = clampf(st[3 + j] + sanitize(a[2 + j], rp.act_lim[2]), rp.qlim[j][0],
                                  rp.qlim[j][1]);
            Fk fk;
            forward_kinematics(rp, q, fk);
#pragma unroll
            for (int j = 1; j < 8; ++j)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    if (t == 20 + 3 * (j - 1) + r) v = fk.f[j].m[4 * r + 3];
                    if (j == 7 && t == 41 + r) v = fk.f[7].m[4 * r + 2];
                }
        }
        row[t] = f2bf(v);
    }
    // candidate base pose, in the robot step's own operation order
    const float pi_f = 0x1.921fb6p+1f, two_pi_f = 0x1.921fb6p+2f;
    float yaw = st[2] + a1;
    if (yaw > pi_f) yaw = yaw - two_pi_f;
    else if (yaw < -pi_f) yaw = yaw + two_pi_f;
    float sy, cy;
    dsincos(yaw, sy, cy);
    const float bx = st[0] + a0 * cy, by = st[1] + a0 * sy;
    const int ox = og.occ_dims[2 * env], oy = og.occ_dims[2 * env + 1];
    const uint8_t *occ = og.occ + og.occ_off[env];
    // patch column c = t: cell (a, b), 8 layers
    const float hx = 0.05f * (fabsf(cy) + fabsf(sy));   // half-extent of a rotated cell's box
    const int pa = t / kPatch, pb = t % kPatch;
    const float px = ((float)pa - 7.5f) * 0.1f, py = ((float)pb - 7.5f) * 0.1f;
    const float wx = bx + (cy * px - sy * py), wy = by + (sy * px + cy * py);
    const float fi0 = floorf(((wx - hx) - gm.x0) / og.occ_cell);
    const float fi1 = floorf(((wx + hx) - gm.x0) / og.occ_cell);
    const float fj0 = floorf(((wy - hx) - gm.y0) / og.occ_cell);
    const float fj1 = floorf(((wy + hx) - gm.y0) / og.occ_cell);
    uint32_t bits = 0xFFu;   // box leaves the grid: every layer blocked
    // the box is under 3 cells wide, so at most 4 x 4 columns: a fixed 4 x 4
    // block of loads (indices clamped into the lattice) issued together, the
    // columns past the box masked out
    if (fi0 >= 0.0f && fj0 >= 0.0f && fi1 < (float)ox && fj1 < (float)oy && fi1 - fi0 < 4.0f &&
        fj1 - fj0 < 4.0f) {
        const int i0 = (int)fi0, i1 = (int)fi1, j0 = (int)fj0, j1 = (int)fj1;
        uint32_t v[4][4];
#pragma unroll
        for (int dj = 0; dj < 4; ++dj)
#pragma unroll
            for (int di = 0; di < 4; ++di) {
                const int i = min(i0 + di, ox - 1), j = min(j0 + dj, oy - 1);
                v[dj][di] = occ[(size_t)j * ox + i];
            }
        bits = 0;
#pragma unroll
        for (int dj = 0; dj < 4; ++dj)
#pragma unroll
            for (int di = 0; di < 4; ++di)
                if (i0 + di <= i1 && j0 + dj <= j1) bits |= v[dj][di];
    }
    // layers 2k and 2k + 1 as BF16 ones or zeros in one word
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = (((bits >> (2 * k)) & 1u) ? 0x3F80u : 0u) | ((((bits >> (2 * k + 1)) & 1u) ? 0x3F80u : 0u) << 16);
    *reinterpret_cast<uint4 *>(row + kFeatPatchBase + t * kPatchZ) = make_uint4(w[0], w[1], w[2], w[3]);
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
