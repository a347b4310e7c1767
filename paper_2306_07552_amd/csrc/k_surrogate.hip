// Surrogate inputs and routing on the device.
//
// Occupancy: per column of the grid and per layer of 0.25 m from the floor
// (8 layers), blocked when the column holds no free layer of the batch's
// last radius class (its largest in a plain batch) at any of four heights
// inside the layer (0.0625 m apart, none below 0.125 m so that the floor
// alone blocks nothing).  Every smaller class's blocked set lies inside the
// largest class's, so a sphere in contact sits in a blocked column
// (Appendix G's structure, summarised).
// Features of one env's next move: the candidate joint angles, normalised
// joint and base offsets, normalised base pose, the held-object flag, the
// origins of the seven joint frames and the end-effector z axis of the
// candidate arm pose in the base frame (the step's own kinematics), and a
// 16 x 16 x 8 patch in the frame of the candidate base pose (0.1 m cells
// centred on the base, so it covers the arm's reach); a patch cell is
// blocked when any column under its rotated footprint's bounding box is, or
// when that box leaves the grid.
// Routing: the exact static check of an env is skipped when the logit is at
// or below the threshold, except for a hashed 1-in-period audit sample.
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

__global__ void k_occ_build(SimBuffers sb, OccGrid og, int num_envs, int max_cells, int num_classes)
{
    const int env = blockIdx.y;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;   // (j * nx + i) * 8 + k
    if (env >= num_envs) return;
    const int ox = og.occ_dims[2 * env], oy = og.occ_dims[2 * env + 1];
    if (cell >= ox * oy * kPatchZ) return;
    const int k = cell % kPatchZ, ij = cell / kPatchZ, i = ij % ox, j = ij / ox;
    const GridMeta gm = sb.grid_meta[env];
    const size_t ek = (size_t)env * num_classes + (num_classes - 1);
    bool blocked = false;
    for (int m = 0; m < 4 && !blocked; ++m) {
        const float z = fmaxf((float)k * 0.25f + 0.0625f * (float)(m + 1), 0.125f);
        blocked = !column_free(sb, gm, ek, i, j, z);
    }
    og.occ[og.occ_off[env] + cell] = blocked ? 1 : 0;
}

// one wave per env
__global__ void k_features(RobotParams rp, SimBuffers sb, OccGrid og, const float *__restrict__ actions,
                           uint16_t *__restrict__ x)
{
    const int env = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (env >= sb.num_envs) return;
    const float *st = sb.state + (size_t)env * 10;
    const float *a = actions + (size_t)env * 9;
    uint16_t *row = x + (size_t)env * kMlpIn;
    const GridMeta gm = sb.grid_meta[env];
    const float a0 = sanitize(a[0], rp.act_lim[0]), a1 = sanitize(a[1], rp.act_lim[1]);
    if (lane < 20) {
        float v = 0.f;
        if (lane < 7)
            v = clampf(st[3 + lane] + sanitize(a[2 + lane], rp.act_lim[2]), rp.qlim[lane][0],
                       rp.qlim[lane][1]);
        else if (lane < 14) v = sanitize(a[2 + lane - 7], rp.act_lim[2]) / rp.act_lim[2];
        else if (lane == 14) v = a0 / rp.act_lim[0];
        else if (lane == 15) v = a1 / rp.act_lim[1];
        else if (lane == 16) v = (st[0] - gm.x0) / ((float)gm.nx * sb.cell);
        else if (lane == 17) v = (st[1] - gm.y0) / ((float)gm.ny * sb.cell);
        else if (lane == 18) v = st[2] * 0.31830988618f;
        else if (lane == 19) v = sb.held[env] ? 1.0f : 0.0f;
        row[lane] = f2bf(v);
    }
    {
        // arm frames of the candidate joint angles with the base at the origin
        float q[10] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 7; ++j)
            q[3 + j] = clampf(st[3 + j] + sanitize(a[2 + j], rp.act_lim[2]), rp.qlim[j][0], rp.qlim[j][1]);
        Fk fk;
        forward_kinematics(rp, q, fk);
        // lanes 20..40: origin of frame 1 + (l - 20) / 3, lanes 41..43: z axis of frame 7
        float v = 0.f;
#pragma unroll
        for (int j = 1; j < 8; ++j)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                if (lane == 20 + 3 * (j - 1) + r) v = fk.f[j].m[4 * r + 3];
                if (j == 7 && lane == 41 + r) v = fk.f[7].m[4 * r + 2];
            }
        if (lane >= 20 && lane < kFeatPatchBase) row[lane] = f2bf(v);
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
    // 256 (a, b) cells of 8 layers; lane takes 4 of them
    const float hx = 0.05f * (fabsf(cy) + fabsf(sy));   // half-extent of a rotated cell's box
    for (int c = lane; c < kPatch * kPatch; c += 64) {
        const int pa = c / kPatch, pb = c % kPatch;
        const float px = ((float)pa - 7.5f) * 0.1f, py = ((float)pb - 7.5f) * 0.1f;
        const float wx = bx + (cy * px - sy * py), wy = by + (sy * px + cy * py);
        const float fi0 = floorf(((wx - hx) - gm.x0) / og.occ_cell);
        const float fi1 = floorf(((wx + hx) - gm.x0) / og.occ_cell);
        const float fj0 = floorf(((wy - hx) - gm.y0) / og.occ_cell);
        const float fj1 = floorf(((wy + hx) - gm.y0) / og.occ_cell);
        uint64_t bits = 0x0101010101010101ull;   // box leaves the grid: blocked
        // the box is under 3 cells wide, so at most 4 x 4 columns
        if (fi0 >= 0.0f && fj0 >= 0.0f && fi1 < (float)ox && fj1 < (float)oy && fi1 - fi0 < 4.0f &&
            fj1 - fj0 < 4.0f) {
            bits = 0;
            for (int j = (int)fj0; j <= (int)fj1; ++j)
                for (int i = (int)fi0; i <= (int)fi1; ++i)
                    bits |= *reinterpret_cast<const uint64_t *>(occ + ((size_t)j * ox + i) * kPatchZ);
        }
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = (((bits >> (16 * k)) & 0xFF) ? 0x3F80u : 0u) |
                   ((((bits >> (16 * k + 8)) & 0xFF) ? 0x3F80u : 0u) << 16);
        *reinterpret_cast<uint4 *>(row + kFeatPatchBase + c * kPatchZ) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

__device__ __forceinline__ uint32_t hash3(uint32_t a, uint32_t b, uint32_t c)
{
    uint64_t x = ((uint64_t)a << 40) ^ ((uint64_t)b << 20) ^ (uint64_t)c;
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return (uint32_t)x;
}

__global__ void k_route(const float *__restrict__ z, const int32_t *__restrict__ counters, int n,
                        float thr, uint32_t period, uint8_t *__restrict__ flags,
                        unsigned long long *__restrict__ stats)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    int skip = 0, audit = 0;
    if (e < n) {
        if (z[e] <= thr) {
            skip = 1;
            if (period > 0 && hash3((uint32_t)e, (uint32_t)counters[2 * e + 1],
                                    (uint32_t)counters[2 * e]) % period == 0)
                audit = 1;
        }
        flags[e] = (uint8_t)(skip ? (audit ? 2 : 1) : 0);
    }
    const uint64_t ms = __ballot(skip), ma = __ballot(audit), mq = __ballot(e < n);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&stats[0], (unsigned long long)__popcll(mq));
        atomicAdd(&stats[1], (unsigned long long)__popcll(ms));
        atomicAdd(&stats[2], (unsigned long long)__popcll(ma));
    }
}

}  // namespace

hipError_t launch_occ_build(const SimBuffers &sb, const OccGrid &og, int num_envs, int num_classes,
                            int max_cells, hipStream_t s)
{
    dim3 grid((max_cells + 255) / 256, num_envs);
    hipLaunchKernelGGL(k_occ_build, grid, dim3(256), 0, s, sb, og, num_envs, max_cells, num_classes);
    return hipGetLastError();
}

hipError_t launch_features(const RobotParams &rp, const SimBuffers &sb, const OccGrid &og,
                           const float *actions, uint16_t *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3((sb.num_envs + 3) / 4), dim3(256), 0, s, rp, sb, og, actions, x);
    return hipGetLastError();
}

hipError_t launch_route(const float *z, const int32_t *counters, int num_envs, float thr_logit,
                        uint32_t audit_period, uint8_t *flags, unsigned long long *stats,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_route, dim3((num_envs + 255) / 256), dim3(256), 0, s, z, counters, num_envs,
                       thr_logit, audit_period, flags, stats);
    return hipGetLastError();
}

}  // namespace gal
