// Surrogate inputs and routing on the device.
//
// Occupancy: a world-aligned lattice of cells (2 x 2 column-grid cells
// laterally, 0.25 m vertically, 8 layers from the floor); a cell is blocked
// when its centre is in contact for the smallest sphere class in the column
// grid (Appendix G's structure, queried as in the step).  Features of one
// env's next move: joint angles, normalised joint / base offsets, normalised
// base pose, and the 16 x 16 x 8 occupancy patch around the base.
// Routing: the exact static check of an env is skipped when the logit is at
// or below the threshold, except for a hashed 1-in-period audit sample.
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

__global__ void k_occ_build(SimBuffers sb, OccGrid og, int num_envs, int max_cells, int num_classes)
{
    const int env = blockIdx.y;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;   // (j * ox + i) * 8 + k
    if (env >= num_envs) return;
    const int ox = og.occ_dims[2 * env], oy = og.occ_dims[2 * env + 1];
    if (cell >= ox * oy * kPatchZ) return;
    const int k = cell % kPatchZ, ij = cell / kPatchZ, i = ij % ox, j = ij / ox;
    const GridMeta gm = sb.grid_meta[env];
    const float x = gm.x0 + ((float)i + 0.5f) * og.occ_cell;
    const float y = gm.y0 + ((float)j + 0.5f) * og.occ_cell;
    const float z = ((float)k + 0.5f) * 0.25f;
    bool blocked = true;
    const float fx = (x - gm.x0) * sb.inv_cell, fy = (y - gm.y0) * sb.inv_cell;
    if (fx >= 0.0f && fx < (float)gm.nx && fy >= 0.0f && fy < (float)gm.ny) {
        const int ci = (int)floorf(fx), cj = (int)floorf(fy);
        const size_t ek = (size_t)env * num_classes + 0;
        const uint32_t *off = sb.grid_offsets + sb.grid_off_base[ek] + (size_t)cj * gm.nx + ci;
        const float2 *lay = sb.grid_layers + sb.grid_layer_base[ek];
        for (uint32_t l = off[0]; l < off[1]; ++l) {
            const float2 L = lay[l];
            if (L.x <= z && z <= L.y) {
                blocked = false;
                break;
            }
        }
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
    if (lane < 32) {
        float v = 0.f;
        if (lane < 7) v = st[3 + lane];
        else if (lane < 14) v = sanitize(a[2 + lane - 7], rp.act_lim[2]) / rp.act_lim[2];
        else if (lane == 14) v = sanitize(a[0], rp.act_lim[0]) / rp.act_lim[0];
        else if (lane == 15) v = sanitize(a[1], rp.act_lim[1]) / rp.act_lim[1];
        else if (lane == 16) v = (st[0] - gm.x0) / ((float)gm.nx * sb.cell);
        else if (lane == 17) v = (st[1] - gm.y0) / ((float)gm.ny * sb.cell);
        else if (lane == 18) v = st[2] * 0.31830988618f;
        row[lane] = f2bf(v);
    }
    const int ox = og.occ_dims[2 * env], oy = og.occ_dims[2 * env + 1];
    const int ci = (int)floorf((st[0] - gm.x0) / og.occ_cell), cj = (int)floorf((st[1] - gm.y0) / og.occ_cell);
    const uint8_t *occ = og.occ + og.occ_off[env];
    // 256 (a, b) cells of 8 layers; lane takes 4 of them
    for (int c = lane; c < kPatch * kPatch; c += 64) {
        const int pa = c / kPatch, pb = c % kPatch;
        const int i = ci + pa - kPatch / 2, j = cj + pb - kPatch / 2;
        uint64_t bits = 0x0101010101010101ull;   // outside the lattice: blocked
        if (i >= 0 && i < ox && j >= 0 && j < oy)
            bits = *reinterpret_cast<const uint64_t *>(occ + ((size_t)j * ox + i) * kPatchZ);
        uint16_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = ((bits >> (8 * k)) & 0xFF) ? 0x3F80u : 0u;
        uint16_t *dst = row + kFeatPatchBase + c * kPatchZ;
#pragma unroll
        for (int k = 0; k < 8; ++k) dst[k] = v[k];
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
