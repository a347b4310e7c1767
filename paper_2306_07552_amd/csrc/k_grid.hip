// Column-grid construction on the device (Appendix G: a dense 2-D array of
// ground-plane columns, one grid per sphere-radius class, each column listing
// its free vertical layers as heights of the query sphere's centre).
//
// For class radius r and column centre c, a static box whose closed XY
// footprint lies within horizontal distance d < r of c blocks sphere centres
// in the open interval (z0 - h, z1 + h), h = sqrt(r^2 - d^2); the floor
// blocks (-inf, r).  The free layers are the maximal closed intervals of the
// complement that have positive length.  One thread per (env, class, column);
// the column's blocking intervals are kept in a small private list and the
// free intervals are produced by repeatedly skipping the blocked run that
// contains the current height and taking the next blocking start.
#include "gal_internal.h"

namespace gal {

namespace {

constexpr int kBoxChunk = 256;

struct ColumnIntervals {
    float a[kGridIvCap];
    float b[kGridIvCap];
    int n;
    bool overflow;
};

__device__ void gather_intervals(const float *__restrict__ sboxes, int nb, float cx, float cy,
                                 float r, ColumnIntervals &iv)
{
    const float r2 = r * r;
    for (int k = 0; k < nb; ++k) {
        const float *B = sboxes + 6 * k;
        float dx = 0.0f, dy = 0.0f;
        if (cx < B[0]) dx = B[0] - cx;
        else if (cx > B[3]) dx = cx - B[3];
        if (cy < B[1]) dy = B[1] - cy;
        else if (cy > B[4]) dy = cy - B[4];
        const float d2 = dx * dx + dy * dy;
        if (d2 < r2) {
            if (iv.n < kGridIvCap) {
                const float h = sqrtf(r2 - d2);
                iv.a[iv.n] = B[2] - h;
                iv.b[iv.n] = B[5] + h;
                ++iv.n;
            } else {
                iv.overflow = true;
            }
        }
    }
}

// Emits the free layers; returns their number.  `out` may be null (count).
__device__ int free_layers(const ColumnIntervals &iv, float r, float2 *out)
{
    int count = 0;
    float lo = r;
    for (;;) {
        bool moved = true;
        while (moved) {
            moved = false;
            for (int i = 0; i < iv.n; ++i) {
                if (iv.a[i] < lo && lo < iv.b[i]) {
                    lo = iv.b[i];
                    moved = true;
                }
            }
        }
        float hi = INFINITY;
        for (int i = 0; i < iv.n; ++i)
            if (iv.a[i] >= lo && iv.a[i] < hi) hi = iv.a[i];
        if (lo < hi) {
            if (out) out[count] = make_float2(lo, hi);
            ++count;
        }
        if (hi == INFINITY) break;
        float next = hi;
        for (int i = 0; i < iv.n; ++i)
            if (iv.a[i] == hi && iv.b[i] > next) next = iv.b[i];
        if (!(next > hi)) break;   // cannot happen for finite boxes; keeps the loop finite
        lo = next;
    }
    return count;
}

// blockIdx.x = (env * K + class) * blocks_per_grid + column block
template <bool kFill>
__global__ __launch_bounds__(256) void k_grid_columns(SimBuffers sb, const float *__restrict__ boxes,
                                                      const uint64_t *__restrict__ box_off,
                                                      int32_t num_classes, ClassRadii radii,
                                                      int32_t blocks_per_grid,
                                                      uint32_t *__restrict__ counts,
                                                      int32_t *__restrict__ overflow)
{
    __shared__ float sboxes[kBoxChunk * 6];
    const int ek = blockIdx.x / blocks_per_grid;
    const int cblock = blockIdx.x % blocks_per_grid;
    const int env = ek / num_classes;
    const int cls = ek % num_classes;
    const GridMeta gm = sb.grid_meta[env];
    const int ncols = gm.nx * gm.ny;
    if (cblock * (int)blockDim.x >= ncols) return;   // whole block idle
    const int col = cblock * blockDim.x + threadIdx.x;
    const float r = radii.r[cls];
    const int i = col % (gm.nx > 0 ? gm.nx : 1);
    const int j = col / (gm.nx > 0 ? gm.nx : 1);
    const float cx = gm.x0 + ((float)i + 0.5f) * sb.cell;
    const float cy = gm.y0 + ((float)j + 0.5f) * sb.cell;

    ColumnIntervals iv;
    iv.n = 0;
    iv.overflow = false;
    const uint64_t b0 = box_off[env], b1 = box_off[env + 1];
    for (uint64_t base = b0; base < b1; base += kBoxChunk) {
        const int nb = (int)((b1 - base) < (uint64_t)kBoxChunk ? (b1 - base) : kBoxChunk);
        __syncthreads();
        for (int k = threadIdx.x; k < nb * 6; k += blockDim.x) sboxes[k] = boxes[base * 6 + k];
        __syncthreads();
        if (col < ncols) gather_intervals(sboxes, nb, cx, cy, r, iv);
    }
    if (col >= ncols) return;
    if (iv.overflow) {
        atomicOr(overflow, 1);
        return;
    }
    const uint64_t ob = sb.grid_off_base[ek];
    if (!kFill) {
        counts[ob + col] = (uint32_t)free_layers(iv, r, nullptr);
    } else {
        float2 *dst = const_cast<float2 *>(sb.grid_layers) + sb.grid_layer_base[ek] +
                      sb.grid_offsets[ob + col];
        free_layers(iv, r, dst);
    }
}

// Exclusive scan of the per-column layer counts of one (env, class) grid,
// in place, with the total stored after the last column.
__global__ __launch_bounds__(1024) void k_grid_scan(const uint64_t *__restrict__ off_base,
                                                    const GridMeta *__restrict__ meta,
                                                    int32_t num_classes, uint32_t *offsets)
{
    __shared__ uint32_t warp_sums[16];
    __shared__ uint32_t carry;
    const int ek = blockIdx.x;
    const int env = ek / num_classes;
    const GridMeta gm = meta[env];
    const int ncols = gm.nx * gm.ny;
    uint32_t *o = offsets + off_base[ek];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < ncols; base += blockDim.x) {
        const int c = base + threadIdx.x;
        uint32_t v = c < ncols ? o[c] : 0u;
        // inclusive scan within the wave
        uint32_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) warp_sums[wid] = x;
        __syncthreads();
        if (wid == 0) {
            uint32_t w = lane < 16 ? warp_sums[lane] : 0u;
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                uint32_t y = __shfl_up(w, d, 64);
                if (lane >= d) w += y;
            }
            if (lane < 16) warp_sums[lane] = w;
        }
        __syncthreads();
        const uint32_t before = carry + (wid > 0 ? warp_sums[wid - 1] : 0u);
        if (c < ncols) o[c] = before + x - v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) o[ncols] = carry;
}

}  // namespace

hipError_t launch_grid_count(const SimBuffers &sb, const float *boxes, const uint64_t *box_off,
                             int32_t num_envs, int32_t num_classes, const ClassRadii &radii,
                             int32_t max_cols, uint32_t *counts, int32_t *overflow, hipStream_t s)
{
    const int bpg = (max_cols + 255) / 256;
    dim3 grid((unsigned)((int64_t)bpg * num_envs * num_classes));
    hipLaunchKernelGGL(k_grid_columns<false>, grid, dim3(256), 0, s, sb, boxes, box_off,
                       num_classes, radii, bpg, counts, overflow);
    return hipGetLastError();
}

hipError_t launch_grid_scan(const uint64_t *off_base, const GridMeta *meta, int32_t num_envs,
                            int32_t num_classes, uint32_t *offsets, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_scan, dim3(num_envs * num_classes), dim3(1024), 0, s, off_base,
                       meta, num_classes, offsets);
    return hipGetLastError();
}

hipError_t launch_grid_fill(const SimBuffers &sb, const float *boxes, const uint64_t *box_off,
                            int32_t num_envs, int32_t num_classes, const ClassRadii &radii,
                            int32_t max_cols, int32_t *overflow, hipStream_t s)
{
    const int bpg = (max_cols + 255) / 256;
    dim3 grid((unsigned)((int64_t)bpg * num_envs * num_classes));
    hipLaunchKernelGGL(k_grid_columns<true>, grid, dim3(256), 0, s, sb, boxes, box_off,
                       num_classes, radii, bpg, nullptr, overflow);
    return hipGetLastError();
}

}  // namespace gal
