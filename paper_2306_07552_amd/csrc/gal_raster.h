// The renderer's device-side interface: the render mesh as clusters, the
// raster parameters and the raster launchers (the rest of the library's
// internal definitions are in gal_internal.h).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

constexpr int kClusterTris = 64;    // triangles per render cluster (one per lane)
constexpr int kClusterVerts = 64;   // unique vertices per render cluster
constexpr int kClusterPlanes = 4;    // distinct face planes per cluster (slot in ctris bits 24..25)
constexpr uint32_t kNoPlane = 0xFFFF; // plane index of clusters built without face planes
constexpr int kMaxPlanes = 4096;     // distinct face planes per env
constexpr int kMaxRegion = 128;     // largest square region rendered by one workgroup

// Render cluster: up to 64 consecutive triangles of one env, the unique
// vertices they use and the (at most 4) face planes they lie on.  Three
// float4 words:
//   w0 = (aabb lo x, y, z, bits of vertex base)
//   w1 = (aabb hi x, y, z, bits of triangle base)
//   w2 = (bits of nverts | ntris << 8, bits of first triangle id,
//         plane index p0 | p1 << 16, p2 | p3 << 16)
// A triangle's slot word holds its three local vertex indices (bits 0..23)
// and the slot of its plane among p0..p3 (bits 24..25); unused plane slots
// repeat p0, and clusters built without planes hold kNoPlane.
struct RenderMesh {
    const float4 *clusters;          // [C][3] AABB lo + slot, hi + slot, counts nv | nt<<8, first tri,
                                     // face-plane indices p0 | p1<<16, p2 | p3<<16
    const float4 *planes;            // [P] distinct face planes per env (normal, offset)
    const uint64_t *env_plane_off;   // [N+1]
    const uint64_t *env_cluster_off; // [N+1]
    const float *cverts;             // [C][64][3] vertex positions of each cluster (unused slots 0)
    const uint32_t *ctris;           // [C][64] packed i0 | i1<<8 | i2<<16 | plane slot<<24
    const uint8_t *tri_rgb;          // [T][3] in original order per env, or null
    const uint64_t *env_tri_off;     // [N+1] for colour lookup
    // movable objects drawn where they are (manipulation; null elsewhere):
    // a box per object, its 12 triangles numbered after the env's mesh
    const float *obj_frames;         // [N][O][12]
    const float *obj_rec;            // [N][O][8] (half extents at [3..5])
    const uint8_t *obj_rgb;          // [N][O][3] or null
    int32_t num_objects;
    // the robot's links drawn as boxes (null link_frames: not drawn)
    const float *link_frames;        // [N][8][12]
    const float *link_box;           // [8][6] centre, half extents in the link frame
    const uint8_t *link_rgb;         // [8][3] or null
    // lit, textured colour (null: flat colour): each triangle's index into
    // its env's face planes, whose normals light it
    const uint16_t *tri_pidx;        // [T] in the caller's order per env
};

struct RasterParams {
    float near_m;
    float invn;        // 1/near
    float kd;          // (2^24-1) / (1/near - 1/far)
    int32_t region;    // square region edge rendered by one workgroup (<= 128)
    int32_t lane_max;  // bbox pixel count rasterised by the triangle's own lane
    int32_t small_max; // bbox pixel count rasterised by the balanced wave pass
    int32_t block;     // threads per workgroup: 256, 512 or 1024
    int32_t refresh;   // clusters a wave draws between occlusion-bound refreshes
    int32_t occlusion; // 1 = cull clusters hidden behind the z-buffer bounds
    int32_t prologue;  // clusters drawn before occlusion culling starts
    int32_t persistent;// 1 = persistent kernel draining the work queue
    int32_t order;     // 1 = the queue follows the last step's item times, longest first
    int32_t bin;       // 1 = mid-sized triangles are binned per 8x8 tile in LDS and drawn tile by tile
    unsigned long long *stats; // optional work counters [8] (null = off)
    uint32_t *item_cost;        // [work] last time of each work item (wall-clock ticks)
    const uint32_t *item_order; // [work] queue position -> work item
};

hipError_t raster_prepare();   // raises the dynamic-LDS limit of the raster kernels
// Workgroups of the persistent raster kernel that fit on the device at once.
int raster_persistent_grid(const RasterParams &rp, int max_region, bool color);
// Whether one workgroup's LDS (z-buffer, bins, shared state) fits a CU.
bool raster_fits(const RasterParams &rp, int max_region, bool color);
hipError_t launch_raster(const RenderMesh &m, const RasterParams &rp, const float *camera,
                         const int32_t *env_res, const uint64_t *env_depth_off,
                         const uint32_t *work, int32_t num_work, int32_t max_region,
                         uint32_t *queue, int32_t persistent_grid, uint32_t *depth, uint8_t *rgb,
                         hipStream_t s);

}  // namespace gal
