// Internal definitions shared by the library's host runtime and its HIP
// kernels (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

constexpr int kMaxClasses = 8;
constexpr int kMaxSpheres = 256;
constexpr int kMaxObjects = 64;
constexpr int kClusterTris = 64;    // triangles per render cluster (one per lane)
constexpr int kClusterVerts = 64;   // unique vertices per render cluster
constexpr int kClusterPlanes = 4;    // distinct face planes per cluster (slot in ctris bits 24..25)
constexpr uint32_t kNoPlane = 0xFFFF; // plane index of clusters built without face planes
constexpr int kMaxPlanes = 4096;     // distinct face planes per env
constexpr int kMaxRegion = 128;     // largest square region rendered by one workgroup
constexpr int kGridIvCap = 64;      // blocking boxes one grid column may see

// Robot constants, passed by value to the step kernel.
struct RobotParams {
    float dh[7][4];
    float qlim[7][2];
    float q_home[7];
    float mount[3];
    float cam_offset[3];
    float cam_pitch_cs[2];
    float class_radius[kMaxClasses];
    float act_lim[3];
    int32_t num_spheres;
    int32_t num_classes;
    int32_t num_objects;
    int32_t num_starts;
    int32_t episode_len;
    int32_t contact_words;
    // manipulation (grasp / release / place / slide); manip = 0 elsewhere
    int32_t manip;              // 1: 11-float actions, movable objects
    int32_t slide;              // 1: a collision slides the base
    float grasp_tip[3];         // end-effector-frame point of the grasp sphere
    float grasp_radius;
    int32_t held_class;         // radius class of a held object's spheres
    float slide_step, place_step;
    uint64_t manip_seed;
    int32_t links;              // 1: write every link's frame for the raster (sb.link_frames)
};

// Spheres of a held object (one per octant of its box).
constexpr int kHeldSpheres = 8;

struct ClassRadii {
    float r[kMaxClasses];
};

// One collision sphere (device table [S]).
struct Sphere {
    float px, py, pz;
    int32_t link;
    int32_t cls;
    int32_t held_only;
};

// Per-env grid placement (device table [N]).
struct GridMeta {
    float x0, y0;
    int32_t nx, ny;
};

// Device pointers of the simulation state and scene tables.
struct SimBuffers {
    float *state;              // [N][10]
    int32_t *counters;         // [N][2]
    float *camera;             // [N][12] position, right, down, forward
    const uint8_t *held;       // [N]
    const float *starts;       // [N][P][3]
    const float *objects;      // [N][O][8]
    const Sphere *spheres;     // [S]
    const GridMeta *grid_meta; // [N]
    const uint64_t *grid_off_base;   // [N*K] base into grid_offsets
    const uint64_t *grid_layer_base; // [N*K] base into grid_layers
    const uint32_t *grid_offsets;    // per (env, class): [nx*ny+1] CSR (relative)
    const float2 *grid_layers;       // free layers (lo, hi)
    float cell;
    float inv_cell;
    int32_t num_envs;
    const uint8_t *skip_flags;       // [N] surrogate routing (null = exact check for all):
                                     // 1 = skip the static check, 2 = skipped but audited
    unsigned long long *sur_stats;   // [4] queries, skipped, audited, audit mismatches
    // manipulation state (null unless RobotParams::manip); `objects` above
    // then holds every object's record at episode start
    float *obj_dyn;                  // [N][O][8] resting records (the held one: before the grasp)
    int32_t *held_obj;               // [N] held object, -1 = none
    float *rel;                      // [N][12] held object's frame in the end-effector frame
    float *obj_frames;               // [N][O][12] object frames after the step (for the raster)
    float *link_frames;              // [N][8][12] link frames after the step (links drawn)
};

// Step outputs (device, caller-owned).
struct StepOutputs {
    uint32_t *contact_static;
    uint32_t *contact_object;
    uint8_t *accepted;
    float *state;
    float *frames;
    int32_t *counters;
    uint8_t *done;
    float *object_frames;   // [N][O][12] (manipulation)
    int32_t *held;          // [N] (manipulation)
};

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
    unsigned long long *stats; // optional work counters [8] (null = off)
    uint32_t *item_cost;        // [work] last time of each work item (wall-clock ticks)
    const uint32_t *item_order; // [work] queue position -> work item
};

// Launchers (defined in the .hip files).
hipError_t launch_robot_step(const RobotParams &rp, const SimBuffers &sb, const float *actions,
                             const StepOutputs &out, uint32_t *queue_reset, int lanes_per_env,
                             hipStream_t s);
hipError_t launch_reset(const RobotParams &rp, const SimBuffers &sb, const uint8_t *mask,
                        hipStream_t s);
// Object frames of the current state (manipulation; after create, reset and
// state restore, so that the raster draws the objects where they are).
hipError_t launch_object_frames(const RobotParams &rp, const SimBuffers &sb, hipStream_t s);
hipError_t raster_prepare();   // raises the dynamic-LDS limit of the raster kernels
// Workgroups of the persistent raster kernel that fit on the device at once.
int raster_persistent_grid(const RasterParams &rp, int max_region, bool color);
hipError_t launch_raster(const RenderMesh &m, const RasterParams &rp, const float *camera,
                         const int32_t *env_res, const uint64_t *env_depth_off,
                         const uint32_t *work, int32_t num_work, int32_t max_region,
                         uint32_t *queue, int32_t persistent_grid, uint32_t *depth, uint8_t *rgb,
                         hipStream_t s);
hipError_t launch_hash_u32(const uint32_t *a, uint64_t n, unsigned long long *out, hipStream_t s);
// Work items the raster queue order handles (the static order beyond).
constexpr int kOrderCap = 32768;
hipError_t launch_grid_count(const SimBuffers &sb, const float *boxes, const uint64_t *box_off,
                             int32_t num_envs, int32_t num_classes, const ClassRadii &radii,
                             int32_t max_cols, uint32_t *counts, int32_t *overflow, hipStream_t s);
hipError_t launch_grid_scan(const uint64_t *off_base, const GridMeta *meta, int32_t num_envs,
                            int32_t num_classes, uint32_t *offsets, hipStream_t s);
hipError_t launch_grid_fill(const SimBuffers &sb, const float *boxes, const uint64_t *box_off,
                            int32_t num_envs, int32_t num_classes, const ClassRadii &radii,
                            int32_t max_cols, int32_t *overflow, hipStream_t s);

}  // namespace gal
