// Internal definitions shared by the library's host runtime and its HIP
// kernels (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gal_raster.h"

namespace gal {

constexpr int kMaxClasses = 8;
constexpr int kMaxSpheres = 256;
constexpr int kMaxObjects = 64;
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
    int32_t objgrid;            // 1: resting objects found through the object grids
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

// Regular grids of the resting objects (Appendix G): four grids of
// kObjCell squares per env, grid g shifted by (g & 1, g >> 1) x kObjCell / 2
// from (x0, y0), nx x ny cells each; a cell's word holds one bit per object
// whose footprint box (grown by kObjMargin) meets the cell.  A sphere of
// radius <= kObjCell / 4 lies wholly inside a cell of at least one grid, so
// that cell's word lists every object the sphere can touch.
constexpr float kObjCell = 0.5f;
constexpr float kObjMargin = 1e-3f;
struct ObjGridMeta {
    float x0, y0;
    int32_t nx, ny;
    uint64_t base;                   // first word of the env's 4 grids in objgrid_mask
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
    // the resting objects' regular grids (null: every object is tested)
    const ObjGridMeta *objgrid_meta; // [N]
    unsigned long long *objgrid_mask;// per env 4 x ny x nx words
    // column-layer cache (Appendix G; null = off): per (env, sphere) the
    // offset, within its column's layer list, of the free layer the sphere's
    // last grid query found; the next query starts there
    uint8_t *layer_hint;             // [N][S]
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

// Launchers (defined in the .hip files).
hipError_t launch_robot_step(const RobotParams &rp, const SimBuffers &sb, const float *actions,
                             const StepOutputs &out, uint32_t *queue_reset, int lanes_per_env,
                             hipStream_t s);
hipError_t launch_reset(const RobotParams &rp, const SimBuffers &sb, const uint8_t *mask,
                        hipStream_t s);
// Object frames of the current state (manipulation; after create, reset and
// state restore, so that the raster draws the objects where they are).
hipError_t launch_object_frames(const RobotParams &rp, const SimBuffers &sb, hipStream_t s);
// The resting objects' grids of every env, from the current object records
// (after create; with manipulation also after reset and state restore).
hipError_t launch_objgrid_build(const RobotParams &rp, const SimBuffers &sb, hipStream_t s);
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
