/*
 * gal.h -- C ABI of the MI355X batched kinematic simulator step.
 *
 * One batch object steps every environment at once, the way the paper's
 * single simulator instance steps physics for a whole batch of environments
 * and a single renderer produces one stacked image per sensor in GPU memory
 * that the learner consumes in place (Galactic, Section 3.1 "Batching").
 * The step itself follows Section 3.2 "Approximate Kinematic
 * Simulation" and Appendix G: action offsets applied directly to the robot
 * state, forward kinematics of the articulated links, sphere-proxy overlap
 * tests against a static-scene column grid (one grid per sphere-radius
 * class) and against the movable objects' oriented boxes, a collision
 * resolved by disallowing all robot movement for the step, and a head-camera
 * depth observation (Section 4.1: 90 degree FoV).
 *
 * Conventions
 *  - Every function returns an int status: GAL_OK (0) or a negative GAL_E*
 *    code; the message of the last failure on the calling thread is returned
 *    by gal_last_error().  Nothing is thrown across the ABI.
 *  - "host" pointers are ordinary CPU memory read during the call only;
 *    "device" pointers are HIP device memory owned by the caller (for
 *    example torch tensors on cuda:0) and must stay valid until the work
 *    enqueued on `stream` has finished.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    gal_step / gal_reset only enqueue work on it: they never synchronise
 *    the device and never copy to the host.
 *  - Coordinates are metres, Z-up, right-handed; angles are radians.
 *  - All floating point is IEEE binary32 evaluated in a fixed order with
 *    round-to-nearest-even, so results are reproducible bit for bit.
 */
#ifndef GAL_H
#define GAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GAL_OK 0
#define GAL_EINVAL (-1)    /* bad argument or configuration                    */
#define GAL_ENOMEM (-2)    /* device or host allocation failed                 */
#define GAL_EDEVICE (-3)   /* a HIP call failed (its text is in gal_last_error) */
#define GAL_ESTATE (-4)    /* state buffer size / layout mismatch              */
#define GAL_EOVERFLOW (-5) /* a fixed-capacity structure overflowed at build   */

#define GAL_MAX_CLASSES 8
#define GAL_MAX_SPHERES 256
#define GAL_MAX_PLANES 4096
#define GAL_STATE_FLOATS 10 /* x, y, yaw, q0..q6 */

/* flags of gal_config.flags */
#define GAL_COLOR 0x1u      /* also produce flat-shaded RGB8 per pixel         */
#define GAL_MANIP 0x2u      /* grasp / carry / release of the movable objects
                               (Section 3.2, Appendix I): 11-float actions,
                               objects move and are drawn where they are     */
#define GAL_SLIDE 0x4u      /* with GAL_MANIP: a collision slides the base
                               instead of stopping it (Appendix I.1)         */
#define GAL_LINKS 0x8u      /* the head camera also sees the robot itself
                               (Section 4.1's observation): each link drawn
                               as its box (gal_robot.link_box)               */
#define GAL_SHADE 0x10u     /* with GAL_COLOR: lit, textured colour instead of
                               flat colour (Section 4.1's RGB; see gal_step);
                               needs scenes->tri_plane (the faces' normals) */

/*
 * Robot (Section 3.2 / Appendix G): a planar base (x, y, yaw) and a 7-DoF
 * revolute arm.  Link frame 0 is the base; link frame j+1 = (link frame j,
 * or for j = 0 the base frame translated by `mount`) * Rz(q_j) Tz(d_j)
 * Tx(a_j) Rx(alpha_j) (standard Denavit-Hartenberg).  alpha_j is given by its
 * cosine and sine.  Each link is proxied by spheres whose radius is one of
 * the configured radius classes; a sphere flagged held-only exists only in
 * environments whose `held` flag is set (a grasped-object proxy carried on
 * the end effector).  Host memory, copied at gal_create_batch.
 */
typedef struct gal_robot {
    float dh[7][4];             /* a, d, cos(alpha), sin(alpha)              */
    float qlim[7][2];           /* joint limits lo, hi                       */
    float q_home[7];            /* joint angles at episode start             */
    float mount[3];             /* arm mount in the base frame               */
    float cam_offset[3];        /* head camera position in the base frame    */
    float cam_pitch_cs[2];      /* cos, sin of the camera's downward pitch   */
    int32_t num_spheres;        /* S, 1..GAL_MAX_SPHERES                     */
    const int32_t *sphere_link; /* [S] link frame 0..7                       */
    const float *sphere_pos;    /* [S][3] centre in the link frame           */
    const int32_t *sphere_class;/* [S] radius class index                    */
    const uint8_t *sphere_held_only; /* [S] or NULL (none held-only)         */
    /* GAL_MANIP (Section 3.2 suction grasp): the grasp sphere at grasp_tip in
       the end-effector frame (link 7), its radius, and the radius class of a
       held object's 8 octant spheres.  Ignored without GAL_MANIP.  With
       GAL_MANIP the held-only spheres above are not used (the held object's
       own spheres replace them). */
    float grasp_tip[3];
    float grasp_radius;
    int32_t held_class;
    /* GAL_LINKS: the render box of each link in its own frame (link 0 = the
       base): centre xyz, half extents xyz (> 0).  Corner k of link l is
       F_l (c + (+-h)) (bit 0 of k: x, bit 1: y, bit 2: z) with F_l the link's
       frame after the step; 12 triangles per link, wound counter-clockwise
       around the outward normals, numbered after the env's mesh triangles
       and (GAL_MANIP) its objects' 12 O, culled by their winding only.
       link_rgb: the flat colour of each link (needed with GAL_COLOR).
       Ignored without GAL_LINKS. */
    const float *link_box;      /* [8][6]                                    */
    const uint8_t *link_rgb;    /* [8][3] or NULL                            */
} gal_robot;

/*
 * Scenes, one per environment, as concatenated host arrays indexed by
 * per-env offsets (CSR).  Copied to the device at gal_create_batch.
 *  - Render mesh: triangles of env-local vertex indices, wound
 *    counter-clockwise around the outward normal (back faces are culled).
 *  - Static collision boxes (axis-aligned, min xyz / max xyz) build the
 *    column grids; the floor z <= 0 is implicit.  Movable objects are not
 *    part of the grid: they are oriented boxes (yaw only).
 *  - The column grid of env e covers nx * ny square cells of `cell_m` from
 *    `grid_origin`; a sphere centre outside it is in contact.
 */
typedef struct gal_scene_set {
    int32_t num_envs;           /* N >= 1                                    */
    const int64_t *vert_offset; /* [N+1]                                     */
    const float *verts;         /* [V][3]                                    */
    const int64_t *tri_offset;  /* [N+1]                                     */
    const int32_t *tris;        /* [T][3] env-local vertex indices           */
    const uint8_t *tri_rgb;     /* [T][3] flat colour, or NULL               */
    const int64_t *box_offset;  /* [N+1]                                     */
    const float *boxes;         /* [B][6] min x,y,z, max x,y,z               */
    int32_t num_objects;        /* O per env, 0..64                          */
    const float *objects;       /* [N][O][8] centre xyz, half extents xyz,
                                   cos(yaw), sin(yaw)                        */
    const float *grid_origin;   /* [N][2]                                    */
    const int32_t *grid_dims;   /* [N][2] nx, ny                             */
    int32_t num_starts;         /* P >= 1 start poses per env                */
    const float *starts;        /* [N][P][3] x, y, yaw                       */
    const uint8_t *held;        /* [N] or NULL (no env holds an object)      */
    const int32_t *res;         /* [N] square depth resolution per env, or
                                   NULL for res0 everywhere; 8..256, a
                                   multiple of 8                             */
    const float *tri_plane;     /* [T][4] or NULL: the plane of the face each
                                   triangle lies on (outward unit normal n,
                                   offset w = n . p on the face).  A triangle
                                   whose face the camera position c is not
                                   strictly in front of, (n0 c0 + n1 c1) +
                                   n2 c2 - w <= 0 in FP32, is culled as a back
                                   face before its winding test; triangles of
                                   one face share one plane (bitwise), which
                                   lets the renderer skip whole groups of them.
                                   At most GAL_MAX_PLANES distinct planes per
                                   env (GAL_EINVAL otherwise).               */
    const uint8_t *obj_rgb;     /* [N][O][3] flat colour of each movable
                                   object (GAL_MANIP with GAL_COLOR), or NULL.
                                   With GAL_MANIP the render mesh holds only
                                   the static scene: every object is drawn as
                                   its box where it is, 12 triangles numbered
                                   after the env's mesh triangles, culled by
                                   their winding only.                       */
} gal_scene_set;

typedef struct gal_config {
    int32_t res0;               /* depth resolution when scenes->res is NULL */
    float near_m, far_m;        /* depth range; the field of view is 90 deg  */
    float cell_m;               /* column-grid cell size                     */
    int32_t num_classes;        /* K, 1..GAL_MAX_CLASSES                     */
    float class_radius[GAL_MAX_CLASSES];
    float act_lim[3];           /* |forward| m, |yaw| rad, |joint delta| rad */
    int32_t episode_len;        /* steps per episode; 0 = never auto-reset   */
    uint32_t flags;             /* GAL_COLOR | GAL_MANIP | GAL_SLIDE |
                                   GAL_LINKS | GAL_SHADE                     */
    /* GAL_MANIP (Appendix I): base jitter per sliding try and object jitter
       per placing try (m), and the seed of the placing jitter's counter-based
       randomness */
    float slide_step, place_step;
    uint64_t manip_seed;
} gal_config;

/*
 * Caller-owned device outputs of one step.  Per-env images are packed one
 * after the other (env e starts at gal_depth_offsets()[e] pixels).  Depth is
 * the 24-bit encoding (1/near - 1/z) * (2^24-1) / (1/near - 1/far) of the
 * camera-space distance z: computed at each triangle's vertices, combined at
 * a pixel centre with the triangle's integer barycentric weights (edge
 * functions / twice the area) in binary32, clamped and truncated; the
 * smallest value over the covering front faces wins, 0xFFFFFF where nothing
 * was hit.  Any pointer except `depth` may be NULL to skip that output.
 */
typedef struct gal_outputs {
    uint32_t *depth;            /* [sum res^2]                               */
    uint8_t *rgb;               /* [sum res^2][3] (needs GAL_COLOR)          */
    uint32_t *contact_static;   /* [N][W], W = ceil(S/32): bit s of word s/32
                                   = sphere s of the candidate pose overlaps
                                   the static scene (column grid)            */
    uint32_t *contact_object;   /* [N][W]: ... overlaps a movable object     */
    uint8_t *accepted;          /* [N] 1 = the move was committed            */
    float *state;               /* [N][10] state after the step              */
    float *frames;              /* [N][8][12] link frames (3x4 row-major)    */
    int32_t *counters;          /* [N][2] step in episode, episode index     */
    uint8_t *done;              /* [N] 1 = the episode ended at this step    */
    float *object_frames;       /* [N][O][12] GAL_MANIP: every object's frame
                                   after the step (3x4 row-major; a held one
                                   is carried by the end effector)           */
    int32_t *held;              /* [N] GAL_MANIP: held object, -1 = none     */
} gal_outputs;

typedef struct gal_batch gal_batch;   /* opaque, owned by the library */

/*
 * Create a batch (Section 3.1 "Batching": one simulator instance and one
 * renderer serve every environment of the batch, and the observations stay
 * stacked in GPU memory): validates the inputs, copies robot and scenes to the
 * device, builds the column grids (one per env and radius class) and the
 * clustered render meshes, and sets every env to episode 0 at its first
 * start pose with the arm at q_home.  Synchronous (returns when done).
 * Errors: GAL_EINVAL (inconsistent sizes, res not a multiple of 8 or out of
 * range, S or K out of range, near/far invalid), GAL_ENOMEM, GAL_EDEVICE,
 * GAL_EOVERFLOW (a grid column blocked by more than 64 boxes).
 */
int gal_create_batch(const gal_config *cfg, const gal_robot *robot,
                     const gal_scene_set *scenes, void *stream, gal_batch **out);

/*
 * Episode reset (Section 4.1: episodes of at most 500 steps; the start pose
 * and arm configuration are this build's reading, Section 3.2 places the
 * robot, it does not say where).
 * Start a new episode in the envs selected by `env_mask_dev` (device u8[N],
 * nonzero = reset; NULL = all envs): episode += 1, pose = start pose
 * (episode mod P), arm at q_home, step counter 0.  Asynchronous on `stream`.
 */
int gal_reset(gal_batch *b, const uint8_t *env_mask_dev, void *stream);

/*
 * One step of every environment (Section 3.2 "Approximate Kinematic
 * Simulation" and Appendix G for steps 1-3; Section 4.1 for the horizon and
 * the 90 degree head-camera depth observation of step 5), asynchronous on
 * `stream`:
 *  1. actions_dev f32 [N][9] = forward offset (m), yaw offset (rad), 7 joint
 *     offsets (rad); NaN components count as 0, then each is clamped to
 *     +-act_lim.  Candidate: yaw' = yaw + a1 wrapped into [-pi, pi]; x, y move
 *     a0 along the new heading; q' = clamp(q + a, qlim).
 *  2. forward kinematics of the candidate; every active sphere is tested
 *     against its class's column grid and every object box;
 *  3. any overlap rejects the whole move (state unchanged), otherwise the
 *     candidate is committed;
 *  4. the step counter advances; at episode_len the env auto-resets
 *     (gal_reset semantics) and `done` is set;
 *  5. frames and the depth (and colour) image are produced for the final
 *     state.  With out->depth NULL only the physics runs (no image).
 * With GAL_MANIP (Section 3.2 grasping and snap-to-surface, Appendix I):
 * actions are [N][11], the 9 above then grasp/release (>= 0.5: grasp when
 * nothing is held -- the nearest object overlapping the grasp sphere is
 * fixed to the end effector -- otherwise a held object is released; NaN
 * counts as 0) and stop (>= 0.5 ends the episode like the horizon).  A held
 * object's 8 octant spheres join the overlap test; resting objects are
 * tested as boxes.  With GAL_SLIDE a rejected move is retried up to 3 times
 * with the base moved slide_step away from the mean centre of the
 * overlapping spheres (accepted = 2 when one of those is taken).  A release
 * sets the object upright (yaw of its x axis), casts 4 spheres of its bottom
 * face down the held class's column grid, lands it on the highest surface
 * they meet, and retries up to 6 times, jittered by place_step, while the
 * cast fails or the landed box overlaps another object; then it returns to
 * where it was grasped.  Contact words then cover S + 8 spheres (bits S..S+7
 * = the held object's).  An episode start restores every object.
 * With GAL_SHADE the colour is lit and textured (a stand-in for the paper's
 * baked textures and lighting), per pixel from the winning triangle's outward
 * unit normal n (its face plane; a box face's frame axis) and colour c and the
 * pixel's D24 depth D: 1/Z = 1/near - D / K (K the depth scale), world point
 * P = cam + Z ((fwd + u right) + v down) at the pixel centre (u, v in
 * [-1, 1]); s = 0.35 + 0.65 max(0, n . (0.36, 0.48, 0.8)); a checker of
 * 0.25 m squares on the two world axes other than n's largest component
 * (z first, then x) darkens odd squares to t = 0.8; each channel
 * min(255, floor(c s t + 1/2)); FP32 in that order.
 * Errors: GAL_EINVAL (NULL batch/actions/outputs, rgb without GAL_COLOR or
 * without depth),
 * GAL_EDEVICE (launch failure).
 */
int gal_step(gal_batch *b, const float *actions_dev, const gal_outputs *out, void *stream);

/*
 * Launch configuration of the raster kernel (this build's extension of the
 * batch renderer of Section 3.1; not in the paper).  Every setting produces
 * the same bits (the outputs are defined independently of how the work is split); the
 * settings only change speed, and an autotuner picks among them.
 *  block      threads per workgroup: 256, 512 or 1024
 *  region     square pixel region owned by one workgroup: 32, 64 or 128 (must
 *             divide every env resolution above it)
 *  lane_max   triangles whose clipped pixel bbox has at most this many pixels
 *             are rasterised by their own lane (0..4096)
 *  small_max  larger ones up to this many pixels are rasterised together by
 *             the wave, pixels spread evenly over the lanes (0..65536); the
 *             rest one at a time by the whole wave, 8x8 tile by tile
 *  refresh    occlusion rounds: how many times the z-buffer bounds are
 *             refreshed and the clusters not drawn yet re-tested against
 *             them (1..16); each round draws half of the survivors (at
 *             least 64), the last one all of them
 *  occlusion  1 = skip clusters provably hidden behind conservative z-buffer
 *             bounds, 0 = frustum culling only
 *  prologue   clusters drawn before the first occlusion test (>= 0)
 *  persistent 1 = one persistent raster kernel whose workgroups drain the
 *             (env, region) work queue, longest items first; 0 = one
 *             workgroup per item
 *  robot_lanes lanes per environment in the robot-step kernel: 64 (one env
 *             per wave) or 32 (two envs per wave)
 *  graph      1 = gal_step replays the whole step as a captured hipGraph
 *             (re-captured when the action/output pointers or the tuning
 *             change; not used while gal_profile is enabled)
 *  split      number of envs (0..N), taken from the cheap end of the
 *             longest-first item order, whose regions are halved (four
 *             items per region instead of one) so that the last items of a
 *             launch are short; envs whose region side is not a multiple of
 *             16 are not split
 *  order      with the persistent queue: 1 = each step drains the items in
 *             the order of their times in the previous step, longest first
 *             (measured on the device; up to 32768 items, the static order
 *             beyond), 0 = the static order by cluster count
 *  objgrid    1 = a sphere's resting-object candidates come from four offset
 *             regular grids of 0.5 m cells (Appendix G: any sphere of
 *             radius <= 12.5 cm lies wholly inside a cell of one of them;
 *             a cell lists the objects whose footprint meets it), 0 = every
 *             object is tested; the contacts are the same either way
 *  bin        1 = the triangles between lane_max and small_max pixels are
 *             binned: each is listed, in LDS, under every 8x8 pixel tile of
 *             the region it can cover, and the tiles are drawn one per wave
 *             (lane = pixel) when the list buffer fills; 0 = they are drawn
 *             by the wave that set them up.  The z-buffer and the bins must
 *             fit one CU's 160 KB of LDS (with colour: region <= 64)
 *  layer_cache 1 = each sphere's column-grid query starts at the layer where
 *             its previous query found free space (Appendix G's layer
 *             cache: a per (env, sphere) offset into the column's layer
 *             list, kept on the device), 0 = at the column's first layer;
 *             the contacts are the same either way.  Not with GAL_MANIP
 * A new batch starts with block 512, region 128 (or the resolution, if
 * smaller), lane_max 8, small_max 1024, occlusion 1 with refresh 1 and
 * prologue 128, persistent 0, robot_lanes 64, graph 0, split 0, order 0,
 * objgrid 1 with 16 or more objects per env (else 0), bin 0, layer_cache 0.
 */
typedef struct gal_tuning {
    int32_t block;
    int32_t region;
    int32_t lane_max;
    int32_t small_max;
    int32_t refresh;
    int32_t occlusion;
    int32_t prologue;
    int32_t persistent;
    int32_t robot_lanes;
    int32_t graph;
    int32_t split;
    int32_t order;
    int32_t objgrid;
    int32_t bin;
    int32_t layer_cache;
} gal_tuning;

/* Read / replace the launch configuration above (Section 3.1 batching
 * extension).  gal_set_tuning errors: GAL_EINVAL for values out of range.
 * Not to be called while a step on the batch is in flight on another
 * stream. */
int gal_get_tuning(const gal_batch *b, gal_tuning *t);
int gal_set_tuning(gal_batch *b, const gal_tuning *t);

/*
 * Autotuner (this build's extension of Section 3.1 "Batching": the paper
 * fixes one batch size per GPU; here the split of the batch's work into
 * workgroups is searched per batch): times the candidate launch configurations (raster workgroup
 * size, region, small-triangle thresholds, occlusion culling, persistent
 * queue, and the 8x8-tile binning wherever its LDS fits) on this batch with
 * the given actions and
 * outputs (`steps` timed steps each, HIP events); then, on the fastest and on
 * it with the other launch mode, `split` at 0, 1/16, 1/8, 1/4 and 1/2 of the
 * workgroups resident at once, each with an occlusion prologue of 128 and 256
 * clusters and, with the queue, both item orders (3 x `steps` each, two
 * interleaved rounds); last, the robot step's 32 or 64 lanes per env on the
 * winner (3 x `steps` each, three interleaved rounds).  It
 * checks that every candidate produces the same depth bits from the same
 * state, keeps the fastest (also written to *best, with its time per step in
 * *best_ms) and restores the simulation state it started from.  The outputs'
 * contents are overwritten.  Synchronous.  GAL_ESTATE if a candidate's output
 * differs.
 */
int gal_autotune(gal_batch *b, const float *actions_dev, const gal_outputs *out, void *stream,
                 int32_t steps, gal_tuning *best, double *best_ms);

/* Number of environments, spheres, contact words, and the packed depth size
 * (the batch's shape, Section 3.1). */
int gal_batch_info(const gal_batch *b, int32_t *num_envs, int32_t *num_spheres,
                   int32_t *contact_words, int64_t *depth_pixels);

/* Host copy of the per-env pixel offsets of the packed depth output, [N+1]
 * (one stacked image per sensor, Section 3.1; envs may differ in resolution). */
int gal_depth_offsets(const gal_batch *b, int64_t *offsets_host, size_t count);

/*
 * Checkpoint / restore of the simulation state of Section 3.2 (the robot's
 * base pose and joint angles; objects and scene are static in this step) and
 * the episode counters of Section 4.1 (synchronises `stream`):
 * host buffer of N * (10 floats + 2 int32) bytes, laid out as f32 state
 * [N][10] followed by i32 counters [N][2]; with GAL_MANIP followed by f32
 * objects [N][O][8] (resting records; a held object's from before its
 * grasp), i32 held [N] and f32 rel [N][12] (the held object's frame in the
 * end-effector frame).  GAL_ESTATE when `bytes` differs.
 */
int gal_get_state(gal_batch *b, void *host, size_t bytes, void *stream);
int gal_set_state(gal_batch *b, const void *host, size_t bytes, void *stream);

/*
 * Inspection of the column grid of Appendix G (free vertical layers per
 * column, one grid per sphere-radius class) built on the device for env `env`
 * and radius class `cls` (synchronous): the layer count of every column as CSR
 * offsets (host u32 [nx*ny+1]) and the free layers (host f32 [L][2] = lowest
 * and highest admissible sphere-centre height; the top one ends at +inf).
 * Pass layers_host = NULL to query L through *num_layers.
 */
int gal_get_grid(gal_batch *b, int32_t env, int32_t cls, uint32_t *offsets_host,
                 size_t offsets_count, float *layers_host, size_t layers_count,
                 int64_t *num_layers);

/*
 * Per-kernel timing of gal_step with HIP events recorded on the step's own
 * stream: the split of Appendix F's rollout-step timing table into physics
 * and rendering, measured here on the device.  While enabled, every gal_step records an event before, between
 * and after its two stages (everything before the raster: the surrogate's
 * kernels when one is attached and the robot step; then the raster);
 * gal_profile_read waits for the recorded events, returns the summed
 * milliseconds of each stage (robot_ms, raster_ms) and the number of timed
 * steps, and clears the record.  Adds no synchronisation to gal_step itself.
 */
int gal_profile_enable(gal_batch *b, int on);
int gal_profile_read(gal_batch *b, double *robot_ms, double *raster_ms, int64_t *steps);
/* The same record split three ways (Appendix F's physics / rendering split,
 * with the learned pre-filter of this build apart): stage_ms_host[0] = the
 * surrogate's kernels (0 when none is attached), [1] = the robot step, [2] =
 * the raster; count must be 3.  Reading clears the record, as above. */
int gal_profile_read_stages(gal_batch *b, double *stage_ms_host, size_t count, int64_t *steps);

/*
 * On-device work counters of the raster kernel (the rendering phase of
 * Appendix F's timing table, broken down by culling stage), summed over the
 * steps run while enabled (reading synchronises the device and clears them).
 * counters_host receives GAL_NUM_COUNTERS values: [0] clusters tested against
 * the frustum, [1] inside it, [2] of those proven hidden by the occlusion
 * bounds, [3] clusters drawn, [4] triangles surviving trivial rejection,
 * [5] of which clipped, [6] front-facing (sub)triangles with pixels in a
 * region, [7] their bbox pixel count.  Counting costs a few atomics per wave.
 */
#define GAL_NUM_COUNTERS 8
int gal_counters_enable(gal_batch *b, int on);
int gal_counters_read(gal_batch *b, int64_t *counters_host, size_t count);

/* Sizes of the device-resident render mesh of the batch renderer
 * (Section 3.1): 64-triangle clusters, their (per-cluster unique) vertices,
 * and triangles. */
int gal_mesh_info(const gal_batch *b, int64_t *clusters, int64_t *cluster_verts,
                  int64_t *tris);

/*
 * ---- Collision surrogate (a learned pre-filter; not in the paper) ----
 *
 * A small MLP predicts, for each environment's next move, whether its
 * candidate pose overlaps the static scene (the column-grid test of Section
 * 3.2).  Input (2112 BF16 values, gal_features): [0..6] the candidate
 * joint angles; [7..13] the joint offsets and [14..15] the base offsets of
 * the action, normalised by their limits; [16..18] the base pose normalised
 * by the grid extent (and yaw / pi); [19] the held-object flag; [20..40] the
 * origins of joint frames 1..7 and [41..43] the end-effector z axis of the
 * candidate arm pose in the base frame (metres); [44..63] zeros; then
 * [64..2111] a 16 x 16 x 8 occupancy patch [a][b][layer] in the frame of the
 * candidate base pose: cells 0.1 m wide centred on ((a - 7.5) 0.1 m,
 * (b - 7.5) 0.1 m) around the base, layers of 0.25 m from the floor.  A
 * patch cell is 1 (blocked) when any grid column under the bounding box of
 * its rotated footprint has, at one of four heights inside the layer (none
 * below 0.125 m), no free layer of the batch's last radius class (the
 * largest in a plain batch), or when that box leaves the grid.  Network
 * 2112 -> 256 -> 256 -> 256 -> 256 -> 1 with ReLU, BF16 weights and
 * activations, FP32 accumulation (matrix cores).
 * Parameters are FP32 [W1 (256 x 2112), b1, W2, b2, W3, b3, W4, b4,
 * W5 (1 x 256), b5], each W one row per output unit.
 */
typedef struct gal_mlp gal_mlp;
#define GAL_MLP_IN 2112

/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Total parameter count (738,561). */
int gal_mlp_num_params(int64_t *n);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Device MLP for up to max_rows rows per call; He-uniform initial weights
 * from `seed`, zero biases, Adam state cleared.  Synchronous. */
int gal_mlp_create(int32_t max_rows, uint64_t seed, gal_mlp **out);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Host FP32 parameters in the layout above (count = gal_mlp_num_params);
 * set also clears the Adam state.  Synchronous.  (The weights arrive as a
 * host array rather than a file path: the caller owns the file format.) */
int gal_mlp_set_weights(gal_mlp *m, const float *host, size_t count);
int gal_mlp_get_weights(gal_mlp *m, float *host, size_t count);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Logits (device f32 [rows]) of x_dev (device BF16 bits, u16 [rows][2112],
 * 16-byte aligned rows).  Up to 8192 rows, the first layer's
 * sum over the 2112 inputs is split over 2, 4 or 8 workgroups per 32 rows
 * whose FP32 partial sums are added in a fixed order, so logits depend on
 * the row count in the last bits and can differ from the training forward
 * pass in the last bits; they are reproducible for a given row count.  The
 * partial sums live in the MLP object: calls on one MLP must not overlap. */
int gal_mlp_forward(gal_mlp *m, const uint16_t *x_dev, int32_t rows, float *logits_dev, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * gal_mlp_forward with its scratch -- the first layer's partial sums, at most
 * 16 MiB -- in a fixed device array of the library instead of the MLP
 * object.  Allocates nothing; each GPU the library runs
 * on holds one such array until the process ends.  Same logits, bit for
 * bit, as gal_mlp_forward for the same rows.  logits_dev must not be NULL;
 * rows above GAL_MLP_STATIC_MAX_ROWS are rejected (GAL_EINVAL).  Every call
 * on one GPU shares that GPU's array (whatever the MLP or the stream):
 * calls that overlap on one GPU race. */
#define GAL_MLP_STATIC_MAX_ROWS (1 << 22)
int gal_mlp_forward_static(gal_mlp *m, const uint16_t *x_dev, int32_t rows, float *logits_dev,
                           void *stream);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Gradients of the weighted logistic loss (1/rows) sum_i w_i l(z_i, y_i),
 * w_i = pos_weight for labels 1, into grads_dev (device f32, parameter
 * layout; may be NULL) and the loss into loss_dev (device f32[1]; may be
 * NULL).  Labels are device f32 0/1. */
int gal_mlp_gradients(gal_mlp *m, const uint16_t *x_dev, const float *labels_dev, int32_t rows,
                      float pos_weight, float *grads_dev, float *loss_dev, void *stream);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * One Adam step (Kingma & Ba; beta 0.9 / 0.999, eps 1e-8) on those
 * gradients. */
int gal_mlp_train_step(gal_mlp *m, const uint16_t *x_dev, const float *labels_dev, int32_t rows,
                       float pos_weight, float lr, float *loss_dev, void *stream);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * The MLP's BF16 matrix-core GEMM alone, FP32 output (for verification):
 * variant 3: C = A B^T, 4: C = A B, 5: C = A^T B, operands BF16 bits with
 * leading dimensions lda / ldb (elements), C [M][ldc]. */
int gal_mlp_gemm_test(int32_t variant, const uint16_t *a_dev, const uint16_t *b_dev, int32_t M,
                      int32_t N, int32_t K, int32_t lda, int32_t ldb, float *c_dev, int32_t ldc,
                      void *stream);
/* Surrogate of the Section 3.2 static-scene test (not in the paper): frees
 * the MLP. */
void gal_mlp_destroy(gal_mlp *m);

/* Surrogate of the Section 3.2 static-scene test (not in the paper); the
 * patch samples the column grid of Appendix G.
 * Surrogate inputs of every env's next move under actions_dev into x_dev
 * (device BF16 u16 [N][2112], 16-byte aligned).  Builds the occupancy
 * lattice on first use (synchronous then). */
int gal_features(gal_batch *b, const float *actions_dev, uint16_t *x_dev, void *stream);
/*
 * Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Put the MLP in front of the static check of gal_step: an env whose
 * predicted contact probability is <= skip_below skips the column-grid test
 * (its static contact mask is then 0), except a hashed 1-in-audit_period
 * sample of those (audit_period 1 = all, 0 = none), for which the exact
 * test runs and a contact counts as a mismatch.  Object checks always run.
 * The MLP must hold >= N rows and outlive the attachment.
 */
int gal_surrogate_attach(gal_batch *b, gal_mlp *m, float skip_below, uint32_t audit_period,
                         void *stream);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * The attached MLP's logits (device f32 [N]) for every env's next move under
 * actions_dev, from the features gal_features would write, computed inside
 * the inference launch the step uses (no routing, no counts).
 * GAL_EINVAL when no surrogate is attached. */
int gal_surrogate_logits(gal_batch *b, const float *actions_dev, float *logits_dev, void *stream);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * Detach restores the exact test for every env. */
int gal_surrogate_detach(gal_batch *b);
/* Surrogate of the Section 3.2 static-scene test (not in the paper).
 * stats_host[4] = queries, skipped, audited, audit mismatches since the last
 * reset (synchronises the device; reset != 0 clears them). */
int gal_surrogate_stats(gal_batch *b, int64_t *stats_host, int reset);

/*
 * The policy that consumes the depth stack (Section 4.2 "Approach: End-to-End
 * RL": the simulator's stacked observation feeds batched DNN inference in
 * place; the SimpleCNN encoder of the appendix on model sizes): 128x128 D24
 * depth, x = D / (2^24 - 1) in BF16 -> conv 8x8 stride 4 (32 channels) ->
 * conv 4x4 stride 2 (64) -> conv 3x3 stride 1 (32), no padding, each with
 * ReLU -> fully connected 4608 -> 512 with ReLU (BF16 weights and
 * activations, FP32 accumulation) -> a Gaussian actor (mean linear in the 512
 * features and the 7 joint angles, a learned log_std per action) and a critic
 * (linear in the same), in FP32.  No recurrent core (a reading: the joint
 * angles carry the state the paper's LSTM would).  Parameter vector (FP32):
 * conv1 W [32][8][8][1], b [32]; conv2 W [64][4][4][32], b [64]; conv3 W
 * [32][3][3][64], b [32]; fc W [512][4608] (input (y * 12 + x) * 32 + c), b
 * [512]; actor W [A][519], b [A]; critic W [519], b [1]; log_std [A].
 * Create: room for max_envs images, act_dim A (1..32), seeded He-uniform
 * encoder weights, small heads, log_std -0.5.  Errors: GAL_EINVAL,
 * GAL_ENOMEM.
 */
typedef struct gal_policy gal_policy;
int gal_policy_create(int32_t max_envs, int32_t act_dim, uint64_t seed, gal_policy **out);
/* The policy of Section 4.2: number of FP32 parameters. */
int gal_policy_num_params(const gal_policy *p, int64_t *n);
/* The policy of Section 4.2: replace / read the parameter vector (host FP32,
 * the layout above; synchronous). */
int gal_policy_set_weights(gal_policy *p, const float *host, size_t count);
int gal_policy_get_weights(gal_policy *p, float *host, size_t count);
/*
 * The policy of Section 4.2 on n_envs envs, asynchronous on `stream`:
 * depth_dev = the batch's depth output of 128x128 images (device u32
 * [n_envs][128][128], 16-byte aligned, read in place), state_dev = its state
 * output (device f32 [n_envs][10], joint angles at 3..9).  actions_dev (f32
 * [n_envs][A]) = mean + exp(log_std) * noise with noise_dev (f32 [n_envs][A],
 * the caller's standard normal draws), or the mean when noise_dev is NULL;
 * value_dev (f32 [n_envs], or NULL) = the critic; logp_dev (f32 [n_envs], or
 * NULL; needs noise) = sum_a (-noise_a^2 / 2 - log_std_a) - A log(2 pi) / 2.
 * Calls that overlap on one policy race on its activation buffers.
 */
int gal_policy_act(gal_policy *p, const uint32_t *depth_dev, const float *state_dev, int32_t n_envs,
                   const float *noise_dev, float *actions_dev, float *value_dev, float *logp_dev,
                   void *stream);
/* Coefficients of the PPO loss below. */
typedef struct gal_ppo_params {
    float clip;                 /* the ratio's clip range, e.g. 0.2          */
    float value_coef;           /* e.g. 0.5                                  */
    float entropy_coef;         /* e.g. 0.01                                 */
} gal_ppo_params;
/*
 * The policy's update (Section 4.2 trains the policy with DD-PPO: PPO with
 * the gradients all-reduced over GPUs; this is one GPU's step).  One
 * gradient of the PPO loss over `samples` (<= max_envs) rollout samples:
 * depth_dev (u32 [S][128][128]) and state_dev (f32 [S][10]) the observations,
 * actions_dev (f32 [S][A]) the actions taken, old_logp_dev (f32 [S]) their
 * log-density under the policy that took them, adv_dev and ret_dev (f32 [S])
 * the advantages and returns (gal_gae).  With r = exp(logp - old_logp):
 *   L = -mean(min(r A, clip(r, 1 - clip, 1 + clip) A))
 *       + value_coef mean((V - R)^2) - entropy_coef H,
 *   H = sum_a (log_std_a + (1 + ln 2 pi) / 2).
 * The gradient (FP32, the parameter layout above) stays in the policy for
 * gal_policy_adam_step and is copied to grads_dev (f32 [n_params]) when not
 * NULL; stats_dev (f32 [4], or NULL) = mean policy loss, mean (V - R)^2, H,
 * mean ratio.  BF16 activations and pre-activation gradients, FP32 weight
 * gradients.  Asynchronous on `stream`.
 */
int gal_policy_ppo_gradients(gal_policy *p, const uint32_t *depth_dev, const float *state_dev,
                             const float *actions_dev, const float *old_logp_dev, const float *adv_dev,
                             const float *ret_dev, int32_t samples, const gal_ppo_params *hp,
                             float *grads_dev, float *stats_dev, void *stream);
/* The policy's update of Section 4.2: one Adam step (beta 0.9 / 0.999, eps
 * 1e-5) of the parameters with the last gradient, learning rate lr; the BF16
 * copy follows.  GAL_ESTATE before any gradient. */
int gal_policy_adam_step(gal_policy *p, float lr, void *stream);
/* Advantages for the update of Section 4.2 (generalised advantage
 * estimation): over a rollout of T steps x N envs (f32 [T][N], dones u8
 * [T][N] = the step ended its episode), last_value_dev (f32 [N]) the critic
 * after the last step:  delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t,
 * A_t = delta_t + gamma lam (1 - d_t) A_{t+1}, returns = A + V (FP32, one
 * thread per env, backwards in time). */
int gal_gae(const float *rewards_dev, const float *values_dev, const uint8_t *dones_dev,
            const float *last_value_dev, int32_t T, int32_t N, float gamma, float lam, float *adv_dev,
            float *ret_dev, void *stream);
/* The policy of Section 4.2: the BF16 activations of layer 1..4 (conv1..3
 * NHWC, fc) of the last gal_policy_act into host memory, count values
 * (synchronous; for checking the encoder layer by layer). */
int gal_policy_activations(gal_policy *p, int32_t layer, uint16_t *host, size_t count);
/* The policy of Section 4.2: frees it. */
void gal_policy_destroy(gal_policy *p);

/* Frees a batch created by gal_create_batch (Section 3.1 batch object). */
void gal_destroy(gal_batch *b);

/* Message of the last failing call on this thread ("" if none); the error
 * convention of every entry point above (Section 3.1 boundary). */
const char *gal_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GAL_H */
