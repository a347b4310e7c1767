/*
 * CPU oracle of the batched kinematic step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct C.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load this library; the product path
 * (the HIP library) shares no code with it.
 *
 * What it computes, for one environment at a time (Galactic, Section 3.2
 * "Approximate Kinematic Simulation" and Appendix G "Additional
 * Collision-Detection Details"):
 *   1. the action offsets are applied directly to the robot state (base
 *      forward/back, base rotation, arm joint deltas) -- kinematic motion, no
 *      velocities or forces;
 *   2. forward kinematics gives the pose of every articulated link;
 *   3. the candidate pose's spheres are tested for overlap against the static
 *      scene's column grid (one grid per sphere-radius class, nearest column,
 *      linear search of the free vertical layers) and against the movable
 *      objects' oriented boxes;
 *   4. a collision is resolved by disallowing all robot movement for the step;
 *   5. the episode counter advances (500-step horizon, Section 4.1);
 *   6. a depth image of the head camera (128x128, 90 degree FoV, Section 4.1)
 *      is rasterised: fixed-point vertices, integer edge functions with a
 *      top-left fill rule, depth interpolated with the barycentric weights
 *      the edge functions give, 24-bit depth, z-min.
 * The paper leaves every numeric detail open; the readings taken here are the
 * ones listed in the design notes (FP32 with a fixed evaluation order, own
 * sincos, Sutherland-Hodgman clipping with canonical endpoint order, ...).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math (no FMA, no
 * reassociation, SSE arithmetic so every float op rounds once to nearest-even).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* sine / cosine: Cody-Waite reduction by pi/2 (two-term split of pi/2) and   */
/* Taylor polynomials on [-pi/4, pi/4] (Cody & Waite 1980).  Used instead of   */
/* any library sinf/cosf so the result is a fixed sequence of float ops.      */
/* ------------------------------------------------------------------------ */
static const float K_TWO_OVER_PI = 0x1.45f306p-1f;   /* 2/pi */
static const float K_PIO2_HI = 0x1.92p+0f;            /* 1.5703125, 8 significant bits */
static const float K_PIO2_LO = 0x1.fb5444p-12f;       /* pi/2 - 1.5703125 */
static const float K_S3 = -0x1.555556p-3f;            /* -1/3! */
static const float K_S5 = 0x1.111112p-7f;             /*  1/5! */
static const float K_S7 = -0x1.a01a02p-13f;           /* -1/7! */
static const float K_S9 = 0x1.71de3ap-19f;            /*  1/9! */
static const float K_C2 = -0.5f;                      /* -1/2! */
static const float K_C4 = 0x1.555556p-5f;             /*  1/4! */
static const float K_C6 = -0x1.6c16c2p-10f;           /* -1/6! */
static const float K_C8 = 0x1.a01a02p-16f;            /*  1/8! */
static const float K_PI = 0x1.921fb6p+1f;
static const float K_TWO_PI = 0x1.921fb6p+2f;

O_EXPORT void o_sincos(float x, float *s, float *c)
{
    float k = rintf(x * K_TWO_OVER_PI);
    float r = (x - k * K_PIO2_HI) - k * K_PIO2_LO;
    float r2 = r * r;
    float ps = ((K_S9 * r2 + K_S7) * r2 + K_S5) * r2 + K_S3;
    float pc = ((K_C8 * r2 + K_C6) * r2 + K_C4) * r2 + K_C2;
    float sr = r + (r * r2) * ps;
    float cr = 1.0f + r2 * pc;
    int q = ((int)k) & 3;
    switch (q) {
    case 0: *s = sr; *c = cr; break;
    case 1: *s = cr; *c = -sr; break;
    case 2: *s = -sr; *c = -cr; break;
    default: *s = -cr; *c = sr; break;
    }
}

O_EXPORT void o_sincos_n(const float *x, float *s, float *c, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) o_sincos(x[i], &s[i], &c[i]);
}

/* ------------------------------------------------------------------------ */
/* 3x4 rigid frames, row-major: [r00 r01 r02 t0 | r10 r11 r12 t1 | ...]       */
/* Products are evaluated as ((a0*b0 + a1*b1) + a2*b2) [+ t].                  */
/* ------------------------------------------------------------------------ */
static void frame_mul(const float *A, const float *B, float *C)
{
    float T[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            T[i * 4 + j] = (A[i * 4 + 0] * B[0 * 4 + j] + A[i * 4 + 1] * B[1 * 4 + j])
                           + A[i * 4 + 2] * B[2 * 4 + j];
        T[i * 4 + 3] = ((A[i * 4 + 0] * B[3] + A[i * 4 + 1] * B[7]) + A[i * 4 + 2] * B[11])
                       + A[i * 4 + 3];
    }
    memcpy(C, T, sizeof(T));
}

static void frame_point(const float *F, const float *p, float *out)
{
    for (int i = 0; i < 3; ++i)
        out[i] = ((F[i * 4 + 0] * p[0] + F[i * 4 + 1] * p[1]) + F[i * 4 + 2] * p[2]) + F[i * 4 + 3];
}

static void frame_vector(const float *F, const float *v, float *out)
{
    for (int i = 0; i < 3; ++i)
        out[i] = (F[i * 4 + 0] * v[0] + F[i * 4 + 1] * v[1]) + F[i * 4 + 2] * v[2];
}

/* ------------------------------------------------------------------------ */
/* robot description and step records (mirrors the library's input arrays)   */
/* ------------------------------------------------------------------------ */
typedef struct {
    float dh[7][4];          /* a, d, cos(alpha), sin(alpha)   (standard DH)  */
    float qlim[7][2];
    float q_home[7];
    float mount[3];
    float cam_offset[3];
    float cam_pitch_cs[2];
    int32_t num_spheres;
    const int32_t *sphere_link;
    const float *sphere_pos;
    const int32_t *sphere_class;
    const uint8_t *sphere_held_only;
} o_robot;

typedef struct {
    int32_t num_classes;
    float class_radius[8];
    float act_lim[3];
    int32_t episode_len;
    float near_m, far_m;
    float cell_m;
} o_params;

/* one environment's collision scene: grids per class (CSR) + objects */
typedef struct {
    float grid_x0, grid_y0, grid_cell;
    int32_t nx, ny;
    const uint32_t *grid_offsets[8];   /* [nx*ny + 1] per class            */
    const float *grid_layers[8];       /* [L][2] per class                 */
    int32_t num_objects;
    const float *objects;              /* [O][8]                           */
    int32_t num_starts;
    const float *starts;               /* [P][3]                           */
    int32_t held;
} o_env;

/* ------------------------------------------------------------------------ */
/* forward kinematics (Section 3.2: offsets applied to the state, then FK)   */
/* ------------------------------------------------------------------------ */
/* frames[8][12]: link 0 = base, links 1..7 = DH joint frames */
O_EXPORT void o_fk(const o_robot *rb, const float *state, float *frames)
{
    float s, c;
    o_sincos(state[2], &s, &c);
    float *F0 = frames;
    F0[0] = c;   F0[1] = -s;  F0[2] = 0.0f;  F0[3] = state[0];
    F0[4] = s;   F0[5] = c;   F0[6] = 0.0f;  F0[7] = state[1];
    F0[8] = 0.0f; F0[9] = 0.0f; F0[10] = 1.0f; F0[11] = 0.0f;
    float T[12] = {1.0f, 0.0f, 0.0f, rb->mount[0],
                   0.0f, 1.0f, 0.0f, rb->mount[1],
                   0.0f, 0.0f, 1.0f, rb->mount[2]};
    float M[12];
    frame_mul(F0, T, M);
    const float *prev = M;
    for (int j = 0; j < 7; ++j) {
        float st, ct;
        o_sincos(state[3 + j], &st, &ct);
        float a = rb->dh[j][0], d = rb->dh[j][1], ca = rb->dh[j][2], sa = rb->dh[j][3];
        /* A_j = Rz(q) Tz(d) Tx(a) Rx(alpha) */
        float A[12] = {ct, -(st * ca), st * sa, a * ct,
                       st, ct * ca, -(ct * sa), a * st,
                       0.0f, sa, ca, d};
        frame_mul(prev, A, frames + 12 * (j + 1));
        prev = frames + 12 * (j + 1);
    }
}

/* camera record: position, right, down, forward (world) */
O_EXPORT void o_camera(const o_robot *rb, const float *state, float *cam)
{
    float frames[8 * 12];
    o_fk(rb, state, frames);
    float cp = rb->cam_pitch_cs[0], sp = rb->cam_pitch_cs[1];
    float right_b[3] = {0.0f, -1.0f, 0.0f};
    float down_b[3] = {-sp, 0.0f, -cp};
    float fwd_b[3] = {cp, 0.0f, -sp};
    frame_point(frames, rb->cam_offset, cam + 0);
    frame_vector(frames, right_b, cam + 3);
    frame_vector(frames, down_b, cam + 6);
    frame_vector(frames, fwd_b, cam + 9);
}

/* ------------------------------------------------------------------------ */
/* column grid (Appendix G): per radius class, per column, the list of free   */
/* vertical layers [lo, hi] of the sphere *centre*.                            */
/* Blocked: floor half-space z <= 0 -> centre in (-inf, r); each static box   */
/* whose closed XY footprint is within r (horizontally) of the column centre   */
/* -> centre in (z0 - h, z1 + h), h = sqrt(r^2 - d^2).  Free layers are the    */
/* maximal closed intervals of the complement with lo < hi.                    */
/* ------------------------------------------------------------------------ */
typedef struct { float a, b; } o_iv;

static int column_layers(const float *boxes, int nb, float cx, float cy, float r,
                         o_iv *scratch, int cap, float *out, int64_t out_cap)
{
    int n = 0;
    float r2 = r * r;
    for (int k = 0; k < nb; ++k) {
        const float *B = boxes + 6 * k;
        float dx = 0.0f, dy = 0.0f;
        if (cx < B[0]) dx = B[0] - cx; else if (cx > B[3]) dx = cx - B[3];
        if (cy < B[1]) dy = B[1] - cy; else if (cy > B[4]) dy = cy - B[4];
        float d2 = dx * dx + dy * dy;
        if (d2 < r2) {
            if (n >= cap) return -1;
            float h = sqrtf(r2 - d2);
            scratch[n].a = B[2] - h;
            scratch[n].b = B[5] + h;
            ++n;
        }
    }
    /* insertion sort by start */
    for (int i = 1; i < n; ++i) {
        o_iv t = scratch[i];
        int j = i - 1;
        while (j >= 0 && scratch[j].a > t.a) { scratch[j + 1] = scratch[j]; --j; }
        scratch[j + 1] = t;
    }
    int L = 0;
    float lo = r;                       /* floor blocks (-inf, r) */
    for (int i = 0; i < n; ++i) {
        if (scratch[i].a >= lo) {
            if (lo < scratch[i].a) {
                if (out) { if (L >= out_cap) return -2; out[2 * L] = lo; out[2 * L + 1] = scratch[i].a; }
                ++L;
            }
        }
        if (scratch[i].b > lo) lo = scratch[i].b;
    }
    if (out) { if (L >= out_cap) return -2; out[2 * L] = lo; out[2 * L + 1] = INFINITY; }
    ++L;
    return L;
}

/* Build one class grid.  offsets[nx*ny+1]; layers may be NULL to count only.
   Column index c = j*nx + i (x fastest).  Returns the total layer count, or
   a negative value when a column has more than `iv_cap` blocking boxes. */
O_EXPORT int64_t o_grid_build(const float *boxes, int nb, float x0, float y0, int nx, int ny,
                              float cell, float r, uint32_t *offsets, float *layers,
                              int64_t layer_cap)
{
    enum { IV_CAP = 256 };
    o_iv iv[IV_CAP];
    int64_t total = 0;
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            float cx = x0 + ((float)i + 0.5f) * cell;
            float cy = y0 + ((float)j + 0.5f) * cell;
            int64_t c = (int64_t)j * nx + i;
            if (offsets) offsets[c] = (uint32_t)total;
            float *dst = layers ? layers + 2 * total : NULL;
            int L = column_layers(boxes, nb, cx, cy, r, iv, IV_CAP, dst, layer_cap - total);
            if (L < 0) return L;
            total += L;
        }
    }
    if (offsets) offsets[(int64_t)nx * ny] = (uint32_t)total;
    return total;
}

/* sphere vs grid: 1 = contact (out of the grid or in no free layer) */
static int grid_contact(const o_env *env, int cls, const float *p)
{
    float inv_h = 1.0f / env->grid_cell;
    float fx = (p[0] - env->grid_x0) * inv_h;
    float fy = (p[1] - env->grid_y0) * inv_h;
    if (!(fx >= 0.0f && fx < (float)env->nx)) return 1;
    if (!(fy >= 0.0f && fy < (float)env->ny)) return 1;
    int i = (int)floorf(fx), j = (int)floorf(fy);
    int64_t c = (int64_t)j * env->nx + i;
    const uint32_t *off = env->grid_offsets[cls];
    const float *lay = env->grid_layers[cls];
    for (uint32_t l = off[c]; l < off[c + 1]; ++l)
        if (lay[2 * l] <= p[2] && p[2] <= lay[2 * l + 1]) return 0;
    return 1;
}

O_EXPORT int o_grid_query(const o_env *env, int cls, float x, float y, float z)
{
    float p[3] = {x, y, z};
    return grid_contact(env, cls, p);
}

/* sphere vs oriented box (yaw only): closest point in the box frame */
static int obb_contact(const float *o, const float *p, float r)
{
    float dx = p[0] - o[0], dy = p[1] - o[1], dz = p[2] - o[2];
    float cps = o[6], sps = o[7];
    float l[3];
    l[0] = cps * dx + sps * dy;
    l[1] = cps * dy - sps * dx;
    l[2] = dz;
    float d[3];
    for (int k = 0; k < 3; ++k) {
        float e = o[3 + k];
        float q = l[k] < -e ? -e : (l[k] > e ? e : l[k]);
        d[k] = l[k] - q;
    }
    float d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return d2 < r * r;
}

O_EXPORT int o_obb_query(const float *obj, float x, float y, float z, float r)
{
    float p[3] = {x, y, z};
    return obb_contact(obj, p, r);
}

/* ------------------------------------------------------------------------ */
/* one kinematic step of one environment                                      */
/* ------------------------------------------------------------------------ */
static float clampf(float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); }

static float sanitize(float a, float lim)
{
    if (a != a) a = 0.0f;
    return clampf(a, -lim, lim);
}

/* state[10] (x, y, yaw, q0..q6) and counters[2] (t, episode) are updated in
   place.  Outputs: contact masks (words of 32 spheres), accepted, done,
   frames[8][12] and cam[12] of the final state. */
O_EXPORT void o_robot_step(const o_robot *rb, const o_params *pr, const o_env *env,
                           float *state, int32_t *counters, const float *action,
                           uint32_t *mask_static, uint32_t *mask_object,
                           uint8_t *accepted, uint8_t *done, float *frames, float *cam)
{
    float a0 = sanitize(action[0], pr->act_lim[0]);
    float a1 = sanitize(action[1], pr->act_lim[1]);
    float cand[10];
    float yaw = state[2] + a1;
    if (yaw > K_PI) yaw = yaw - K_TWO_PI;
    else if (yaw < -K_PI) yaw = yaw + K_TWO_PI;
    float sy, cy;
    o_sincos(yaw, &sy, &cy);
    cand[0] = state[0] + a0 * cy;
    cand[1] = state[1] + a0 * sy;
    cand[2] = yaw;
    for (int j = 0; j < 7; ++j) {
        float aj = sanitize(action[2 + j], pr->act_lim[2]);
        cand[3 + j] = clampf(state[3 + j] + aj, rb->qlim[j][0], rb->qlim[j][1]);
    }

    float fr[8 * 12];
    o_fk(rb, cand, fr);
    int S = rb->num_spheres;
    int words = (S + 31) / 32;
    for (int w = 0; w < words; ++w) { mask_static[w] = 0; mask_object[w] = 0; }
    int any = 0;
    for (int s = 0; s < S; ++s) {
        if (rb->sphere_held_only && rb->sphere_held_only[s] && !env->held) continue;
        float c[3];
        frame_point(fr + 12 * rb->sphere_link[s], rb->sphere_pos + 3 * s, c);
        int cls = rb->sphere_class[s];
        float r = pr->class_radius[cls];
        if (grid_contact(env, cls, c)) { mask_static[s >> 5] |= 1u << (s & 31); any = 1; }
        for (int o = 0; o < env->num_objects; ++o) {
            if (obb_contact(env->objects + 8 * o, c, r)) {
                mask_object[s >> 5] |= 1u << (s & 31);
                any = 1;
                break;
            }
        }
    }
    *accepted = any ? 0 : 1;
    if (!any) memcpy(state, cand, sizeof(cand));

    /* episode bookkeeping: 500-step horizon (Section 4.1), auto-reset */
    *done = 0;
    counters[0] += 1;
    if (pr->episode_len > 0 && counters[0] >= pr->episode_len) {
        counters[1] += 1;
        int p = counters[1] % env->num_starts;
        state[0] = env->starts[3 * p + 0];
        state[1] = env->starts[3 * p + 1];
        state[2] = env->starts[3 * p + 2];
        for (int j = 0; j < 7; ++j) state[3 + j] = rb->q_home[j];
        counters[0] = 0;
        *done = 1;
    }
    o_fk(rb, state, frames);
    o_camera(rb, state, cam);
}

/* ------------------------------------------------------------------------ */
/* manipulation (Section 3.2: suction grasp with a small sphere at the end-   */
/* effector tip, the grasped object fixed to the end effector, snap-to-       */
/* surface on release; Appendix I: sliding and object-placing heuristics)     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t slide;             /* resolve a collision by sliding the base       */
    float grasp_tip[3];        /* end-effector-frame point of the grasp sphere  */
    float grasp_radius;
    int32_t held_class;        /* radius class of the held object's spheres     */
    float slide_step;          /* base jitter per sliding try (m)               */
    float place_step;          /* object jitter per placing try (m)             */
    uint64_t seed;             /* counter-based jitter randomness               */
} o_manip;

/* dynamic state of one environment's movable objects */
typedef struct {
    float *objects;            /* [O][8] resting records; the held object keeps
                                  its record from before the grasp              */
    const float *objects0;     /* [O][8] records at episode start               */
    int32_t *held;             /* held object index, -1 = none                   */
    float *rel;                /* [12] held object's frame in the EE frame       */
} o_dyn;

enum { O_SLIDE_TRIES = 3, O_PLACE_TRIES = 6, O_HELD_SPHERES = 8 };

/* frame of a resting object: Rz(yaw) about its centre */
static void object_frame(const float *o, float *F)
{
    float c = o[6], s = o[7];
    F[0] = c;    F[1] = -s;   F[2] = 0.0f;  F[3] = o[0];
    F[4] = s;    F[5] = c;    F[6] = 0.0f;  F[7] = o[1];
    F[8] = 0.0f; F[9] = 0.0f; F[10] = 1.0f; F[11] = o[2];
}

/* inverse of a rigid frame: R^T | -R^T t */
static void frame_inverse(const float *F, float *G)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i * 4 + j] = F[j * 4 + i];
    for (int i = 0; i < 3; ++i)
        G[i * 4 + 3] = -((F[0 * 4 + i] * F[3] + F[1 * 4 + i] * F[7]) + F[2 * 4 + i] * F[11]);
}

/* octant k of a box of half extents e: (+-e0/2, +-e1/2, +-e2/2), bit 0 = x */
static void octant(const float *e, int k, float *p)
{
    p[0] = (k & 1) ? 0.5f * e[0] : -(0.5f * e[0]);
    p[1] = (k & 2) ? 0.5f * e[1] : -(0.5f * e[1]);
    p[2] = (k & 4) ? 0.5f * e[2] : -(0.5f * e[2]);
}

/* squared distance from p to an oriented box (the test of obb_contact) */
static float obb_dist2(const float *o, const float *p)
{
    float dx = p[0] - o[0], dy = p[1] - o[1], dz = p[2] - o[2];
    float cps = o[6], sps = o[7];
    float l[3];
    l[0] = cps * dx + sps * dy;
    l[1] = cps * dy - sps * dx;
    l[2] = dz;
    float d[3];
    for (int k = 0; k < 3; ++k) {
        float e = o[3 + k];
        float q = l[k] < -e ? -e : (l[k] > e ? e : l[k]);
        d[k] = l[k] - q;
    }
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* SplitMix64 (Steele, Lea & Flood 2014) of a counter; uniform in [0, 1) with
   24 bits */
static float o_hash01(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, uint64_t d)
{
    uint64_t x = seed + 0x9E3779B97F4A7C15ull * (((a << 40) ^ (b << 24) ^ (c << 8) ^ d) + 1ull);
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x = x ^ (x >> 31);
    return (float)(x >> 40) * 0x1p-24f;
}

/* Overlap test of a candidate pose (robot spheres, and with a held object its
   8 spheres at the octant centres of its box) against the column grids and
   the resting objects.  Masks: bit s = robot sphere s, bits S..S+7 = the held
   object's spheres.  With sum != NULL, the x, y of every overlapping sphere's
   centre is summed in sphere order (robot spheres, then held) and counted. */
static int pose_contacts(const o_robot *rb, const o_params *pr, const o_env *env,
                         const o_manip *mp, const o_dyn *dy, const float *cand,
                         uint32_t *mask_static, uint32_t *mask_object, float *sum, int *count)
{
    float fr[8 * 12];
    o_fk(rb, cand, fr);
    int S = rb->num_spheres;
    int words = (S + O_HELD_SPHERES + 31) / 32;
    for (int w = 0; w < words; ++w) { mask_static[w] = 0; mask_object[w] = 0; }
    int any = 0;
    float sx = 0.0f, sy = 0.0f;
    int n = 0;
    int held = *dy->held;
    for (int s = 0; s < S + O_HELD_SPHERES; ++s) {
        float c[3];
        int cls;
        if (s < S) {
            if (rb->sphere_held_only && rb->sphere_held_only[s]) continue;   /* replaced by the object */
            frame_point(fr + 12 * rb->sphere_link[s], rb->sphere_pos + 3 * s, c);
            cls = rb->sphere_class[s];
        } else {
            if (held < 0) continue;
            float F[12], p[3];
            frame_mul(fr + 12 * 7, dy->rel, F);
            octant(dy->objects + 8 * held + 3, s - S, p);
            frame_point(F, p, c);
            cls = mp->held_class;
        }
        float r = pr->class_radius[cls];
        int hit = 0;
        if (grid_contact(env, cls, c)) { mask_static[s >> 5] |= 1u << (s & 31); hit = 1; }
        for (int o = 0; o < env->num_objects; ++o) {
            if (o == held) continue;
            if (obb_contact(dy->objects + 8 * o, c, r)) {
                mask_object[s >> 5] |= 1u << (s & 31);
                hit = 1;
                break;
            }
        }
        if (hit) {
            any = 1;
            sx = sx + c[0];
            sy = sy + c[1];
            ++n;
        }
    }
    if (sum) { sum[0] = sx; sum[1] = sy; *count = n; }
    return any;
}

/* Snap-to-surface of object h released at frame F (Section 3.2), then the
   placing heuristic (Appendix I): the object lands upright with the yaw of
   its x axis; four spheres of the held class touching its bottom face from
   inside (octant x, y; z = -e2 + r) are cast straight down through the
   column grid: each drops to the bottom of the free layer holding its centre,
   the object by the smallest of those drops.  The cast fails when a sphere
   centre is outside the grid or in no free layer; the landed object fails
   when one of its 8 octant spheres overlaps another resting object.  On a
   failure the drop point moves by place_step along a jitter direction -- away
   from the overlapped object, turned by a random angle in [-pi/4, pi/4), or
   a random direction when the grid refused the cast -- and the cast is
   repeated, up to O_PLACE_TRIES jitters.  If every try fails the object goes
   back to its resting record from before the grasp. */
static void place_object(const o_params *pr, const o_env *env, const o_manip *mp, const o_dyn *dy,
                         int h, const float *F, uint64_t env_id, int32_t episode, int32_t t)
{
    float *ob = dy->objects + 8 * h;
    const float *e = ob + 3;
    float cx = F[0], sx = F[4];
    float n2 = cx * cx + sx * sx;
    float c = 1.0f, s = 0.0f;
    if (n2 > 1e-12f) {
        float len = sqrtf(n2);
        c = cx / len;
        s = sx / len;
    }
    float px = F[3], py = F[7], z0 = F[11];
    float r = pr->class_radius[mp->held_class];
    int cls = mp->held_class;
    for (int k = 0; k <= O_PLACE_TRIES; ++k) {
        int fail_static = 0, fail_obj = -1;
        float drop = INFINITY;
        for (int q = 0; q < 4; ++q) {
            float p[3];
            octant(e, q, p);
            float w[3];
            w[0] = px + (c * p[0] - s * p[1]);
            w[1] = py + (s * p[0] + c * p[1]);
            w[2] = z0 + (r - e[2]);
            float inv_h = 1.0f / env->grid_cell;
            float fx = (w[0] - env->grid_x0) * inv_h;
            float fy = (w[1] - env->grid_y0) * inv_h;
            if (!(fx >= 0.0f && fx < (float)env->nx && fy >= 0.0f && fy < (float)env->ny)) {
                fail_static = 1;
                break;
            }
            int i = (int)floorf(fx), j = (int)floorf(fy);
            int64_t col = (int64_t)j * env->nx + i;
            const uint32_t *off = env->grid_offsets[cls];
            const float *lay = env->grid_layers[cls];
            int found = 0;
            for (uint32_t l = off[col]; l < off[col + 1]; ++l)
                if (lay[2 * l] <= w[2] && w[2] <= lay[2 * l + 1]) {
                    float d = w[2] - lay[2 * l];
                    if (d < drop) drop = d;
                    found = 1;
                    break;
                }
            if (!found) { fail_static = 1; break; }
        }
        float rec[8] = {px, py, 0.0f, e[0], e[1], e[2], c, s};
        if (!fail_static) {
            rec[2] = z0 - drop;
            float Fo[12];
            object_frame(rec, Fo);
            for (int q = 0; q < O_HELD_SPHERES && fail_obj < 0; ++q) {
                float p[3], w[3];
                octant(e, q, p);
                frame_point(Fo, p, w);
                for (int o = 0; o < env->num_objects; ++o) {
                    if (o == h) continue;
                    if (obb_contact(dy->objects + 8 * o, w, r)) { fail_obj = o; break; }
                }
            }
            if (fail_obj < 0) {
                memcpy(ob, rec, sizeof(rec));
                return;
            }
        }
        if (k == O_PLACE_TRIES) break;
        float u = o_hash01(mp->seed, env_id, (uint64_t)(uint32_t)episode, (uint64_t)(uint32_t)t,
                           (uint64_t)(16 + k));
        float dx, dy2;
        if (fail_obj >= 0) {
            const float *oo = dy->objects + 8 * fail_obj;
            float vx = px - oo[0], vy = py - oo[1];
            float vn = sqrtf(vx * vx + vy * vy);
            float bx = 1.0f, by = 0.0f;
            if (vn > 1e-6f) { bx = vx / vn; by = vy / vn; }
            float sphi, cphi;
            o_sincos((u - 0.5f) * 0x1.921fb6p+0f, &sphi, &cphi);   /* [-pi/4, pi/4) */
            dx = cphi * bx - sphi * by;
            dy2 = sphi * bx + cphi * by;
        } else {
            float sphi, cphi;
            o_sincos(u * K_TWO_PI - K_PI, &sphi, &cphi);
            dx = cphi;
            dy2 = sphi;
        }
        px = px + mp->place_step * dx;
        py = py + mp->place_step * dy2;
    }
    /* every try failed: the object keeps its record from before the grasp */
}

/* One step with manipulation.  action: 11 floats, the 9 of o_robot_step, then
   grasp/release (>= 0.5: grasp when nothing is held; otherwise a held object
   is released; NaN counts as 0) and stop (>= 0.5 ends the episode).
   accepted: 0 = no movement, 1 = the candidate, 2 = a slid candidate.
   obj_frames [O][12]: every object's frame after the step (held: carried by
   the end effector). */
O_EXPORT void o_robot_step_manip(const o_robot *rb, const o_params *pr, const o_env *env,
                                 const o_manip *mp, const o_dyn *dy, int32_t env_id,
                                 float *state, int32_t *counters, const float *action,
                                 uint32_t *mask_static, uint32_t *mask_object,
                                 uint8_t *accepted, uint8_t *done, float *frames, float *cam,
                                 float *obj_frames)
{
    float a0 = sanitize(action[0], pr->act_lim[0]);
    float a1 = sanitize(action[1], pr->act_lim[1]);
    float ag = action[9], as = action[10];
    int grasp = ag == ag && ag >= 0.5f;
    int stop = as == as && as >= 0.5f;
    float cand[10];
    float yaw = state[2] + a1;
    if (yaw > K_PI) yaw = yaw - K_TWO_PI;
    else if (yaw < -K_PI) yaw = yaw + K_TWO_PI;
    float sy, cy;
    o_sincos(yaw, &sy, &cy);
    cand[0] = state[0] + a0 * cy;
    cand[1] = state[1] + a0 * sy;
    cand[2] = yaw;
    for (int j = 0; j < 7; ++j) {
        float aj = sanitize(action[2 + j], pr->act_lim[2]);
        cand[3 + j] = clampf(state[3 + j] + aj, rb->qlim[j][0], rb->qlim[j][1]);
    }

    float sum[2];
    int cnt = 0;
    int any = pose_contacts(rb, pr, env, mp, dy, cand, mask_static, mask_object, sum, &cnt);
    if (!any) {
        memcpy(state, cand, sizeof(cand));
        *accepted = 1;
    } else {
        *accepted = 0;
        if (mp->slide) {
            /* sliding (Appendix I): push the base away from the mean of the
               overlapping spheres' centres, up to O_SLIDE_TRIES jitters */
            int words = (rb->num_spheres + O_HELD_SPHERES + 31) / 32;
            uint32_t ms[16], mo[16];
            for (int k = 0; k < O_SLIDE_TRIES && words <= 16; ++k) {
                float mx = sum[0] / (float)cnt, my = sum[1] / (float)cnt;
                float vx = cand[0] - mx, vy = cand[1] - my;
                float vn = sqrtf(vx * vx + vy * vy);
                if (!(vn > 1e-6f)) break;
                cand[0] = cand[0] + mp->slide_step * (vx / vn);
                cand[1] = cand[1] + mp->slide_step * (vy / vn);
                if (!pose_contacts(rb, pr, env, mp, dy, cand, ms, mo, sum, &cnt)) {
                    memcpy(state, cand, sizeof(cand));
                    *accepted = 2;
                    break;
                }
            }
        }
    }

    /* grasp / release at the resolved pose */
    {
        float fr[8 * 12];
        o_fk(rb, state, fr);
        const float *Fee = fr + 12 * 7;
        int held = *dy->held;
        if (grasp && held < 0) {
            float tip[3];
            frame_point(Fee, mp->grasp_tip, tip);
            float r2 = mp->grasp_radius * mp->grasp_radius;
            int best = -1;
            float bd = 0.0f;
            for (int o = 0; o < env->num_objects; ++o) {
                float d2 = obb_dist2(dy->objects + 8 * o, tip);
                if (d2 < r2 && (best < 0 || d2 < bd)) { best = o; bd = d2; }
            }
            if (best >= 0) {
                float Fo[12], G[12];
                object_frame(dy->objects + 8 * best, Fo);
                frame_inverse(Fee, G);
                frame_mul(G, Fo, dy->rel);
                *dy->held = best;
            }
        } else if (!grasp && held >= 0) {
            float F[12];
            frame_mul(Fee, dy->rel, F);
            place_object(pr, env, mp, dy, held, F, (uint64_t)(uint32_t)env_id, counters[1], counters[0]);
            *dy->held = -1;
        }
    }

    /* episode bookkeeping: horizon or stop action, auto-reset */
    *done = 0;
    counters[0] += 1;
    if (stop || (pr->episode_len > 0 && counters[0] >= pr->episode_len)) {
        counters[1] += 1;
        int p = counters[1] % env->num_starts;
        state[0] = env->starts[3 * p + 0];
        state[1] = env->starts[3 * p + 1];
        state[2] = env->starts[3 * p + 2];
        for (int j = 0; j < 7; ++j) state[3 + j] = rb->q_home[j];
        counters[0] = 0;
        memcpy(dy->objects, dy->objects0, sizeof(float) * 8 * (size_t)env->num_objects);
        *dy->held = -1;
        *done = 1;
    }
    o_fk(rb, state, frames);
    o_camera(rb, state, cam);
    for (int o = 0; o < env->num_objects; ++o) {
        if (o == *dy->held) frame_mul(frames + 12 * 7, dy->rel, obj_frames + 12 * o);
        else object_frame(dy->objects + 8 * o, obj_frames + 12 * o);
    }
}

/* The movable objects as render triangles: box corner k of object o =
   F_o (+-e0, +-e1, +-e2) (bit 0 of k: x, bit 1: y, bit 2: z) at vertex 8 o + k;
   12 triangles per object, wound counter-clockwise around the outward
   normals, vertex indices offset by vbase.  verts [8 O][3], tris [12 O][3]. */
O_EXPORT void o_object_mesh(const float *obj_frames, const float *objects, int O, int32_t vbase,
                            float *verts, int32_t *tris)
{
    static const int faces[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                    {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
    for (int o = 0; o < O; ++o) {
        const float *e = objects + 8 * o + 3;
        for (int k = 0; k < 8; ++k) {
            float p[3] = {(k & 1) ? e[0] : -e[0], (k & 2) ? e[1] : -e[1], (k & 4) ? e[2] : -e[2]};
            frame_point(obj_frames + 12 * o, p, verts + 3 * (8 * o + k));
        }
        for (int f = 0; f < 6; ++f) {
            const int *q = faces[f];
            int32_t *t0 = tris + 3 * (12 * o + 2 * f), *t1 = t0 + 3;
            t0[0] = vbase + 8 * o + q[0]; t0[1] = vbase + 8 * o + q[1]; t0[2] = vbase + 8 * o + q[2];
            t1[0] = vbase + 8 * o + q[0]; t1[1] = vbase + 8 * o + q[2]; t1[2] = vbase + 8 * o + q[3];
        }
    }
}

/* The robot's links as render triangles (the head camera sees the robot's own
   body and arm): link l (frame l of the step's kinematics, 0 = base) is the box
   centred at c_l with half extents h_l in its own frame (link_box [8][6] =
   c xyz, h xyz).  Corner k of link l = F_l (c_l + (+-h_l)) (bit 0 of k: x,
   bit 1: y, bit 2: z; the sum in FP32 before the frame product) at vertex
   8 l + k; 12 triangles per link in the object boxes' face order, vertex
   indices offset by vbase.  verts [64][3], tris [96][3]. */
O_EXPORT void o_link_mesh(const float *frames, const float *link_box, int32_t vbase, float *verts,
                          int32_t *tris)
{
    static const int faces[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                    {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
    for (int l = 0; l < 8; ++l) {
        const float *c = link_box + 6 * l, *h = c + 3;
        for (int k = 0; k < 8; ++k) {
            float p[3];
            p[0] = c[0] + ((k & 1) ? h[0] : -h[0]);
            p[1] = c[1] + ((k & 2) ? h[1] : -h[1]);
            p[2] = c[2] + ((k & 4) ? h[2] : -h[2]);
            frame_point(frames + 12 * l, p, verts + 3 * (8 * l + k));
        }
        for (int f = 0; f < 6; ++f) {
            const int *q = faces[f];
            int32_t *t0 = tris + 3 * (12 * l + 2 * f), *t1 = t0 + 3;
            t0[0] = vbase + 8 * l + q[0]; t0[1] = vbase + 8 * l + q[1]; t0[2] = vbase + 8 * l + q[2];
            t1[0] = vbase + 8 * l + q[0]; t1[1] = vbase + 8 * l + q[2]; t1[2] = vbase + 8 * l + q[3];
        }
    }
}

/* reset one environment to the start pose of its (incremented) episode */
O_EXPORT void o_reset_env(const o_robot *rb, const o_env *env, float *state, int32_t *counters,
                          int new_episode)
{
    if (new_episode) counters[1] += 1;
    int p = counters[1] % env->num_starts;
    state[0] = env->starts[3 * p + 0];
    state[1] = env->starts[3 * p + 1];
    state[2] = env->starts[3 * p + 2];
    for (int j = 0; j < 7; ++j) state[3 + j] = rb->q_home[j];
    counters[0] = 0;
}

/* ------------------------------------------------------------------------ */
/* depth rasteriser                                                           */
/* ------------------------------------------------------------------------ */
typedef struct { float X, Y, Z; } o_cv;   /* camera-space vertex */

typedef struct {
    int64_t tris_in;       /* triangles that survive trivial rejection         */
    int64_t tris_front;    /* front-facing, non-degenerate (after clipping)    */
    int64_t cand_px;       /* bbox-in-viewport candidate pixels                */
    int64_t frags;         /* covered pixel samples                            */
    int64_t clipped;       /* triangles that needed clipping                   */
} o_rstats;

static float plane_value(const o_cv *v, int k, float near_m)
{
    switch (k) {
    case 0: return v->Z - near_m;
    case 1: return v->X + 2.0f * v->Z;
    case 2: return 2.0f * v->Z - v->X;
    case 3: return v->Y + 2.0f * v->Z;
    default: return 2.0f * v->Z - v->Y;
    }
}

static uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* canonical order of two endpoints: by the bit patterns of (X, Y, Z) */
static int vless(const o_cv *a, const o_cv *b)
{
    if (fbits(a->X) != fbits(b->X)) return fbits(a->X) < fbits(b->X);
    if (fbits(a->Y) != fbits(b->Y)) return fbits(a->Y) < fbits(b->Y);
    return fbits(a->Z) < fbits(b->Z);
}

static o_cv intersect(const o_cv *p, const o_cv *q, int k, float near_m)
{
    const o_cv *s = p, *e = q;
    if (vless(q, p)) { s = q; e = p; }
    float ps = plane_value(s, k, near_m), pe = plane_value(e, k, near_m);
    float t = ps / (ps - pe);
    o_cv v;
    v.X = s->X + t * (e->X - s->X);
    v.Y = s->Y + t * (e->Y - s->Y);
    v.Z = s->Z + t * (e->Z - s->Z);
    return v;
}

typedef struct {
    int W, H;
    float hw, hh;
    float near_m, invn, kd;
    uint32_t *depth;
    uint32_t *tri_win;      /* winning triangle per pixel (colour)   */
    uint8_t *cover;         /* per-pixel coverage count (debug)      */
    o_rstats *st;
} o_rctx;

static int32_t snap(float v)
{
    float s = v * 16.0f;
    s = clampf(s, -1048576.0f, 1048576.0f);
    return (int32_t)rintf(s);
}

static void raster_tri(o_rctx *cx, const o_cv *in, uint32_t id)
{
    int32_t x[3], y[3];
    float d[3];
    for (int k = 0; k < 3; ++k) {
        float xs = cx->hw + cx->hw * (in[k].X / in[k].Z);
        float ys = cx->hh + cx->hh * (in[k].Y / in[k].Z);
        x[k] = snap(xs);
        y[k] = snap(ys);
        float inv = 1.0f / in[k].Z;
        d[k] = (cx->invn - inv) * cx->kd;
    }
    int32_t A2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    if (A2 >= 0) return;                /* back face or degenerate: culled */
    /* front face: swap v1, v2 so the signed area is positive */
    { int32_t t = x[1]; x[1] = x[2]; x[2] = t; }
    { int32_t t = y[1]; y[1] = y[2]; y[2] = t; }
    { float t = d[1]; d[1] = d[2]; d[2] = t; }
    A2 = -A2;
    cx->st->tris_front += 1;

    int32_t minx = x[0], maxx = x[0], miny = y[0], maxy = y[0];
    for (int k = 1; k < 3; ++k) {
        if (x[k] < minx) minx = x[k];
        if (x[k] > maxx) maxx = x[k];
        if (y[k] < miny) miny = y[k];
        if (y[k] > maxy) maxy = y[k];
    }
    int px0 = (minx + 7) >> 4, px1 = (maxx - 8) >> 4;
    int py0 = (miny + 7) >> 4, py1 = (maxy - 8) >> 4;
    if (px0 < 0) px0 = 0;
    if (py0 < 0) py0 = 0;
    if (px1 > cx->W - 1) px1 = cx->W - 1;
    if (py1 > cx->H - 1) py1 = cx->H - 1;
    if (px0 > px1 || py0 > py1) return;

    /* edges k: from vertex i to vertex j, (i, j) = (1,2), (2,0), (0,1) */
    static const int EI[3] = {1, 2, 0}, EJ[3] = {2, 0, 1};
    int32_t bias[3];
    for (int k = 0; k < 3; ++k) {
        int32_t ex = x[EJ[k]] - x[EI[k]], ey = y[EJ[k]] - y[EI[k]];
        int top_left = (ey < 0) || (ey == 0 && ex > 0);
        bias[k] = top_left ? 0 : 1;
    }
    /* depth: convex combination of the vertex depths with the barycentric
       weights E_k / A2 given by the integer edge functions (edge k is opposite
       vertex k); the weights are non-negative on covered pixels, so the
       result stays within a few LSB of the vertices' depth range */
    float invA = 1.0f / (float)A2;
    float q[3] = {d[0] * invA, d[1] * invA, d[2] * invA};

    for (int py = py0; py <= py1; ++py) {
        for (int px = px0; px <= px1; ++px) {
            int32_t Px = 16 * px + 8, Py = 16 * py + 8;
            cx->st->cand_px += 1;
            int inside = 1;
            int32_t E[3];
            for (int k = 0; k < 3; ++k) {
                int i = EI[k], j = EJ[k];
                E[k] = (x[j] - x[i]) * (Py - y[i]) - (y[j] - y[i]) * (Px - x[i]);
                if (E[k] < bias[k]) inside = 0;
            }
            if (!inside) continue;
            cx->st->frags += 1;
            float dv = ((float)E[0] * q[0] + (float)E[1] * q[1]) + (float)E[2] * q[2];
            uint32_t D;
            if (!(dv > 0.0f)) D = 0;
            else if (dv >= 16777215.0f) D = 16777215u;
            else D = (uint32_t)dv;
            size_t p = (size_t)py * cx->W + px;
            if (cx->cover && cx->cover[p] < 255) cx->cover[p] += 1;
            if (D < cx->depth[p] || (D == cx->depth[p] && cx->tri_win && id < cx->tri_win[p])) {
                if (D < 16777215u) {
                    cx->depth[p] = D;
                    if (cx->tri_win) cx->tri_win[p] = id;
                }
            }
        }
    }
}

/* Render one environment.  depth[H*W] (cleared to 0xFFFFFF here); tri_win
   (optional) receives the winning triangle id (0xFFFFFFFF = none); cover
   (optional) counts covering fragments per pixel (saturating at 255).
   tri_plane (optional, [ntri][4]): the outward unit normal n and offset w of
   each triangle's face; a triangle whose face the camera position c is not
   strictly in front of ((n0 c0 + n1 c1) + n2 c2 - w <= 0) is culled as a back
   face, before the winding test of its snapped vertices. */
O_EXPORT void o_render(const float *verts, const int32_t *tris, int64_t ntri, const float *tri_plane,
                       const float *cam,
                       int W, int H, float near_m, float far_m, uint32_t *depth,
                       uint32_t *tri_win, uint8_t *cover, o_rstats *stats)
{
    o_rstats local;
    memset(&local, 0, sizeof(local));
    o_rctx cx;
    cx.W = W; cx.H = H;
    cx.hw = (float)W * 0.5f;
    cx.hh = (float)H * 0.5f;
    cx.near_m = near_m;
    cx.invn = 1.0f / near_m;
    float invf = 1.0f / far_m;
    cx.kd = 16777215.0f / (cx.invn - invf);
    cx.depth = depth;
    cx.tri_win = tri_win;
    cx.cover = cover;
    cx.st = &local;
    for (int64_t p = 0; p < (int64_t)W * H; ++p) {
        depth[p] = 16777215u;
        if (tri_win) tri_win[p] = 0xFFFFFFFFu;
        if (cover) cover[p] = 0;
    }
    const float *P = cam, *Rt = cam + 3, *Dn = cam + 6, *Fw = cam + 9;
    for (int64_t t = 0; t < ntri; ++t) {
        if (tri_plane) {
            const float *pl = tri_plane + 4 * t;
            const float side = ((pl[0] * P[0] + pl[1] * P[1]) + pl[2] * P[2]) - pl[3];
            if (!(side > 0.0f)) continue;
        }
        o_cv v[3];
        for (int k = 0; k < 3; ++k) {
            const float *w = verts + 3 * (int64_t)tris[3 * t + k];
            float dx = w[0] - P[0], dy = w[1] - P[1], dz = w[2] - P[2];
            v[k].X = (Rt[0] * dx + Rt[1] * dy) + Rt[2] * dz;
            v[k].Y = (Dn[0] * dx + Dn[1] * dy) + Dn[2] * dz;
            v[k].Z = (Fw[0] * dx + Fw[1] * dy) + Fw[2] * dz;
        }
        int reject = 0, all_in = 1;
        for (int k = 0; k < 5 && !reject; ++k) {
            int out = 0;
            for (int m = 0; m < 3; ++m) out += plane_value(&v[m], k, near_m) < 0.0f;
            if (out == 3) reject = 1;
            if (out) all_in = 0;
        }
        if (reject) continue;
        local.tris_in += 1;
        if (all_in) {
            raster_tri(&cx, v, (uint32_t)t);
            continue;
        }
        /* Sutherland-Hodgman: planes near, left, right, top, bottom */
        local.clipped += 1;
        /* a convex triangle clipped by 5 planes has at most 3 + 5 = 8 vertices;
           should rounding ever emit more, the extra vertices are dropped */
        o_cv poly[8], tmp[8];
        int n = 3;
        memcpy(poly, v, sizeof(v));
        for (int k = 0; k < 5 && n > 0; ++k) {
            int m = 0;
            for (int i = 0; i < n; ++i) {
                const o_cv *cur = &poly[i];
                const o_cv *prv = &poly[(i + n - 1) % n];
                int cin = plane_value(cur, k, near_m) >= 0.0f;
                int pin = plane_value(prv, k, near_m) >= 0.0f;
                if (cin) {
                    if (!pin && m < 8) tmp[m++] = intersect(prv, cur, k, near_m);
                    if (m < 8) tmp[m++] = *cur;
                } else if (pin) {
                    if (m < 8) tmp[m++] = intersect(prv, cur, k, near_m);
                }
            }
            n = m;
            memcpy(poly, tmp, sizeof(o_cv) * (size_t)n);
        }
        for (int i = 1; i + 1 < n; ++i) {
            o_cv tri[3] = {poly[0], poly[i], poly[i + 1]};
            raster_tri(&cx, tri, (uint32_t)t);
        }
    }
    if (stats) *stats = local;
}

/* ------------------------------------------------------------------------ */
/* lit, textured colour                                                       */
/* ------------------------------------------------------------------------ */
/* The RGB half of the RGBD observation (Section 4.1) with lighting and a
   texture: the paper's scenes carry baked textures and lighting, which are not
   available, so a procedural stand-in is computed per pixel from what the
   depth pass leaves (the winning triangle and its D24 depth):
     - the pixel's camera-space depth from its D24 value, 1/Z = 1/n - D / K
       (K the depth scale of the rasteriser), and its world position
       P = c + Z ((f + u r) + v d) along the pixel-centre ray, u = (x + 1/2 -
       W/2) / (W/2), v likewise in y;
     - Lambert lighting from one directional light L = (0.36, 0.48, 0.8) (a
       unit vector) with an ambient term: s = 0.35 + 0.65 max(0, n . L), n the
       winning triangle's outward unit normal;
     - a world-space checker texture of 0.25 m squares on the plane the face
       most nearly lies in (the two world axes other than n's largest
       component: z first, then x), dark squares at 0.8 of the colour:
       t = 0.8 when floor(4 a) + floor(4 b) is odd, else 1;
     - each channel min(255, floor(c s t + 1/2)) of the triangle's flat
       colour c; background (0, 0, 0).
   FP32 throughout in the order written.  depth and win as o_render leaves
   them (win = winning triangle id); tri_n [T][3] the outward unit normals;
   rgb [H][W][3] out. */
O_EXPORT void o_shade(const uint32_t *depth, const uint32_t *win, int W, int H, const float *cam,
                      float near_m, float far_m, const float *tri_n, const uint8_t *tri_rgb,
                      uint8_t *rgb)
{
    const float invn = 1.0f / near_m, invf = 1.0f / far_m;
    const float kd = 16777215.0f / (invn - invf);
    const float invk = 1.0f / kd;
    const float hw = (float)W * 0.5f, hh = (float)H * 0.5f;
    const float L0 = 0.36f, L1 = 0.48f, L2 = 0.8f;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int64_t p = (int64_t)y * W + x;
            uint8_t *out = rgb + 3 * p;
            const uint32_t D = depth[p];
            if (D >= 16777215u) {
                out[0] = out[1] = out[2] = 0;
                continue;
            }
            const uint32_t id = win[p];
            const float invz = invn - (float)D * invk;
            const float z = 1.0f / invz;
            const float u = (((float)x + 0.5f) - hw) / hw;
            const float v = (((float)y + 0.5f) - hh) / hh;
            float P[3];
            for (int i = 0; i < 3; ++i) P[i] = cam[i] + z * ((cam[9 + i] + u * cam[3 + i]) + v * cam[6 + i]);
            const float *n = tri_n + 3 * (int64_t)id;
            const float ndl = (n[0] * L0 + n[1] * L1) + n[2] * L2;
            const float s = 0.35f + 0.65f * (ndl > 0.0f ? ndl : 0.0f);
            const float a0 = fabsf(n[0]), a1 = fabsf(n[1]), a2 = fabsf(n[2]);
            float ta, tb;
            if (a2 >= a0 && a2 >= a1) { ta = P[0]; tb = P[1]; }
            else if (a0 >= a1) { ta = P[1]; tb = P[2]; }
            else { ta = P[0]; tb = P[2]; }
            const int ia = (int)floorf(ta * 4.0f), ib = (int)floorf(tb * 4.0f);
            const float t = ((ia + ib) & 1) ? 0.8f : 1.0f;
            const float f = s * t;
            for (int c = 0; c < 3; ++c) {
                const float val = floorf((float)tri_rgb[3 * (int64_t)id + c] * f + 0.5f);
                out[c] = (uint8_t)(val >= 255.0f ? 255.0f : val);
            }
        }
}

/* Outward unit normals of the 12 triangles of each of nbox boxes in the order
   of o_object_mesh / o_link_mesh (faces -x, +x, -y, +y, -z, +z, two triangles
   each): the box frame's axis column, negated for the minus faces.
   frames [nbox][12], tri_n [12 nbox][3]. */
O_EXPORT void o_box_normals(const float *frames, int nbox, float *tri_n)
{
    for (int b = 0; b < nbox; ++b)
        for (int j = 0; j < 12; ++j) {
            const int face = j >> 1, axis = face >> 1;
            const float *F = frames + 12 * b;
            float *n = tri_n + 3 * (12 * b + j);
            for (int i = 0; i < 3; ++i) n[i] = (face & 1) ? F[4 * i + axis] : -F[4 * i + axis];
        }
}
