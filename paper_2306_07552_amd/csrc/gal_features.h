// Inputs of the collision surrogate for one environment's next move, as
// device functions shared by the feature kernel (k_features) and the fused
// inference kernel (k_sur_infer), so both produce the same bits.
//
// Layout of one input row (2112 BF16 values):
//   [0..6]    candidate joint angles
//   [7..13]   joint offsets / their limit, [14..15] base offsets / their limits
//   [16..18]  base pose: x, y over the grid extent, yaw / pi
//   [19]      held-object flag
//   [20..40]  origins of joint frames 1..7, [41..43] end-effector z axis, of the
//             candidate arm pose with the base at the origin (the step's own
//             kinematics)
//   [44..63]  zero
//   [64..]    16 x 16 x 8 occupancy patch, column c = a * 16 + b at 64 + 8 c
#pragma once

#include "gal_fk.h"
#include "gal_math.h"
#include "gal_mlp.h"

namespace gal {

__device__ __forceinline__ float feat_clampf(float v, float lo, float hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ float feat_sanitize(float a, float lim)
{
    if (a != a) a = 0.0f;
    return feat_clampf(a, -lim, lim);
}

__device__ __forceinline__ uint16_t feat_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Candidate base pose of the move, in the robot step's own operation order.
struct CandBase {
    float bx, by, cy, sy;
};

__device__ __forceinline__ CandBase cand_base(const RobotParams &rp, const float *st, const float *a)
{
    const float a0 = feat_sanitize(a[0], rp.act_lim[0]), a1 = feat_sanitize(a[1], rp.act_lim[1]);
    const float pi_f = 0x1.921fb6p+1f, two_pi_f = 0x1.921fb6p+2f;
    float yaw = st[2] + a1;
    if (yaw > pi_f) yaw = yaw - two_pi_f;
    else if (yaw < -pi_f) yaw = yaw + two_pi_f;
    CandBase cb;
    dsincos(yaw, cb.sy, cb.cy);
    cb.bx = st[0] + a0 * cb.cy;
    cb.by = st[1] + a0 * cb.sy;
    return cb;
}

// Features 20..43: the origins of joint frames 1..7 and the end-effector z
// axis of the candidate joint angles, base at the origin.
__device__ __forceinline__ void arm_frame_features(const RobotParams &rp, const float *st, const float *a,
                                                   float (&out)[24])
{
    float q[10] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 7; ++j)
        q[3 + j] = feat_clampf(st[3 + j] + feat_sanitize(a[2 + j], rp.act_lim[2]), rp.qlim[j][0],
                               rp.qlim[j][1]);
    Fk fk;
    forward_kinematics(rp, q, fk);
#pragma unroll
    for (int j = 1; j < 8; ++j)
#pragma unroll
        for (int r = 0; r < 3; ++r) out[3 * (j - 1) + r] = fk.f[j].m[4 * r + 3];
#pragma unroll
    for (int r = 0; r < 3; ++r) out[21 + r] = fk.f[7].m[4 * r + 2];
}

// Scalar feature t (0 <= t < 64) of env `env`; `arm` holds features 20..43.
__device__ __forceinline__ float scalar_feature(const RobotParams &rp, const SimBuffers &sb,
                                                const GridMeta &gm, int env, const float *st,
                                                const float *a, int t, const float *arm)
{
    if (t < 7)
        return feat_clampf(st[3 + t] + feat_sanitize(a[2 + t], rp.act_lim[2]), rp.qlim[t][0],
                           rp.qlim[t][1]);
    if (t < 14) return feat_sanitize(a[2 + t - 7], rp.act_lim[2]) / rp.act_lim[2];
    if (t == 14) return feat_sanitize(a[0], rp.act_lim[0]) / rp.act_lim[0];
    if (t == 15) return feat_sanitize(a[1], rp.act_lim[1]) / rp.act_lim[1];
    if (t == 16) return (st[0] - gm.x0) / ((float)gm.nx * sb.cell);
    if (t == 17) return (st[1] - gm.y0) / ((float)gm.ny * sb.cell);
    if (t == 18) return st[2] * 0.31830988618f;
    if (t == 19) return sb.held[env] ? 1.0f : 0.0f;
    if (t < 44) return arm[t - 20];
    return 0.0f;
}

// Lattice box of patch column c = a * 16 + b around the candidate base pose:
// the columns i0..i1 x j0..j1 under the bounding box of the rotated 0.1 m
// cell.  False when the box leaves the grid (every layer blocked).  The box
// is under 3 columns wide, so at most 4 x 4 columns.
__device__ __forceinline__ bool patch_box(const CandBase &cb, float x0, float y0, float cell, int ox,
                                          int oy, int c, int &i0, int &i1, int &j0, int &j1)
{
    const float hx = 0.05f * (fabsf(cb.cy) + fabsf(cb.sy));   // half-extent of a rotated cell's box
    const int pa = c / kPatch, pb = c % kPatch;
    const float px = ((float)pa - 7.5f) * 0.1f, py = ((float)pb - 7.5f) * 0.1f;
    const float wx = cb.bx + (cb.cy * px - cb.sy * py), wy = cb.by + (cb.sy * px + cb.cy * py);
    const float fi0 = floorf(((wx - hx) - x0) / cell);
    const float fi1 = floorf(((wx + hx) - x0) / cell);
    const float fj0 = floorf(((wy - hx) - y0) / cell);
    const float fj1 = floorf(((wy + hx) - y0) / cell);
    if (!(fi0 >= 0.0f && fj0 >= 0.0f && fi1 < (float)ox && fj1 < (float)oy && fi1 - fi0 < 4.0f &&
          fj1 - fj0 < 4.0f))
        return false;
    i0 = (int)fi0;
    i1 = (int)fi1;
    j0 = (int)fj0;
    j1 = (int)fj1;
    return true;
}

// Occupancy bits (bit k = layer k blocked) of a patch column: the OR of the
// lattice bytes of its box, all 0xFF outside the grid.  Each of the box's
// (at most 4) rows is read as the 4 bytes from column i0 on, cut out of the
// two aligned words that hold them; the bytes past column i1 are masked out.
// The loads are a fixed 4 x 2 block (row indices clamped into the lattice,
// box 0..0 when outside) issued without a branch, so that the loads of
// several columns can be in flight together.  The lattice's allocation has 8
// bytes of slack past its end for the second word of its last bytes.
__device__ __forceinline__ uint32_t patch_or(const uint8_t *occ, int ox, int oy, bool inside, int i0,
                                             int i1, int j0, int j1)
{
    uint32_t lo[4], hi[4], sh[4];
#pragma unroll
    for (int dj = 0; dj < 4; ++dj) {
        const int j = min(j0 + dj, oy - 1);
        const uintptr_t a = (uintptr_t)(occ + (size_t)j * ox + i0);
        const uint32_t *w = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
        lo[dj] = w[0];
        hi[dj] = w[1];
        sh[dj] = (uint32_t)(a & 3);
    }
    const uint32_t keep = i1 - i0 >= 3 ? 0xFFFFFFFFu : (1u << (8 * (i1 - i0 + 1))) - 1u;
    uint32_t acc = 0;
#pragma unroll
    for (int dj = 0; dj < 4; ++dj)
        if (j0 + dj <= j1) acc |= __builtin_amdgcn_alignbyte(hi[dj], lo[dj], sh[dj]) & keep;
    acc |= acc >> 16;
    acc |= acc >> 8;
    return inside ? (acc & 0xFFu) : 0xFFu;
}

__device__ __forceinline__ uint32_t patch_bits(const OccGrid &og, const GridMeta &gm, int env,
                                               const CandBase &cb, int c)
{
    const int ox = og.occ_dims[2 * env], oy = og.occ_dims[2 * env + 1];
    int i0 = 0, i1 = 0, j0 = 0, j1 = 0;
    const bool in = patch_box(cb, gm.x0, gm.y0, og.occ_cell, ox, oy, c, i0, i1, j0, j1);
    return patch_or(og.occ + og.occ_off[env], ox, oy, in, i0, i1, j0, j1);
}

// The 8 layers of a patch column as BF16 ones and zeros, two per word.
__device__ __forceinline__ uint4 patch_words(uint32_t bits)
{
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = (((bits >> (2 * k)) & 1u) ? 0x3F80u : 0u) |
               ((((bits >> (2 * k + 1)) & 1u) ? 0x3F80u : 0u) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

}  // namespace gal
