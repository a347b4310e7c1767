// Depth rasteriser of the head camera (the per-env depth observation of
// Galactic, Section 4.1: 90 degree FoV; the paper's batch renderer is
// replaced by this fixed-point rasteriser).
//
// Semantics (identical, bit for bit, for any launch shape):
//  * a triangle whose face plane (supplied with the mesh) does not have the
//    camera strictly in front of it is culled;
//  * camera space X = right.(v-p), Y = down.(v-p), Z = fwd.(v-p);
//  * trivial reject against the near plane Z = n and a guard band of half a
//    viewport per side (X + 2Z, 2Z - X, Y + 2Z, 2Z - Y >= 0); triangles that
//    straddle a plane are clipped (Sutherland-Hodgman, planes in that order,
//    each intersection computed from the endpoints in a canonical order) and
//    fan-triangulated;
//  * projection x = w/2 + (w/2) X/Z (focal length w/2 for 90 degrees),
//    snapped to 1/16 pixel; triangles whose snapped winding is not front
//    facing, or whose area is zero, are culled;
//  * coverage at pixel centres by integer edge functions with the top-left
//    rule; per-vertex depth d = (1/n - 1/Z) (2^24-1)/(1/n - 1/f), combined
//    per pixel with the edge functions as barycentric weights, clamped and
//    truncated to 24 bits; the image keeps the minimum (0xFFFFFF = nothing;
//    with colour, the smallest (depth, triangle id)).
//
// Launch: one workgroup per (env, square region of <= 128x128 pixels), as a
// grid of items or as a persistent queue (longest items first, by cluster
// count or by the previous step's measured item times; the cheapest envs may
// be split into quarter regions).  The region's z-buffer lives in LDS and is
// updated with ds_min.  The env's mesh is stored as clusters of <= 64
// consecutive triangles, <= 64 unique vertices and <= 4 face planes, with an
// AABB.  The workgroup keeps the clusters inside the region's frustum with a
// face plane towards the camera, draws them in mesh order and, after a
// prologue, re-tests the rest against conservative z-buffer bounds
// (occlusion culling).  Per cluster: lane = vertex (transform, outcodes,
// projection once per vertex), lane = triangle (gathers its vertices with
// ds_bpermute); triangles whose pixel bbox is small are rasterised by their
// own lane, mid-sized ones by the whole wave with the pixels spread over the
// lanes (or, with binning, listed per 8x8 tile in LDS and drawn tile by tile,
// lane = pixel), large ones one 8x8 tile (lane = pixel) at a time.  Every
// extra rejection only removes triangles that cannot change a pixel of the
// region.
#include "gal_raster.h"

#include <algorithm>
#include <type_traits>

namespace gal {

namespace {

constexpr uint32_t kFar = 0xFFFFFFu;
constexpr uint32_t kClipBits = 0x1Fu;
constexpr int kVisCap = 3072;   // clusters per visibility window (u16 list in LDS)

// Products of edge-function terms: snapped coordinates lie in the guard band
// (|x| < 3 * 16 * 256 / 2 < 2^13 at the largest resolution, 256), so every
// factor fits in 24 signed bits and v_mul_i32_i24 (full rate) returns the same
// low 32 bits as a 32-bit multiply, which is the exact product.
__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }

struct Cam {
    float px, py, pz, rx, ry, rz, dx, dy, dz, fx, fy, fz;
};

struct Proj {
    float hw;     // half width (= half height)
    float near_m;
    float invn;
    float kd;
};

__device__ __forceinline__ int snap16(float v)
{
    float s = v * 16.0f;
    s = s < -1048576.0f ? -1048576.0f : (s > 1048576.0f ? 1048576.0f : s);
    return (int)rintf(s);
}

__device__ __forceinline__ void project(const Proj &pj, float X, float Y, float Z, int &xi, int &yi,
                                        float &d)
{
    float xs = pj.hw + pj.hw * (X / Z);
    float ys = pj.hw + pj.hw * (Y / Z);
    xi = snap16(xs);
    yi = snap16(ys);
    float inv = 1.0f / Z;
    d = (pj.invn - inv) * pj.kd;
}

__device__ __forceinline__ float clip_plane(float X, float Y, float Z, int k, float near_m)
{
    switch (k) {
    case 0: return Z - near_m;
    case 1: return X + 2.0f * Z;
    case 2: return 2.0f * Z - X;
    case 3: return Y + 2.0f * Z;
    default: return 2.0f * Z - Y;
    }
}

__device__ __forceinline__ uint32_t depth24(float dv)
{
    if (!(dv > 0.0f)) return 0u;
    if (dv >= 16777215.0f) return kFar;
    return (uint32_t)dv;
}

struct Poly {
    float X[8], Y[8], Z[8];
    int n;
};

__device__ __forceinline__ bool before(float ax, float ay, float az, float bx, float by, float bz)
{
    uint32_t a0 = __float_as_uint(ax), b0 = __float_as_uint(bx);
    if (a0 != b0) return a0 < b0;
    uint32_t a1 = __float_as_uint(ay), b1 = __float_as_uint(by);
    if (a1 != b1) return a1 < b1;
    return __float_as_uint(az) < __float_as_uint(bz);
}

// Sutherland-Hodgman against near, left, right, top, bottom.  A convex
// triangle gains at most one vertex per plane (<= 8); should rounding ever
// emit more, the extra vertices are dropped.
__device__ __noinline__ void clip_polygon(Poly &p, float near_m)
{
    for (int k = 0; k < 5 && p.n > 0; ++k) {
        Poly q;
        q.n = 0;
        for (int i = 0; i < p.n; ++i) {
            const int j = (i + p.n - 1) % p.n;   // previous vertex
            const float cX = p.X[i], cY = p.Y[i], cZ = p.Z[i];
            const float pX = p.X[j], pY = p.Y[j], pZ = p.Z[j];
            const bool cin = clip_plane(cX, cY, cZ, k, near_m) >= 0.0f;
            const bool pin = clip_plane(pX, pY, pZ, k, near_m) >= 0.0f;
            if (cin != pin && q.n < 8) {
                // endpoints in canonical order
                float sX = pX, sY = pY, sZ = pZ, eX = cX, eY = cY, eZ = cZ;
                if (before(cX, cY, cZ, pX, pY, pZ)) {
                    sX = cX; sY = cY; sZ = cZ; eX = pX; eY = pY; eZ = pZ;
                }
                const float ps = clip_plane(sX, sY, sZ, k, near_m);
                const float pe = clip_plane(eX, eY, eZ, k, near_m);
                const float t = ps / (ps - pe);
                q.X[q.n] = sX + t * (eX - sX);
                q.Y[q.n] = sY + t * (eY - sY);
                q.Z[q.n] = sZ + t * (eZ - sZ);
                ++q.n;
            }
            if (cin && q.n < 8) {
                q.X[q.n] = cX;
                q.Y[q.n] = cY;
                q.Z[q.n] = cZ;
                ++q.n;
            }
        }
        p = q;
    }
}

// Triangle set up for rasterisation: snapped vertices (after the winding
// swap), per-vertex depth scaled by 1/A2 (barycentric weights are the edge
// functions), pixel bbox clipped to the region.
struct Setup {
    int x0, y0, x1, y1, x2, y2;
    int bias;                 // bit k set: edge k is not top-left (needs E >= 1)
    float q0, q1, q2;         // vertex depth / A2
    int px0, px1, py0, py1;
};

// Returns 0 = nothing to draw, 1 = drawable.
__device__ __forceinline__ int setup_triangle(int x0, int y0, float d0, int x1, int y1, float d1,
                                              int x2, int y2, float d2, int rx0, int ry0, int R,
                                              Setup &S)
{
    const int A2 = mul24(x1 - x0, y2 - y0) - mul24(x2 - x0, y1 - y0);
    if (A2 >= 0) return 0;   // back face or degenerate
    // front face: swap v1 and v2 so the signed area is positive
    S.x0 = x0; S.y0 = y0;
    S.x1 = x2; S.y1 = y2;
    S.x2 = x1; S.y2 = y1;
    const int minx = min(x0, min(x1, x2)), maxx = max(x0, max(x1, x2));
    const int miny = min(y0, min(y1, y2)), maxy = max(y0, max(y1, y2));
    S.px0 = max((minx + 7) >> 4, rx0);
    S.px1 = min((maxx - 8) >> 4, rx0 + R - 1);
    S.py0 = max((miny + 7) >> 4, ry0);
    S.py1 = min((maxy - 8) >> 4, ry0 + R - 1);
    if (S.px0 > S.px1 || S.py0 > S.py1) return 0;
    // edges (1->2), (2->0), (0->1) of the swapped triangle
    int bias = 0;
    {
        const int ex = S.x2 - S.x1, ey = S.y2 - S.y1;
        if (!((ey < 0) || (ey == 0 && ex > 0))) bias |= 1;
    }
    {
        const int ex = S.x0 - S.x2, ey = S.y0 - S.y2;
        if (!((ey < 0) || (ey == 0 && ex > 0))) bias |= 2;
    }
    {
        const int ex = S.x1 - S.x0, ey = S.y1 - S.y0;
        if (!((ey < 0) || (ey == 0 && ex > 0))) bias |= 4;
    }
    S.bias = bias;
    const float invA = 1.0f / (float)(-A2);
    S.q0 = d0 * invA;
    S.q1 = d2 * invA;   // swapped vertex 1 is the original vertex 2
    S.q2 = d1 * invA;
    return 1;
}

__device__ __forceinline__ uint32_t frag_depth(int e0, int e1, int e2, float q0, float q1, float q2)
{
    const float dv = ((float)e0 * q0 + (float)e1 * q1) + (float)e2 * q2;
    return depth24(dv);
}

// Row pitch (words) of a region's z-buffer in LDS: R padded so that 8
// consecutive rows start 8 banks apart (pitch/8 odd), so the 64 pixels of an
// 8x8 tile fall in 64 different banks instead of the 8 that a pitch of
// R = 128 or 64 would give.
__host__ __device__ constexpr int zpitch(int R) { return 8 * (((R >> 3) + 1) | 1); }

// Z-buffer sinks in LDS: depth only (u32, 24-bit depth) or depth and colour
// (u64 key = depth << 32 | triangle id: the smallest depth wins, ties go to
// the smallest triangle id).
// key_at / set_key / make: plain access for a wave that owns a pixel tile
// while no other wave writes it (the binned pass).
struct DepthSink {
    typedef uint32_t Key;
    uint32_t *z;
    __device__ __forceinline__ void put(int p, uint32_t D, uint32_t) const { atomicMin(&z[p], D); }
    __device__ __forceinline__ uint32_t depth_at(int p) const { return z[p]; }
    __device__ __forceinline__ void clear(int p) const { z[p] = kFar; }
    __device__ __forceinline__ Key key_at(int p) const { return z[p]; }
    __device__ __forceinline__ void set_key(int p, Key k) const { z[p] = k; }
    static __device__ __forceinline__ Key make(uint32_t D, uint32_t) { return D; }
};

struct ColorSink {
    typedef unsigned long long Key;
    unsigned long long *k;
    __device__ __forceinline__ void put(int p, uint32_t D, uint32_t id) const
    {
        atomicMin(&k[p], ((unsigned long long)D << 32) | (unsigned long long)id);
    }
    __device__ __forceinline__ uint32_t depth_at(int p) const { return (uint32_t)(k[p] >> 32); }
    __device__ __forceinline__ void clear(int p) const
    {
        k[p] = ((unsigned long long)kFar << 32) | 0xFFFFFFFFull;
    }
    __device__ __forceinline__ Key key_at(int p) const { return k[p]; }
    __device__ __forceinline__ void set_key(int p, Key v) const { k[p] = v; }
    static __device__ __forceinline__ Key make(uint32_t D, uint32_t id)
    {
        return ((unsigned long long)D << 32) | (unsigned long long)id;
    }
};

template <class Sink>
__device__ __forceinline__ void raster_small(const Setup &S, uint32_t id, int rx0, int ry0, int P,
                                             const Sink &zb)
{
    // edge k from vertex i to j: E = (xj-xi)(Py-yi) - (yj-yi)(Px-xi)
    const int ex0 = S.x2 - S.x1, ey0 = S.y2 - S.y1;
    const int ex1 = S.x0 - S.x2, ey1 = S.y0 - S.y2;
    const int ex2 = S.x1 - S.x0, ey2 = S.y1 - S.y0;
    const int b0 = S.bias & 1, b1 = (S.bias >> 1) & 1, b2 = (S.bias >> 2) & 1;
    const int Px0 = 16 * S.px0 + 8;
    const int Py0 = 16 * S.py0 + 8;
    int r0 = mul24(ex0, Py0 - S.y1) - mul24(ey0, Px0 - S.x1);
    int r1 = mul24(ex1, Py0 - S.y2) - mul24(ey1, Px0 - S.x2);
    int r2 = mul24(ex2, Py0 - S.y0) - mul24(ey2, Px0 - S.x0);
    for (int py = S.py0; py <= S.py1; ++py) {
        int e0 = r0, e1 = r1, e2 = r2;
        for (int px = S.px0; px <= S.px1; ++px) {
            if (e0 >= b0 && e1 >= b1 && e2 >= b2) {
                const uint32_t D = frag_depth(e0, e1, e2, S.q0, S.q1, S.q2);
                if (D < kFar) zb.put((py - ry0) * P + (px - rx0), D, id);
            }
            e0 -= 16 * ey0;
            e1 -= 16 * ey1;
            e2 -= 16 * ey2;
        }
        r0 += 16 * ex0;
        r1 += 16 * ex1;
        r2 += 16 * ex2;
    }
}

__device__ __forceinline__ int rl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rlf(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// One triangle's record, uniform over the wave.
struct TriRec {
    int x0, y0, x1, y1, x2, y2;
    int bias;
    float q0, q1, q2;
    int px0, px1, py0, py1;
    uint32_t id;
};

// The whole wave rasterises one triangle over 8-pixel tile rows ty_first ..
// ty_last, in 16 x 8 double tiles (lane = pixel pair (lx, ly), (lx + 8, ly)).
// The double tiles of its bbox in those rows (at most 8 per row in a
// 128-pixel region) are first tested lane-parallel, four tile rows at a time:
// a tile is skipped when some edge function is below its threshold even at
// the tile's pixel centre where that edge is largest (the functions are
// linear), so only tiles that can hold a covered pixel are visited.  Within a
// tile the edge values are the tile origin's plus a per-lane offset, and the
// right half's are the left half's minus 8 pixel steps (the same integers as
// evaluating them per pixel).
template <class Sink>
__device__ __forceinline__ void raster_tiles(const TriRec &t, int ty_first, int ty_last, int lane,
                                             int ry0, int rx0, int P, const Sink &zb)
{
    const int x0 = t.x0, y0 = t.y0, x1 = t.x1, y1 = t.y1, x2 = t.x2, y2 = t.y2;
    const int ex0 = x2 - x1, ey0 = y2 - y1;
    const int ex1 = x0 - x2, ey1 = y0 - y2;
    const int ex2 = x1 - x0, ey2 = y1 - y0;
    const int b0 = t.bias & 1, b1 = (t.bias >> 1) & 1, b2 = (t.bias >> 2) & 1;
    const int lx = lane & 7, ly = lane >> 3;
    // offset of pixel (lx, ly) from its tile's origin pixel, per edge
    const int o0 = mul24(16 * ex0, ly) - mul24(16 * ey0, lx);
    const int o1 = mul24(16 * ex1, ly) - mul24(16 * ey1, lx);
    const int o2 = mul24(16 * ex2, ly) - mul24(16 * ey2, lx);
    // corner offsets of a 16 x 8 tile (pixel-centre units) where each edge is largest
    const int c0x = ey0 < 0 ? 240 : 0, c0y = ex0 > 0 ? 112 : 0;
    const int c1x = ey1 < 0 ? 240 : 0, c1y = ex1 > 0 ? 112 : 0;
    const int c2x = ey2 < 0 ? 240 : 0, c2y = ex2 > 0 ? 112 : 0;
    const int tx0 = t.px0 >> 4, tx1 = t.px1 >> 4;
    for (int tyb = ty_first; tyb <= ty_last; tyb += 4) {
        bool live = false;
        {
            const int tx = tx0 + (lane & 15), ty = tyb + (lane >> 4);
            if (tx <= tx1 && ty <= ty_last) {
                const int Pxb = 256 * tx + 8, Pyb = 128 * ty + 8;
                const int m0 = mul24(ex0, Pyb + c0y - y1) - mul24(ey0, Pxb + c0x - x1);
                const int m1 = mul24(ex1, Pyb + c1y - y2) - mul24(ey1, Pxb + c1x - x2);
                const int m2 = mul24(ex2, Pyb + c2y - y0) - mul24(ey2, Pxb + c2x - x0);
                live = m0 >= b0 && m1 >= b1 && m2 >= b2;
            }
        }
        uint64_t mask = __ballot(live);
        while (mask) {
            const int k = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int tx = tx0 + (k & 15), ty = tyb + (k >> 4);
            const int Pxb = 256 * tx + 8, Pyb = 128 * ty + 8;
            int e0 = mul24(ex0, Pyb - y1) - mul24(ey0, Pxb - x1) + o0;
            int e1 = mul24(ex1, Pyb - y2) - mul24(ey1, Pxb - x2) + o1;
            int e2 = mul24(ex2, Pyb - y0) - mul24(ey2, Pxb - x0) + o2;
            const int py = ty * 8 + ly;
            const int zrow = mul24(py - ry0, P) - rx0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int px = tx * 16 + 8 * h + lx;
                if (px >= t.px0 && px <= t.px1 && py >= t.py0 && py <= t.py1 && e0 >= b0 && e1 >= b1 &&
                    e2 >= b2) {
                    const uint32_t D = frag_depth(e0, e1, e2, t.q0, t.q1, t.q2);
                    if (D < kFar) zb.put(zrow + px, D, t.id);
                }
                e0 -= 128 * ey0;
                e1 -= 128 * ey1;
                e2 -= 128 * ey2;
            }
        }
    }
}

// Lane L's triangle record, read into every lane.
__device__ __forceinline__ TriRec lane_record(const Setup &S, uint32_t myid, int L)
{
    TriRec t;
    t.id = (uint32_t)rl((int)myid, L);
    t.x0 = rl(S.x0, L); t.y0 = rl(S.y0, L);
    t.x1 = rl(S.x1, L); t.y1 = rl(S.y1, L);
    t.x2 = rl(S.x2, L); t.y2 = rl(S.y2, L);
    t.bias = rl(S.bias, L);
    t.q0 = rlf(S.q0, L); t.q1 = rlf(S.q1, L); t.q2 = rlf(S.q2, L);
    t.px0 = rl(S.px0, L); t.px1 = rl(S.px1, L);
    t.py0 = rl(S.py0, L); t.py1 = rl(S.py1, L);
    return t;
}

// Large triangles (bbox above small_max pixels) are not drawn by the wave that
// sets them up: their records go to a list in LDS and, at the end of each
// drawing round, every wave of the workgroup takes groups of four tile rows
// of them in turn, so that a floor or wall triangle covering half the region
// does not keep one wave busy while the others wait at the round's barrier.
// A full list falls back to drawing by the wave itself.
constexpr int kBigCap = 32;
struct BigRec {
    int xy0, xy1, xy2;   // snapped x | y << 16
    int box;             // px0 | px1 << 8 | py0 << 16 | py1 << 24
    int bias;
    float q0, q1, q2;
    uint32_t id;
};

// (the record is the same for every lane: kept in scalar registers)
__device__ __forceinline__ TriRec unpack_big(const BigRec &b)
{
    const int xy0 = __builtin_amdgcn_readfirstlane(b.xy0);
    const int xy1 = __builtin_amdgcn_readfirstlane(b.xy1);
    const int xy2 = __builtin_amdgcn_readfirstlane(b.xy2);
    const int box = __builtin_amdgcn_readfirstlane(b.box);
    TriRec t;
    t.x0 = (int)(short)(xy0 & 0xFFFF); t.y0 = xy0 >> 16;
    t.x1 = (int)(short)(xy1 & 0xFFFF); t.y1 = xy1 >> 16;
    t.x2 = (int)(short)(xy2 & 0xFFFF); t.y2 = xy2 >> 16;
    t.bias = __builtin_amdgcn_readfirstlane(b.bias);
    t.q0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(b.q0)));
    t.q1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(b.q1)));
    t.q2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(b.q2)));
    t.px0 = box & 0xFF; t.px1 = (box >> 8) & 0xFF;
    t.py0 = (box >> 16) & 0xFF; t.py1 = (box >> 24) & 0xFF;
    t.id = (uint32_t)__builtin_amdgcn_readfirstlane((int)b.id);
    return t;
}

// Row-shifted copy of v (DPP, no LDS traffic); lanes whose source lies
// outside their row of 16 get `fill`.
template <int kCtrl>
__device__ __forceinline__ int dpp_shift(int v, int fill)
{
    return __builtin_amdgcn_update_dpp(fill, v, kCtrl, 0xF, 0xF, false);
}

// Maximum over the (fully active) wave, returned to every lane: prefix
// maxima within each row of 16 (DPP row_shr 1, 2, 4, 8), then the four row
// maxima read from lanes 15, 31, 47 and 63.
__device__ __forceinline__ int wave_max(int v)
{
    constexpr int kMin = -2147483647 - 1;
    v = max(v, dpp_shift<0x111>(v, kMin));
    v = max(v, dpp_shift<0x112>(v, kMin));
    v = max(v, dpp_shift<0x114>(v, kMin));
    v = max(v, dpp_shift<0x118>(v, kMin));
    const int a = max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31));
    const int b = max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63));
    return max(a, b);
}

// Inclusive prefix sum / maximum over the (fully active) wave: prefixes within
// each row of 16 lanes (DPP row_shr 1, 2, 4, 8), then the totals of the
// earlier rows (lanes 15, 31, 47) folded into rows 1..3.
__device__ __forceinline__ int wave_incl_sum(int v, int lane)
{
    v += dpp_shift<0x111>(v, 0);
    v += dpp_shift<0x112>(v, 0);
    v += dpp_shift<0x114>(v, 0);
    v += dpp_shift<0x118>(v, 0);
    const int r0 = __builtin_amdgcn_readlane(v, 15);
    const int r1 = __builtin_amdgcn_readlane(v, 31);
    const int r2 = __builtin_amdgcn_readlane(v, 47);
    const int row = lane >> 4;
    return v + (row >= 1 ? r0 : 0) + (row >= 2 ? r1 : 0) + (row >= 3 ? r2 : 0);
}

__device__ __forceinline__ int wave_incl_max(int v, int lane)
{
    constexpr int kMin = -2147483647 - 1;
    v = max(v, dpp_shift<0x111>(v, kMin));
    v = max(v, dpp_shift<0x112>(v, kMin));
    v = max(v, dpp_shift<0x114>(v, kMin));
    v = max(v, dpp_shift<0x118>(v, kMin));
    const int r0 = __builtin_amdgcn_readlane(v, 15);
    const int r1 = max(r0, __builtin_amdgcn_readlane(v, 31));
    const int r2 = max(r1, __builtin_amdgcn_readlane(v, 47));
    const int row = lane >> 4;
    return max(v, row == 0 ? kMin : row == 1 ? r0 : row == 2 ? r1 : r2);
}

// Load-balanced rasterisation of every lane's triangle at once.  Each bbox row
// is cut into spans of 4 pixels; the spans of all bboxes are numbered by a
// wave prefix sum and lane l takes spans l, l + 64, ...  For each window of
// 64 spans, every triangle starting inside it writes (first span, lane) at its
// start position in the wave's 64 LDS words `own`, and a wave maximum-scan
// over the positions gives every span its triangle (the last start at or
// before it; position 0 inherits the previous window's last owner).  The
// triangle's record is then fetched from its lane once for the span's 4
// pixels, whose edge functions step by the exact integer increments.
constexpr int kSpan = 4;

template <class Sink>
__device__ __forceinline__ void raster_balanced(const Setup &S, uint32_t myid, bool mine, int lane,
                                                int rx0, int ry0, int P, int *own_generic,
                                                const Sink &zb)
{
    // LDS pointer, volatile: the writes of other lanes must be re-read
    typedef __attribute__((address_space(3))) volatile int lds_int;
    lds_int *own = (lds_int *)own_generic;
    const int w = mine ? S.px1 - S.px0 + 1 : 0;
    const int h = mine ? S.py1 - S.py0 + 1 : 0;
    const int ns = (w + kSpan - 1) / kSpan;   // spans per bbox row
    const int cnt = ns * h;
    const int incl = wave_incl_sum(cnt, lane);
    const int excl = incl - cnt;
    const int total = __builtin_amdgcn_readlane(incl, 63);
    if (total == 0) return;
    // packed record of this lane's triangle
    const int xy0 = (S.x0 & 0xFFFF) | (S.y0 << 16);
    const int xy1 = (S.x1 & 0xFFFF) | (S.y1 << 16);
    const int xy2 = (S.x2 & 0xFFFF) | (S.y2 << 16);
    const int meta = S.px0 | (S.py0 << 9) | ((ns > 0 ? ns - 1 : 0) << 18) | (S.bias << 27);
    const float invns = 1.0f / (float)(ns > 0 ? ns : 1);
    // (first span << 6 | lane): increasing along the lanes with spans
    const int start = (excl << 6) | lane;
    int carry = 0;
    for (int base = 0; base < total; base += 64) {
        const int g = base + lane;
        own[lane] = -1;
        if (cnt > 0 && excl >= base && excl < base + 64) own[excl - base] = start;
        int o = own[lane];
        if (lane == 0 && o < 0) o = carry;
        const int packed = wave_incl_max(o, lane);
        carry = __builtin_amdgcn_readlane(packed, 63);
        const int t = packed & 63;
        const int local = g - (packed >> 6);
        const int txy0 = __shfl(xy0, t, 64), txy1 = __shfl(xy1, t, 64), txy2 = __shfl(xy2, t, 64);
        const int tmeta = __shfl(meta, t, 64);
        const int tpx1 = __shfl(S.px1, t, 64);
        const float tq0 = __shfl(S.q0, t, 64), tq1 = __shfl(S.q1, t, 64), tq2 = __shfl(S.q2, t, 64);
        const float tinvns = __shfl(invns, t, 64);
        const uint32_t tid = (uint32_t)__shfl((int)myid, t, 64);
        if (g >= total) continue;
        const int tns = ((tmeta >> 18) & 0x1FF) + 1;
        // span (row oy, span ox) of the triangle's bbox; the float quotient is
        // within 0.002 of (local + 0.5) / tns, whose fraction is at least
        // 0.5 / 64 from an integer, and the step below settles any doubt
        int oy = (int)(((float)local + 0.5f) * tinvns);
        int ox = local - mul24(oy, tns);
        if (ox < 0) { oy -= 1; ox += tns; }
        else if (ox >= tns) { oy += 1; ox -= tns; }
        const int px = (tmeta & 0x1FF) + kSpan * ox, py = ((tmeta >> 9) & 0x1FF) + oy;
        const int x0 = (int)(short)(txy0 & 0xFFFF), y0 = txy0 >> 16;
        const int x1 = (int)(short)(txy1 & 0xFFFF), y1 = txy1 >> 16;
        const int x2 = (int)(short)(txy2 & 0xFFFF), y2 = txy2 >> 16;
        const int tb = tmeta >> 27;
        const int b0 = tb & 1, b1 = (tb >> 1) & 1, b2 = (tb >> 2) & 1;
        const int Px = 16 * px + 8, Py = 16 * py + 8;
        int e0 = mul24(x2 - x1, Py - y1) - mul24(y2 - y1, Px - x1);
        int e1 = mul24(x0 - x2, Py - y2) - mul24(y0 - y2, Px - x2);
        int e2 = mul24(x1 - x0, Py - y0) - mul24(y1 - y0, Px - x0);
        // one pixel to the right: E decreases by 16 (y_j - y_i)
        const int d0 = 16 * (y2 - y1), d1 = 16 * (y0 - y2), d2 = 16 * (y1 - y0);
        const int zrow = mul24(py - ry0, P) - rx0;
#pragma unroll
        for (int k = 0; k < kSpan; ++k) {
            if (px + k <= tpx1 && e0 >= b0 && e1 >= b1 && e2 >= b2) {
                const uint32_t D = frag_depth(e0, e1, e2, tq0, tq1, tq2);
                if (D < kFar) zb.put(zrow + px + k, D, tid);
            }
            e0 -= d0;
            e1 -= d1;
            e2 -= d2;
        }
    }
}


// Conservative frustum test of a cluster AABB (world) against the near plane
// and the region's four side planes; margins cover float rounding.
struct RegionPlanes {
    float n[5][3];
    float off[5];
};

__device__ __forceinline__ bool aabb_visible(const RegionPlanes &P, float lx, float ly, float lz,
                                             float hx, float hy, float hz)
{
    const float cx = 0.5f * (lx + hx), cy = 0.5f * (ly + hy), cz = 0.5f * (lz + hz);
    const float ex = 0.5f * (hx - lx), ey = 0.5f * (hy - ly), ez = 0.5f * (hz - lz);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float c = P.n[k][0] * cx + P.n[k][1] * cy + P.n[k][2] * cz + P.off[k];
        const float r = fabsf(P.n[k][0]) * ex + fabsf(P.n[k][1]) * ey + fabsf(P.n[k][2]) * ez;
        if (c + r < -1e-2f) return false;
    }
    return true;
}

// Occlusion bounds: maxima of the z-buffer over 8x8 tiles and 32x32 blocks,
// taken between drawing rounds; the z-buffer only decreases, so they stay
// upper bounds of the current maxima while the next round draws.
struct Occl {
    uint32_t *tilemax;   // [TW*TW]
    uint32_t *blockmax;  // [BW*BW]
    int TW, BW;
    int P;               // z-buffer row pitch
};

// True when every fragment the cluster could produce in the region is
// provably behind the current z-buffer.  Fragment depths are convex
// combinations of vertex depths (a few LSB of rounding), vertex depth grows
// with camera distance, and all vertices lie in the AABB; the screen bbox of
// the projected AABB (plus a pixel) contains every covered pixel centre.
__device__ __forceinline__ bool cluster_hidden(const Cam &cam, const Proj &pj, const Occl &oc,
                                               int rx0, int ry0, int R, float lx, float ly,
                                               float lz, float hx, float hy, float hz)
{
    const float ddx = lx - cam.px, ddy = ly - cam.py, ddz = lz - cam.pz;
    const float X0 = cam.rx * ddx + cam.ry * ddy + cam.rz * ddz;
    const float Y0 = cam.dx * ddx + cam.dy * ddy + cam.dz * ddz;
    const float Z0 = cam.fx * ddx + cam.fy * ddy + cam.fz * ddz;
    const float ex = hx - lx, ey = hy - ly, ez = hz - lz;
    const float aX = cam.rx * ex, bX = cam.ry * ey, cX = cam.rz * ez;
    const float aY = cam.dx * ex, bY = cam.dy * ey, cY = cam.dz * ez;
    const float aZ = cam.fx * ex, bZ = cam.fy * ey, cZ = cam.fz * ez;
    const float zmin = Z0 + fminf(aZ, 0.f) + fminf(bZ, 0.f) + fminf(cZ, 0.f);
    if (!(zmin > 1.01f * pj.near_m + 1e-3f)) return false;
    float nxmin = 1e30f, nxmax = -1e30f, nymin = 1e30f, nymax = -1e30f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float X = X0 + ((c & 1) ? aX : 0.f) + ((c & 2) ? bX : 0.f) + ((c & 4) ? cX : 0.f);
        const float Y = Y0 + ((c & 1) ? aY : 0.f) + ((c & 2) ? bY : 0.f) + ((c & 4) ? cY : 0.f);
        const float Z = Z0 + ((c & 1) ? aZ : 0.f) + ((c & 2) ? bZ : 0.f) + ((c & 4) ? cZ : 0.f);
        const float r = __builtin_amdgcn_rcpf(Z);
        nxmin = fminf(nxmin, X * r);
        nxmax = fmaxf(nxmax, X * r);
        nymin = fminf(nymin, Y * r);
        nymax = fmaxf(nymax, Y * r);
    }
    const float fx0 = pj.hw + pj.hw * nxmin, fx1 = pj.hw + pj.hw * nxmax;
    const float fy0 = pj.hw + pj.hw * nymin, fy1 = pj.hw + pj.hw * nymax;
    // pixel ranges relative to the region, one pixel of margin
    const int px0 = max((int)floorf(fmaxf(fx0, -1e6f)) - 1 - rx0, 0);
    const int px1 = min((int)floorf(fminf(fx1, 1e6f)) + 1 - rx0, R - 1);
    const int py0 = max((int)floorf(fmaxf(fy0, -1e6f)) - 1 - ry0, 0);
    const int py1 = min((int)floorf(fminf(fy1, 1e6f)) + 1 - ry0, R - 1);
    if (px0 > px1 || py0 > py1) return true;   // projects outside the region
    const float zlb = zmin * (1.0f - 1e-5f) - 1e-4f;
    const float dlb = (pj.invn - 1.0f / zlb) * pj.kd - 16.0f;
    uint32_t m = 0;
    const int tx0 = px0 >> 3, tx1 = px1 >> 3, ty0 = py0 >> 3, ty1 = py1 >> 3;
    if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) <= 16) {
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) m = max(m, oc.tilemax[ty * oc.TW + tx]);
    } else {
        for (int by = py0 >> 5; by <= (py1 >> 5); ++by)
            for (int bx = px0 >> 5; bx <= (px1 >> 5); ++bx) m = max(m, oc.blockmax[by * oc.BW + bx]);
    }
    return dlb > (float)m;
}

// Refresh of the occlusion bounds by the whole workgroup (no cluster is being
// drawn): tiles w, w+W, ... per wave, then the blocks from the tiles.
template <class Sink>
__device__ __forceinline__ void refresh_bounds(const Sink &zb, const Occl &oc, int R,
                                               int wave, int nwaves, int lane)
{
    if constexpr (std::is_same<Sink, DepthSink>::value) {
        // four tiles per wave and pass: a row of 16 lanes per tile, each lane
        // four pixels of one tile row (one 16-byte LDS read; R, the pitch and
        // the tile origins are multiples of 8), the row maximum by DPP
        constexpr int kMin = -2147483647 - 1;
        const int q = lane >> 4, row = (lane >> 1) & 7, half = lane & 1;
        const int ntile = oc.TW * oc.TW;
        for (int t0 = wave * 4; t0 < ntile; t0 += nwaves * 4) {
            const int t = t0 + q;
            int v = 0;
            if (t < ntile) {
                const int tx = t % oc.TW, ty = t / oc.TW;
                const uint4 w = *reinterpret_cast<const uint4 *>(zb.z + (8 * ty + row) * oc.P + 8 * tx + 4 * half);
                v = (int)max(max(w.x, w.y), max(w.z, w.w));
            }
            v = max(v, dpp_shift<0x111>(v, kMin));
            v = max(v, dpp_shift<0x112>(v, kMin));
            v = max(v, dpp_shift<0x114>(v, kMin));
            v = max(v, dpp_shift<0x118>(v, kMin));
            if ((lane & 15) == 15 && t < ntile) oc.tilemax[t] = (uint32_t)v;
        }
    } else {
        const int lx = lane & 7, ly = lane >> 3;
        for (int t = wave; t < oc.TW * oc.TW; t += nwaves) {
            const int tx = t % oc.TW, ty = t / oc.TW;
            const int px = tx * 8 + lx, py = ty * 8 + ly;
            const int v = (px < R && py < R) ? (int)zb.depth_at(py * oc.P + px) : 0;
            const int m = wave_max(v);
            if (lane == 0) oc.tilemax[t] = (uint32_t)m;
        }
    }
    __syncthreads();
    for (int b = wave; b < oc.BW * oc.BW; b += nwaves) {
        const int bx = b % oc.BW, by = b / oc.BW;
        const int tx = bx * 4 + (lane & 3), ty = by * 4 + ((lane >> 2) & 3);
        const int v = (lane < 16 && tx < oc.TW && ty < oc.TW) ? (int)oc.tilemax[ty * oc.TW + tx] : 0;
        const int m = wave_max(v);
        if (lane == 0) oc.blockmax[b] = (uint32_t)m;
    }
    __syncthreads();
}

// Whether the camera is strictly in front of face plane p, from the item's
// bits (kNoPlane: a mesh without face planes, never culled by a plane).
__device__ __forceinline__ bool plane_front(const uint32_t *bits, uint32_t p)
{
    return p == kNoPlane || ((bits[p >> 5] >> (p & 31u)) & 1u) != 0u;
}

// Whether any of a cluster's face planes (p0 | p1 << 16, p2 | p3 << 16) faces
// the camera; when none does, every triangle of the cluster is culled.
__device__ __forceinline__ bool any_plane_front(const uint32_t *bits, uint32_t p01, uint32_t p23)
{
    return plane_front(bits, p01 & 0xFFFFu) || plane_front(bits, p01 >> 16) ||
           plane_front(bits, p23 & 0xFFFFu) || plane_front(bits, p23 >> 16);
}

// 8x8-tile binning (tuning `bin`).  Mid-sized triangles are not drawn by the
// wave that sets them up: their edge functions go to a record buffer in LDS
// and the record's index to the list of every 8x8 tile of the region that can
// hold one of their pixels.  When the buffer is nearly full, and at the end of
// each occlusion round, the workgroup synchronises and every wave draws whole
// tiles: lane = pixel, looping over the tile's list with the pixel's key in a
// register (no other wave writes the tile meanwhile, so no atomics).  A
// triangle that finds the buffer or one of its tiles' lists full is drawn by
// the balanced pass instead; drawing a triangle twice changes nothing, the
// z-buffer keeping a minimum.
constexpr int kBinTris = 256;   // records per flush
constexpr int kBinCap = 24;     // list entries per tile

// A binned triangle: per edge k, E_k = C + A * px + B * py at the pixel
// (px, py) relative to the region origin (the same integer as the edge
// function at that pixel centre), covered iff E_k >= b_k (top-left rule).
struct BinRec {
    int4 e0, e1, e2;   // A, B, C, b
    float4 q;          // q0, q1, q2, bits of the triangle id
};

struct Bins {
    BinRec *rec;       // [kBinTris]
    int *cnt;          // [tiles] list entries claimed (above kBinCap: overflowed)
    uint16_t *list;    // [tiles][kBinCap] record indices
    int *ntri;         // records claimed
    int TW;            // tiles per region row
};

// Bytes of a region's bins in dynamic LDS (after the z-buffer).
__host__ __device__ constexpr size_t bin_bytes(int R)
{
    return sizeof(BinRec) * kBinTris + (size_t)(R / 8) * (R / 8) * (4 + 2 * kBinCap) + 16;
}

// Whether the edge function can reach its threshold somewhere in tile
// (tx, ty): its largest value over the tile's 64 pixel centres (it is linear).
__device__ __forceinline__ bool tile_live(const int4 &e, int tx, int ty)
{
    const int px = 8 * tx + (e.x > 0 ? 7 : 0), py = 8 * ty + (e.y > 0 ? 7 : 0);
    return e.z + mul24(e.x, px) + mul24(e.y, py) >= e.w;
}

// Draw the binned triangles: wave w takes tiles w, w + nwaves, ...
template <class Sink>
__device__ void flush_bins(const Bins &bn, int wave, int nwaves, int lane, int P, const Sink &zb)
{
    const int lx = lane & 7, ly = lane >> 3;
    const int ntiles = bn.TW * bn.TW;
    for (int t = wave; t < ntiles; t += nwaves) {
        const int n = __builtin_amdgcn_readfirstlane(min(bn.cnt[t], kBinCap));
        if (n == 0) continue;
        const int ty = t / bn.TW, tx = t - ty * bn.TW;
        const int px = 8 * tx + lx, py = 8 * ty + ly;
        const int zi = py * P + px;
        typename Sink::Key best = zb.key_at(zi);
        const uint16_t *L = bn.list + t * kBinCap;
        for (int j = 0; j < n; ++j) {
            const int k = __builtin_amdgcn_readfirstlane((int)L[j]);
            const BinRec r = bn.rec[k];
            const int e0 = r.e0.z + mul24(r.e0.x, px) + mul24(r.e0.y, py);
            const int e1 = r.e1.z + mul24(r.e1.x, px) + mul24(r.e1.y, py);
            const int e2 = r.e2.z + mul24(r.e2.x, px) + mul24(r.e2.y, py);
            if (e0 >= r.e0.w && e1 >= r.e1.w && e2 >= r.e2.w) {
                const uint32_t D = frag_depth(e0, e1, e2, r.q.x, r.q.y, r.q.z);
                if (D < kFar) {
                    const typename Sink::Key key = Sink::make(D, __float_as_uint(r.q.w));
                    best = key < best ? key : best;
                }
            }
        }
        zb.set_key(zi, best);
    }
}

// Everything a wave needs to draw clusters of one (env, region) item.
struct Ctx {
    Cam cam;
    Proj pj;
    float kl, kr, kt, kb;
    int rx0, ry0, R;
    int P;           // z-buffer row pitch in LDS
    int *own;        // this wave's 64 words of LDS scratch (balanced raster)
    const uint32_t *planefront;   // bit per env face plane: camera strictly in front
    int small_max;   // bbox pixels: <= lane_max per lane, <= small_max balanced, else tiles
    int lane_max;
    BigRec *big;     // the workgroup's list of deferred large triangles
    int *nbig;
    bool binning;    // mid-sized triangles go to the 8x8-tile bins
    Bins bins;
};

// The record of one set-up triangle.
__device__ __forceinline__ BinRec bin_record(const Ctx &c, const Setup &S, uint32_t id)
{
    const int ex0 = S.x2 - S.x1, ey0 = S.y2 - S.y1;
    const int ex1 = S.x0 - S.x2, ey1 = S.y0 - S.y2;
    const int ex2 = S.x1 - S.x0, ey2 = S.y1 - S.y0;
    const int Px = 16 * c.rx0 + 8, Py = 16 * c.ry0 + 8;   // centre of the region's first pixel
    BinRec r;
    r.e0 = make_int4(-16 * ey0, 16 * ex0, mul24(ex0, Py - S.y1) - mul24(ey0, Px - S.x1), S.bias & 1);
    r.e1 = make_int4(-16 * ey1, 16 * ex1, mul24(ex1, Py - S.y2) - mul24(ey1, Px - S.x2), (S.bias >> 1) & 1);
    r.e2 = make_int4(-16 * ey2, 16 * ex2, mul24(ex2, Py - S.y0) - mul24(ey2, Px - S.x0), (S.bias >> 2) & 1);
    r.q = make_float4(S.q0, S.q1, S.q2, __uint_as_float(id));
    return r;
}

// Bin the wave's mid-sized triangles (lanes with `bal`): one record each,
// then each lane lists its record under every tile of its bbox that can hold
// one of its pixels.  Clears `bal` for the triangles binned whole; the others
// (record buffer or a tile's list full) stay with the caller, which draws
// them itself.  (Listing tile by tile over the union of the wave's ranges,
// one atomic per tile and wave, measured slower: the unions are wide.)
__device__ __forceinline__ void bin_wave(const Ctx &c, const Setup &S, uint32_t id, int lane, bool &bal)
{
    const uint64_t mm = __ballot(bal);
    if (!mm) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(c.bins.ntri, __popcll(mm));
    base = __builtin_amdgcn_readlane(base, 0);
    const int slot = base + __popcll(mm & ((1ull << lane) - 1ull));
    if (!bal || slot >= kBinTris) return;
    const BinRec r = bin_record(c, S, id);
    c.bins.rec[slot] = r;
    const int tx0 = (S.px0 - c.rx0) >> 3, tx1 = (S.px1 - c.rx0) >> 3;
    const int ty0 = (S.py0 - c.ry0) >> 3, ty1 = (S.py1 - c.ry0) >> 3;
    bool full = false;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            if (!(tile_live(r.e0, tx, ty) && tile_live(r.e1, tx, ty) && tile_live(r.e2, tx, ty))) continue;
            const int t = ty * c.bins.TW + tx;
            const int pos = atomicAdd(&c.bins.cnt[t], 1);
            if (pos < kBinCap) c.bins.list[t * kBinCap + pos] = (uint16_t)slot;
            else full = true;
        }
    if (!full) bal = false;
}

// One cluster's per-lane inputs: lane l holds vertex l and triangle l.
struct ClusterData {
    float vx, vy, vz;
    uint32_t packed;
    int nv, nt;
    uint32_t first;   // env-local index of the cluster's first triangle
    uint32_t p01, p23; // face-plane indices p0 | p1 << 16, p2 | p3 << 16
};

// Loads of cluster ci: its counts and first triangle (record word 8..9) and
// its 64 vertex and triangle slots, addressed from ci alone so that all of
// them are in flight at once; the counts only mask lanes later.
__device__ __forceinline__ void fetch_cluster(const RenderMesh &m, uint64_t ci, int lane, ClusterData &d)
{
    const uint4 cf = *reinterpret_cast<const uint4 *>(&m.clusters[ci * 3 + 2]);
    const size_t slot = (size_t)ci * kClusterVerts + lane;
    d.vx = m.cverts[slot * 3 + 0];
    d.vy = m.cverts[slot * 3 + 1];
    d.vz = m.cverts[slot * 3 + 2];
    d.packed = m.ctris[slot];
    d.nv = (int)(cf.x & 0xFF);
    d.nt = (int)((cf.x >> 8) & 0xFF);
    d.first = cf.y;
    d.p01 = cf.z;
    d.p23 = cf.w;
}

// Movable objects drawn where they are: a box per object, its 8 corners
// F_o (+-e0, +-e1, +-e2) (bit 0 of the corner index = x, 1 = y, 2 = z) and 12
// triangles wound counter-clockwise around the outward normals, numbered
// after the env's mesh triangles (12 per object, in object order), with no
// face plane.  Four objects (32 vertices, 48 triangles) make one cluster.
__device__ __forceinline__ void object_cluster(const RenderMesh &m, int env, int cidx, int lane,
                                               uint32_t first_id, ClusterData &d)
{
    const int O = m.num_objects;
    const int nobj = min(4, O - 4 * cidx);
    d.nv = 8 * nobj;
    d.nt = 12 * nobj;
    d.first = first_id + 48u * (uint32_t)cidx;
    d.p01 = kNoPlane | (kNoPlane << 16);
    d.p23 = d.p01;
    d.vx = d.vy = d.vz = 0.0f;
    d.packed = 0u;
    if (lane < d.nv) {
        const int o = 4 * cidx + (lane >> 3), k = lane & 7;
        const float *e = m.obj_rec + ((size_t)env * O + o) * 8 + 3;
        const float *F = m.obj_frames + ((size_t)env * O + o) * 12;
        const float px = (k & 1) ? e[0] : -e[0];
        const float py = (k & 2) ? e[1] : -e[1];
        const float pz = (k & 4) ? e[2] : -e[2];
        d.vx = ((F[0] * px + F[1] * py) + F[2] * pz) + F[3];
        d.vy = ((F[4] * px + F[5] * py) + F[6] * pz) + F[7];
        d.vz = ((F[8] * px + F[9] * py) + F[10] * pz) + F[11];
    }
    if (lane < d.nt) {
        // faces -x, +x, -y, +y, -z, +z as corner quads, two triangles each
        const int ol = lane / 12, f2 = lane - 12 * ol;
        const int face = f2 >> 1;
        // corner quads (a, b, c, d) of the six faces
        const int q[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
        int a = q[0][0], b = q[0][1], c = q[0][2], dd = q[0][3];
#pragma unroll
        for (int f = 1; f < 6; ++f)
            if (face == f) { a = q[f][0]; b = q[f][1]; c = q[f][2]; dd = q[f][3]; }
        const int i0 = 8 * ol + a;
        const int i1 = 8 * ol + ((f2 & 1) ? c : b);
        const int i2 = 8 * ol + ((f2 & 1) ? dd : c);
        d.packed = (uint32_t)i0 | ((uint32_t)i1 << 8) | ((uint32_t)i2 << 16);
    }
}

// The robot's links drawn where they are: link l's box has centre c_l and
// half extents h_l in link frame l, corner k = F_l (c_l + (+-h_l)) (bit 0 of
// k = x, 1 = y, 2 = z; the sum in FP32 before the frame product), the same
// 12 triangles per box as the objects, numbered from first_id in link order,
// with no face plane.  Four links (32 vertices, 48 triangles) make one
// cluster, two clusters per env.
__device__ __forceinline__ void link_cluster(const RenderMesh &m, int env, int cidx, int lane,
                                             uint32_t first_id, ClusterData &d)
{
    d.nv = 32;
    d.nt = 48;
    d.first = first_id + 48u * (uint32_t)cidx;
    d.p01 = kNoPlane | (kNoPlane << 16);
    d.p23 = d.p01;
    d.vx = d.vy = d.vz = 0.0f;
    d.packed = 0u;
    if (lane < 32) {
        const int l = 4 * cidx + (lane >> 3), k = lane & 7;
        const float *c = m.link_box + 6 * l, *h = c + 3;
        const float *F = m.link_frames + ((size_t)env * 8 + l) * 12;
        const float px = c[0] + ((k & 1) ? h[0] : -h[0]);
        const float py = c[1] + ((k & 2) ? h[1] : -h[1]);
        const float pz = c[2] + ((k & 4) ? h[2] : -h[2]);
        d.vx = ((F[0] * px + F[1] * py) + F[2] * pz) + F[3];
        d.vy = ((F[4] * px + F[5] * py) + F[6] * pz) + F[7];
        d.vz = ((F[8] * px + F[9] * py) + F[10] * pz) + F[11];
    }
    if (lane < 48) {
        const int ol = lane / 12, f2 = lane - 12 * ol;
        const int face = f2 >> 1;
        const int q[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
        int a = q[0][0], b = q[0][1], c = q[0][2], dd = q[0][3];
#pragma unroll
        for (int f = 1; f < 6; ++f)
            if (face == f) { a = q[f][0]; b = q[f][1]; c = q[f][2]; dd = q[f][3]; }
        const int i0 = 8 * ol + a;
        const int i1 = 8 * ol + ((f2 & 1) ? c : b);
        const int i2 = 8 * ol + ((f2 & 1) ? dd : c);
        d.packed = (uint32_t)i0 | ((uint32_t)i1 << 8) | ((uint32_t)i2 << 16);
    }
}

// Lit, textured colour of one pixel (a stand-in for baked textures and
// lighting), from its D24 depth D, its pixel (X, Y) in a res x res image, the
// env camera (position, right, down, forward), the winning triangle's outward
// unit normal n and flat colour: the world point along the pixel-centre ray at
// the depth's distance, Lambert from the light (0.36, 0.48, 0.8) over 0.35
// ambient, a 0.25 m world checker (0.8 on odd squares) on the two axes other
// than n's largest component; FP32, no contraction.
__device__ __forceinline__ void shade_pixel(uint32_t D, int X, int Y, int res, const float *cam,
                                            const RasterParams &rp, float n0, float n1, float n2, uint8_t &r,
                                            uint8_t &g, uint8_t &b)
{
    const float invk = 1.0f / rp.kd;
    const float invz = rp.invn - (float)D * invk;
    const float z = 1.0f / invz;
    const float hw = (float)res * 0.5f;
    const float u = (((float)X + 0.5f) - hw) / hw;
    const float v = (((float)Y + 0.5f) - hw) / hw;
    float P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = cam[i] + z * ((cam[9 + i] + u * cam[3 + i]) + v * cam[6 + i]);
    const float ndl = (n0 * 0.36f + n1 * 0.48f) + n2 * 0.8f;
    const float s = 0.35f + 0.65f * (ndl > 0.0f ? ndl : 0.0f);
    const float a0 = fabsf(n0), a1 = fabsf(n1), a2 = fabsf(n2);
    float ta, tb;
    if (a2 >= a0 && a2 >= a1) {
        ta = P[0];
        tb = P[1];
    } else if (a0 >= a1) {
        ta = P[1];
        tb = P[2];
    } else {
        ta = P[0];
        tb = P[2];
    }
    const int ia = (int)floorf(ta * 4.0f), ib = (int)floorf(tb * 4.0f);
    const float t = ((ia + ib) & 1) ? 0.8f : 1.0f;
    const float f = s * t;
    const float vr = floorf((float)r * f + 0.5f), vg = floorf((float)g * f + 0.5f), vb = floorf((float)b * f + 0.5f);
    r = (uint8_t)(vr >= 255.0f ? 255.0f : vr);
    g = (uint8_t)(vg >= 255.0f ? 255.0f : vg);
    b = (uint8_t)(vb >= 255.0f ? 255.0f : vb);
}

// Work counters (debug / roofline accounting), summed per wave.
enum {
    kStatBatchClusters = 0,  // clusters tested against the frustum
    kStatFrustumVisible,     // ... inside it
    kStatOccluded,           // ... and then proven hidden
    kStatDrawn,              // clusters drawn
    kStatTrisValid,          // triangles surviving trivial rejection
    kStatTrisClipped,        // ... of which clipped
    kStatTrisSetup,          // front-facing (sub)triangles with pixels in the region
    kStatCandPixels,         // their bbox pixels
    kNumStats
};

__device__ __forceinline__ void stat_add(unsigned long long *stats, int k, int lane, uint64_t v)
{
    if (stats && lane == 0 && v) atomicAdd(&stats[k], (unsigned long long)v);
}

// Draw one cluster.
template <bool kBin, class Sink>
__device__ void draw_cluster(const Ctx &c, const ClusterData &d, int lane, const Sink &zb,
                             unsigned long long *stats)
{
    const uint32_t myid = d.first + (uint32_t)lane;
    const Cam &cam = c.cam;
    const int nv = d.nv, nt = d.nt;

    // ---- per vertex: camera space, outcodes, projection
    float X = 0.f, Y = 0.f, Z = 1.f;
    uint32_t oc = 0;
    int xi = 0, yi = 0;
    float dv = 0.f;
    if (lane < nv) {
        const float ddx = d.vx - cam.px, ddy = d.vy - cam.py, ddz = d.vz - cam.pz;
        X = (cam.rx * ddx + cam.ry * ddy) + cam.rz * ddz;
        Y = (cam.dx * ddx + cam.dy * ddy) + cam.dz * ddz;
        Z = (cam.fx * ddx + cam.fy * ddy) + cam.fz * ddz;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            if (clip_plane(X, Y, Z, k, c.pj.near_m) < 0.0f) oc |= 1u << k;
        if (X - c.kl * Z < 0.0f) oc |= 1u << 5;
        if (c.kr * Z - X < 0.0f) oc |= 1u << 6;
        if (Y - c.kt * Z < 0.0f) oc |= 1u << 7;
        if (c.kb * Z - Y < 0.0f) oc |= 1u << 8;
        if ((oc & 1u) == 0) project(c.pj, X, Y, Z, xi, yi, dv);
    }

    // ---- per triangle
    const uint32_t packed = d.packed;
    const int i0 = (int)(packed & 0xFF), i1 = (int)((packed >> 8) & 0xFF),
              i2 = (int)((packed >> 16) & 0xFF);
    const uint32_t o0 = (uint32_t)__shfl((int)oc, i0, 64);
    const uint32_t o1 = (uint32_t)__shfl((int)oc, i1, 64);
    const uint32_t o2 = (uint32_t)__shfl((int)oc, i2, 64);
    // face plane of this triangle (its slot among the cluster's four)
    const uint32_t pslot = (packed >> 24) & 3u;
    const uint32_t pidx = ((pslot & 2u) ? d.p23 : d.p01) >> (16u * (pslot & 1u)) & 0xFFFFu;
    const bool valid = lane < nt && (o0 & o1 & o2) == 0u && plane_front(c.planefront, pidx);
    const bool allin = valid && ((o0 | o1 | o2) & kClipBits) == 0u;
    const bool clipped = valid && !allin;
    const uint64_t vmask = __ballot(valid);
    if (!vmask) return;
    const uint64_t cmask = __ballot(clipped);
    stat_add(stats, kStatTrisValid, lane, __popcll(vmask));
    stat_add(stats, kStatTrisClipped, lane, __popcll(cmask));
    const int vx0 = __shfl(xi, i0, 64), vy0 = __shfl(yi, i0, 64);
    const int vx1 = __shfl(xi, i1, 64), vy1 = __shfl(yi, i1, 64);
    const int vx2 = __shfl(xi, i2, 64), vy2 = __shfl(yi, i2, 64);
    const float vd0 = __shfl(dv, i0, 64), vd1 = __shfl(dv, i1, 64), vd2 = __shfl(dv, i2, 64);

    int nsub = allin ? 1 : 0;
    Poly poly;
    poly.n = 0;
    if (cmask) {
        const float X0 = __shfl(X, i0, 64), Y0 = __shfl(Y, i0, 64), Z0 = __shfl(Z, i0, 64);
        const float X1 = __shfl(X, i1, 64), Y1 = __shfl(Y, i1, 64), Z1 = __shfl(Z, i1, 64);
        const float X2 = __shfl(X, i2, 64), Y2 = __shfl(Y, i2, 64), Z2 = __shfl(Z, i2, 64);
        if (clipped) {
            poly.n = 3;
            poly.X[0] = X0; poly.Y[0] = Y0; poly.Z[0] = Z0;
            poly.X[1] = X1; poly.Y[1] = Y1; poly.Z[1] = Z1;
            poly.X[2] = X2; poly.Y[2] = Y2; poly.Z[2] = Z2;
            clip_polygon(poly, c.pj.near_m);
            nsub = poly.n >= 3 ? poly.n - 2 : 0;
        }
    }
    const int maxsub = cmask ? wave_max(nsub) : 1;
    for (int s = 0; s < maxsub; ++s) {
        Setup S = {};
        int ok = 0;
        if (s < nsub) {
            if (allin) {
                ok = setup_triangle(vx0, vy0, vd0, vx1, vy1, vd1, vx2, vy2, vd2, c.rx0, c.ry0, c.R, S);
            } else {
                int ax, ay, bx, by, cx2, cy2;
                float ad, bd, cd;
                project(c.pj, poly.X[0], poly.Y[0], poly.Z[0], ax, ay, ad);
                project(c.pj, poly.X[s + 1], poly.Y[s + 1], poly.Z[s + 1], bx, by, bd);
                project(c.pj, poly.X[s + 2], poly.Y[s + 2], poly.Z[s + 2], cx2, cy2, cd);
                ok = setup_triangle(ax, ay, ad, bx, by, bd, cx2, cy2, cd, c.rx0, c.ry0, c.R, S);
            }
        }
        bool big = false, bal = false;
        int npx = 0;
        if (ok) {
            npx = (S.px1 - S.px0 + 1) * (S.py1 - S.py0 + 1);
            if (npx <= c.lane_max) raster_small(S, myid, c.rx0, c.ry0, c.P, zb);
            else if (npx <= c.small_max) bal = true;
            else big = true;
        }
        if (stats) {
            stat_add(stats, kStatTrisSetup, lane, __popcll(__ballot(ok != 0)));
            const int tot = wave_incl_sum(npx, lane);
            stat_add(stats, kStatCandPixels, lane, (uint64_t)__builtin_amdgcn_readlane(tot, 63));
        }
        if (kBin && c.binning) bin_wave(c, S, myid, lane, bal);
        if (__ballot(bal)) raster_balanced(S, myid, bal, lane, c.rx0, c.ry0, c.P, c.own, zb);
        bool spill = false;
        if (big) {
            const int slot = atomicAdd(c.nbig, 1);
            if (slot < kBigCap) {
                BigRec &r = c.big[slot];
                r.xy0 = (S.x0 & 0xFFFF) | (S.y0 << 16);
                r.xy1 = (S.x1 & 0xFFFF) | (S.y1 << 16);
                r.xy2 = (S.x2 & 0xFFFF) | (S.y2 << 16);
                r.box = S.px0 | (S.px1 << 8) | (S.py0 << 16) | (S.py1 << 24);
                r.bias = S.bias;
                r.q0 = S.q0;
                r.q1 = S.q1;
                r.q2 = S.q2;
                r.id = myid;
            } else {
                spill = true;
            }
        }
        uint64_t bmask = __ballot(spill);
        while (bmask) {
            const int L = __ffsll((unsigned long long)bmask) - 1;
            bmask &= bmask - 1;
            const TriRec t = lane_record(S, myid, L);
            raster_tiles(t, t.py0 >> 3, t.py1 >> 3, lane, c.ry0, c.rx0, c.P, zb);
        }
    }
}

// Every wave of the workgroup draws the deferred large triangles, groups of
// four tile rows at a time, then the list is emptied (called by the whole
// workgroup right after a barrier).
template <class Sink>
__device__ __forceinline__ void drain_big(BigRec *big, int *nbig, int *gofs, int wave, int nwaves,
                                          int lane, int rx0, int ry0, int P, const Sink &zb)
{
    const int n = min(*nbig, kBigCap);
    if (n == 0) return;
    if (wave == 0) {
        int ng = 0;
        if (lane < n) {
            const int box = big[lane].box;
            ng = ((((box >> 24) & 0xFF) >> 3) - (((box >> 16) & 0xFF) >> 3) + 4) >> 2;
        }
        const int incl = wave_incl_sum(ng, lane);
        if (lane < n) gofs[lane + 1] = incl;
        if (lane == 0) gofs[0] = 0;
    }
    __syncthreads();
    const int G = gofs[n];
    for (int g = wave; g < G; g += nwaves) {
        int k = 0;
        while (gofs[k + 1] <= g) ++k;
        const TriRec t = unpack_big(big[k]);
        const int ty = (t.py0 >> 3) + 4 * (g - gofs[k]);
        raster_tiles(t, ty, min(ty + 3, t.py1 >> 3), lane, ry0, rx0, P, zb);
    }
    __syncthreads();
    if (threadIdx.x == 0) *nbig = 0;
    __syncthreads();
}

// LDS of one workgroup besides the z-buffer.
template <int kBlock>
struct ItemShared {
    uint32_t tilemax[(kMaxRegion / 8) * (kMaxRegion / 8)];
    uint32_t blockmax[(kMaxRegion / 32) * (kMaxRegion / 32)];
    uint16_t vis[kVisCap];
    int wave_cnt[kBlock / 64];
    int wave_cnt2[2][kBlock / 64];   // per wave, the two halves of a frustum compaction pass
    int own[kBlock];   // 64 words per wave, balanced raster
    RegionPlanes rplanes;   // the item's region frustum in world space
    uint32_t planefront[kMaxPlanes / 32];   // camera strictly in front of face plane p
    BigRec big[kBigCap];
    int big_gofs[kBigCap + 1];
    int nbig;
    int next;
    int queue_item;
};

// Render one (env, region) work item into the depth (and colour) output.
template <int kBlock, bool kColor, bool kBin>
__device__ __forceinline__ void raster_item(const RenderMesh &m, const RasterParams &rp,
                                            const float *__restrict__ camera,
                                            const int32_t *__restrict__ env_res,
                                            const uint64_t *__restrict__ env_depth_off,
                                            uint32_t item, uint32_t *__restrict__ depth,
                                            uint8_t *__restrict__ rgb, unsigned long long *zdyn,
                                            ItemShared<kBlock> &sh)
{
    using SinkT = typename std::conditional<kColor, ColorSink, DepthSink>::type;
    SinkT zb;
    if constexpr (kColor) zb.k = zdyn;
    else zb.z = reinterpret_cast<uint32_t *>(zdyn);
    uint32_t *tilemax = sh.tilemax;
    uint32_t *blockmax = sh.blockmax;
    uint16_t *vis = sh.vis;
    int *wave_cnt = sh.wave_cnt;
    int &next = sh.next;
    constexpr int kWaves = kBlock / 64;
    const int env = (int)(item & 0xFFFFFu);
    const int reg = (int)((item >> 20) & 0x7FFu);
    const int res = env_res[env];
    Ctx c;
    c.R = min(res, rp.region) >> (item >> 31);
    const int nr = res / c.R;
    c.rx0 = (reg % nr) * c.R;
    c.ry0 = (reg / nr) * c.R;
    c.P = zpitch(c.R);
    c.own = sh.own + (threadIdx.x & ~63);
    c.big = sh.big;
    c.nbig = &sh.nbig;
    if (threadIdx.x == 0) sh.nbig = 0;
    c.planefront = sh.planefront;
    c.small_max = rp.small_max;
    c.lane_max = rp.lane_max;
    c.binning = false;   // objects and links are drawn directly
    const int R = c.R;
    if (kBin) {
        unsigned char *after = reinterpret_cast<unsigned char *>(zdyn) + (size_t)R * c.P * (kColor ? 8 : 4);
        const int TW = R >> 3;
        c.bins.rec = reinterpret_cast<BinRec *>(after);
        c.bins.cnt = reinterpret_cast<int *>(after + sizeof(BinRec) * kBinTris);
        c.bins.list = reinterpret_cast<uint16_t *>(c.bins.cnt + TW * TW);
        c.bins.ntri = reinterpret_cast<int *>(c.bins.list + (size_t)TW * TW * kBinCap);
        c.bins.TW = TW;
        for (int i = threadIdx.x; i < TW * TW; i += kBlock) c.bins.cnt[i] = 0;
        if (threadIdx.x == 0) *c.bins.ntri = 0;
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    Occl oc;
    oc.tilemax = tilemax;
    oc.blockmax = blockmax;
    oc.TW = (R + 7) >> 3;
    oc.BW = (R + 31) >> 5;
    oc.P = c.P;

    if constexpr (kColor) {
        for (int i = threadIdx.x; i < R * c.P; i += kBlock) zb.clear(i);
    } else {
        // 16-byte stores (R P is a multiple of 4 words, the buffer 16-byte aligned)
        uint4 *z4 = reinterpret_cast<uint4 *>(zdyn);
        for (int i = threadIdx.x; i < (R * c.P) >> 2; i += kBlock) z4[i] = make_uint4(kFar, kFar, kFar, kFar);
    }
    for (int i = threadIdx.x; i < oc.TW * oc.TW; i += kBlock) tilemax[i] = kFar;
    for (int i = threadIdx.x; i < oc.BW * oc.BW; i += kBlock) blockmax[i] = kFar;

    {
        const float *cp = camera + (size_t)env * 12;
        c.cam.px = cp[0]; c.cam.py = cp[1]; c.cam.pz = cp[2];
        c.cam.rx = cp[3]; c.cam.ry = cp[4]; c.cam.rz = cp[5];
        c.cam.dx = cp[6]; c.cam.dy = cp[7]; c.cam.dz = cp[8];
        c.cam.fx = cp[9]; c.cam.fy = cp[10]; c.cam.fz = cp[11];
    }
    const Cam &cam = c.cam;
    c.pj.hw = (float)res * 0.5f;
    c.pj.near_m = rp.near_m;
    c.pj.invn = rp.invn;
    c.pj.kd = rp.kd;
    // region side planes in normalised device units: x_ndc in [kl, kr]
    c.kl = ((float)c.rx0 - c.pj.hw) / c.pj.hw;
    c.kr = ((float)(c.rx0 + R) - c.pj.hw) / c.pj.hw;
    c.kt = ((float)c.ry0 - c.pj.hw) / c.pj.hw;
    c.kb = ((float)(c.ry0 + R) - c.pj.hw) / c.pj.hw;
    // the region's frustum planes, the same for every thread: kept in LDS (the
    // compaction passes read them; registers are the persistent kernel's
    // scarce resource)
    RegionPlanes &P = sh.rplanes;
    if (threadIdx.x == 0) {
        // camera-space plane  a*X + b*Y + c*Z + e >= 0  ->  world normal, offset
        const float pa[5][4] = {{0.f, 0.f, 1.f, -c.pj.near_m},
                                {1.f, 0.f, -c.kl, 0.f},
                                {-1.f, 0.f, c.kr, 0.f},
                                {0.f, 1.f, -c.kt, 0.f},
                                {0.f, -1.f, c.kb, 0.f}};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const float nx = pa[k][0] * cam.rx + pa[k][1] * cam.dx + pa[k][2] * cam.fx;
            const float ny = pa[k][0] * cam.ry + pa[k][1] * cam.dy + pa[k][2] * cam.fy;
            const float nz = pa[k][0] * cam.rz + pa[k][1] * cam.dz + pa[k][2] * cam.fz;
            P.n[k][0] = nx;
            P.n[k][1] = ny;
            P.n[k][2] = nz;
            P.off[k] = pa[k][3] - (nx * cam.px + ny * cam.py + nz * cam.pz);
        }
    }
    __syncthreads();

    // ---- the env's face planes the camera is strictly in front of, one bit
    // each ((n0 c0 + n1 c1) + n2 c2 - w > 0 at the camera position c)
    {
        const uint64_t pb = m.env_plane_off[env];
        const int np = (int)(m.env_plane_off[env + 1] - pb);
        for (int base = wave * 64; base < np; base += kBlock) {
            const int k = base + lane;
            bool front = false;
            if (k < np) {
                const float4 pl = m.planes[pb + k];
                const float side = ((pl.x * cam.px + pl.y * cam.py) + pl.z * cam.pz) - pl.w;
                front = side > 0.0f;
            }
            const uint64_t bm = __ballot(front);
            if (lane == 0) {
                sh.planefront[base >> 5] = (uint32_t)bm;
                sh.planefront[(base >> 5) + 1] = (uint32_t)(bm >> 32);
            }
        }
    }
    __syncthreads();

    const uint64_t c0 = m.env_cluster_off[env], c1 = m.env_cluster_off[env + 1];
    unsigned long long *stats = rp.stats;
    // ---- the movable objects first (one wave per four objects)
    if (m.obj_frames) {
        const int nc = (m.num_objects + 3) / 4;
        const uint32_t first_id = (uint32_t)(m.env_tri_off[env + 1] - m.env_tri_off[env]);
        for (int cidx = wave; cidx < nc; cidx += kWaves) {
            ClusterData cd;
            object_cluster(m, env, cidx, lane, first_id, cd);
            draw_cluster<kBin>(c, cd, lane, zb, stats);
        }
    }
    // ---- the robot's links (four links per cluster, on the last two waves)
    if (m.link_frames && wave >= kWaves - 2) {
        const uint32_t first_id = (uint32_t)(m.env_tri_off[env + 1] - m.env_tri_off[env]) +
                                  (m.obj_frames ? 12u * (uint32_t)m.num_objects : 0u);
        ClusterData cd;
        link_cluster(m, env, kWaves - 1 - wave, lane, first_id, cd);
        draw_cluster<kBin>(c, cd, lane, zb, stats);
    }
    c.binning = kBin;
    // Clusters are processed in windows of up to kVisCap: the workgroup tests
    // a window against the region frustum and compacts the visible ones, in
    // mesh order, into an LDS list; waves then pull list entries one at a
    // time (LDS counter), prefetching the next while drawing the current, and
    // test each against the occlusion bounds just before drawing it.
    for (uint64_t wbase = c0; wbase < c1; wbase += kVisCap) {
        const int wn = (int)min((uint64_t)kVisCap, c1 - wbase);
        // ---- ordered compaction of the frustum-visible clusters
        // (two clusters per thread and pass, k and k + kBlock: both records in
        // flight together, one pair of barriers per 2 kBlock clusters)
        int vis_total = 0;
        for (int off = 0; off < wn; off += 2 * kBlock) {
            bool fr[2];
            uint64_t bm[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = off + h * kBlock + (int)threadIdx.x;
                fr[h] = false;
                if (k < wn) {
                    const uint64_t ci = wbase + k;
                    const float4 w0 = m.clusters[ci * 3 + 0];
                    const float4 w1 = m.clusters[ci * 3 + 1];
                    const uint4 w2 = *reinterpret_cast<const uint4 *>(&m.clusters[ci * 3 + 2]);
                    fr[h] = aabb_visible(P, w0.x, w0.y, w0.z, w1.x, w1.y, w1.z) &&
                            any_plane_front(sh.planefront, w2.z, w2.w);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                bm[h] = __ballot(fr[h]);
                if (lane == 0) sh.wave_cnt2[h][wave] = __popcll(bm[h]);
            }
            __syncthreads();
            int before0 = vis_total, all0 = vis_total;
            for (int w = 0; w < kWaves; ++w) {
                if (w < wave) before0 += sh.wave_cnt2[0][w];
                all0 += sh.wave_cnt2[0][w];
            }
            int before1 = all0, all1 = all0;
            for (int w = 0; w < kWaves; ++w) {
                if (w < wave) before1 += sh.wave_cnt2[1][w];
                all1 += sh.wave_cnt2[1][w];
            }
            const uint64_t below = (1ull << lane) - 1ull;
            if (fr[0]) vis[before0 + __popcll(bm[0] & below)] = (uint16_t)(off + (int)threadIdx.x);
            if (fr[1]) vis[before1 + __popcll(bm[1] & below)] = (uint16_t)(off + kBlock + (int)threadIdx.x);
            __syncthreads();
            vis_total = all1;
        }
        if (stats) {
            if (threadIdx.x == 0) {
                atomicAdd(&stats[kStatBatchClusters], (unsigned long long)wn);
                atomicAdd(&stats[kStatFrustumVisible], (unsigned long long)vis_total);
            }
        }
        // ---- draw in rounds: without occlusion culling one round of every
        // visible cluster; with it, the prologue first (the mesh order puts
        // the large occluders early), then after each refresh of the bounds
        // the remaining clusters are re-tested lane-parallel, the survivors
        // compacted in order, and half of them (at least 64) drawn, until
        // `refresh` refreshes have been spent and the rest is drawn
        int drawn = 0, hidden = 0;
        int pos = 0, V = vis_total, rounds = 0;
        int end = rp.occlusion ? min(V, rp.prologue) : V;
        for (;;) {
            if (threadIdx.x == 0) next = pos;
            __syncthreads();
            int idx = 0;
            if (lane == 0) idx = atomicAdd(&next, 1);
            idx = __builtin_amdgcn_readfirstlane(idx);
            ClusterData cd;
            if (idx < end) fetch_cluster(m, wbase + vis[idx], lane, cd);
            // with bins: sub-rounds that end when the record buffer is nearly
            // full; the cluster a wave has fetched waits for the next one
            for (;;) {
                while (idx < end) {
                    int nidx = 0;
                    if (lane == 0) nidx = atomicAdd(&next, 1);
                    nidx = __builtin_amdgcn_readfirstlane(nidx);
                    ClusterData nd;
                    if (nidx < end) fetch_cluster(m, wbase + vis[nidx], lane, nd);
                    draw_cluster<kBin>(c, cd, lane, zb, stats);
                    ++drawn;
                    idx = nidx;
                    cd = nd;
                    if (kBin && __builtin_amdgcn_readfirstlane(*(volatile int *)c.bins.ntri) > kBinTris - 64)
                        break;
                }
                __syncthreads();
                if (kBin) {
                    flush_bins(c.bins, wave, kWaves, lane, c.P, zb);
                    __syncthreads();
                }
                drain_big(sh.big, &sh.nbig, sh.big_gofs, wave, kWaves, lane, c.rx0, c.ry0, c.P, zb);
                if (!kBin) break;
                for (int i = threadIdx.x; i < c.bins.TW * c.bins.TW; i += kBlock) c.bins.cnt[i] = 0;
                if (threadIdx.x == 0) *c.bins.ntri = 0;
                if (!__syncthreads_or(idx < end)) break;
            }
            pos = end;
            if (pos >= V) break;
            refresh_bounds(zb, oc, R, wave, kWaves, lane);
            // re-test vis[pos, V) against the fresh bounds, compacting in place
            int kept = 0;
            for (int base = pos; base < V; base += kBlock) {
                const int k = base + (int)threadIdx.x;
                bool keep = false;
                uint16_t v = 0;
                if (k < V) {
                    v = vis[k];
                    const uint64_t ci = wbase + v;
                    const float4 w0 = m.clusters[ci * 3 + 0];
                    const float4 w1 = m.clusters[ci * 3 + 1];
                    keep = !cluster_hidden(cam, c.pj, oc, c.rx0, c.ry0, R, w0.x, w0.y, w0.z, w1.x, w1.y,
                                           w1.z);
                }
                const uint64_t bm = __ballot(keep);
                if (lane == 0) wave_cnt[wave] = __popcll(bm);
                __syncthreads();
                int before = pos + kept;
                for (int w = 0; w < wave; ++w) before += wave_cnt[w];
                int all = kept;
                for (int w = 0; w < kWaves; ++w) all += wave_cnt[w];
                if (keep) vis[before + __popcll(bm & ((1ull << lane) - 1ull))] = v;
                __syncthreads();
                kept = all;
            }
            hidden += (threadIdx.x == 0) ? (V - pos - kept) : 0;
            V = pos + kept;
            ++rounds;
            end = rounds >= rp.refresh ? V : min(V, pos + max(64, (V - pos + 1) / 2));
        }
        if (stats) {
            if (threadIdx.x == 0 && hidden) atomicAdd(&stats[kStatOccluded], (unsigned long long)hidden);
            stat_add(stats, kStatDrawn, lane, (uint64_t)drawn);
        }
        __syncthreads();
    }
    __syncthreads();
    const uint64_t doff = env_depth_off[env];
    uint32_t *dst = depth + doff;
    if constexpr (!kColor) {
        // depth only: four pixels of a row per thread, one 16-byte LDS read and
        // one 16-byte store each (R, the pitch and res are multiples of 8, the
        // region origin a multiple of R); a thread keeps its column
        const int tw = R >> 2;
        const int rows_per_pass = kBlock / tw;
        const int x = ((int)threadIdx.x % tw) * 4;
        const uint32_t *z = reinterpret_cast<const uint32_t *>(zdyn);
        if ((int)threadIdx.x < rows_per_pass * tw) {
            for (int y = (int)threadIdx.x / tw; y < R; y += rows_per_pass) {
                const uint4 v = *reinterpret_cast<const uint4 *>(z + y * c.P + x);
                *reinterpret_cast<uint4 *>(dst + (size_t)(c.ry0 + y) * res + (c.rx0 + x)) = v;
            }
        }
    }
    for (int i = threadIdx.x; kColor && i < R * R; i += kBlock) {
        const int y = i / R, x = i - y * R;
        const size_t o = (size_t)(c.ry0 + y) * res + (c.rx0 + x);
        const int zi = y * c.P + x;
        if constexpr (kColor) {
            const unsigned long long key = zdyn[zi];
            const uint32_t D = (uint32_t)(key >> 32);
            dst[o] = D;
            if (rgb) {
                uint8_t r = 0, g = 0, bch = 0;
                if (D < kFar) {
                    const uint64_t id = key & 0xFFFFFFFFull;
                    const uint64_t ntri = m.env_tri_off[env + 1] - m.env_tri_off[env];
                    const uint64_t nobj = m.obj_frames ? 12ull * (uint64_t)m.num_objects : 0ull;
                    const uint8_t *cc = id < ntri          ? m.tri_rgb + (m.env_tri_off[env] + id) * 3
                                        : id < ntri + nobj ? m.obj_rgb + ((size_t)env * m.num_objects + (id - ntri) / 12) * 3
                                                           : m.link_rgb + ((id - ntri - nobj) / 12) * 3;
                    r = cc[0];
                    g = cc[1];
                    bch = cc[2];
                    if (m.tri_pidx) {
                        // lit, textured: the winner's outward normal (face
                        // plane, or the frame axis of a box face)
                        float n0, n1, n2;
                        if (id < ntri) {
                            const float4 pl = m.planes[m.env_plane_off[env] + m.tri_pidx[m.env_tri_off[env] + id]];
                            n0 = pl.x;
                            n1 = pl.y;
                            n2 = pl.z;
                        } else {
                            const float *F = id < ntri + nobj
                                                 ? m.obj_frames + ((size_t)env * m.num_objects + (id - ntri) / 12) * 12
                                                 : m.link_frames + ((size_t)env * 8 + (id - ntri - nobj) / 12) * 12;
                            const int face = (int)((id - ntri - (id < ntri + nobj ? 0 : nobj)) % 12) >> 1;
                            const int axis = face >> 1;
                            n0 = F[axis];
                            n1 = F[4 + axis];
                            n2 = F[8 + axis];
                            if (!(face & 1)) {
                                n0 = -n0;
                                n1 = -n1;
                                n2 = -n2;
                            }
                        }
                        shade_pixel(D, c.rx0 + x, c.ry0 + y, res, camera + (size_t)env * 12, rp, n0, n1, n2, r, g,
                                    bch);
                    }
                }
                uint8_t *px = rgb + (doff + o) * 3;
                px[0] = r;
                px[1] = g;
                px[2] = bch;
            }
        } else {
            dst[o] = zb.depth_at(zi);
        }
    }
    __syncthreads();   // the LDS is reused by the next item
}

// One workgroup per work item.
// Waves per SIMD the register allocation is sized for: 4 at 512 and 1024
// threads (two workgroups' or one workgroup's waves per CU); with bins a
// 512-thread workgroup's z-buffer and bins at the largest region leave LDS for
// one workgroup per CU, so its waves may use twice the registers.
template <int kBlock, bool kBin>
constexpr int raster_waves_per_eu()
{
    return kBlock >= 1024 ? 4 : kBlock >= 512 ? (kBin ? 2 : 4) : 2;
}

template <int kBlock, bool kColor, bool kBin>
__global__ __launch_bounds__(kBlock, (raster_waves_per_eu<kBlock, kBin>())) void k_raster(
    RenderMesh m, RasterParams rp, const float *__restrict__ camera,
    const int32_t *__restrict__ env_res, const uint64_t *__restrict__ env_depth_off,
    const uint32_t *__restrict__ work, int32_t num_work, uint32_t *__restrict__ queue,
    uint32_t *__restrict__ depth, uint8_t *__restrict__ rgb)
{
    extern __shared__ __attribute__((aligned(16))) unsigned long long zdyn[];
    __shared__ ItemShared<kBlock> sh;
    raster_item<kBlock, kColor, kBin>(m, rp, camera, env_res, env_depth_off, work[blockIdx.x], depth, rgb,
                                zdyn, sh);
}

// Persistent: as many workgroups as fit on the chip drain the work queue
// (items in longest-first order; the counter is reset by the robot kernel
// that precedes this launch in the step).
template <int kBlock, bool kColor, bool kBin>
__global__ __launch_bounds__(kBlock, (raster_waves_per_eu<kBlock, kBin>())) void k_raster_persistent(
    RenderMesh m, RasterParams rp, const float *__restrict__ camera,
    const int32_t *__restrict__ env_res, const uint64_t *__restrict__ env_depth_off,
    const uint32_t *__restrict__ work, int32_t num_work, uint32_t *__restrict__ queue,
    uint32_t *__restrict__ depth, uint8_t *__restrict__ rgb)
{
    extern __shared__ __attribute__((aligned(16))) unsigned long long zdyn[];
    __shared__ ItemShared<kBlock> sh;
    for (;;) {
        if (threadIdx.x == 0) sh.queue_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int i = sh.queue_item;
        __syncthreads();
        if (i >= num_work) break;
        // the queue position's work item (static order: the position itself)
        int idx = i;
        if (rp.order && rp.item_order) {
            idx = (int)rp.item_order[i];
            if ((unsigned)idx >= (unsigned)num_work) idx = i;
        }
        const uint64_t t0 = wall_clock64();
        raster_item<kBlock, kColor, kBin>(m, rp, camera, env_res, env_depth_off, work[idx], depth, rgb, zdyn,
                                    sh);
        // the item's time, which orders the next step's queue (raster_item
        // ends with a barrier, so every wave is done)
        if (threadIdx.x == 0 && rp.item_cost) {
            const uint64_t dt = wall_clock64() - t0;
            rp.item_cost[idx] = (uint32_t)(dt < 0xFFFFFFFFull ? dt : 0xFFFFFFFFull);
        }
    }
}

template <bool kColor, bool kPersist, bool kBin>
hipError_t launch_raster_t(const RenderMesh &m, const RasterParams &rp, const float *camera,
                           const int32_t *env_res, const uint64_t *env_depth_off,
                           const uint32_t *work, int32_t num_work, uint32_t *queue,
                           uint32_t *depth, uint8_t *rgb, size_t lds, int grid, hipStream_t s)
{
    const int g = kPersist ? grid : num_work;
#define GAL_RASTER_LAUNCH(B)                                                                     \
    hipLaunchKernelGGL((kPersist ? k_raster_persistent<B, kColor, kBin> : k_raster<B, kColor, kBin>), dim3(g), \
                       dim3(B), lds, s, m, rp, camera, env_res, env_depth_off, work, num_work,     \
                       queue, depth, rgb)
    switch (rp.block) {
    case 256: GAL_RASTER_LAUNCH(256); break;
    case 1024: GAL_RASTER_LAUNCH(1024); break;
    default: GAL_RASTER_LAUNCH(512); break;
    }
#undef GAL_RASTER_LAUNCH
    return hipGetLastError();
}

size_t lds_bytes(int region, bool color, bool bin)
{
    return (size_t)region * zpitch(region) * (color ? 8 : 4) + (bin ? bin_bytes(region) : 0);
}

// LDS a workgroup of kernel f may use beside its static LDS (the device's
// per-workgroup limit, 160 KB on gfx950, less the kernel's own static LDS).
template <class K>
hipError_t lds_room(K f, size_t *room)
{
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, (const void *)f);
    if (e != hipSuccess) return e;
    int dev = 0, max_lds = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
    *room = (size_t)max_lds > fa.sharedSizeBytes ? (size_t)max_lds - fa.sharedSizeBytes : 0;
    return hipSuccess;
}

// The largest dynamic LDS any tuning asks of kernel f: the largest region's
// z-buffer (and bins, for the binned kernels), within the room there is.
template <class K>
hipError_t allow(K f, bool color, bool bin)
{
    size_t room = 0;
    hipError_t e = lds_room(f, &room);
    if (e != hipSuccess) return e;
    const size_t want = std::min(lds_bytes(kMaxRegion, color, bin), room);
    return hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want);
}

}  // namespace

hipError_t raster_prepare()
{
    hipError_t e = hipSuccess;
#define GAL_ALLOW(B, C)                                                                  \
    if ((e = allow(k_raster<B, C, false>, C, false)) != hipSuccess) return e;            \
    if ((e = allow(k_raster_persistent<B, C, false>, C, false)) != hipSuccess) return e; \
    if ((e = allow(k_raster<B, C, true>, C, true)) != hipSuccess) return e;              \
    if ((e = allow(k_raster_persistent<B, C, true>, C, true)) != hipSuccess) return e;
    GAL_ALLOW(256, false) GAL_ALLOW(512, false) GAL_ALLOW(1024, false)
    GAL_ALLOW(256, true) GAL_ALLOW(512, true) GAL_ALLOW(1024, true)
#undef GAL_ALLOW
    return e;
}

bool raster_fits(const RasterParams &rp, int max_region, bool color)
{
    const int R = max_region < rp.region ? max_region : rp.region;
    size_t room = 0, room2 = 0;
    hipError_t e = hipSuccess;
#define GAL_ROOM(B, C, BIN)                                                   \
    e = lds_room(k_raster<B, C, BIN>, &room);                                 \
    if (e == hipSuccess) e = lds_room(k_raster_persistent<B, C, BIN>, &room2)
#define GAL_ROOM_B(B)                                                         \
    if (color) {                                                              \
        if (rp.bin) { GAL_ROOM(B, true, true); } else { GAL_ROOM(B, true, false); } \
    } else {                                                                  \
        if (rp.bin) { GAL_ROOM(B, false, true); } else { GAL_ROOM(B, false, false); } \
    }
    switch (rp.block) {
    case 256: GAL_ROOM_B(256); break;
    case 1024: GAL_ROOM_B(1024); break;
    default: GAL_ROOM_B(512); break;
    }
#undef GAL_ROOM_B
#undef GAL_ROOM
    return e == hipSuccess && lds_bytes(R, color, rp.bin != 0) <= std::min(room, room2);
}

int raster_persistent_grid(const RasterParams &rp, int max_region, bool color)
{
    const int R = max_region < rp.region ? max_region : rp.region;
    const size_t lds = lds_bytes(R, color, rp.bin != 0);
    int per_cu = 0;
    hipError_t e = hipSuccess;
#define GAL_OCC(B)                                                                              \
    e = rp.bin ? (color ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raster_persistent<B, true, true>, B, lds) \
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raster_persistent<B, false, true>, B, lds)) \
               : (color ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raster_persistent<B, true, false>, B, lds) \
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raster_persistent<B, false, false>, B, lds))
    switch (rp.block) {
    case 256: GAL_OCC(256); break;
    case 1024: GAL_OCC(1024); break;
    default: GAL_OCC(512); break;
    }
#undef GAL_OCC
    int dev = 0, cus = 0;
    if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    return (per_cu < 1 ? 1 : per_cu) * cus;
}

hipError_t launch_raster(const RenderMesh &m, const RasterParams &rp, const float *camera,
                         const int32_t *env_res, const uint64_t *env_depth_off,
                         const uint32_t *work, int32_t num_work, int32_t max_region,
                         uint32_t *queue, int32_t persistent_grid, uint32_t *depth, uint8_t *rgb,
                         hipStream_t s)
{
    if (num_work <= 0) return hipSuccess;
    const int R = max_region < rp.region ? max_region : rp.region;
    const size_t lds = lds_bytes(R, rgb != nullptr, rp.bin != 0);
    const bool persist = rp.persistent && queue && persistent_grid > 0;
    const int grid = persist ? persistent_grid : 0;
#define GAL_RASTER_SELECT(C, P)                                                                         \
    return rp.bin ? launch_raster_t<C, P, true>(m, rp, camera, env_res, env_depth_off, work, num_work,   \
                                                queue, depth, rgb, lds, grid, s)                          \
                  : launch_raster_t<C, P, false>(m, rp, camera, env_res, env_depth_off, work, num_work,  \
                                                 queue, depth, rgb, lds, grid, s)
    if (rgb) {
        if (persist) GAL_RASTER_SELECT(true, true);
        GAL_RASTER_SELECT(true, false);
    }
    if (persist) GAL_RASTER_SELECT(false, true);
    GAL_RASTER_SELECT(false, false);
#undef GAL_RASTER_SELECT
}

}  // namespace gal
