// Depth rasteriser of the head camera (the per-env depth observation of
// Galactic, Section 4.1: 90 degree FoV; the paper's batch renderer is
// replaced by this fixed-point tile rasteriser).
//
// Semantics (identical, bit for bit, for any launch shape):
//  * camera space X = right.(v-p), Y = down.(v-p), Z = fwd.(v-p);
//  * trivial reject against the near plane Z = n and a guard band of half a
//    viewport per side (X + 2Z, 2Z - X, Y + 2Z, 2Z - Y >= 0); triangles that
//    straddle a plane are clipped (Sutherland-Hodgman, planes in that order,
//    each intersection computed from the endpoints in a canonical order) and
//    fan-triangulated;
//  * projection x = w/2 + (w/2) X/Z (focal length w/2 for 90 degrees),
//    snapped to 1/16 pixel; back faces and zero-area triangles are culled;
//  * coverage at pixel centres by integer edge functions with the top-left
//    rule; depth d = (1/n - 1/Z) (2^24-1)/(1/n - 1/f) per vertex,
//    interpolated as a plane in screen space, clamped and truncated to 24
//    bits; the image keeps the minimum (0xFFFFFF = nothing).
//
// Launch: one workgroup per (env, square region of <= 128x128 pixels); the
// region's z-buffer lives in LDS and is updated with ds_min_u32.  The env's
// mesh is stored as clusters of <= 64 consecutive triangles and <= 64 unique
// vertices with an AABB.  Each wave culls 64 clusters at a time against the
// region's frustum, then per cluster: lane = vertex (transform, outcodes,
// projection once per vertex), lane = triangle (gathers its vertices with
// ds_bpermute); triangles whose pixel bbox is small are rasterised by their
// own lane, large ones by the whole wave, one 8x8 tile (lane = pixel) at a
// time.  Every extra rejection (cluster AABB, region planes) only removes
// triangles that cannot cover a pixel centre of the region.
#include "gal_internal.h"

namespace gal {

namespace {

constexpr uint32_t kFar = 0xFFFFFFu;
constexpr uint32_t kClipBits = 0x1Fu;

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
// swap), depth plane, pixel bbox clipped to the region.
struct Setup {
    int x0, y0, x1, y1, x2, y2;
    int bias;                 // bit k set: edge k is not top-left (needs E >= 1)
    float d0, a, b;
    int px0, px1, py0, py1;
};

// Returns 0 = nothing to draw, 1 = drawable.
__device__ __forceinline__ int setup_triangle(int x0, int y0, float d0, int x1, int y1, float d1,
                                              int x2, int y2, float d2, int rx0, int ry0, int R,
                                              Setup &S)
{
    const int A2 = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
    if (A2 >= 0) return 0;   // back face or degenerate
    // front face: swap v1 and v2 so the signed area is positive
    S.x0 = x0; S.y0 = y0; S.d0 = d0;
    S.x1 = x2; S.y1 = y2;
    S.x2 = x1; S.y2 = y1;
    const float e1 = d2 - d0, e2 = d1 - d0;
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
    const float fx1 = (float)(S.x1 - S.x0), fy1 = (float)(S.y1 - S.y0);
    const float fx2 = (float)(S.x2 - S.x0), fy2 = (float)(S.y2 - S.y0);
    const float fA = (float)(-A2);
    S.a = (e1 * fy2 - e2 * fy1) / fA;
    S.b = (e2 * fx1 - e1 * fx2) / fA;
    return 1;
}

__device__ __forceinline__ void raster_small(const Setup &S, int rx0, int ry0, int R,
                                             uint32_t *zbuf)
{
    // edge k from vertex i to j: E = (xj-xi)(Py-yi) - (yj-yi)(Px-xi)
    const int ex0 = S.x2 - S.x1, ey0 = S.y2 - S.y1;
    const int ex1 = S.x0 - S.x2, ey1 = S.y0 - S.y2;
    const int ex2 = S.x1 - S.x0, ey2 = S.y1 - S.y0;
    const int b0 = S.bias & 1, b1 = (S.bias >> 1) & 1, b2 = (S.bias >> 2) & 1;
    const int Px0 = 16 * S.px0 + 8;
    int Py = 16 * S.py0 + 8;
    int r0 = ex0 * (Py - S.y1) - ey0 * (Px0 - S.x1);
    int r1 = ex1 * (Py - S.y2) - ey1 * (Px0 - S.x2);
    int r2 = ex2 * (Py - S.y0) - ey2 * (Px0 - S.x0);
    for (int py = S.py0; py <= S.py1; ++py, Py += 16) {
        int e0 = r0, e1 = r1, e2 = r2;
        int Px = Px0;
        for (int px = S.px0; px <= S.px1; ++px, Px += 16) {
            if (e0 >= b0 && e1 >= b1 && e2 >= b2) {
                const float dv = S.d0 + (S.a * (float)(Px - S.x0) + S.b * (float)(Py - S.y0));
                const uint32_t D = depth24(dv);
                if (D < kFar) atomicMin(&zbuf[(py - ry0) * R + (px - rx0)], D);
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

// The whole wave rasterises lane L's triangle, one 8x8 tile at a time.
__device__ __forceinline__ void raster_big(const Setup &S, int L, int lane, int rx0, int ry0,
                                           int R, uint32_t *zbuf)
{
    const int x0 = rl(S.x0, L), y0 = rl(S.y0, L);
    const int x1 = rl(S.x1, L), y1 = rl(S.y1, L);
    const int x2 = rl(S.x2, L), y2 = rl(S.y2, L);
    const int bias = rl(S.bias, L);
    const float d0 = rlf(S.d0, L), a = rlf(S.a, L), b = rlf(S.b, L);
    const int px0 = rl(S.px0, L), px1 = rl(S.px1, L);
    const int py0 = rl(S.py0, L), py1 = rl(S.py1, L);
    const int ex0 = x2 - x1, ey0 = y2 - y1;
    const int ex1 = x0 - x2, ey1 = y0 - y2;
    const int ex2 = x1 - x0, ey2 = y1 - y0;
    const int b0 = bias & 1, b1 = (bias >> 1) & 1, b2 = (bias >> 2) & 1;
    const int lx = lane & 7, ly = lane >> 3;
    for (int ty = py0 >> 3; ty <= (py1 >> 3); ++ty) {
        const int py = ty * 8 + ly;
        const int Py = 16 * py + 8;
        for (int tx = px0 >> 3; tx <= (px1 >> 3); ++tx) {
            const int px = tx * 8 + lx;
            if (px < px0 || px > px1 || py < py0 || py > py1) continue;
            const int Px = 16 * px + 8;
            const int e0 = ex0 * (Py - y1) - ey0 * (Px - x1);
            const int e1 = ex1 * (Py - y2) - ey1 * (Px - x2);
            const int e2 = ex2 * (Py - y0) - ey2 * (Px - x0);
            if (e0 >= b0 && e1 >= b1 && e2 >= b2) {
                const float dv = d0 + (a * (float)(Px - x0) + b * (float)(Py - y0));
                const uint32_t D = depth24(dv);
                if (D < kFar) atomicMin(&zbuf[(py - ry0) * R + (px - rx0)], D);
            }
        }
    }
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return v;
}

// Conservative frustum test of a cluster AABB (world) against the near plane
// and the region's four side planes; margins cover float rounding.
struct RegionPlanes {
    // plane value = nx*(p-c).x + ... in camera terms; stored as world normals
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

template <int kBlock>
__global__ __launch_bounds__(kBlock) void k_raster(RenderMesh m, RasterParams rp,
                                                   const float *__restrict__ camera,
                                                   const int32_t *__restrict__ env_res,
                                                   const uint64_t *__restrict__ env_depth_off,
                                                   const uint32_t *__restrict__ work,
                                                   uint32_t *__restrict__ depth)
{
    __shared__ uint32_t zbuf[kMaxRegion * kMaxRegion];
    const uint32_t item = work[blockIdx.x];
    const int env = (int)(item & 0xFFFFFu);
    const int reg = (int)(item >> 20);
    const int res = env_res[env];
    const int R = min(res, rp.region);
    const int nr = res / R;
    const int rx0 = (reg % nr) * R, ry0 = (reg / nr) * R;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int kWaves = kBlock / 64;

    for (int i = threadIdx.x; i < R * R; i += kBlock) zbuf[i] = kFar;

    Cam cam;
    {
        const float *c = camera + (size_t)env * 12;
        cam.px = c[0]; cam.py = c[1]; cam.pz = c[2];
        cam.rx = c[3]; cam.ry = c[4]; cam.rz = c[5];
        cam.dx = c[6]; cam.dy = c[7]; cam.dz = c[8];
        cam.fx = c[9]; cam.fy = c[10]; cam.fz = c[11];
    }
    Proj pj;
    pj.hw = (float)res * 0.5f;
    pj.near_m = rp.near_m;
    pj.invn = rp.invn;
    pj.kd = rp.kd;
    // region side planes in normalised device units: x_ndc in [kl, kr]
    const float kl = ((float)rx0 - pj.hw) / pj.hw, kr = ((float)(rx0 + R) - pj.hw) / pj.hw;
    const float kt = ((float)ry0 - pj.hw) / pj.hw, kb = ((float)(ry0 + R) - pj.hw) / pj.hw;
    RegionPlanes P;
    {
        // camera-space plane  a*X + b*Y + c*Z + e >= 0  ->  world normal, offset
        const float pa[5][4] = {{0.f, 0.f, 1.f, -pj.near_m},
                                {1.f, 0.f, -kl, 0.f},
                                {-1.f, 0.f, kr, 0.f},
                                {0.f, 1.f, -kt, 0.f},
                                {0.f, -1.f, kb, 0.f}};
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

    const uint64_t c0 = m.env_cluster_off[env], c1 = m.env_cluster_off[env + 1];
    for (uint64_t cb = c0 + (uint64_t)wave * 64; cb < c1; cb += (uint64_t)kWaves * 64) {
        bool vis = false;
        const uint64_t myc = cb + lane;
        if (myc < c1) {
            const float4 w0 = m.clusters[myc * 3 + 0];
            const float4 w1 = m.clusters[myc * 3 + 1];
            vis = aabb_visible(P, w0.x, w0.y, w0.z, w1.x, w1.y, w1.z);
        }
        uint64_t vmask = __ballot(vis);
        while (vmask) {
            const int bit = __ffsll((unsigned long long)vmask) - 1;
            vmask &= vmask - 1;
            const uint64_t ci = cb + bit;
            const float4 w0 = m.clusters[ci * 3 + 0];
            const float4 w1 = m.clusters[ci * 3 + 1];
            const float4 w2 = m.clusters[ci * 3 + 2];
            const uint32_t vbase = __float_as_uint(w0.w);
            const uint32_t tbase = __float_as_uint(w1.w);
            const uint32_t cnt = __float_as_uint(w2.x);
            const int nv = (int)(cnt & 0xFF), nt = (int)((cnt >> 8) & 0xFF);

            // ---- per vertex: camera space, outcodes, projection
            float X = 0.f, Y = 0.f, Z = 1.f;
            uint32_t oc = 0;
            int xi = 0, yi = 0;
            float dv = 0.f;
            if (lane < nv) {
                const float *v = m.cverts + ((size_t)vbase + lane) * 3;
                const float ddx = v[0] - cam.px, ddy = v[1] - cam.py, ddz = v[2] - cam.pz;
                X = (cam.rx * ddx + cam.ry * ddy) + cam.rz * ddz;
                Y = (cam.dx * ddx + cam.dy * ddy) + cam.dz * ddz;
                Z = (cam.fx * ddx + cam.fy * ddy) + cam.fz * ddz;
#pragma unroll
                for (int k = 0; k < 5; ++k)
                    if (clip_plane(X, Y, Z, k, pj.near_m) < 0.0f) oc |= 1u << k;
                if (X - kl * Z < 0.0f) oc |= 1u << 5;
                if (kr * Z - X < 0.0f) oc |= 1u << 6;
                if (Y - kt * Z < 0.0f) oc |= 1u << 7;
                if (kb * Z - Y < 0.0f) oc |= 1u << 8;
                if ((oc & 1u) == 0) project(pj, X, Y, Z, xi, yi, dv);
            }

            // ---- per triangle
            const uint32_t packed = lane < nt ? m.ctris[(size_t)tbase + lane] : 0u;
            const int i0 = (int)(packed & 0xFF), i1 = (int)((packed >> 8) & 0xFF),
                      i2 = (int)((packed >> 16) & 0xFF);
            const uint32_t o0 = (uint32_t)__shfl((int)oc, i0, 64);
            const uint32_t o1 = (uint32_t)__shfl((int)oc, i1, 64);
            const uint32_t o2 = (uint32_t)__shfl((int)oc, i2, 64);
            const bool valid = lane < nt && (o0 & o1 & o2) == 0u;
            const bool allin = valid && ((o0 | o1 | o2) & kClipBits) == 0u;
            const bool clipped = valid && !allin;
            const int vx0 = __shfl(xi, i0, 64), vy0 = __shfl(yi, i0, 64);
            const int vx1 = __shfl(xi, i1, 64), vy1 = __shfl(yi, i1, 64);
            const int vx2 = __shfl(xi, i2, 64), vy2 = __shfl(yi, i2, 64);
            const float vd0 = __shfl(dv, i0, 64), vd1 = __shfl(dv, i1, 64), vd2 = __shfl(dv, i2, 64);

            int nsub = allin ? 1 : 0;
            Poly poly;
            poly.n = 0;
            if (__ballot(clipped)) {
                const float X0 = __shfl(X, i0, 64), Y0 = __shfl(Y, i0, 64), Z0 = __shfl(Z, i0, 64);
                const float X1 = __shfl(X, i1, 64), Y1 = __shfl(Y, i1, 64), Z1 = __shfl(Z, i1, 64);
                const float X2 = __shfl(X, i2, 64), Y2 = __shfl(Y, i2, 64), Z2 = __shfl(Z, i2, 64);
                if (clipped) {
                    poly.n = 3;
                    poly.X[0] = X0; poly.Y[0] = Y0; poly.Z[0] = Z0;
                    poly.X[1] = X1; poly.Y[1] = Y1; poly.Z[1] = Z1;
                    poly.X[2] = X2; poly.Y[2] = Y2; poly.Z[2] = Z2;
                    clip_polygon(poly, pj.near_m);
                    nsub = poly.n >= 3 ? poly.n - 2 : 0;
                }
            }
            const int maxsub = wave_max(nsub);
            for (int s = 0; s < maxsub; ++s) {
                Setup S;
                int ok = 0;
                if (s < nsub) {
                    if (allin) {
                        ok = setup_triangle(vx0, vy0, vd0, vx1, vy1, vd1, vx2, vy2, vd2, rx0, ry0,
                                            R, S);
                    } else {
                        int ax, ay, bx, by, cx2, cy2;
                        float ad, bd, cd;
                        project(pj, poly.X[0], poly.Y[0], poly.Z[0], ax, ay, ad);
                        project(pj, poly.X[s + 1], poly.Y[s + 1], poly.Z[s + 1], bx, by, bd);
                        project(pj, poly.X[s + 2], poly.Y[s + 2], poly.Z[s + 2], cx2, cy2, cd);
                        ok = setup_triangle(ax, ay, ad, bx, by, bd, cx2, cy2, cd, rx0, ry0, R, S);
                    }
                }
                bool big = false;
                if (ok) {
                    const int npx = (S.px1 - S.px0 + 1) * (S.py1 - S.py0 + 1);
                    if (npx <= rp.small_max) raster_small(S, rx0, ry0, R, zbuf);
                    else big = true;
                }
                uint64_t bmask = __ballot(big);
                while (bmask) {
                    const int L = __ffsll((unsigned long long)bmask) - 1;
                    bmask &= bmask - 1;
                    raster_big(S, L, lane, rx0, ry0, R, zbuf);
                }
            }
        }
    }
    __syncthreads();
    uint32_t *dst = depth + env_depth_off[env];
    for (int i = threadIdx.x; i < R * R; i += kBlock) {
        const int y = i / R, x = i - y * R;
        dst[(size_t)(ry0 + y) * res + (rx0 + x)] = zbuf[i];
    }
}

}  // namespace

hipError_t launch_raster(const RenderMesh &m, const RasterParams &rp, const float *camera,
                         const int32_t *env_res, const uint64_t *env_depth_off,
                         const uint32_t *work, int32_t num_work, uint32_t *depth, hipStream_t s)
{
    if (num_work <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster<256>, dim3(num_work), dim3(256), 0, s, m, rp, camera, env_res,
                       env_depth_off, work, depth);
    return hipGetLastError();
}

}  // namespace gal
