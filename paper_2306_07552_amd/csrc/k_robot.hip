// Robot step kernel: action decode, kinematic update, forward kinematics,
// sphere-proxy collision against the column grid and the object boxes,
// resolution, episode bookkeeping and the head-camera pose (Galactic,
// Section 3.2 and Appendix G).  One wave64 (or half-wave) per environment:
// the chain of seven joint frames is evaluated redundantly by every lane (it
// is a short serial chain), each lane owns every 64th (32nd) sphere, and the
// accept/reject decision is a ballot.
#include "gal_fk.h"
#include "gal_internal.h"
#include "gal_math.h"
#include "gal_order.h"

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

// Frame of `link` (0..7), selected element by element.  Each candidate value
// passes through an empty asm so that the compiler cannot turn the selects
// into a load from a selected address, which would keep all eight frames in
// scratch memory instead of registers.
__device__ __forceinline__ Frame pick(const Fk &fk, int link)
{
    Frame r;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        float v = fk.f[0].m[k];
        asm("" : "+v"(v));
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            float c = fk.f[j].m[k];
            asm("" : "+v"(c));
            v = link == j ? c : v;
        }
        r.m[k] = v;
    }
    return r;
}

// Column-grid test of one sphere centre, split into stages so that the
// dependent loads of several spheres are in flight together: the column's
// layer range, then two of its layers, then (rarely) the rest.  Contact
// when the centre is outside the grid or inside no free layer [lo, hi]
// (touching a layer bound counts as free).  The two layers loaded first are
// the column's first two, or, with the layer cache, the one at the sphere's
// cached offset and the next: which layers are read first changes no result.
struct GridProbe {
    bool outside;
    uint32_t l0, l1;
    uint32_t s0;   // first of the two layers loaded up front
    float z;
    float2 a, b;   // layers s0 and s0 + 1 when present
};

__device__ __forceinline__ void grid_probe_column(const SimBuffers &sb, const GridMeta &gm,
                                                  uint64_t off_base, float x, float y, float z,
                                                  GridProbe &g)
{
    g.z = z;
    g.l0 = g.l1 = g.s0 = 0;
    const float fx = (x - gm.x0) * sb.inv_cell;
    const float fy = (y - gm.y0) * sb.inv_cell;
    g.outside = !(fx >= 0.0f && fx < (float)gm.nx) || !(fy >= 0.0f && fy < (float)gm.ny);
    if (g.outside) return;
    const int i = (int)floorf(fx), j = (int)floorf(fy);
    const uint64_t col = (uint64_t)j * (uint64_t)gm.nx + (uint64_t)i;
    const uint32_t *off = sb.grid_offsets + off_base + col;
    g.l0 = off[0];
    g.l1 = off[1];
}

// hint: the layer cache's offset for this sphere (0 without the cache)
__device__ __forceinline__ void grid_probe_layers(const SimBuffers &sb, uint64_t layer_base, GridProbe &g,
                                                  uint32_t hint = 0)
{
    const float2 *lay = sb.grid_layers + layer_base;
    g.s0 = g.l0 + hint < g.l1 ? g.l0 + hint : g.l0;
    if (g.s0 < g.l1) g.a = lay[g.s0];
    if (g.s0 + 1 < g.l1) g.b = lay[g.s0 + 1];
}

// found: the index of the free layer holding the centre (l1 if none)
__device__ __forceinline__ bool grid_probe_contact(const SimBuffers &sb, uint64_t layer_base,
                                                   const GridProbe &g, uint32_t &found)
{
    found = g.l1;
    if (g.outside) return true;
    const float z = g.z;
    if (g.s0 < g.l1 && g.a.x <= z && z <= g.a.y) {
        found = g.s0;
        return false;
    }
    if (g.s0 + 1 < g.l1 && g.b.x <= z && z <= g.b.y) {
        found = g.s0 + 1;
        return false;
    }
    const float2 *lay = sb.grid_layers + layer_base;
    for (uint32_t l = g.l0; l < g.l1; ++l) {
        if (l == g.s0 || l == g.s0 + 1) continue;
        const float2 L = lay[l];
        if (L.x <= z && z <= L.y) {
            found = l;
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ bool grid_probe_contact(const SimBuffers &sb, uint64_t layer_base,
                                                   const GridProbe &g)
{
    uint32_t found;
    return grid_probe_contact(sb, layer_base, g, found);
}

__device__ __forceinline__ bool obb_contact(const float *o, float x, float y, float z, float r)
{
    float dx = x - o[0], dy = y - o[1], dz = z - o[2];
    float cps = o[6], sps = o[7];
    float l0 = cps * dx + sps * dy;
    float l1 = cps * dy - sps * dx;
    float l2 = dz;
    float q0 = clampf(l0, -o[3], o[3]);
    float q1 = clampf(l1, -o[4], o[4]);
    float q2 = clampf(l2, -o[5], o[5]);
    float d0 = l0 - q0, d1 = l1 - q1, d2 = l2 - q2;
    float dd = (d0 * d0 + d1 * d1) + d2 * d2;
    return dd < r * r;
}

// Objects a sphere (x, y, radius r) may touch: the word of the first object
// grid cell that holds the sphere's whole disk (x +- r, y +- r inside the
// cell), or every object when no cell does (a sphere wider than a quarter
// cell, or outside the grids) or the grids are not in use.  Every object whose
// box the sphere meets has its footprint in that cell, so testing the word's
// objects finds exactly the contacts of testing them all.
__device__ __forceinline__ uint64_t objgrid_candidates(const RobotParams &rp, const SimBuffers &sb, int env,
                                                        float x, float y, float r)
{
    const int O = rp.num_objects;
    const uint64_t all = O >= 64 ? ~0ull : ((1ull << O) - 1ull);
    if (!rp.objgrid || !sb.objgrid_mask) return all;
    const ObjGridMeta gm = sb.objgrid_meta[env];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float ox = gm.x0 + (float)(g & 1) * (0.5f * kObjCell);
        const float oy = gm.y0 + (float)(g >> 1) * (0.5f * kObjCell);
        const float fx = (x - ox) * (1.0f / kObjCell), fy = (y - oy) * (1.0f / kObjCell);
        if (!(fx >= 0.0f && fx < (float)gm.nx && fy >= 0.0f && fy < (float)gm.ny)) continue;
        const float i = floorf(fx), j = floorf(fy);
        const float lx = x - (ox + i * kObjCell), ly = y - (oy + j * kObjCell);
        if (lx >= r && kObjCell - lx >= r && ly >= r && kObjCell - ly >= r)
            return sb.objgrid_mask[gm.base + ((uint64_t)g * (uint64_t)gm.ny + (uint64_t)j) * (uint64_t)gm.nx +
                                   (uint64_t)i];
    }
    return all;
}

// The object grids of one env from its object records (one wave): clear the
// words, then set object o's bit in every cell, of every grid, that its
// footprint box (grown by kObjMargin) meets.  Objects wholly outside a grid,
// or with non-finite records (which no sphere can touch), set no bit there.
__device__ void objgrid_rebuild(const RobotParams &rp, const SimBuffers &sb, int env, const float *objs, int lane)
{
    const ObjGridMeta gm = sb.objgrid_meta[env];
    unsigned long long *w = sb.objgrid_mask + gm.base;
    const int per = gm.nx * gm.ny;
    for (int i = lane; i < 4 * per; i += 64) w[i] = 0ull;
    __threadfence_block();
    for (int p = lane; p < 4 * rp.num_objects; p += 64) {
        const int o = p >> 2, g = p & 3;
        const float *ob = objs + 8 * o;
        const float c = fabsf(ob[6]), sn = fabsf(ob[7]);
        const float ax = (c * ob[3] + sn * ob[4]) + kObjMargin;
        const float ay = (sn * ob[3] + c * ob[4]) + kObjMargin;
        const float ox = gm.x0 + (float)(g & 1) * (0.5f * kObjCell);
        const float oy = gm.y0 + (float)(g >> 1) * (0.5f * kObjCell);
        const float fi0 = floorf(((ob[0] - ax) - ox) * (1.0f / kObjCell));
        const float fi1 = floorf(((ob[0] + ax) - ox) * (1.0f / kObjCell));
        const float fj0 = floorf(((ob[1] - ay) - oy) * (1.0f / kObjCell));
        const float fj1 = floorf(((ob[1] + ay) - oy) * (1.0f / kObjCell));
        if (!(fi1 >= 0.0f && fj1 >= 0.0f && fi0 < (float)gm.nx && fj0 < (float)gm.ny)) continue;
        const int i0 = (int)fmaxf(fi0, 0.0f), i1 = (int)fminf(fi1, (float)(gm.nx - 1));
        const int j0 = (int)fmaxf(fj0, 0.0f), j1 = (int)fminf(fj1, (float)(gm.ny - 1));
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) atomicOr(&w[(size_t)g * per + (size_t)j * gm.nx + i], 1ull << o);
    }
}

__device__ __forceinline__ void load_start(const RobotParams &rp, const SimBuffers &sb, int env,
                                           int episode, float *st)
{
    int p = episode % rp.num_starts;
    const float *s0 = sb.starts + ((size_t)env * rp.num_starts + p) * 3;
    st[0] = s0[0];
    st[1] = s0[1];
    st[2] = s0[2];
#pragma unroll
    for (int j = 0; j < 7; ++j) st[3 + j] = rp.q_home[j];
}

__device__ __forceinline__ void write_camera(const RobotParams &rp, const Frame &F0, float *cam)
{
    const float cp = rp.cam_pitch_cs[0], sp = rp.cam_pitch_cs[1];
    fpoint(F0, rp.cam_offset[0], rp.cam_offset[1], rp.cam_offset[2], cam[0], cam[1], cam[2]);
    fvec(F0, 0.0f, -1.0f, 0.0f, cam[3], cam[4], cam[5]);
    fvec(F0, -sp, 0.0f, -cp, cam[6], cam[7], cam[8]);
    fvec(F0, cp, 0.0f, -sp, cam[9], cam[10], cam[11]);
}

// The spheres of two consecutive passes owned by one lane: records, whether
// they take part (a held-object proxy only while an object is held), and the
// bases of their class's grid in the offset and layer tables.
constexpr int kSlots = 2;
struct SphereSlots {
    Sphere sp[kSlots];
    bool live[kSlots];
    uint64_t off_base[kSlots], layer_base[kSlots];
    int idx[kSlots];         // sphere index
    uint32_t hint[kSlots];   // layer-cache offset (0 without the cache)
};

template <int kLanes>
__device__ __forceinline__ void load_slots(const RobotParams &rp, const SimBuffers &sb, int env, bool held,
                                           bool active, int sub, int base, SphereSlots &sl)
{
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int s = base + k * kLanes + sub;
        sl.live[k] = false;
        sl.off_base[k] = sl.layer_base[k] = 0;
        sl.idx[k] = s;
        sl.hint[k] = 0;
        if (active && s < rp.num_spheres) {
            sl.sp[k] = sb.spheres[s];
            if (!(sl.sp[k].held_only && !held)) {
                sl.live[k] = true;
                const size_t gk = (size_t)env * rp.num_classes + sl.sp[k].cls;
                sl.off_base[k] = sb.grid_off_base[gk];
                sl.layer_base[k] = sb.grid_layer_base[gk];
                if (sb.layer_hint) sl.hint[k] = sb.layer_hint[(size_t)env * rp.num_spheres + s];
            }
        }
    }
}

// Queue order of the raster work items by descending cost, to within 1/256
// of the largest: a counting sort of the costs quantised to 256 buckets by
// one 256-thread workgroup (three passes over the costs; the order inside a
// bucket is whatever the LDS atomics give, and the order of the items changes
// no output).
__device__ void order_items_block(const ItemOrder &ord)
{
    constexpr int kBuckets = 256;
    __shared__ uint32_t cmax;
    __shared__ uint32_t count[kBuckets];
    const int t = (int)threadIdx.x, n = ord.n;
    if (t == 0) cmax = 1u;
    count[t] = 0u;
    __syncthreads();
    for (int i = t; i < n; i += 256) atomicMax(&cmax, ord.cost[i]);
    __syncthreads();
    const uint64_t m = cmax;
    auto bucket = [&](uint32_t c) {   // longest first: bucket 0 holds the largest costs
        return (uint32_t)(kBuckets - 1) - (uint32_t)(((uint64_t)c * (kBuckets - 1)) / m);
    };
    for (int i = t; i < n; i += 256) atomicAdd(&count[bucket(ord.cost[i])], 1u);
    __syncthreads();
    if (t < 64) {   // exclusive prefix over the buckets, 4 per lane
        const uint32_t a = count[4 * t], b = count[4 * t + 1], d = count[4 * t + 2], e = count[4 * t + 3];
        const uint32_t sum = a + b + d + e;
        uint32_t incl = sum;
#pragma unroll
        for (int k = 1; k < 64; k <<= 1) {
            const uint32_t y = __shfl_up(incl, k, 64);
            if (t >= k) incl += y;
        }
        const uint32_t ex = incl - sum;
        count[4 * t] = ex;
        count[4 * t + 1] = ex + a;
        count[4 * t + 2] = ex + a + b;
        count[4 * t + 3] = ex + a + b + d;
    }
    __syncthreads();
    for (int i = t; i < n; i += 256) ord.order[atomicAdd(&count[bucket(ord.cost[i])], 1u)] = (uint32_t)i;
}

// kLanes lanes per environment: 64 (one env per wave, spheres lane + 64k) or
// 32 (two envs per wave, spheres lane + 32k); the ballot's 32-bit halves are
// then exactly the envs' contact words.
template <int kLanes>
__global__ __launch_bounds__(256) void k_robot_step(RobotParams rp, SimBuffers sb,
                                                    const float *__restrict__ actions,
                                                    StepOutputs out, uint32_t *queue_reset,
                                                    ItemOrder ord)
{
    // the launch's extra last workgroup orders the raster queue
    if (ord.n > 0 && blockIdx.x == gridDim.x - 1) {
        order_items_block(ord);
        return;
    }
    // the raster work queue of this step starts empty (a kernel store rather
    // than a memset, so the step can be captured as a graph)
    if (queue_reset && blockIdx.x == 0 && threadIdx.x == 0) *queue_reset = 0u;
    constexpr int kEnvsPerBlock = 256 / kLanes;
    const int lane = threadIdx.x & 63;
    const int sub = (int)threadIdx.x % kLanes;
    const int half = kLanes == 32 ? (lane >> 5) : 0;
    int env = (int)blockIdx.x * kEnvsPerBlock + (int)threadIdx.x / kLanes;
    if (kLanes == 64) env = __builtin_amdgcn_readfirstlane(env);
    // The object records of the workgroup's envs, staged in LDS once: every
    // sphere may test all of them, and read from global memory each test of
    // the chain would wait on a load of its own.
    __shared__ float4 obj_lds[kEnvsPerBlock * kMaxObjects * 2];
    const int env0 = (int)blockIdx.x * kEnvsPerBlock;
    {
        const int ne = min(kEnvsPerBlock, sb.num_envs - env0);
        const int n4 = ne * rp.num_objects * 2;
        const float4 *src = reinterpret_cast<const float4 *>(sb.objects + (size_t)env0 * rp.num_objects * 8);
        for (int i = (int)threadIdx.x; i < n4; i += 256) obj_lds[i] = src[i];
        __syncthreads();
    }
    if (kLanes == 64 && env >= sb.num_envs) return;
    // with two envs per wave, a half-wave past the end still joins the ballots
    const bool active = env < sb.num_envs;
    if (!active) env = 0;

    float st[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) st[k] = sb.state[(size_t)env * 10 + k];
    int t = sb.counters[(size_t)env * 2 + 0];
    int episode = sb.counters[(size_t)env * 2 + 1];
    const float *act = actions + (size_t)env * 9;

    // 1. kinematic update: offsets applied directly to the state
    float cand[10];
    {
        float a0 = sanitize(act[0], rp.act_lim[0]);
        float a1 = sanitize(act[1], rp.act_lim[1]);
        const float pi_f = 0x1.921fb6p+1f, two_pi_f = 0x1.921fb6p+2f;
        float yaw = st[2] + a1;
        if (yaw > pi_f) yaw = yaw - two_pi_f;
        else if (yaw < -pi_f) yaw = yaw + two_pi_f;
        float sy, cy;
        dsincos(yaw, sy, cy);
        cand[0] = st[0] + a0 * cy;
        cand[1] = st[1] + a0 * sy;
        cand[2] = yaw;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            float aj = sanitize(act[2 + j], rp.act_lim[2]);
            cand[3 + j] = clampf(st[3 + j] + aj, rp.qlim[j][0], rp.qlim[j][1]);
        }
    }

    // 2. forward kinematics of the candidate, sphere tests.  Each lane owns
    // spheres sub + kLanes * p; two passes p are processed together, and the
    // sphere records and grid bases of the first two are loaded before the
    // kinematics (they do not depend on it).
    const bool held = sb.held ? (sb.held[env] != 0) : false;
    SphereSlots sl;
    load_slots<kLanes>(rp, sb, env, held, active, sub, 0, sl);
    Fk fk;
    forward_kinematics(rp, cand, fk);
    const GridMeta gm = sb.grid_meta[env];
    const float *objs = reinterpret_cast<const float *>(obj_lds) + (active ? env - env0 : 0) * rp.num_objects * 8;
    // surrogate routing: 1 = static check skipped (no contact assumed),
    // 2 = skipped but audited (exact check runs; a contact is a mismatch)
    const int route = sb.skip_flags ? sb.skip_flags[env] : 0;
    bool any = false, any_static = false;
    for (int base = 0; base < rp.num_spheres; base += kSlots * kLanes) {
        GridProbe g[kSlots];
        float cx[kSlots], cy[kSlots], cz[kSlots];
        const bool grid = route != 1;
        uint64_t cm[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            g[k].outside = false;
            g[k].l0 = g[k].l1 = 0;
            cx[k] = cy[k] = cz[k] = 0.0f;
            cm[k] = 0ull;
            if (sl.live[k]) {
                const Frame F = pick(fk, sl.sp[k].link);
                fpoint(F, sl.sp[k].px, sl.sp[k].py, sl.sp[k].pz, cx[k], cy[k], cz[k]);
                if (grid) grid_probe_column(sb, gm, sl.off_base[k], cx[k], cy[k], cz[k], g[k]);
                cm[k] = objgrid_candidates(rp, sb, env, cx[k], cy[k], rp.class_radius[sl.sp[k].cls]);
            }
        }
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (sl.live[k] && grid) grid_probe_layers(sb, sl.layer_base[k], g[k], sl.hint[k]);
        bool hit_static[kSlots], hit_object[kSlots];
        // object boxes: one pass over the candidates of every slot of the
        // env's lanes (the OR of their masks), each record read from LDS once
        // for all of its tests; the tests are pure, so testing a lane's
        // candidates past its first contact changes nothing
        {
            uint64_t m[kSlots], u = 0ull;
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                hit_object[k] = false;
                m[k] = sl.live[k] ? cm[k] : 0ull;
                u |= m[k];
            }
            uint32_t ulo = (uint32_t)u, uhi = (uint32_t)(u >> 32);
#pragma unroll
            for (int d = kLanes / 2; d >= 1; d >>= 1) {
                ulo |= (uint32_t)__shfl_xor((int)ulo, d, 64);
                uhi |= (uint32_t)__shfl_xor((int)uhi, d, 64);
            }
            float r[kSlots];
#pragma unroll
            for (int k = 0; k < kSlots; ++k) r[k] = sl.live[k] ? rp.class_radius[sl.sp[k].cls] : 0.0f;
            for (u = ((uint64_t)uhi << 32) | ulo; u; u &= u - 1) {
                const int o = __ffsll((unsigned long long)u) - 1;
#pragma unroll
                for (int k = 0; k < kSlots; ++k)
                    if ((m[k] >> o) & 1ull)
                        hit_object[k] = hit_object[k] | obb_contact(objs + 8 * o, cx[k], cy[k], cz[k], r[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            hit_static[k] = false;
            if (sl.live[k]) {
                if (grid) {
                    uint32_t found;
                    hit_static[k] = grid_probe_contact(sb, sl.layer_base[k], g[k], found);
                    // the layer cache: where this sphere's free layer was
                    // found (kept when the centre is in no free layer)
                    if (sb.layer_hint && found < g[k].l1) {
                        const uint32_t off = found - g[k].l0;
                        const uint32_t h = off < 255u ? off : 0u;
                        if (h != sl.hint[k]) sb.layer_hint[(size_t)env * rp.num_spheres + sl.idx[k]] = (uint8_t)h;
                    }
                }
            }
        }
        // records of the next two passes
        if (base + kSlots * kLanes < rp.num_spheres)
            load_slots<kLanes>(rp, sb, env, held, active, sub, base + kSlots * kLanes, sl);
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int pb = base + k * kLanes;
            if (pb >= rp.num_spheres) break;
            const uint64_t ms = __ballot(hit_static[k]);
            const uint64_t mo = __ballot(hit_object[k]);
            const int w = pb >> 5;
            if (kLanes == 64) {
                any = any || (ms | mo) != 0;
                any_static = any_static || ms != 0;
                if (lane == 0) {
                    if (out.contact_static) {
                        uint32_t *cs = out.contact_static + (size_t)env * rp.contact_words;
                        if (w < rp.contact_words) cs[w] = (uint32_t)ms;
                        if (w + 1 < rp.contact_words) cs[w + 1] = (uint32_t)(ms >> 32);
                    }
                    if (out.contact_object) {
                        uint32_t *co = out.contact_object + (size_t)env * rp.contact_words;
                        if (w < rp.contact_words) co[w] = (uint32_t)mo;
                        if (w + 1 < rp.contact_words) co[w + 1] = (uint32_t)(mo >> 32);
                    }
                }
            } else {
                const uint32_t hs = (uint32_t)(ms >> (32 * half)), ho = (uint32_t)(mo >> (32 * half));
                any = any || (hs | ho) != 0u;
                any_static = any_static || hs != 0u;
                if (sub == 0 && active && w < rp.contact_words) {
                    if (out.contact_static) out.contact_static[(size_t)env * rp.contact_words + w] = hs;
                    if (out.contact_object) out.contact_object[(size_t)env * rp.contact_words + w] = ho;
                }
            }
        }
    }
    if (!active) return;
    if (route == 2 && any_static && sub == 0) atomicAdd(&sb.sur_stats[3], 1ull);

    // 3. resolve: any overlap rejects the whole move
    const bool accepted = !any;
    if (accepted) {
#pragma unroll
        for (int k = 0; k < 10; ++k) st[k] = cand[k];
    }

    // 4. episode bookkeeping (auto-reset at the horizon)
    bool done = false;
    t += 1;
    if (rp.episode_len > 0 && t >= rp.episode_len) {
        episode += 1;
        load_start(rp, sb, env, episode, st);
        t = 0;
        done = true;
    }

    // 5. frames and camera of the final state
    if (!accepted || done) forward_kinematics(rp, st, fk);
    if (sub == 0) {
#pragma unroll
        for (int k = 0; k < 10; ++k) sb.state[(size_t)env * 10 + k] = st[k];
        sb.counters[(size_t)env * 2 + 0] = t;
        sb.counters[(size_t)env * 2 + 1] = episode;
        float cam[12];
        write_camera(rp, fk.f[0], cam);
#pragma unroll
        for (int k = 0; k < 12; ++k) sb.camera[(size_t)env * 12 + k] = cam[k];
        if (out.state) {
#pragma unroll
            for (int k = 0; k < 10; ++k) out.state[(size_t)env * 10 + k] = st[k];
        }
        if (out.counters) {
            out.counters[(size_t)env * 2 + 0] = t;
            out.counters[(size_t)env * 2 + 1] = episode;
        }
        if (out.accepted) out.accepted[env] = accepted ? 1 : 0;
        if (out.done) out.done[env] = done ? 1 : 0;
    }
    if ((out.frames || rp.links) && sub < 8) {
        Frame F = pick(fk, sub);
        if (out.frames) {
            float *dst = out.frames + ((size_t)env * 8 + sub) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) dst[k] = F.m[k];
        }
        if (rp.links) {
            float *dst = sb.link_frames + ((size_t)env * 8 + sub) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) dst[k] = F.m[k];
        }
    }
}

// ---- manipulation: grasp / carry / release with snap-to-surface and
// placing, sliding (Section 3.2 grasping paragraphs, Appendix I) ----------

__device__ __forceinline__ float rlf(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Frame of a resting object: Rz(yaw) about its centre.
__device__ __forceinline__ Frame object_frame(const float *o)
{
    Frame F;
    F.m[0] = o[6];  F.m[1] = -o[7]; F.m[2] = 0.0f;  F.m[3] = o[0];
    F.m[4] = o[7];  F.m[5] = o[6];  F.m[6] = 0.0f;  F.m[7] = o[1];
    F.m[8] = 0.0f;  F.m[9] = 0.0f;  F.m[10] = 1.0f; F.m[11] = o[2];
    return F;
}

// R^T | -R^T t
__device__ __forceinline__ Frame frame_inverse(const Frame &F)
{
    Frame G;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) G.m[i * 4 + j] = F.m[j * 4 + i];
        G.m[i * 4 + 3] = -((F.m[0 * 4 + i] * F.m[3] + F.m[1 * 4 + i] * F.m[7]) + F.m[2 * 4 + i] * F.m[11]);
    }
    return G;
}

// Octant k of a box of half extents e (bit 0 = x, 1 = y, 2 = z).
__device__ __forceinline__ void octant(const float *e, int k, float &x, float &y, float &z)
{
    x = (k & 1) ? 0.5f * e[0] : -(0.5f * e[0]);
    y = (k & 2) ? 0.5f * e[1] : -(0.5f * e[1]);
    z = (k & 4) ? 0.5f * e[2] : -(0.5f * e[2]);
}

__device__ __forceinline__ float obb_dist2(const float *o, float x, float y, float z)
{
    float dx = x - o[0], dy = y - o[1], dz = z - o[2];
    float cps = o[6], sps = o[7];
    float l0 = cps * dx + sps * dy;
    float l1 = cps * dy - sps * dx;
    float l2 = dz;
    float q0 = clampf(l0, -o[3], o[3]);
    float q1 = clampf(l1, -o[4], o[4]);
    float q2 = clampf(l2, -o[5], o[5]);
    float d0 = l0 - q0, d1 = l1 - q1, d2 = l2 - q2;
    return (d0 * d0 + d1 * d1) + d2 * d2;
}

// SplitMix64 (Steele, Lea & Flood 2014) of a counter, as a uniform in [0, 1)
// with 24 bits.
__device__ __forceinline__ float hash01(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, uint64_t d)
{
    uint64_t x = seed + 0x9E3779B97F4A7C15ull * (((a << 40) ^ (b << 24) ^ (c << 8) ^ d) + 1ull);
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x = x ^ (x >> 31);
    return (float)(x >> 40) * 0x1p-24f;
}

// Full column-grid test of one point for class k of env e.
__device__ __forceinline__ bool grid_point_contact(const RobotParams &rp, const SimBuffers &sb,
                                                   const GridMeta &gm, int env, int cls, float x,
                                                   float y, float z)
{
    const size_t gk = (size_t)env * rp.num_classes + cls;
    GridProbe g;
    grid_probe_column(sb, gm, sb.grid_off_base[gk], x, y, z, g);
    if (!g.outside) grid_probe_layers(sb, sb.grid_layer_base[gk], g);
    return grid_probe_contact(sb, sb.grid_layer_base[gk], g);
}

// Overlap test of a pose (frames fk) of one env, one wave: lane l takes
// spheres l + 64 p of the robot's S spheres followed, with an object held,
// by the held object's 8 octant spheres.  Returns whether any sphere
// overlaps the grid or a resting object; with masks, writes the contact
// words; the x, y of every overlapping sphere centre are summed in sphere
// order (the same in every lane).
__device__ __forceinline__ bool manip_pose_contacts(const RobotParams &rp, const SimBuffers &sb,
                                                    const GridMeta &gm, int env, const Fk &fk,
                                                    int held, const Frame &rel, const float *objs,
                                                    int lane, uint32_t *ms_out, uint32_t *mo_out,
                                                    float &sx, float &sy, int &n)
{
    const int S = rp.num_spheres;
    const int total = S + (held >= 0 ? kHeldSpheres : 0);
    Frame Fh;
    const float *eh = nullptr;
    if (held >= 0) {
        Fh = fmul(fk.f[7], rel);
        eh = objs + 8 * held + 3;
    }
    bool any = false;
    sx = 0.0f;
    sy = 0.0f;
    n = 0;
    for (int base = 0; base < S + kHeldSpheres; base += 64) {
        const int s = base + lane;
        bool live = false;
        float cx = 0.f, cy = 0.f, cz = 0.f;
        int cls = 0;
        if (s < S) {
            const Sphere sp = sb.spheres[s];
            if (!sp.held_only) {
                live = true;
                const Frame F = pick(fk, sp.link);
                fpoint(F, sp.px, sp.py, sp.pz, cx, cy, cz);
                cls = sp.cls;
            }
        } else if (s < total) {
            live = true;
            float px, py, pz;
            octant(eh, s - S, px, py, pz);
            fpoint(Fh, px, py, pz, cx, cy, cz);
            cls = rp.held_class;
        }
        bool hs = false, ho = false;
        if (live) {
            hs = grid_point_contact(rp, sb, gm, env, cls, cx, cy, cz);
            const float r = rp.class_radius[cls];
            uint64_t m = objgrid_candidates(rp, sb, env, cx, cy, r);
            if (held >= 0) m &= ~(1ull << held);
            for (; m; m &= m - 1) {
                const int o = __ffsll((unsigned long long)m) - 1;
                if (obb_contact(objs + 8 * o, cx, cy, cz, r)) {
                    ho = true;
                    break;
                }
            }
        }
        const uint64_t ms = __ballot(hs), mo = __ballot(ho);
        if (lane == 0) {
            const int w = base >> 5;
            if (ms_out && w < rp.contact_words) ms_out[w] = (uint32_t)ms;
            if (ms_out && w + 1 < rp.contact_words) ms_out[w + 1] = (uint32_t)(ms >> 32);
            if (mo_out && w < rp.contact_words) mo_out[w] = (uint32_t)mo;
            if (mo_out && w + 1 < rp.contact_words) mo_out[w + 1] = (uint32_t)(mo >> 32);
        }
        uint64_t hm = ms | mo;
        any = any || hm != 0;
        while (hm) {
            const int l = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            sx = sx + rlf(cx, l);
            sy = sy + rlf(cy, l);
            ++n;
        }
    }
    return any;
}

// Release of held object h at frame F: snap-to-surface and the placing
// heuristic.  The object lands upright with the yaw of its x axis; four
// spheres of the held class touching its bottom face from inside are cast
// down the column grid (each drops to the bottom of the free layer holding
// its centre; the object drops by the least of those); the landed object
// must not overlap another resting object with its octant spheres.  A failed
// try moves the drop point by place_step: away from the blocking object,
// turned by a hashed angle in [-pi/4, pi/4), or in a hashed direction when
// the grid refused the cast; after kPlaceTries jitters the object keeps its
// record from before the grasp.  Uniform over the wave; lanes share the
// sphere tests.
constexpr int kPlaceTries = 6;
constexpr int kSlideTries = 3;

__device__ __forceinline__ void place_object(const RobotParams &rp, const SimBuffers &sb,
                                             const GridMeta &gm, int env, int h, const Frame &F,
                                             float *objs, int episode, int t, int lane)
{
    float e[3] = {objs[8 * h + 3], objs[8 * h + 4], objs[8 * h + 5]};
    const float cx0 = F.m[0], sx0 = F.m[4];
    const float n2 = cx0 * cx0 + sx0 * sx0;
    float c = 1.0f, s = 0.0f;
    if (n2 > 1e-12f) {
        const float len = sqrtf(n2);
        c = cx0 / len;
        s = sx0 / len;
    }
    float px = F.m[3], py = F.m[7];
    const float z0 = F.m[11];
    const int cls = rp.held_class;
    const float r = rp.class_radius[cls];
    const size_t gk = (size_t)env * rp.num_classes + cls;
    for (int k = 0; k <= kPlaceTries; ++k) {
        // the bottom-face cast: lanes 0..3
        bool fail = false;
        float d = INFINITY;
        if (lane < 4) {
            float ox, oy, oz;
            octant(e, lane, ox, oy, oz);
            const float wx = px + (c * ox - s * oy);
            const float wy = py + (s * ox + c * oy);
            const float wz = z0 + (r - e[2]);
            const float fx = (wx - gm.x0) * sb.inv_cell;
            const float fy = (wy - gm.y0) * sb.inv_cell;
            if (!(fx >= 0.0f && fx < (float)gm.nx && fy >= 0.0f && fy < (float)gm.ny)) {
                fail = true;
            } else {
                const int i = (int)floorf(fx), j = (int)floorf(fy);
                const uint64_t col = (uint64_t)j * (uint64_t)gm.nx + (uint64_t)i;
                const uint32_t *off = sb.grid_offsets + sb.grid_off_base[gk] + col;
                const float2 *lay = sb.grid_layers + sb.grid_layer_base[gk];
                bool found = false;
                for (uint32_t l = off[0]; l < off[1]; ++l) {
                    const float2 L = lay[l];
                    if (L.x <= wz && wz <= L.y) {
                        d = wz - L.x;
                        found = true;
                        break;
                    }
                }
                fail = !found;
            }
        }
        const bool fail_static = __ballot(fail) != 0;
        int fail_obj = -1;
        if (!fail_static) {
            float drop = d;
            drop = fminf(drop, rlf(d, 1));
            drop = fminf(drop, rlf(d, 2));
            drop = fminf(drop, rlf(d, 3));
            drop = fminf(rlf(d, 0), drop);
            float rec[8] = {px, py, z0 - drop, e[0], e[1], e[2], c, s};
            const Frame Fo = object_frame(rec);
            int hit = -1;
            if (lane < kHeldSpheres) {
                float ox, oy, oz, wx, wy, wz;
                octant(e, lane, ox, oy, oz);
                fpoint(Fo, ox, oy, oz, wx, wy, wz);
                // candidates in ascending order: the first hit is the lowest
                // index of the objects the sphere touches
                for (uint64_t m = objgrid_candidates(rp, sb, env, wx, wy, r) & ~(1ull << h); m; m &= m - 1) {
                    const int o = __ffsll((unsigned long long)m) - 1;
                    if (obb_contact(objs + 8 * o, wx, wy, wz, r)) {
                        hit = o;
                        break;
                    }
                }
            }
            const uint64_t hm = __ballot(hit >= 0);
            if (hm) {
                fail_obj = __builtin_amdgcn_readlane(hit, __ffsll((unsigned long long)hm) - 1);
            } else {
                if (lane < 8) objs[8 * h + lane] = rec[lane];
                return;
            }
        }
        if (k == kPlaceTries) break;
        const float u = hash01(rp.manip_seed, (uint64_t)(uint32_t)env, (uint64_t)(uint32_t)episode,
                               (uint64_t)(uint32_t)t, (uint64_t)(16 + k));
        float dx, dy;
        if (fail_obj >= 0) {
            const float *oo = objs + 8 * fail_obj;
            const float vx = px - oo[0], vy = py - oo[1];
            const float vn = sqrtf(vx * vx + vy * vy);
            float bx = 1.0f, by = 0.0f;
            if (vn > 1e-6f) {
                bx = vx / vn;
                by = vy / vn;
            }
            float sphi, cphi;
            dsincos((u - 0.5f) * 0x1.921fb6p+0f, sphi, cphi);
            dx = cphi * bx - sphi * by;
            dy = sphi * bx + cphi * by;
        } else {
            float sphi, cphi;
            dsincos(u * 0x1.921fb6p+2f - 0x1.921fb6p+1f, sphi, cphi);
            dx = cphi;
            dy = sphi;
        }
        px = px + rp.place_step * dx;
        py = py + rp.place_step * dy;
    }
}

// One manipulation step per wave (4 envs per 256-thread workgroup).
__global__ __launch_bounds__(256) void k_robot_step_manip(RobotParams rp, SimBuffers sb,
                                                          const float *__restrict__ actions,
                                                          StepOutputs out, uint32_t *queue_reset,
                                                          ItemOrder ord)
{
    if (ord.n > 0 && blockIdx.x == gridDim.x - 1) {
        order_items_block(ord);
        return;
    }
    if (queue_reset && blockIdx.x == 0 && threadIdx.x == 0) *queue_reset = 0u;
    const int lane = threadIdx.x & 63;
    const int env = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)threadIdx.x / 64);
    if (env >= sb.num_envs) return;
    const int O = rp.num_objects;
    float st[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) st[k] = sb.state[(size_t)env * 10 + k];
    int t = sb.counters[(size_t)env * 2 + 0];
    int episode = sb.counters[(size_t)env * 2 + 1];
    const float *act = actions + (size_t)env * 11;
    float *objs = sb.obj_dyn + (size_t)env * O * 8;
    int held = sb.held_obj[env];
    Frame rel;
#pragma unroll
    for (int k = 0; k < 12; ++k) rel.m[k] = sb.rel[(size_t)env * 12 + k];
    const float ag = act[9], as = act[10];
    bool moved = false;   // a resting object changed place (its grids are rebuilt)
    const bool grasp = ag == ag && ag >= 0.5f;
    const bool stop = as == as && as >= 0.5f;

    // 1. kinematic update
    float cand[10];
    {
        float a0 = sanitize(act[0], rp.act_lim[0]);
        float a1 = sanitize(act[1], rp.act_lim[1]);
        const float pi_f = 0x1.921fb6p+1f, two_pi_f = 0x1.921fb6p+2f;
        float yaw = st[2] + a1;
        if (yaw > pi_f) yaw = yaw - two_pi_f;
        else if (yaw < -pi_f) yaw = yaw + two_pi_f;
        float sy, cy;
        dsincos(yaw, sy, cy);
        cand[0] = st[0] + a0 * cy;
        cand[1] = st[1] + a0 * sy;
        cand[2] = yaw;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            float aj = sanitize(act[2 + j], rp.act_lim[2]);
            cand[3 + j] = clampf(st[3 + j] + aj, rp.qlim[j][0], rp.qlim[j][1]);
        }
    }
    // 2. overlap test of the candidate (its masks are reported)
    const GridMeta gm = sb.grid_meta[env];
    Fk fk;
    forward_kinematics(rp, cand, fk);
    float sx, sy;
    int n;
    uint32_t *ms_out = out.contact_static ? out.contact_static + (size_t)env * rp.contact_words : nullptr;
    uint32_t *mo_out = out.contact_object ? out.contact_object + (size_t)env * rp.contact_words : nullptr;
    const bool any = manip_pose_contacts(rp, sb, gm, env, fk, held, rel, objs, lane, ms_out, mo_out,
                                         sx, sy, n);
    // 3. resolve: commit, or slide the base (up to kSlideTries jitters away
    // from the mean overlapping sphere centre), or keep the old state
    int accepted = 0;
    if (!any) {
#pragma unroll
        for (int k = 0; k < 10; ++k) st[k] = cand[k];
        accepted = 1;
    } else if (rp.slide) {
        for (int k = 0; k < kSlideTries; ++k) {
            const float mx = sx / (float)n, my = sy / (float)n;
            const float vx = cand[0] - mx, vy = cand[1] - my;
            const float vn = sqrtf(vx * vx + vy * vy);
            if (!(vn > 1e-6f)) break;
            cand[0] = cand[0] + rp.slide_step * (vx / vn);
            cand[1] = cand[1] + rp.slide_step * (vy / vn);
            forward_kinematics(rp, cand, fk);
            if (!manip_pose_contacts(rp, sb, gm, env, fk, held, rel, objs, lane, nullptr, nullptr, sx,
                                     sy, n)) {
#pragma unroll
                for (int q = 0; q < 10; ++q) st[q] = cand[q];
                accepted = 2;
                break;
            }
        }
    }
    // 4. grasp / release at the resolved pose
    forward_kinematics(rp, st, fk);
    if (grasp && held < 0) {
        float tx, ty, tz;
        fpoint(fk.f[7], rp.grasp_tip[0], rp.grasp_tip[1], rp.grasp_tip[2], tx, ty, tz);
        const float r2 = rp.grasp_radius * rp.grasp_radius;
        unsigned long long key = ~0ull;
        if (lane < O) {
            const float d2 = obb_dist2(objs + 8 * lane, tx, ty, tz);
            if (d2 < r2) key = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned long long)lane;
        }
        // the nearest overlapping object (d2 >= 0, so its bits order like the
        // values), the smallest index among equals
        uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const uint32_t h2 = (uint32_t)__shfl_xor((int)hi, off, 64);
            const uint32_t l2 = (uint32_t)__shfl_xor((int)lo, off, 64);
            if (h2 < hi || (h2 == hi && l2 < lo)) { hi = h2; lo = l2; }
        }
        if (hi != 0xFFFFFFFFu || lo != 0xFFFFFFFFu) {
            const int best = __builtin_amdgcn_readfirstlane((int)lo);
            rel = fmul(frame_inverse(fk.f[7]), object_frame(objs + 8 * best));
            held = best;
        }
    } else if (!grasp && held >= 0) {
        const Frame F = fmul(fk.f[7], rel);
        place_object(rp, sb, gm, env, held, F, objs, episode, t, lane);
        held = -1;
        moved = true;
    }
    // 5. episode bookkeeping: horizon or stop, auto-reset (objects back too)
    bool done = false;
    t += 1;
    if (stop || (rp.episode_len > 0 && t >= rp.episode_len)) {
        episode += 1;
        load_start(rp, sb, env, episode, st);
        t = 0;
        done = true;
        held = -1;
        const float *o0 = sb.objects + (size_t)env * O * 8;
        for (int i = lane; i < O * 8; i += 64) objs[i] = o0[i];
        forward_kinematics(rp, st, fk);
        moved = true;
    }
    if (moved) {
        // the records other lanes wrote are read below: fence the wave
        __threadfence_block();
        if (sb.objgrid_mask) objgrid_rebuild(rp, sb, env, objs, lane);
    }
    // 6. outputs
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 10; ++k) sb.state[(size_t)env * 10 + k] = st[k];
        sb.counters[(size_t)env * 2 + 0] = t;
        sb.counters[(size_t)env * 2 + 1] = episode;
        sb.held_obj[env] = held;
#pragma unroll
        for (int k = 0; k < 12; ++k) sb.rel[(size_t)env * 12 + k] = rel.m[k];
        float cam[12];
        write_camera(rp, fk.f[0], cam);
#pragma unroll
        for (int k = 0; k < 12; ++k) sb.camera[(size_t)env * 12 + k] = cam[k];
        if (out.state)
#pragma unroll
            for (int k = 0; k < 10; ++k) out.state[(size_t)env * 10 + k] = st[k];
        if (out.counters) {
            out.counters[(size_t)env * 2 + 0] = t;
            out.counters[(size_t)env * 2 + 1] = episode;
        }
        if (out.accepted) out.accepted[env] = (uint8_t)accepted;
        if (out.done) out.done[env] = done ? 1 : 0;
        if (out.held) out.held[env] = held;
    }
    if ((out.frames || rp.links) && lane < 8) {
        Frame F = pick(fk, lane);
        if (out.frames) {
            float *dst = out.frames + ((size_t)env * 8 + lane) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) dst[k] = F.m[k];
        }
        if (rp.links) {
            float *dst = sb.link_frames + ((size_t)env * 8 + lane) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) dst[k] = F.m[k];
        }
    }
    if (lane < O) {
        const Frame Fo = lane == held ? fmul(fk.f[7], rel) : object_frame(objs + 8 * lane);
        float *dst = sb.obj_frames + ((size_t)env * O + lane) * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) dst[k] = Fo.m[k];
        if (out.object_frames) {
            float *d2 = out.object_frames + ((size_t)env * O + lane) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) d2[k] = Fo.m[k];
        }
    }
}

// Object frames of the current state (one wave per env).
__global__ __launch_bounds__(256) void k_object_frames(RobotParams rp, SimBuffers sb)
{
    const int lane = threadIdx.x & 63;
    const int env = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)threadIdx.x / 64);
    if (env >= sb.num_envs) return;
    const int O = rp.num_objects;
    float st[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) st[k] = sb.state[(size_t)env * 10 + k];
    const int held = sb.held_obj[env];
    Fk fk;
    forward_kinematics(rp, st, fk);
    Frame rel;
#pragma unroll
    for (int k = 0; k < 12; ++k) rel.m[k] = sb.rel[(size_t)env * 12 + k];
    if (lane < O) {
        const Frame Fo = lane == held ? fmul(fk.f[7], rel)
                                      : object_frame(sb.obj_dyn + ((size_t)env * O + lane) * 8);
        float *dst = sb.obj_frames + ((size_t)env * O + lane) * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) dst[k] = Fo.m[k];
    }
    if (sb.objgrid_mask) objgrid_rebuild(rp, sb, env, sb.obj_dyn + (size_t)env * O * 8, lane);
}

// The object grids of every env (one wave per env) from the resting records.
__global__ __launch_bounds__(256) void k_objgrid_build(RobotParams rp, SimBuffers sb)
{
    const int lane = threadIdx.x & 63;
    const int env = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)threadIdx.x / 64);
    if (env >= sb.num_envs) return;
    const float *objs = (rp.manip ? sb.obj_dyn : sb.objects) + (size_t)env * rp.num_objects * 8;
    objgrid_rebuild(rp, sb, env, objs, lane);
}

// New episode for the selected envs (mask null = all): episode += 1, start
// pose of that episode, arm at home, step counter 0; camera refreshed.
__global__ void k_reset(RobotParams rp, SimBuffers sb, const uint8_t *__restrict__ mask)
{
    const int env = blockIdx.x * blockDim.x + threadIdx.x;
    if (env >= sb.num_envs) return;
    if (mask && !mask[env]) return;
    int episode = sb.counters[(size_t)env * 2 + 1] + 1;
    float st[10];
    load_start(rp, sb, env, episode, st);
    for (int k = 0; k < 10; ++k) sb.state[(size_t)env * 10 + k] = st[k];
    sb.counters[(size_t)env * 2 + 0] = 0;
    sb.counters[(size_t)env * 2 + 1] = episode;
    if (rp.manip) {
        // the movable objects return to their places, nothing is held
        const int O = rp.num_objects;
        for (int i = 0; i < O * 8; ++i) sb.obj_dyn[(size_t)env * O * 8 + i] = sb.objects[(size_t)env * O * 8 + i];
        sb.held_obj[env] = -1;
    }
    float s, c;
    dsincos(st[2], s, c);
    Frame F0;
    F0.m[0] = c;    F0.m[1] = -s;   F0.m[2] = 0.0f;  F0.m[3] = st[0];
    F0.m[4] = s;    F0.m[5] = c;    F0.m[6] = 0.0f;  F0.m[7] = st[1];
    F0.m[8] = 0.0f; F0.m[9] = 0.0f; F0.m[10] = 1.0f; F0.m[11] = 0.0f;
    float cam[12];
    write_camera(rp, F0, cam);
    for (int k = 0; k < 12; ++k) sb.camera[(size_t)env * 12 + k] = cam[k];
}

}  // namespace

hipError_t launch_robot_step(const RobotParams &rp, const SimBuffers &sb, const float *actions,
                             const StepOutputs &out, uint32_t *queue_reset, int lanes_per_env,
                             const ItemOrder &ord, hipStream_t s)
{
    if (ord.n < 0 || ord.n > kOrderCap || (ord.n > 0 && (!ord.cost || !ord.order)))
        return hipErrorInvalidValue;
    const int extra = ord.n > 0 ? 1 : 0;
    if (rp.manip) {
        const int blocks = (sb.num_envs + 3) / 4 + extra;
        hipLaunchKernelGGL(k_robot_step_manip, dim3(blocks), dim3(256), 0, s, rp, sb, actions, out,
                           queue_reset, ord);
        return hipGetLastError();
    }
    if (lanes_per_env == 32) {
        const int blocks = (sb.num_envs + 7) / 8 + extra;
        hipLaunchKernelGGL(k_robot_step<32>, dim3(blocks), dim3(256), 0, s, rp, sb, actions, out,
                           queue_reset, ord);
    } else {
        const int blocks = (sb.num_envs + 3) / 4 + extra;
        hipLaunchKernelGGL(k_robot_step<64>, dim3(blocks), dim3(256), 0, s, rp, sb, actions, out,
                           queue_reset, ord);
    }
    return hipGetLastError();
}

hipError_t launch_robot_step(const RobotParams &rp, const SimBuffers &sb, const float *actions,
                             const StepOutputs &out, uint32_t *queue_reset, int lanes_per_env,
                             hipStream_t s)
{
    return launch_robot_step(rp, sb, actions, out, queue_reset, lanes_per_env, ItemOrder{nullptr, 0, nullptr},
                             s);
}

hipError_t launch_reset(const RobotParams &rp, const SimBuffers &sb, const uint8_t *mask,
                        hipStream_t s)
{
    const int blocks = (sb.num_envs + 255) / 256;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, s, rp, sb, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !rp.manip) return e;
    return launch_object_frames(rp, sb, s);
}

hipError_t launch_objgrid_build(const RobotParams &rp, const SimBuffers &sb, hipStream_t s)
{
    if (!sb.objgrid_mask || sb.num_envs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_objgrid_build, dim3((sb.num_envs + 3) / 4), dim3(256), 0, s, rp, sb);
    return hipGetLastError();
}

hipError_t launch_object_frames(const RobotParams &rp, const SimBuffers &sb, hipStream_t s)
{
    if (!rp.manip || sb.num_envs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_object_frames, dim3((sb.num_envs + 3) / 4), dim3(256), 0, s, rp, sb);
    return hipGetLastError();
}

}  // namespace gal
