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
// layer range, then its first two layers, then (rarely) the rest.  Contact
// when the centre is outside the grid or inside no free layer [lo, hi]
// (touching a layer bound counts as free).
struct GridProbe {
    bool outside;
    uint32_t l0, l1;
    float z;
    float2 a, b;   // layers l0 and l0 + 1 when present
};

__device__ __forceinline__ void grid_probe_column(const SimBuffers &sb, const GridMeta &gm,
                                                  uint64_t off_base, float x, float y, float z,
                                                  GridProbe &g)
{
    g.z = z;
    g.l0 = g.l1 = 0;
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

__device__ __forceinline__ void grid_probe_layers(const SimBuffers &sb, uint64_t layer_base, GridProbe &g)
{
    const float2 *lay = sb.grid_layers + layer_base;
    if (g.l0 < g.l1) g.a = lay[g.l0];
    if (g.l0 + 1 < g.l1) g.b = lay[g.l0 + 1];
}

__device__ __forceinline__ bool grid_probe_contact(const SimBuffers &sb, uint64_t layer_base,
                                                   const GridProbe &g)
{
    if (g.outside) return true;
    const float z = g.z;
    if (g.l0 < g.l1 && g.a.x <= z && z <= g.a.y) return false;
    if (g.l0 + 1 < g.l1 && g.b.x <= z && z <= g.b.y) return false;
    const float2 *lay = sb.grid_layers + layer_base;
    for (uint32_t l = g.l0 + 2; l < g.l1; ++l) {
        const float2 L = lay[l];
        if (L.x <= z && z <= L.y) return false;
    }
    return true;
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
        if (active && s < rp.num_spheres) {
            sl.sp[k] = sb.spheres[s];
            if (!(sl.sp[k].held_only && !held)) {
                sl.live[k] = true;
                const size_t gk = (size_t)env * rp.num_classes + sl.sp[k].cls;
                sl.off_base[k] = sb.grid_off_base[gk];
                sl.layer_base[k] = sb.grid_layer_base[gk];
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
    const float *objs = sb.objects + (size_t)env * rp.num_objects * 8;
    // surrogate routing: 1 = static check skipped (no contact assumed),
    // 2 = skipped but audited (exact check runs; a contact is a mismatch)
    const int route = sb.skip_flags ? sb.skip_flags[env] : 0;
    bool any = false, any_static = false;
    for (int base = 0; base < rp.num_spheres; base += kSlots * kLanes) {
        GridProbe g[kSlots];
        float cx[kSlots], cy[kSlots], cz[kSlots];
        const bool grid = route != 1;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            g[k].outside = false;
            g[k].l0 = g[k].l1 = 0;
            cx[k] = cy[k] = cz[k] = 0.0f;
            if (sl.live[k]) {
                const Frame F = pick(fk, sl.sp[k].link);
                fpoint(F, sl.sp[k].px, sl.sp[k].py, sl.sp[k].pz, cx[k], cy[k], cz[k]);
                if (grid) grid_probe_column(sb, gm, sl.off_base[k], cx[k], cy[k], cz[k], g[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (sl.live[k] && grid) grid_probe_layers(sb, sl.layer_base[k], g[k]);
        bool hit_static[kSlots], hit_object[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            hit_static[k] = false;
            hit_object[k] = false;
            if (sl.live[k]) {
                if (grid) hit_static[k] = grid_probe_contact(sb, sl.layer_base[k], g[k]);
                const float r = rp.class_radius[sl.sp[k].cls];
                for (int o = 0; o < rp.num_objects; ++o) {
                    if (obb_contact(objs + 8 * o, cx[k], cy[k], cz[k], r)) {
                        hit_object[k] = true;
                        break;
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
    if (out.frames && sub < 8) {
        Frame F = pick(fk, sub);
        float *dst = out.frames + ((size_t)env * 8 + sub) * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) dst[k] = F.m[k];
    }
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
    return hipGetLastError();
}

}  // namespace gal
