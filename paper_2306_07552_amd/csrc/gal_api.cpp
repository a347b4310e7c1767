// Host runtime of the C ABI declared in include/gal.h: validation, device
// buffers, render-cluster construction, column-grid construction (on the
// device) and the asynchronous step / reset launches.
#include "gal.h"
#include "gal_internal.h"
#include "gal_mlp.h"
#include "gal_order.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

static_assert(GAL_MAX_PLANES == gal::kMaxPlanes, "plane table bound of the ABI and the kernels");

namespace {

// events of one profiled step: before the surrogate, before the robot step,
// before the raster, after the raster
constexpr int kProfileEvents = 4;

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(GAL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

struct DevAlloc {
    std::vector<void *> ptrs;
    ~DevAlloc()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    int alloc(T **out, size_t count)
    {
        void *p = nullptr;
        size_t bytes = std::max<size_t>(count * sizeof(T), 16);
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess)
            return fail(GAL_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        ptrs.push_back(p);
        *out = static_cast<T *>(p);
        return GAL_OK;
    }
};

// Clusters of one env: <= 64 consecutive triangles using <= 64 unique vertices
// and lying on <= 4 distinct face planes.
struct EnvClusters {
    std::vector<float> cl;        // [C][12] words (see RenderMesh), bases relative to env
    std::vector<float> verts;     // [Vc][3]
    std::vector<uint32_t> tris;   // [T]
    std::vector<float> planes;    // [P][4] distinct face planes of the env (bit patterns)
    std::vector<uint16_t> pidx;   // [T] each triangle's index in `planes` (with face planes)
    int bad = 0;                  // 1 = triangle index out of range, 2 = too many planes
};

// Index of plane `pl` in the env's table (added when new), or -1 when the
// table is full.
int plane_index(const float *pl, std::vector<float> &table, std::unordered_map<std::string, int> &seen)
{
    const std::string key(reinterpret_cast<const char *>(pl), 4 * sizeof(float));
    auto it = seen.find(key);
    if (it != seen.end()) return it->second;
    const int idx = (int)(table.size() / 4);
    if (idx >= GAL_MAX_PLANES) return -1;
    table.insert(table.end(), pl, pl + 4);
    seen.emplace(key, idx);
    return idx;
}

constexpr int kFaceSplitMin = 24;

void build_env_clusters(const float *verts, int64_t nverts, const int32_t *tris, int64_t ntris,
                        const float *tri_plane, EnvClusters &out)
{
    std::vector<int64_t> mark(std::max<int64_t>(nverts, 1), -1);
    std::vector<int32_t> lidx(std::max<int64_t>(nverts, 1), 0);
    out.tris.reserve(ntris);
    out.verts.reserve(ntris * 3 / 2 + 64);
    int64_t cid = 0;
    int nv = 0, nt = 0;
    int64_t vstart = 0, tstart = 0;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    // the cluster's face planes (env table indices); without planes every
    // slot is gal::kNoPlane (never culled by a plane)
    int cpl[gal::kClusterPlanes];
    int ncpl = 0;
    std::unordered_map<std::string, int> seen;
    auto close = [&]() {
        if (nt == 0) return;
        float w[12];
        uint32_t vb = (uint32_t)vstart, tb = (uint32_t)tstart, cnt = (uint32_t)nv | ((uint32_t)nt << 8);
        uint32_t first = (uint32_t)tstart;
        // unused plane slots repeat the first plane, so "any plane in front" is unchanged
        uint32_t ps[gal::kClusterPlanes];
        for (int k = 0; k < gal::kClusterPlanes; ++k)
            ps[k] = ncpl ? (uint32_t)cpl[k < ncpl ? k : 0] : gal::kNoPlane;
        const uint32_t p01 = ps[0] | (ps[1] << 16), p23 = ps[2] | (ps[3] << 16);
        w[0] = lo[0]; w[1] = lo[1]; w[2] = lo[2]; memcpy(&w[3], &vb, 4);
        w[4] = hi[0]; w[5] = hi[1]; w[6] = hi[2]; memcpy(&w[7], &tb, 4);
        memcpy(&w[8], &cnt, 4); memcpy(&w[9], &first, 4); memcpy(&w[10], &p01, 4);
        memcpy(&w[11], &p23, 4);
        out.cl.insert(out.cl.end(), w, w + 12);
        ++cid;
        nv = nt = 0;
        ncpl = 0;
        vstart = (int64_t)out.verts.size() / 3;
        tstart = (int64_t)out.tris.size();
        for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    };
    for (int64_t t = 0; t < ntris; ++t) {
        int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
        for (int k = 0; k < 3; ++k)
            if (v[k] < 0 || v[k] >= nverts) { out.bad = 1; return; }
        int fresh = 0;
        for (int k = 0; k < 3; ++k) {
            bool was = mark[v[k]] == cid;
            for (int q = 0; q < k; ++q) was = was || v[q] == v[k];
            fresh += was ? 0 : 1;
        }
        int pidx = -1, pslot = -1;
        if (tri_plane) {
            pidx = plane_index(tri_plane + 4 * t, out.planes, seen);
            if (pidx < 0) { out.bad = 2; return; }
            for (int k = 0; k < ncpl; ++k)
                if (cpl[k] == pidx) pslot = k;
        }
        // a new face plane also starts a new cluster once the current one holds
        // kFaceSplitMin triangles, so that most clusters lie on one face and are
        // culled whole when it faces away
        if (nt == gal::kClusterTris || nv + fresh > gal::kClusterVerts ||
            (tri_plane && pslot < 0 && ncpl == gal::kClusterPlanes) ||
            (tri_plane && pslot < 0 && ncpl > 0 && nt >= kFaceSplitMin)) {
            close();
            pslot = -1;
        }
        if (tri_plane && pslot < 0) {
            pslot = ncpl;
            cpl[ncpl++] = pidx;
        }
        if (tri_plane) out.pidx.push_back((uint16_t)pidx);
        uint32_t packed = tri_plane ? (uint32_t)pslot << 24 : 0u;
        for (int k = 0; k < 3; ++k) {
            if (mark[v[k]] != cid) {
                mark[v[k]] = cid;
                lidx[v[k]] = nv++;
                const float *p = verts + 3 * (int64_t)v[k];
                out.verts.insert(out.verts.end(), p, p + 3);
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], p[a]);
                    hi[a] = std::max(hi[a], p[a]);
                }
            }
            packed |= (uint32_t)lidx[v[k]] << (8 * k);
        }
        out.tris.push_back(packed);
        ++nt;
    }
    close();
}

template <class F>
void parallel_for(int64_t n, F &&f)
{
    unsigned hc = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    for (unsigned i = 0; i < hc; ++i)
        th.emplace_back([&]() {
            for (;;) {
                int64_t k = next.fetch_add(1);
                if (k >= n) break;
                f(k);
            }
        });
    for (auto &t : th) t.join();
}

}  // namespace

namespace gal {
int api_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
int mlp_max_rows(const gal_mlp *m);
}  // namespace gal

struct gal_batch {
    DevAlloc mem;
    int32_t N = 0, S = 0, K = 0, O = 0, P = 0, words = 0;
    uint32_t flags = 0;
    gal::RobotParams rp{};
    gal::SimBuffers sb{};
    gal::RenderMesh mesh{};
    gal::RasterParams rast{};
    std::vector<int64_t> depth_off_host;   // [N+1]
    std::vector<int32_t> res_host;
    std::vector<gal::GridMeta> meta_host;
    std::vector<uint64_t> off_base_host, layer_base_host;
    int32_t *d_res = nullptr;
    uint64_t *d_depth_off = nullptr;
    uint32_t *d_work = nullptr;
    uint32_t *d_item_cost = nullptr;        // last step's time per work item
    uint32_t *d_item_order = nullptr;       // queue position -> work item
    int32_t num_work = 0;
    int32_t max_res = 0;
    int64_t n_clusters = 0, n_cverts = 0, n_tris = 0;
    unsigned long long *d_stats = nullptr;  // raster work counters (allocated on demand)
    std::vector<int64_t> cl_count_host;    // clusters per env
    int32_t work_cap = 0;
    uint32_t *d_queue = nullptr;            // persistent raster work-queue counter
    // surrogate pre-filter
    gal_mlp *sur = nullptr;
    float sur_thr_logit = 0.0f;
    uint32_t sur_audit = 16;
    uint8_t *d_flags = nullptr;             // [N] routing
    uint8_t *d_layer_hint = nullptr;        // [N][S] column-layer cache (allocated when first enabled)
    unsigned long long *d_sur_stats = nullptr;
    uint8_t *d_occ = nullptr;               // occupancy lattice (built on first use)
    uint64_t *d_occ_off = nullptr;
    int32_t *d_occ_dims = nullptr;
    int32_t occ_max_cells = 0;
    int32_t persist_grid = 0;
    int32_t robot_lanes = 64;
    int32_t use_graph = 0;
    int32_t split = 0;   // cheapest envs rendered with halved regions
    uint64_t tune_gen = 1;                  // bumps on every tuning change
    // autotuner scratch (allocated on the first gal_autotune, reused after)
    float *tune_st0 = nullptr;
    int32_t *tune_cnt0 = nullptr;
    float *tune_obj0 = nullptr;      // manipulation: objects, held, rel
    int32_t *tune_held0 = nullptr;
    float *tune_rel0 = nullptr;
    unsigned long long *tune_hash = nullptr;
    // captured step graph and what it was captured for
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const float *g_actions = nullptr;
    gal_outputs g_out{};
    uint64_t g_gen = 0;
    // per-kernel timing
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;     // free events
    std::vector<hipEvent_t> ev_rec;      // recorded triples (start, mid, end)
    ~gal_batch()
    {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_rec) (void)hipEventDestroy(e);
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
    }
    hipEvent_t take_event()
    {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

namespace {

int enqueue_step(gal_batch *b, const float *actions_dev, const gal_outputs *out, hipStream_t s,
                 hipEvent_t *ev);

// Region side of env e's items: the tuned region (or the resolution, if
// smaller), halved for the `split` cheapest envs when it stays a multiple of 8.
int item_region(const gal_batch *b, int e, bool half)
{
    const int R = std::min(b->res_host[e], b->rast.region);
    return (half && R % 16 == 0) ? R / 2 : R;
}

// (env, region) work items, longest envs first (so the tail of the launch is
// short), regions of one env 8 items apart (same XCD, shared L2).  Item word:
// env (bits 0..19), region index (20..30), halved region (31).
int build_work(gal_batch *b)
{
    const int N = b->N;
    std::vector<int32_t> order(N);
    for (int e = 0; e < N; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        const double ca = (double)b->cl_count_host[a] + 1e-3 * b->res_host[a] * b->res_host[a];
        const double cc = (double)b->cl_count_host[c] + 1e-3 * b->res_host[c] * b->res_host[c];
        return ca > cc;
    });
    std::vector<uint32_t> work;
    const int first_half = N - std::min(std::max(b->split, 0), N);
    for (int g = 0; g < N; g += 8) {
        int maxreg = 0;
        for (int k = g; k < std::min(N, g + 8); ++k) {
            const int r = b->res_host[order[k]];
            const int R = item_region(b, order[k], k >= first_half);
            maxreg = std::max(maxreg, (r / R) * (r / R));
        }
        for (int reg = 0; reg < maxreg; ++reg)
            for (int k = g; k < std::min(N, g + 8); ++k) {
                const int e = order[k];
                const int r = b->res_host[e];
                const int R = item_region(b, e, k >= first_half);
                const uint32_t half = R < std::min(r, b->rast.region) ? 1u : 0u;
                if (reg < (r / R) * (r / R))
                    work.push_back((uint32_t)e | ((uint32_t)reg << 20) | (half << 31));
            }
    }
    if ((int32_t)work.size() > b->work_cap) {
        int rc;
        if ((rc = b->mem.alloc(&b->d_work, work.size())) || (rc = b->mem.alloc(&b->d_item_cost, work.size())) ||
            (rc = b->mem.alloc(&b->d_item_order, work.size())))
            return rc;
        b->work_cap = (int32_t)work.size();
    }
    b->num_work = (int32_t)work.size();
    // until items have been timed: the static order (costs decreasing along it)
    std::vector<uint32_t> cost(work.size()), ord(work.size());
    for (size_t i = 0; i < work.size(); ++i) {
        cost[i] = (uint32_t)(work.size() - i);
        ord[i] = (uint32_t)i;
    }
    hipError_t e = hipMemcpy(b->d_work, work.data(), sizeof(uint32_t) * work.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_item_cost, cost.data(), sizeof(uint32_t) * cost.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_item_order, ord.data(), sizeof(uint32_t) * ord.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(GAL_EDEVICE, "hipMemcpy(work) failed: %s", hipGetErrorString(e));
    b->rast.item_cost = b->d_item_cost;
    b->rast.item_order = b->d_item_order;
    return GAL_OK;
}

}  // namespace

extern "C" {

const char *gal_last_error(void) { return g_last_error.c_str(); }

int gal_get_tuning(const gal_batch *b, gal_tuning *t)
{
    if (!b || !t) return fail(GAL_EINVAL, "null argument");
    t->block = b->rast.block;
    t->region = b->rast.region;
    t->lane_max = b->rast.lane_max;
    t->small_max = b->rast.small_max;
    t->refresh = b->rast.refresh;
    t->occlusion = b->rast.occlusion;
    t->prologue = b->rast.prologue;
    t->persistent = b->rast.persistent;
    t->robot_lanes = b->robot_lanes;
    t->graph = b->use_graph;
    t->split = b->split;
    t->order = b->rast.order;
    t->objgrid = b->rp.objgrid;
    t->bin = b->rast.bin;
    t->layer_cache = b->sb.layer_hint != nullptr ? 1 : 0;
    return GAL_OK;
}

int gal_set_tuning(gal_batch *b, const gal_tuning *t)
{
    if (!b || !t) return fail(GAL_EINVAL, "null argument");
    if (t->block != 256 && t->block != 512 && t->block != 1024)
        return fail(GAL_EINVAL, "block must be 256, 512 or 1024");
    if (t->region != 32 && t->region != 64 && t->region != 128)
        return fail(GAL_EINVAL, "region must be 32, 64 or 128");
    for (int e = 0; e < b->N; ++e)
        if (b->res_host[e] > t->region && b->res_host[e] % t->region != 0)
            return fail(GAL_EINVAL, "region %d does not divide resolution %d", t->region, b->res_host[e]);
    if (t->small_max < 0 || t->small_max > 65536) return fail(GAL_EINVAL, "small_max out of range");
    if (t->lane_max < 0 || t->lane_max > 4096) return fail(GAL_EINVAL, "lane_max out of range");
    if (t->refresh < 1 || t->refresh > 16) return fail(GAL_EINVAL, "refresh must be in 1..16");
    if (t->prologue < 0) return fail(GAL_EINVAL, "prologue must be >= 0");
    if (t->robot_lanes != 32 && t->robot_lanes != 64) return fail(GAL_EINVAL, "robot_lanes must be 32 or 64");
    if (t->split < 0 || t->split > b->N) return fail(GAL_EINVAL, "split must be in 0..num_envs");
    if (t->order != 0 && t->order != 1) return fail(GAL_EINVAL, "order must be 0 or 1");
    if (t->objgrid != 0 && t->objgrid != 1) return fail(GAL_EINVAL, "objgrid must be 0 or 1");
    if (t->bin != 0 && t->bin != 1) return fail(GAL_EINVAL, "bin must be 0 or 1");
    if (t->layer_cache != 0 && t->layer_cache != 1) return fail(GAL_EINVAL, "layer_cache must be 0 or 1");
    if (t->layer_cache && b->rp.manip) return fail(GAL_EINVAL, "the layer cache serves the plain robot step, not GAL_MANIP");
    if (t->layer_cache && !b->d_layer_hint) {
        int rc = b->mem.alloc(&b->d_layer_hint, (size_t)b->N * (size_t)b->S);
        if (rc) return rc;
        HIP_TRY(hipMemset(b->d_layer_hint, 0, (size_t)b->N * (size_t)b->S));
    }
    {
        gal::RasterParams probe = b->rast;
        probe.block = t->block;
        probe.region = t->region;
        probe.bin = t->bin;
        if (!gal::raster_fits(probe, b->max_res, (b->flags & GAL_COLOR) != 0))
            return fail(GAL_EINVAL, "block %d region %d%s: the z-buffer and bins exceed the 160 KB of LDS",
                        t->block, t->region, (b->flags & GAL_COLOR) ? " with colour" : "");
    }
    const bool rebuild = t->region != b->rast.region || t->split != b->split;
    b->rast.block = t->block;
    b->rast.region = t->region;
    b->rast.lane_max = t->lane_max;
    b->rast.small_max = t->small_max;
    b->rast.refresh = t->refresh;
    b->rast.occlusion = t->occlusion ? 1 : 0;
    b->rast.prologue = t->prologue;
    b->rast.persistent = t->persistent ? 1 : 0;
    b->robot_lanes = t->robot_lanes;
    b->use_graph = t->graph ? 1 : 0;
    b->split = t->split;
    b->rast.order = t->order;
    b->rp.objgrid = t->objgrid;
    b->rast.bin = t->bin;
    b->sb.layer_hint = t->layer_cache ? b->d_layer_hint : nullptr;
    b->tune_gen += 1;
    b->persist_grid = gal::raster_persistent_grid(b->rast, b->max_res, (b->flags & GAL_COLOR) != 0);
    if (b->persist_grid <= 0) return fail(GAL_EDEVICE, "occupancy query for the persistent raster kernel failed");
    if (rebuild) {
        HIP_TRY(hipDeviceSynchronize());
        return build_work(b);
    }
    return GAL_OK;
}

int gal_autotune(gal_batch *b, const float *actions_dev, const gal_outputs *out, void *stream,
                 int32_t steps, gal_tuning *best, double *best_ms)
{
    if (!b || !actions_dev || !out || !out->depth) return fail(GAL_EINVAL, "null argument");
    if (steps < 1) return fail(GAL_EINVAL, "steps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    gal_tuning orig;
    gal_get_tuning(b, &orig);
    const bool was_profiling = b->profiling;
    b->profiling = false;
    // saved simulation state (restored before every candidate and at the end);
    // the buffers are allocated once per batch and reused by later calls
    int rc;
    if (!b->tune_st0 &&
        ((rc = b->mem.alloc(&b->tune_st0, (size_t)b->N * 10)) ||
         (rc = b->mem.alloc(&b->tune_cnt0, (size_t)b->N * 2)) || (rc = b->mem.alloc(&b->tune_hash, 1))))
        return rc;
    const size_t nobj = (size_t)b->N * b->O * 8;
    if (b->rp.manip && !b->tune_obj0 &&
        ((rc = b->mem.alloc(&b->tune_obj0, std::max<size_t>(nobj, 1))) ||
         (rc = b->mem.alloc(&b->tune_held0, (size_t)b->N)) || (rc = b->mem.alloc(&b->tune_rel0, (size_t)b->N * 12))))
        return rc;
    float *st0 = b->tune_st0;
    int32_t *cnt0 = b->tune_cnt0;
    unsigned long long *hash = b->tune_hash;
    HIP_TRY(hipMemcpyAsync(st0, b->sb.state, sizeof(float) * b->N * 10, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(cnt0, b->sb.counters, sizeof(int32_t) * b->N * 2, hipMemcpyDeviceToDevice, s));
    if (b->rp.manip) {
        HIP_TRY(hipMemcpyAsync(b->tune_obj0, b->sb.obj_dyn, sizeof(float) * nobj, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->tune_held0, b->sb.held_obj, sizeof(int32_t) * b->N, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->tune_rel0, b->sb.rel, sizeof(float) * b->N * 12, hipMemcpyDeviceToDevice, s));
    }
    // the surrogate's query counters are not the tuner's to change: saved here,
    // restored at the end
    unsigned long long sur_stats0[4] = {0, 0, 0, 0};
    if (b->d_sur_stats) {
        HIP_TRY(hipMemcpyAsync(sur_stats0, b->d_sur_stats, sizeof(sur_stats0), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // likewise the raster work counters: off while tuning
    unsigned long long *stats_on = b->rast.stats;
    b->rast.stats = nullptr;
    auto restore = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(b->sb.state, st0, sizeof(float) * b->N * 10, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->sb.counters, cnt0, sizeof(int32_t) * b->N * 2, hipMemcpyDeviceToDevice, s));
        if (b->rp.manip) {
            HIP_TRY(hipMemcpyAsync(b->sb.obj_dyn, b->tune_obj0, sizeof(float) * nobj, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(b->sb.held_obj, b->tune_held0, sizeof(int32_t) * b->N, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(b->sb.rel, b->tune_rel0, sizeof(float) * b->N * 12, hipMemcpyDeviceToDevice, s));
            HIP_TRY(gal::launch_object_frames(b->rp, b->sb, s));
        }
        return GAL_OK;
    };
    std::vector<gal_tuning> cands;
    const int regions[2] = {64, 128};
    for (int block : {256, 512, 1024})
        for (int region : regions)
            for (int lane_max : {4, 8, 16})
                for (int small_max : {256, 1024})
                    for (int occl : {0, 1})   // 1: one refresh after a 128-cluster prologue
                        for (int persist : {0, 1})
                            for (int rl : {64}) {
                                bool ok = true;
                                for (int e = 0; e < b->N && ok; ++e)
                                    if (b->res_host[e] > region && b->res_host[e] % region) ok = false;
                                if (!ok) continue;
                                gal_tuning t = orig;
                                t.block = block;
                                t.region = region;
                                t.lane_max = lane_max;
                                t.small_max = small_max;
                                t.occlusion = occl;
                                t.refresh = 1;
                                t.prologue = 128;
                                t.persistent = persist;
                                t.robot_lanes = rl;
                                t.graph = 0;
                                t.split = 0;
                                t.order = 0;
                                t.bin = 0;
                                cands.push_back(t);
                            }
    // binned candidates (mid-sized triangles listed per 8x8 tile in LDS)
    for (int block : {256, 512, 1024})
        for (int region : regions)
            for (int lane_max : {4, 8})
                for (int small_max : {256})
                    for (int persist : {0, 1}) {
                        bool ok = true;
                        for (int e = 0; e < b->N && ok; ++e)
                            if (b->res_host[e] > region && b->res_host[e] % region) ok = false;
                        gal::RasterParams probe = b->rast;
                        probe.block = block;
                        probe.region = region;
                        probe.bin = 1;
                        if (!ok || !gal::raster_fits(probe, b->max_res, (b->flags & GAL_COLOR) != 0)) continue;
                        gal_tuning t = orig;
                        t.block = block;
                        t.region = region;
                        t.lane_max = lane_max;
                        t.small_max = small_max;
                        t.occlusion = 1;
                        t.refresh = 1;
                        t.prologue = 128;
                        t.persistent = persist;
                        t.robot_lanes = 64;
                        t.graph = 0;
                        t.split = 0;
                        t.order = 0;
                        t.bin = 1;
                        cands.push_back(t);
                    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        b->rast.stats = stats_on;
        b->profiling = was_profiling;
        return fail(GAL_EDEVICE, "autotune: hipEventCreate failed");
    }
    double best_t = 1e30;
    gal_tuning best_c = orig;
    unsigned long long ref_hash = 0;
    bool have_ref = false;
    // One candidate: one step from the saved state (its depth hash must equal
    // the first candidate's), then `steps` timed steps.
    auto evaluate = [&](const gal_tuning &t, int nsteps) -> int {
        int r;
        if ((r = gal_set_tuning(b, &t))) return r;
        if ((r = restore())) return r;
        if ((r = enqueue_step(b, actions_dev, out, s, nullptr))) return r;
        if (hipSuccess != gal::launch_hash_u32(out->depth, (uint64_t)b->depth_off_host[b->N], hash, s))
            return fail(GAL_EDEVICE, "hash launch failed");
        unsigned long long h = 0;
        if (hipMemcpyAsync(&h, hash, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(GAL_EDEVICE, "autotune: device error");
        if (!have_ref) {
            ref_hash = h;
            have_ref = true;
        } else if (h != ref_hash) {
            return fail(GAL_ESTATE, "autotune: candidate (block %d region %d lane_max %d small_max %d "
                        "occlusion %d persistent %d split %d bin %d) changed the output bits",
                        t.block, t.region, t.lane_max, t.small_max, t.occlusion, t.persistent, t.split, t.bin);
        }
        (void)hipEventRecord(e0, s);
        for (int k = 0; k < nsteps; ++k)
            if ((r = enqueue_step(b, actions_dev, out, s, nullptr))) return r;
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(GAL_EDEVICE, "autotune: event timing failed");
        if (ms / nsteps < best_t) {
            best_t = ms / nsteps;
            best_c = t;
        }
        return GAL_OK;
    };
    int result = GAL_OK;
    for (const gal_tuning &t : cands)
        if ((result = evaluate(t, steps))) break;
    // Second stage: halve the regions of the cheapest envs, in fractions of
    // the number of workgroups resident at once (the launch's last items), so
    // that the tail of the launch is made of short items; tried on the winner
    // and on the winner with the other launch mode (queue or one workgroup
    // per item), whose tails differ.  The winner is timed again beside them
    // (the first stage's minimum over many candidates is biased low by
    // noise), with three times the steps, in two interleaved rounds, each
    // candidate keeping its best.
    if (result == GAL_OK && (result = gal_set_tuning(b, &best_c)) == GAL_OK) {
        const int slots = b->persist_grid;
        const gal_tuning w = best_c;
        std::vector<gal_tuning> c2;
        for (int flip : {0, 1})
            for (int div : {0, 16, 8, 4, 2})
                for (int pro : {128, 256})
                    for (int ord : {0, 1}) {
                        if (!w.occlusion && pro != w.prologue) continue;
                        gal_tuning t = w;
                        if (flip) t.persistent = 1 - w.persistent;
                        if (ord && !t.persistent) continue;
                        t.split = div ? std::min(b->N, std::max(1, slots / div)) : 0;
                        if (w.occlusion) t.prologue = pro;
                        t.order = ord;
                        c2.push_back(t);
                    }
        std::vector<double> t2(c2.size(), 1e30);
        for (int round = 0; round < 2 && result == GAL_OK; ++round)
            for (size_t i = 0; i < c2.size(); ++i) {
                best_t = 1e30;
                if ((result = evaluate(c2[i], 3 * steps))) break;
                t2[i] = std::min(t2[i], best_t);
            }
        if (result == GAL_OK) {
            size_t k = 0;
            for (size_t i = 1; i < c2.size(); ++i)
                if (t2[i] < t2[k]) k = i;
            best_c = c2[k];
            best_t = t2[k];
        }
    }
    // Third stage: the robot step's lanes per env (32 or 64) on the winner,
    // in three interleaved rounds of 3 x `steps`; their difference of a few
    // microseconds per step is smaller than the spread between raster
    // candidates, so the first stage does not vary them.
    if (result == GAL_OK) {
        gal_tuning c3[2] = {best_c, best_c};
        c3[0].robot_lanes = 64;
        c3[1].robot_lanes = 32;
        double t3[2] = {1e30, 1e30};
        for (int round = 0; round < 3 && result == GAL_OK; ++round)
            for (int i = 0; i < 2; ++i) {
                best_t = 1e30;
                if ((result = evaluate(c3[i], 3 * steps))) break;
                t3[i] = std::min(t3[i], best_t);
            }
        if (result == GAL_OK) {
            const int k = t3[1] < t3[0] ? 1 : 0;
            best_c = c3[k];
            best_t = t3[k];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    best_c.graph = orig.graph;
    int rc2 = gal_set_tuning(b, result == GAL_OK ? &best_c : &orig);
    int rc3 = restore();
    (void)hipStreamSynchronize(s);
    b->profiling = was_profiling;
    b->rast.stats = stats_on;
    b->tune_gen += 1;
    if (b->d_sur_stats &&
        (hipMemcpy(b->d_sur_stats, sur_stats0, sizeof(sur_stats0), hipMemcpyHostToDevice) != hipSuccess))
        return fail(GAL_EDEVICE, "autotune: restoring the surrogate counters failed");
    if (result) return result;
    if (rc2) return rc2;
    if (rc3) return rc3;
    if (best) *best = best_c;
    if (best_ms) *best_ms = best_t;
    return GAL_OK;
}

int gal_create_batch(const gal_config *cfg, const gal_robot *robot, const gal_scene_set *sc,
                     void *stream, gal_batch **out)
{
    g_last_error.clear();
    if (!cfg || !robot || !sc || !out) return fail(GAL_EINVAL, "null argument");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    const int N = sc->num_envs;
    if (N < 1 || N > (1 << 20)) return fail(GAL_EINVAL, "num_envs %d out of range", N);
    if (cfg->num_classes < 1 || cfg->num_classes > GAL_MAX_CLASSES)
        return fail(GAL_EINVAL, "num_classes %d out of range", cfg->num_classes);
    if (robot->num_spheres < 1 || robot->num_spheres > GAL_MAX_SPHERES)
        return fail(GAL_EINVAL, "num_spheres %d out of range", robot->num_spheres);
    if (!(cfg->near_m > 0.0f) || !(cfg->far_m > cfg->near_m))
        return fail(GAL_EINVAL, "need 0 < near < far");
    if (!(cfg->cell_m > 0.0f)) return fail(GAL_EINVAL, "cell_m must be positive");
    if (sc->num_objects < 0 || sc->num_objects > gal::kMaxObjects)
        return fail(GAL_EINVAL, "num_objects %d out of range", sc->num_objects);
    if (sc->num_starts < 1) return fail(GAL_EINVAL, "need at least one start pose");
    if (cfg->episode_len < 0) return fail(GAL_EINVAL, "episode_len must be >= 0");
    if (!sc->vert_offset || !sc->verts || !sc->tri_offset || !sc->tris || !sc->box_offset ||
        !sc->grid_origin || !sc->grid_dims || !sc->starts || (sc->num_objects > 0 && !sc->objects))
        return fail(GAL_EINVAL, "missing scene array");
    if (!robot->sphere_link || !robot->sphere_pos || !robot->sphere_class)
        return fail(GAL_EINVAL, "missing sphere array");
    if ((cfg->flags & GAL_COLOR) && !sc->tri_rgb)
        return fail(GAL_EINVAL, "GAL_COLOR needs tri_rgb");
    for (int i = 0; i < robot->num_spheres; ++i) {
        if (robot->sphere_link[i] < 0 || robot->sphere_link[i] > 7)
            return fail(GAL_EINVAL, "sphere %d: link out of range", i);
        if (robot->sphere_class[i] < 0 || robot->sphere_class[i] >= cfg->num_classes)
            return fail(GAL_EINVAL, "sphere %d: class out of range", i);
    }
    for (int k = 0; k < cfg->num_classes; ++k)
        if (!(cfg->class_radius[k] > 0.0f)) return fail(GAL_EINVAL, "class radius must be > 0");
    const bool manip = (cfg->flags & GAL_MANIP) != 0;
    const bool links = (cfg->flags & GAL_LINKS) != 0;
    const bool shade = (cfg->flags & GAL_SHADE) != 0;
    if (shade && (!(cfg->flags & GAL_COLOR) || !sc->tri_plane))
        return fail(GAL_EINVAL, "GAL_SHADE needs GAL_COLOR and tri_plane (the faces' normals)");
    if ((cfg->flags & GAL_SLIDE) && !manip) return fail(GAL_EINVAL, "GAL_SLIDE needs GAL_MANIP");
    if (links) {
        if (!robot->link_box) return fail(GAL_EINVAL, "GAL_LINKS needs link_box");
        for (int l = 0; l < 8; ++l)
            for (int k = 3; k < 6; ++k)
                if (!(robot->link_box[6 * l + k] > 0.0f) || !std::isfinite(robot->link_box[6 * l + k]))
                    return fail(GAL_EINVAL, "link %d: half extents must be finite and > 0", l);
        if ((cfg->flags & GAL_COLOR) && !robot->link_rgb)
            return fail(GAL_EINVAL, "GAL_LINKS with GAL_COLOR needs link_rgb");
    }
    if (manip) {
        if (robot->held_class < 0 || robot->held_class >= cfg->num_classes)
            return fail(GAL_EINVAL, "held_class out of range");
        if (!(robot->grasp_radius > 0.0f)) return fail(GAL_EINVAL, "grasp_radius must be > 0");
        if (!(cfg->slide_step >= 0.0f) || !(cfg->place_step >= 0.0f))
            return fail(GAL_EINVAL, "slide_step and place_step must be >= 0");
        if ((cfg->flags & GAL_COLOR) && sc->num_objects > 0 && !sc->obj_rgb)
            return fail(GAL_EINVAL, "GAL_MANIP with GAL_COLOR needs obj_rgb");
    }

    gal_batch *b = new gal_batch();
    auto cleanup = [&](int code) {
        delete b;
        return code;
    };
    b->N = N;
    b->S = robot->num_spheres;
    b->K = cfg->num_classes;
    b->O = sc->num_objects;
    b->P = sc->num_starts;
    b->words = (b->S + (manip ? gal::kHeldSpheres : 0) + 31) / 32;
    b->flags = cfg->flags;

    // ---- per-env resolution, depth offsets
    b->res_host.resize(N);
    b->depth_off_host.resize(N + 1);
    b->depth_off_host[0] = 0;
    for (int e = 0; e < N; ++e) {
        int r = sc->res ? sc->res[e] : cfg->res0;
        if (r < 8 || r > 256 || (r % 8) != 0)
            return cleanup(fail(GAL_EINVAL, "env %d: resolution %d must be a multiple of 8 in [8, 256]", e, r));
        if (r > gal::kMaxRegion && (r % gal::kMaxRegion) != 0)
            return cleanup(fail(GAL_EINVAL, "env %d: resolution %d must be a multiple of %d", e, r, gal::kMaxRegion));
        b->res_host[e] = r;
        b->max_res = std::max(b->max_res, r);
        b->depth_off_host[e + 1] = b->depth_off_host[e] + (int64_t)r * r;
    }
    for (int64_t i = 0; i < sc->box_offset[N]; ++i) {
        const float *B = sc->boxes + 6 * i;
        for (int k = 0; k < 6; ++k)
            if (!std::isfinite(B[k])) return cleanup(fail(GAL_EINVAL, "static box %lld: non-finite coordinate", (long long)i));
        if (!(B[0] <= B[3] && B[1] <= B[4] && B[2] <= B[5]))
            return cleanup(fail(GAL_EINVAL, "static box %lld: min > max", (long long)i));
    }
    for (int e = 0; e < N; ++e) {
        if (sc->vert_offset[e + 1] < sc->vert_offset[e] || sc->tri_offset[e + 1] < sc->tri_offset[e] ||
            sc->box_offset[e + 1] < sc->box_offset[e])
            return cleanup(fail(GAL_EINVAL, "env %d: offsets not monotone", e));
        if (sc->grid_dims[2 * e] < 1 || sc->grid_dims[2 * e + 1] < 1 ||
            (int64_t)sc->grid_dims[2 * e] * sc->grid_dims[2 * e + 1] > (1 << 26))
            return cleanup(fail(GAL_EINVAL, "env %d: grid dims out of range", e));
    }

    // ---- robot parameters
    gal::RobotParams &rp = b->rp;
    memcpy(rp.dh, robot->dh, sizeof(rp.dh));
    memcpy(rp.qlim, robot->qlim, sizeof(rp.qlim));
    memcpy(rp.q_home, robot->q_home, sizeof(rp.q_home));
    memcpy(rp.mount, robot->mount, sizeof(rp.mount));
    memcpy(rp.cam_offset, robot->cam_offset, sizeof(rp.cam_offset));
    memcpy(rp.cam_pitch_cs, robot->cam_pitch_cs, sizeof(rp.cam_pitch_cs));
    for (int k = 0; k < gal::kMaxClasses; ++k)
        rp.class_radius[k] = k < cfg->num_classes ? cfg->class_radius[k] : 0.0f;
    memcpy(rp.act_lim, cfg->act_lim, sizeof(rp.act_lim));
    rp.num_spheres = b->S;
    rp.num_classes = b->K;
    rp.num_objects = b->O;
    rp.num_starts = b->P;
    rp.episode_len = cfg->episode_len;
    rp.contact_words = b->words;
    rp.manip = manip ? 1 : 0;
    rp.slide = (cfg->flags & GAL_SLIDE) ? 1 : 0;
    rp.links = links ? 1 : 0;
    if (manip) {
        memcpy(rp.grasp_tip, robot->grasp_tip, sizeof(rp.grasp_tip));
        rp.grasp_radius = robot->grasp_radius;
        rp.held_class = robot->held_class;
        rp.slide_step = cfg->slide_step;
        rp.place_step = cfg->place_step;
        rp.manip_seed = cfg->manip_seed;
    }

    int rc;
    // ---- spheres, per-env tables
    std::vector<gal::Sphere> sph(b->S);
    for (int i = 0; i < b->S; ++i) {
        sph[i].px = robot->sphere_pos[3 * i];
        sph[i].py = robot->sphere_pos[3 * i + 1];
        sph[i].pz = robot->sphere_pos[3 * i + 2];
        sph[i].link = robot->sphere_link[i];
        sph[i].cls = robot->sphere_class[i];
        sph[i].held_only = robot->sphere_held_only ? robot->sphere_held_only[i] : 0;
    }
    gal::Sphere *d_sph;
    float *d_state, *d_cam, *d_starts, *d_obj;
    int32_t *d_counters;
    uint8_t *d_held;
    gal::GridMeta *d_meta;
    if ((rc = b->mem.alloc(&d_sph, b->S)) || (rc = b->mem.alloc(&d_state, (size_t)N * 10)) ||
        (rc = b->mem.alloc(&d_cam, (size_t)N * 12)) || (rc = b->mem.alloc(&d_counters, (size_t)N * 2)) ||
        (rc = b->mem.alloc(&d_starts, (size_t)N * b->P * 3)) ||
        (rc = b->mem.alloc(&d_obj, (size_t)N * std::max(b->O, 1) * 8)) ||
        (rc = b->mem.alloc(&d_held, (size_t)N)) || (rc = b->mem.alloc(&d_meta, (size_t)N)))
        return cleanup(rc);
    HIP_TRY(hipMemcpy(d_sph, sph.data(), sizeof(gal::Sphere) * b->S, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_starts, sc->starts, sizeof(float) * (size_t)N * b->P * 3, hipMemcpyHostToDevice));
    if (b->O > 0)
        HIP_TRY(hipMemcpy(d_obj, sc->objects, sizeof(float) * (size_t)N * b->O * 8, hipMemcpyHostToDevice));
    {
        std::vector<uint8_t> held(N, 0);
        if (sc->held)
            for (int e = 0; e < N; ++e) held[e] = sc->held[e] ? 1 : 0;
        HIP_TRY(hipMemcpy(d_held, held.data(), N, hipMemcpyHostToDevice));
    }
    b->meta_host.resize(N);
    int32_t max_cols = 0;
    for (int e = 0; e < N; ++e) {
        b->meta_host[e].x0 = sc->grid_origin[2 * e];
        b->meta_host[e].y0 = sc->grid_origin[2 * e + 1];
        b->meta_host[e].nx = sc->grid_dims[2 * e];
        b->meta_host[e].ny = sc->grid_dims[2 * e + 1];
        max_cols = std::max(max_cols, b->meta_host[e].nx * b->meta_host[e].ny);
    }
    HIP_TRY(hipMemcpy(d_meta, b->meta_host.data(), sizeof(gal::GridMeta) * N, hipMemcpyHostToDevice));

    gal::SimBuffers &sb = b->sb;
    sb.state = d_state;
    sb.counters = d_counters;
    sb.camera = d_cam;
    sb.held = d_held;
    sb.starts = d_starts;
    sb.objects = d_obj;
    sb.spheres = d_sph;
    sb.grid_meta = d_meta;
    sb.cell = cfg->cell_m;
    sb.inv_cell = 1.0f / cfg->cell_m;
    sb.num_envs = N;
    if (manip) {
        // movable objects: resting records (a copy of those at episode start),
        // the held object and its pose in the end-effector frame, the frames
        const size_t no = (size_t)N * std::max(b->O, 1);
        if ((rc = b->mem.alloc(&sb.obj_dyn, no * 8)) || (rc = b->mem.alloc(&sb.held_obj, (size_t)N)) ||
            (rc = b->mem.alloc(&sb.rel, (size_t)N * 12)) || (rc = b->mem.alloc(&sb.obj_frames, no * 12)))
            return cleanup(rc);
        if (b->O > 0)
            HIP_TRY(hipMemcpy(sb.obj_dyn, d_obj, sizeof(float) * (size_t)N * b->O * 8, hipMemcpyDeviceToDevice));
        HIP_TRY(hipMemset(sb.held_obj, 0xFF, sizeof(int32_t) * N));
        HIP_TRY(hipMemset(sb.rel, 0, sizeof(float) * N * 12));
        HIP_TRY(hipMemset(sb.obj_frames, 0, sizeof(float) * no * 12));
    }
    if (links) {
        // link frames after each step (written by the robot step, read by the raster)
        if ((rc = b->mem.alloc(&sb.link_frames, (size_t)N * 8 * 12))) return cleanup(rc);
        HIP_TRY(hipMemset(sb.link_frames, 0, sizeof(float) * N * 8 * 12));
    }
    if (b->O > 0) {
        // the resting objects' four offset grids per env, over the column
        // grid's rectangle with a cell of margin on every side
        std::vector<gal::ObjGridMeta> og(N);
        uint64_t words = 0;
        for (int e = 0; e < N; ++e) {
            const gal::GridMeta &gm = b->meta_host[e];
            og[e].x0 = gm.x0 - gal::kObjCell;
            og[e].y0 = gm.y0 - gal::kObjCell;
            og[e].nx = (int32_t)std::ceil((double)gm.nx * cfg->cell_m / gal::kObjCell) + 3;
            og[e].ny = (int32_t)std::ceil((double)gm.ny * cfg->cell_m / gal::kObjCell) + 3;
            og[e].base = words;
            words += 4ull * (uint64_t)og[e].nx * (uint64_t)og[e].ny;
        }
        gal::ObjGridMeta *d_og;
        unsigned long long *d_mask;
        if ((rc = b->mem.alloc(&d_og, (size_t)N)) || (rc = b->mem.alloc(&d_mask, (size_t)words)))
            return cleanup(rc);
        HIP_TRY(hipMemcpy(d_og, og.data(), sizeof(gal::ObjGridMeta) * N, hipMemcpyHostToDevice));
        sb.objgrid_meta = d_og;
        sb.objgrid_mask = d_mask;
        rp.objgrid = b->O >= 16 ? 1 : 0;
        HIP_TRY(gal::launch_objgrid_build(rp, sb, nullptr));
    }

    // ---- column grids: count, scan, fill (on the device)
    {
        const int K = b->K;
        b->off_base_host.resize((size_t)N * K);
        uint64_t total_cols = 0;
        for (int e = 0; e < N; ++e)
            for (int k = 0; k < K; ++k) {
                b->off_base_host[(size_t)e * K + k] = total_cols;
                total_cols += (uint64_t)b->meta_host[e].nx * b->meta_host[e].ny + 1;
            }
        uint32_t *d_offsets;
        uint64_t *d_off_base, *d_layer_base, *d_box_off;
        float *d_boxes;
        int32_t *d_overflow;
        const int64_t nbox = sc->box_offset[N];
        std::vector<uint64_t> box_off(N + 1);
        for (int e = 0; e <= N; ++e) box_off[e] = (uint64_t)sc->box_offset[e];
        if ((rc = b->mem.alloc(&d_offsets, total_cols)) || (rc = b->mem.alloc(&d_off_base, (size_t)N * K)) ||
            (rc = b->mem.alloc(&d_layer_base, (size_t)N * K)) || (rc = b->mem.alloc(&d_box_off, (size_t)N + 1)) ||
            (rc = b->mem.alloc(&d_boxes, (size_t)std::max<int64_t>(nbox, 1) * 6)) ||
            (rc = b->mem.alloc(&d_overflow, 1)))
            return cleanup(rc);
        HIP_TRY(hipMemcpy(d_off_base, b->off_base_host.data(), sizeof(uint64_t) * N * K, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_box_off, box_off.data(), sizeof(uint64_t) * (N + 1), hipMemcpyHostToDevice));
        if (nbox > 0)
            HIP_TRY(hipMemcpy(d_boxes, sc->boxes, sizeof(float) * nbox * 6, hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(d_overflow, 0, sizeof(int32_t)));
        gal::ClassRadii radii{};
        for (int k = 0; k < K; ++k) radii.r[k] = cfg->class_radius[k];
        sb.grid_offsets = d_offsets;
        sb.grid_off_base = d_off_base;
        HIP_TRY(gal::launch_grid_count(sb, d_boxes, d_box_off, N, K, radii, max_cols, d_offsets,
                                       d_overflow, s));
        HIP_TRY(gal::launch_grid_scan(d_off_base, d_meta, N, K, d_offsets, s));
        HIP_TRY(hipStreamSynchronize(s));
        int32_t ovf = 0;
        HIP_TRY(hipMemcpy(&ovf, d_overflow, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (ovf)
            return cleanup(fail(GAL_EOVERFLOW, "a grid column is blocked by more than %d boxes",
                                gal::kGridIvCap));
        // totals -> layer bases
        b->layer_base_host.resize((size_t)N * K);
        uint64_t total_layers = 0;
        for (size_t ek = 0; ek < (size_t)N * K; ++ek) {
            const int e = (int)(ek / K);
            const uint64_t ncols = (uint64_t)b->meta_host[e].nx * b->meta_host[e].ny;
            uint32_t tot = 0;
            HIP_TRY(hipMemcpy(&tot, d_offsets + b->off_base_host[ek] + ncols, sizeof(uint32_t),
                              hipMemcpyDeviceToHost));
            b->layer_base_host[ek] = total_layers;
            total_layers += tot;
        }
        float2 *d_layers;
        if ((rc = b->mem.alloc(&d_layers, (size_t)std::max<uint64_t>(total_layers, 1))))
            return cleanup(rc);
        HIP_TRY(hipMemcpy(d_layer_base, b->layer_base_host.data(), sizeof(uint64_t) * N * K,
                          hipMemcpyHostToDevice));
        sb.grid_layers = d_layers;
        sb.grid_layer_base = d_layer_base;
        HIP_TRY(gal::launch_grid_fill(sb, d_boxes, d_box_off, N, K, radii, max_cols, d_overflow, s));
        HIP_TRY(hipStreamSynchronize(s));
    }

    // ---- render clusters (host), then upload
    {
        std::vector<EnvClusters> ec(N);
        parallel_for(N, [&](int64_t e) {
            const int64_t v0 = sc->vert_offset[e], v1 = sc->vert_offset[e + 1];
            const int64_t t0 = sc->tri_offset[e], t1 = sc->tri_offset[e + 1];
            build_env_clusters(sc->verts + 3 * v0, v1 - v0, sc->tris + 3 * t0, t1 - t0,
                               sc->tri_plane ? sc->tri_plane + 4 * t0 : nullptr, ec[e]);
        });
        std::vector<uint64_t> cl_off(N + 1, 0), tri_off(N + 1, 0), pl_off(N + 1, 0);
        uint64_t nv_tot = 0, nt_tot = 0;
        for (int e = 0; e < N; ++e) {
            if (ec[e].bad == 1) return cleanup(fail(GAL_EINVAL, "env %d: triangle index out of range", e));
            if (ec[e].bad == 2)
                return cleanup(fail(GAL_EINVAL, "env %d: more than %d distinct face planes", e, GAL_MAX_PLANES));
            pl_off[e + 1] = pl_off[e] + ec[e].planes.size() / 4;
            cl_off[e + 1] = cl_off[e] + ec[e].cl.size() / 12;
            tri_off[e + 1] = tri_off[e] + ec[e].tris.size();
            nv_tot += ec[e].verts.size() / 3;
            nt_tot += ec[e].tris.size();
        }
        // every cluster owns 64 vertex and 64 triangle slots, so the raster
        // kernel addresses them from the cluster index alone and issues those
        // loads together with the cluster record's (unused slots are zero)
        const uint64_t slots = (uint64_t)cl_off[N] * gal::kClusterVerts;
        if (slots >= (1ull << 32))
            return cleanup(fail(GAL_EINVAL, "scene set too large for 32-bit cluster slots"));
        float4 *d_cl, *d_pl;
        float *d_cv;
        uint32_t *d_ct;
        uint64_t *d_cl_off, *d_tri_off, *d_pl_off;
        if ((rc = b->mem.alloc(&d_cl, (size_t)cl_off[N] * 3)) || (rc = b->mem.alloc(&d_cv, slots * 3)) ||
            (rc = b->mem.alloc(&d_ct, slots)) || (rc = b->mem.alloc(&d_cl_off, (size_t)N + 1)) ||
            (rc = b->mem.alloc(&d_tri_off, (size_t)N + 1)) ||
            (rc = b->mem.alloc(&d_pl, (size_t)std::max<uint64_t>(pl_off[N], 1))) ||
            (rc = b->mem.alloc(&d_pl_off, (size_t)N + 1)))
            return cleanup(rc);
        {
            std::vector<float> pl_all((size_t)std::max<uint64_t>(pl_off[N], 1) * 4, 0.0f);
            for (int e = 0; e < N; ++e)
                std::copy(ec[e].planes.begin(), ec[e].planes.end(), pl_all.begin() + pl_off[e] * 4);
            HIP_TRY(hipMemcpy(d_pl, pl_all.data(), sizeof(float) * pl_all.size(), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(d_pl_off, pl_off.data(), sizeof(uint64_t) * (N + 1), hipMemcpyHostToDevice));
        }
        if (shade) {
            // each triangle's face-plane index (its normal), in the caller's order
            uint16_t *d_pidx;
            if ((rc = b->mem.alloc(&d_pidx, (size_t)std::max<uint64_t>(tri_off[N], 1)))) return cleanup(rc);
            std::vector<uint16_t> all((size_t)std::max<uint64_t>(tri_off[N], 1), 0);
            for (int e = 0; e < N; ++e) {
                std::copy(ec[e].pidx.begin(), ec[e].pidx.end(), all.begin() + tri_off[e]);
                std::vector<uint16_t>().swap(ec[e].pidx);
            }
            HIP_TRY(hipMemcpy(d_pidx, all.data(), sizeof(uint16_t) * all.size(), hipMemcpyHostToDevice));
            b->mesh.tri_pidx = d_pidx;
        }
        std::vector<float> cl_all((size_t)cl_off[N] * 12);
        std::vector<float> cv_all(slots * 3, 0.0f);
        std::vector<uint32_t> ct_all(slots, 0u);
        parallel_for(N, [&](int64_t e) {
            EnvClusters &c = ec[e];
            const size_t nc = c.cl.size() / 12;
            for (size_t i = 0; i < nc; ++i) {
                float *w = &c.cl[i * 12];
                uint32_t v, t, cnt;
                memcpy(&v, &w[3], 4);
                memcpy(&t, &w[7], 4);
                memcpy(&cnt, &w[8], 4);
                const uint64_t slot = (cl_off[e] + i) * (uint64_t)gal::kClusterVerts;
                const uint32_t nv = cnt & 0xFF, nt = (cnt >> 8) & 0xFF;
                std::copy(c.verts.begin() + (size_t)v * 3, c.verts.begin() + (size_t)(v + nv) * 3,
                          cv_all.begin() + slot * 3);
                std::copy(c.tris.begin() + t, c.tris.begin() + t + nt, ct_all.begin() + slot);
                const uint32_t s32 = (uint32_t)slot;
                memcpy(&w[3], &s32, 4);
                memcpy(&w[7], &s32, 4);
            }
            std::copy(c.cl.begin(), c.cl.end(), cl_all.begin() + cl_off[e] * 12);
            std::vector<float>().swap(c.cl);
            std::vector<float>().swap(c.verts);
            std::vector<uint32_t>().swap(c.tris);
            std::vector<float>().swap(c.planes);
        });
        HIP_TRY(hipMemcpy(d_cl, cl_all.data(), sizeof(float) * cl_all.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_cv, cv_all.data(), sizeof(float) * cv_all.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_ct, ct_all.data(), sizeof(uint32_t) * ct_all.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_cl_off, cl_off.data(), sizeof(uint64_t) * (N + 1), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_tri_off, tri_off.data(), sizeof(uint64_t) * (N + 1), hipMemcpyHostToDevice));
        b->mesh.clusters = d_cl;
        b->mesh.env_cluster_off = d_cl_off;
        b->mesh.cverts = d_cv;
        b->mesh.ctris = d_ct;
        b->mesh.env_tri_off = d_tri_off;
        b->mesh.planes = d_pl;
        b->mesh.env_plane_off = d_pl_off;
        b->mesh.tri_rgb = nullptr;
        b->n_clusters = (int64_t)cl_off[N];
        b->cl_count_host.resize(N);
        for (int e = 0; e < N; ++e) b->cl_count_host[e] = (int64_t)(cl_off[e + 1] - cl_off[e]);
        b->n_cverts = (int64_t)nv_tot;
        b->n_tris = (int64_t)nt_tot;
        if (cfg->flags & GAL_COLOR) {
            uint8_t *d_rgb;
            if ((rc = b->mem.alloc(&d_rgb, (size_t)std::max<uint64_t>(nt_tot, 1) * 3))) return cleanup(rc);
            HIP_TRY(hipMemcpy(d_rgb, sc->tri_rgb, nt_tot * 3, hipMemcpyHostToDevice));
            b->mesh.tri_rgb = d_rgb;
        }
        if (links) {
            float *d_box;
            if ((rc = b->mem.alloc(&d_box, (size_t)8 * 6))) return cleanup(rc);
            HIP_TRY(hipMemcpy(d_box, robot->link_box, sizeof(float) * 8 * 6, hipMemcpyHostToDevice));
            b->mesh.link_box = d_box;
            b->mesh.link_frames = b->sb.link_frames;
            if ((cfg->flags & GAL_COLOR) && robot->link_rgb) {
                uint8_t *d_lrgb;
                if ((rc = b->mem.alloc(&d_lrgb, (size_t)8 * 3))) return cleanup(rc);
                HIP_TRY(hipMemcpy(d_lrgb, robot->link_rgb, 8 * 3, hipMemcpyHostToDevice));
                b->mesh.link_rgb = d_lrgb;
            }
        }
        if (manip && b->O > 0) {
            b->mesh.obj_frames = b->sb.obj_frames;
            b->mesh.obj_rec = b->sb.objects;
            b->mesh.num_objects = b->O;
            if ((cfg->flags & GAL_COLOR) && sc->obj_rgb) {
                uint8_t *d_orgb;
                if ((rc = b->mem.alloc(&d_orgb, (size_t)N * b->O * 3))) return cleanup(rc);
                HIP_TRY(hipMemcpy(d_orgb, sc->obj_rgb, (size_t)N * b->O * 3, hipMemcpyHostToDevice));
                b->mesh.obj_rgb = d_orgb;
            }
        }
    }

    // ---- raster parameters and the (env, region) work list
    {
        b->rast.near_m = cfg->near_m;
        b->rast.invn = 1.0f / cfg->near_m;
        const float invf = 1.0f / cfg->far_m;
        b->rast.kd = 16777215.0f / (b->rast.invn - invf);
        b->rast.region = gal::kMaxRegion;
        b->rast.lane_max = 8;
        b->rast.small_max = 1024;
        b->rast.block = 512;
        b->rast.refresh = 1;
        b->rast.occlusion = 1;
        b->rast.prologue = 128;
        b->rast.order = 0;
        b->rast.stats = nullptr;
        if ((rc = b->mem.alloc(&b->d_res, (size_t)N)) || (rc = b->mem.alloc(&b->d_depth_off, (size_t)N + 1)))
            return cleanup(rc);
        HIP_TRY(hipMemcpy(b->d_res, b->res_host.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice));
        std::vector<uint64_t> doff(N + 1);
        for (int e = 0; e <= N; ++e) doff[e] = (uint64_t)b->depth_off_host[e];
        HIP_TRY(hipMemcpy(b->d_depth_off, doff.data(), sizeof(uint64_t) * (N + 1), hipMemcpyHostToDevice));
        if ((rc = build_work(b))) return cleanup(rc);
        HIP_TRY(gal::raster_prepare());
        b->rast.persistent = 0;
        if ((rc = b->mem.alloc(&b->d_queue, 1))) return cleanup(rc);
        HIP_TRY(hipMemset(b->d_queue, 0, sizeof(uint32_t)));
        b->persist_grid = gal::raster_persistent_grid(b->rast, b->max_res, (cfg->flags & GAL_COLOR) != 0);
        HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    }

    // ---- initial state: episode 0 at the first start pose (reset from episode -1)
    {
        std::vector<int32_t> cnt((size_t)N * 2);
        for (int e = 0; e < N; ++e) {
            cnt[2 * e] = 0;
            cnt[2 * e + 1] = -1;
        }
        HIP_TRY(hipMemcpy(d_counters, cnt.data(), sizeof(int32_t) * N * 2, hipMemcpyHostToDevice));
        HIP_TRY(gal::launch_reset(b->rp, b->sb, nullptr, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    *out = b;
    return GAL_OK;
}

int gal_reset(gal_batch *b, const uint8_t *env_mask_dev, void *stream)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    HIP_TRY(gal::launch_reset(b->rp, b->sb, env_mask_dev, (hipStream_t)stream));
    return GAL_OK;
}

}  // extern "C"

namespace {

gal::OccGrid occ_grid(const gal_batch *b)
{
    gal::OccGrid og;
    og.occ = b->d_occ;
    og.occ_off = b->d_occ_off;
    og.occ_dims = b->d_occ_dims;
    og.occ_cell = b->sb.cell;
    return og;
}

// Occupancy lattice of the surrogate features (built once per batch).
int ensure_occupancy(gal_batch *b, hipStream_t s)
{
    if (b->d_occ) return GAL_OK;
    std::vector<uint64_t> off(b->N);
    std::vector<int32_t> dims(2 * (size_t)b->N);
    uint64_t tot = 0;
    int32_t maxc = 0;
    for (int e = 0; e < b->N; ++e) {
        const int ox = b->meta_host[e].nx, oy = b->meta_host[e].ny;
        dims[2 * e] = ox;
        dims[2 * e + 1] = oy;
        off[e] = tot;
        tot += (uint64_t)ox * oy;   // one byte per column, a bit per layer
        maxc = std::max(maxc, ox * oy);
    }
    int rc;
    // 8 bytes of slack: the feature kernels read each lattice row as the two
    // aligned words around its first byte
    if ((rc = b->mem.alloc(&b->d_occ, tot + 8)) || (rc = b->mem.alloc(&b->d_occ_off, (size_t)b->N)) ||
        (rc = b->mem.alloc(&b->d_occ_dims, 2 * (size_t)b->N)))
        return rc;
    HIP_TRY(hipMemcpy(b->d_occ_off, off.data(), sizeof(uint64_t) * b->N, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_occ_dims, dims.data(), sizeof(int32_t) * 2 * b->N, hipMemcpyHostToDevice));
    b->occ_max_cells = maxc;
    HIP_TRY(gal::launch_occ_build(b->sb, occ_grid(b), b->N, b->K, maxc, s));
    HIP_TRY(hipStreamSynchronize(s));
    return GAL_OK;
}

// The feature source of the fused surrogate inference: every env of the
// batch, its next move under actions_dev.
gal::SurInferArgs batch_features(const gal_batch *b, const float *actions_dev)
{
    gal::SurInferArgs a{};
    a.rp = b->rp;
    a.sb = b->sb;
    a.og = occ_grid(b);
    a.actions = actions_dev;
    return a;
}

// Enqueue one step (robot kernel, then raster) on stream s.
int enqueue_step(gal_batch *b, const float *actions_dev, const gal_outputs *out, hipStream_t s,
                 hipEvent_t *ev)
{
    gal::StepOutputs so;
    so.contact_static = out->contact_static;
    so.contact_object = out->contact_object;
    so.accepted = out->accepted;
    so.state = out->state;
    so.frames = out->frames;
    so.counters = out->counters;
    so.done = out->done;
    so.object_frames = out->object_frames;
    so.held = out->held;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    gal::SimBuffers sb = b->sb;
    if (b->sur) {
        // surrogate pre-filter: features -> MLP -> routing flags for the robot
        // kernel, one launch
        const gal::RouteArgs ra{b->sb.counters, b->sur_thr_logit, b->sur_audit, b->d_flags,
                                b->d_sur_stats, 0};
        const gal::SurInferArgs src = batch_features(b, actions_dev);
        int rc = gal::mlp_infer_rows(b->sur, nullptr, &src, b->N, nullptr, &ra, s);
        if (rc) return rc;
        sb.skip_flags = b->d_flags;
        sb.sur_stats = b->d_sur_stats;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    // the raster queue order (from the previous step's item times) is computed
    // by an extra workgroup of the robot launch
    const bool order_items =
        out->depth && b->rast.persistent && b->rast.order && b->num_work <= gal::kOrderCap;
    const gal::ItemOrder ord{b->d_item_cost, order_items ? b->num_work : 0, b->d_item_order};
    HIP_TRY(gal::launch_robot_step(b->rp, sb, actions_dev, so, b->d_queue, b->robot_lanes, ord, s));
    if (ev) HIP_TRY(hipEventRecord(ev[2], s));
    if (out->depth)
        HIP_TRY(gal::launch_raster(b->mesh, b->rast, b->sb.camera, b->d_res, b->d_depth_off, b->d_work,
                                   b->num_work, b->max_res, b->d_queue, b->persist_grid, out->depth,
                                   out->rgb, s));
    if (ev) HIP_TRY(hipEventRecord(ev[3], s));
    return GAL_OK;
}

bool same_outputs(const gal_outputs &a, const gal_outputs &c)
{
    return a.depth == c.depth && a.rgb == c.rgb && a.contact_static == c.contact_static &&
           a.contact_object == c.contact_object && a.accepted == c.accepted && a.state == c.state &&
           a.frames == c.frames && a.counters == c.counters && a.done == c.done &&
           a.object_frames == c.object_frames && a.held == c.held;
}

// Replay the step graph, capturing it first if the pointers or tuning changed.
int graph_step(gal_batch *b, const float *actions_dev, const gal_outputs *out, hipStream_t s)
{
    if (!b->graph_exec || b->g_actions != actions_dev || !same_outputs(b->g_out, *out) ||
        b->g_gen != b->tune_gen) {
        b->drop_graph();
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_step(b, actions_dev, out, b->cap_stream, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (rc != GAL_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(GAL_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
        b->g_actions = actions_dev;
        b->g_out = *out;
        b->g_gen = b->tune_gen;
    }
    HIP_TRY(hipGraphLaunch(b->graph_exec, s));
    return GAL_OK;
}

}  // namespace

extern "C" {

int gal_step(gal_batch *b, const float *actions_dev, const gal_outputs *out, void *stream)
{
    if (!b || !actions_dev || !out)
        return fail(GAL_EINVAL, "gal_step needs a batch, actions and outputs");
    if (out->rgb && !out->depth) return fail(GAL_EINVAL, "rgb output needs the depth output");
    if (!b->rp.manip && (out->object_frames || out->held))
        return fail(GAL_EINVAL, "object frames and held outputs need GAL_MANIP");
    if (out->rgb && !(b->flags & GAL_COLOR))
        return fail(GAL_EINVAL, "rgb output requested but the batch was created without GAL_COLOR");
    hipStream_t s = (hipStream_t)stream;
    if (b->profiling) {
        hipEvent_t ev[kProfileEvents];
        for (int i = 0; i < kProfileEvents; ++i)
            if (!(ev[i] = b->take_event())) return fail(GAL_EDEVICE, "hipEventCreate failed");
        int rc = enqueue_step(b, actions_dev, out, s, ev);
        b->ev_rec.insert(b->ev_rec.end(), ev, ev + kProfileEvents);
        return rc;
    }
    if (b->use_graph) return graph_step(b, actions_dev, out, s);
    return enqueue_step(b, actions_dev, out, s, nullptr);
}

int gal_profile_enable(gal_batch *b, int on)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    b->profiling = on != 0;
    return GAL_OK;
}

int gal_profile_read_stages(gal_batch *b, double *stage_ms, size_t count, int64_t *steps)
{
    if (!b || (count && !stage_ms)) return fail(GAL_EINVAL, "null argument");
    if (count != 3) return fail(GAL_EINVAL, "need 3 stage times");
    double acc[3] = {0.0, 0.0, 0.0};
    const size_t n = b->ev_rec.size() / kProfileEvents;
    for (size_t i = 0; i < n; ++i) {
        hipEvent_t *e = &b->ev_rec[kProfileEvents * i];
        HIP_TRY(hipEventSynchronize(e[kProfileEvents - 1]));
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e[k], e[k + 1]));
            acc[k] += ms;
        }
    }
    b->ev_pool.insert(b->ev_pool.end(), b->ev_rec.begin(), b->ev_rec.end());
    b->ev_rec.clear();
    for (int k = 0; k < 3; ++k) stage_ms[k] = acc[k];
    if (steps) *steps = (int64_t)n;
    return GAL_OK;
}

int gal_profile_read(gal_batch *b, double *robot_ms, double *raster_ms, int64_t *steps)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    double st[3];
    const int rc = gal_profile_read_stages(b, st, 3, steps);
    if (rc) return rc;
    if (robot_ms) *robot_ms = st[0] + st[1];
    if (raster_ms) *raster_ms = st[2];
    return GAL_OK;
}

int gal_counters_enable(gal_batch *b, int on)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    if (on && !b->d_stats) {
        int rc = b->mem.alloc(&b->d_stats, GAL_NUM_COUNTERS);
        if (rc) return rc;
        HIP_TRY(hipMemset(b->d_stats, 0, sizeof(unsigned long long) * GAL_NUM_COUNTERS));
    }
    b->rast.stats = on ? b->d_stats : nullptr;
    b->tune_gen += 1;   // a captured step graph holds the raster parameters by value
    return GAL_OK;
}

int gal_counters_read(gal_batch *b, int64_t *counters_host, size_t count)
{
    if (!b || !counters_host) return fail(GAL_EINVAL, "null argument");
    if (count != GAL_NUM_COUNTERS) return fail(GAL_EINVAL, "need %d counters", GAL_NUM_COUNTERS);
    if (!b->d_stats) {
        memset(counters_host, 0, sizeof(int64_t) * GAL_NUM_COUNTERS);
        return GAL_OK;
    }
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(counters_host, b->d_stats, sizeof(int64_t) * GAL_NUM_COUNTERS, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(b->d_stats, 0, sizeof(unsigned long long) * GAL_NUM_COUNTERS));
    return GAL_OK;
}

int gal_features(gal_batch *b, const float *actions_dev, uint16_t *x_dev, void *stream)
{
    if (!b || !actions_dev || !x_dev) return fail(GAL_EINVAL, "null argument");
    if ((uintptr_t)x_dev % 16) return fail(GAL_EINVAL, "x_dev must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_occupancy(b, s);
    if (rc) return rc;
    HIP_TRY(gal::launch_features(b->rp, b->sb, occ_grid(b), actions_dev, x_dev, s));
    return GAL_OK;
}

int gal_surrogate_attach(gal_batch *b, gal_mlp *m, float skip_below, uint32_t audit_period,
                         void *stream)
{
    if (!b || !m) return fail(GAL_EINVAL, "null argument");
    if (!(skip_below >= 0.0f && skip_below < 1.0f)) return fail(GAL_EINVAL, "skip_below must be in [0, 1)");
    if (b->rp.manip) return fail(GAL_EINVAL, "the surrogate pre-filter is not available with GAL_MANIP");
    if (gal::mlp_max_rows(m) < b->N)
        return fail(GAL_EINVAL, "the MLP was created for %d rows, the batch has %d envs", gal::mlp_max_rows(m), b->N);
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_occupancy(b, s);
    if (rc) return rc;
    if (!b->d_flags) {
        if ((rc = b->mem.alloc(&b->d_flags, (size_t)b->N)) || (rc = b->mem.alloc(&b->d_sur_stats, 4)))
            return rc;
        HIP_TRY(hipMemset(b->d_sur_stats, 0, sizeof(unsigned long long) * 4));
    }
    b->sur = m;
    // skip iff sigmoid(z) <= skip_below  <=>  z <= logit(skip_below)
    b->sur_thr_logit = skip_below > 0.0f ? std::log(skip_below / (1.0f - skip_below)) : -INFINITY;
    b->sur_audit = audit_period;
    b->tune_gen += 1;   // the captured graph changes
    return GAL_OK;
}

int gal_surrogate_logits(gal_batch *b, const float *actions_dev, float *logits_dev, void *stream)
{
    if (!b || !actions_dev || !logits_dev) return fail(GAL_EINVAL, "null argument");
    if (!b->sur) return fail(GAL_EINVAL, "no surrogate is attached to the batch");
    const gal::SurInferArgs src = batch_features(b, actions_dev);
    return gal::mlp_infer_rows(b->sur, nullptr, &src, b->N, logits_dev, nullptr, (hipStream_t)stream);
}

int gal_surrogate_detach(gal_batch *b)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    b->sur = nullptr;
    b->tune_gen += 1;
    return GAL_OK;
}

int gal_surrogate_stats(gal_batch *b, int64_t *stats_host, int reset)
{
    if (!b || !stats_host) return fail(GAL_EINVAL, "null argument");
    if (!b->d_sur_stats) {
        memset(stats_host, 0, sizeof(int64_t) * 4);
        return GAL_OK;
    }
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(stats_host, b->d_sur_stats, sizeof(int64_t) * 4, hipMemcpyDeviceToHost));
    if (reset) HIP_TRY(hipMemset(b->d_sur_stats, 0, sizeof(unsigned long long) * 4));
    return GAL_OK;
}

int gal_mesh_info(const gal_batch *b, int64_t *clusters, int64_t *cluster_verts, int64_t *tris)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    if (clusters) *clusters = b->n_clusters;
    if (cluster_verts) *cluster_verts = b->n_cverts;
    if (tris) *tris = b->n_tris;
    return GAL_OK;
}

int gal_batch_info(const gal_batch *b, int32_t *num_envs, int32_t *num_spheres,
                   int32_t *contact_words, int64_t *depth_pixels)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    if (num_envs) *num_envs = b->N;
    if (num_spheres) *num_spheres = b->S;
    if (contact_words) *contact_words = b->words;
    if (depth_pixels) *depth_pixels = b->depth_off_host[b->N];
    return GAL_OK;
}

int gal_depth_offsets(const gal_batch *b, int64_t *offsets_host, size_t count)
{
    if (!b || !offsets_host) return fail(GAL_EINVAL, "null argument");
    if (count != (size_t)b->N + 1) return fail(GAL_EINVAL, "need %d offsets", b->N + 1);
    memcpy(offsets_host, b->depth_off_host.data(), sizeof(int64_t) * (b->N + 1));
    return GAL_OK;
}

namespace {
// bytes of the manipulation part of the state (0 without GAL_MANIP)
size_t manip_state_bytes(const gal_batch *b)
{
    if (!b->rp.manip) return 0;
    return (size_t)b->N * (sizeof(float) * 8 * b->O + sizeof(int32_t) + sizeof(float) * 12);
}
}  // namespace

int gal_get_state(gal_batch *b, void *host, size_t bytes, void *stream)
{
    if (!b || !host) return fail(GAL_EINVAL, "null argument");
    const size_t need = (size_t)b->N * (10 * sizeof(float) + 2 * sizeof(int32_t)) + manip_state_bytes(b);
    if (bytes != need) return fail(GAL_ESTATE, "state buffer must be %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    char *h = static_cast<char *>(host);
    HIP_TRY(hipMemcpy(h, b->sb.state, sizeof(float) * b->N * 10, hipMemcpyDeviceToHost));
    h += sizeof(float) * b->N * 10;
    HIP_TRY(hipMemcpy(h, b->sb.counters, sizeof(int32_t) * b->N * 2, hipMemcpyDeviceToHost));
    h += sizeof(int32_t) * b->N * 2;
    if (b->rp.manip) {
        HIP_TRY(hipMemcpy(h, b->sb.obj_dyn, sizeof(float) * b->N * b->O * 8, hipMemcpyDeviceToHost));
        h += sizeof(float) * b->N * b->O * 8;
        HIP_TRY(hipMemcpy(h, b->sb.held_obj, sizeof(int32_t) * b->N, hipMemcpyDeviceToHost));
        h += sizeof(int32_t) * b->N;
        HIP_TRY(hipMemcpy(h, b->sb.rel, sizeof(float) * b->N * 12, hipMemcpyDeviceToHost));
    }
    return GAL_OK;
}

int gal_set_state(gal_batch *b, const void *host, size_t bytes, void *stream)
{
    if (!b || !host) return fail(GAL_EINVAL, "null argument");
    const size_t need = (size_t)b->N * (10 * sizeof(float) + 2 * sizeof(int32_t)) + manip_state_bytes(b);
    if (bytes != need) return fail(GAL_ESTATE, "state buffer must be %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    const char *h = static_cast<const char *>(host);
    HIP_TRY(hipMemcpy(b->sb.state, h, sizeof(float) * b->N * 10, hipMemcpyHostToDevice));
    h += sizeof(float) * b->N * 10;
    HIP_TRY(hipMemcpy(b->sb.counters, h, sizeof(int32_t) * b->N * 2, hipMemcpyHostToDevice));
    h += sizeof(int32_t) * b->N * 2;
    if (b->rp.manip) {
        const int32_t *held = reinterpret_cast<const int32_t *>(h + sizeof(float) * b->N * b->O * 8);
        for (int e = 0; e < b->N; ++e)
            if (held[e] < -1 || held[e] >= b->O) return fail(GAL_ESTATE, "env %d: held object %d out of range", e, held[e]);
        HIP_TRY(hipMemcpy(b->sb.obj_dyn, h, sizeof(float) * b->N * b->O * 8, hipMemcpyHostToDevice));
        h += sizeof(float) * b->N * b->O * 8;
        HIP_TRY(hipMemcpy(b->sb.held_obj, h, sizeof(int32_t) * b->N, hipMemcpyHostToDevice));
        h += sizeof(int32_t) * b->N;
        HIP_TRY(hipMemcpy(b->sb.rel, h, sizeof(float) * b->N * 12, hipMemcpyHostToDevice));
        HIP_TRY(gal::launch_object_frames(b->rp, b->sb, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return GAL_OK;
}

int gal_get_grid(gal_batch *b, int32_t env, int32_t cls, uint32_t *offsets_host,
                 size_t offsets_count, float *layers_host, size_t layers_count, int64_t *num_layers)
{
    if (!b) return fail(GAL_EINVAL, "null batch");
    if (env < 0 || env >= b->N || cls < 0 || cls >= b->K)
        return fail(GAL_EINVAL, "env or class out of range");
    const size_t ek = (size_t)env * b->K + cls;
    const uint64_t ncols = (uint64_t)b->meta_host[env].nx * b->meta_host[env].ny;
    uint32_t total = 0;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(&total, b->sb.grid_offsets + b->off_base_host[ek] + ncols, sizeof(uint32_t),
                      hipMemcpyDeviceToHost));
    if (num_layers) *num_layers = total;
    if (offsets_host) {
        if (offsets_count != ncols + 1) return fail(GAL_EINVAL, "need %llu offsets", (unsigned long long)(ncols + 1));
        HIP_TRY(hipMemcpy(offsets_host, b->sb.grid_offsets + b->off_base_host[ek],
                          sizeof(uint32_t) * (ncols + 1), hipMemcpyDeviceToHost));
    }
    if (layers_host) {
        if (layers_count != (size_t)total) return fail(GAL_EINVAL, "need %u layers", total);
        if (total > 0)
            HIP_TRY(hipMemcpy(layers_host, b->sb.grid_layers + b->layer_base_host[ek],
                              sizeof(float2) * total, hipMemcpyDeviceToHost));
    }
    return GAL_OK;
}

void gal_destroy(gal_batch *b) { delete b; }

}  // extern "C"
