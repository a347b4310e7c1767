/*
 * Sanitizer driver of the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Compiled together with oracle.c and oracle_mlp.c (one translation unit)
 * under AddressSanitizer and UndefinedBehaviorSanitizer by the CPU test suite,
 * then run: it drives every exported oracle routine over a small seeded
 * workload (a box room, a 7-DoF robot, random moves, a depth render with
 * clipping through the near and guard planes, a tiny MLP forward / backward
 * and Adam step), so out-of-bounds accesses, overflows of the signed integer
 * edge functions, or uses of uninitialised values in those paths abort the run.
 * Prints "sanitize ok <checksum>" and exits 0 when nothing fired.
 */
#include <stdio.h>

#include "oracle.c"
#include "oracle_mlp.c"

static uint64_t lcg_state = 0x9E3779B97F4A7C15ull;

static float urand(float lo, float hi)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    float u = (float)(lcg_state >> 40) * (1.0f / 16777216.0f);
    return lo + (hi - lo) * u;
}

/* closed box [lo, hi] as 12 outward counter-clockwise triangles */
static int add_box(const float *lo, const float *hi, float *verts, int nv, int32_t *tris, int nt,
                   float *planes)
{
    for (int k = 0; k < 8; ++k) {
        verts[3 * (nv + k) + 0] = (k & 1) ? hi[0] : lo[0];
        verts[3 * (nv + k) + 1] = (k & 2) ? hi[1] : lo[1];
        verts[3 * (nv + k) + 2] = (k & 4) ? hi[2] : lo[2];
    }
    static const int F[12][3] = {{0, 2, 1}, {1, 2, 3}, {4, 5, 6}, {5, 7, 6},
                                 {0, 1, 4}, {1, 5, 4}, {2, 6, 3}, {3, 6, 7},
                                 {0, 4, 2}, {2, 4, 6}, {1, 3, 5}, {3, 7, 5}};
    static const float N[6][3] = {{0, 0, -1}, {0, 0, 1}, {0, -1, 0}, {0, 1, 0}, {-1, 0, 0}, {1, 0, 0}};
    for (int f = 0; f < 12; ++f) {
        for (int k = 0; k < 3; ++k) tris[3 * (nt + f) + k] = nv + F[f][k];
        const float *n = N[f / 2];
        const float *on = (n[0] + n[1] + n[2]) > 0 ? hi : lo;
        int ax = n[0] != 0 ? 0 : (n[1] != 0 ? 1 : 2);
        planes[4 * (nt + f) + 0] = n[0];
        planes[4 * (nt + f) + 1] = n[1];
        planes[4 * (nt + f) + 2] = n[2];
        planes[4 * (nt + f) + 3] = n[ax] * on[ax];
    }
    return 12;
}

int main(void)
{
    double checksum = 0.0;
    /* ---- robot: seeded DH chain, 24 spheres over 8 links, one held-only */
    enum { S = 24 };
    int32_t sl[S], sc[S];
    float sp[S * 3];
    uint8_t sh[S];
    o_robot rb;
    memset(&rb, 0, sizeof(rb));
    for (int j = 0; j < 7; ++j) {
        int a = (int)urand(0.0f, 2.999f);
        rb.dh[j][0] = urand(0.05f, 0.15f);
        rb.dh[j][1] = urand(0.0f, 0.12f);
        rb.dh[j][2] = a == 1 ? 1.0f : 0.0f;
        rb.dh[j][3] = a == 0 ? -1.0f : (a == 2 ? 1.0f : 0.0f);
        rb.qlim[j][0] = -1.5f;
        rb.qlim[j][1] = 1.5f;
        rb.q_home[j] = urand(-0.3f, 0.3f);
    }
    rb.mount[0] = 0.15f; rb.mount[2] = 0.95f;
    rb.cam_offset[0] = 0.10f; rb.cam_offset[2] = 1.10f;
    rb.cam_pitch_cs[0] = 0.98f; rb.cam_pitch_cs[1] = 0.2f;
    for (int s = 0; s < S; ++s) {
        sl[s] = s / 3;
        sc[s] = s % 4;
        sp[3 * s] = urand(-0.1f, 0.1f); sp[3 * s + 1] = urand(-0.04f, 0.04f);
        sp[3 * s + 2] = sl[s] == 0 ? urand(0.3f, 1.0f) : urand(-0.04f, 0.04f);
        sh[s] = s == S - 1;
    }
    rb.num_spheres = S;
    rb.sphere_link = sl; rb.sphere_pos = sp; rb.sphere_class = sc; rb.sphere_held_only = sh;

    o_params pr;
    memset(&pr, 0, sizeof(pr));
    pr.num_classes = 4;
    pr.class_radius[0] = 0.06f; pr.class_radius[1] = 0.08f;
    pr.class_radius[2] = 0.10f; pr.class_radius[3] = 0.12f;
    pr.act_lim[0] = 0.1f; pr.act_lim[1] = 0.1f; pr.act_lim[2] = 0.05f;
    pr.episode_len = 7;
    pr.near_m = 0.1f; pr.far_m = 10.0f; pr.cell_m = 0.05f;

    /* ---- scene: a 4 x 6 m room of 12 boxes (walls + furniture) */
    enum { NB = 12, NX = 80, NY = 120 };
    float boxes[NB * 6];
    for (int k = 0; k < NB; ++k) {
        float x = urand(0.2f, 3.5f), y = urand(0.2f, 5.5f), z = k % 3 == 0 ? urand(0.5f, 1.0f) : 0.0f;
        float w = urand(0.3f, 1.2f), d = urand(0.3f, 1.2f), h = urand(0.3f, 1.5f);
        float *B = boxes + 6 * k;
        B[0] = x; B[1] = y; B[2] = z; B[3] = x + w; B[4] = y + d; B[5] = z + h;
    }
    o_env env;
    memset(&env, 0, sizeof(env));
    env.grid_x0 = 0.0f; env.grid_y0 = 0.0f; env.grid_cell = 0.05f;
    env.nx = NX; env.ny = NY;
    uint32_t *offs[4];
    float *lays[4];
    for (int c = 0; c < 4; ++c) {
        int64_t L = o_grid_build(boxes, NB, 0.0f, 0.0f, NX, NY, 0.05f, pr.class_radius[c], NULL, NULL, 0);
        if (L < 0) { printf("grid build failed\n"); return 1; }
        offs[c] = malloc(sizeof(uint32_t) * (NX * NY + 1));
        lays[c] = malloc(sizeof(float) * 2 * (size_t)L);
        if (o_grid_build(boxes, NB, 0.0f, 0.0f, NX, NY, 0.05f, pr.class_radius[c], offs[c], lays[c], L) != L)
            return 1;
        env.grid_offsets[c] = offs[c];
        env.grid_layers[c] = lays[c];
        checksum += (double)L;
    }
    float objects[5 * 8];
    for (int o = 0; o < 5; ++o) {
        float *ob = objects + 8 * o;
        float psi = urand(-3.0f, 3.0f), s, c;
        o_sincos(psi, &s, &c);
        ob[0] = urand(0.5f, 3.5f); ob[1] = urand(0.5f, 5.5f); ob[2] = 0.05f;
        ob[3] = 0.05f; ob[4] = 0.07f; ob[5] = 0.05f; ob[6] = c; ob[7] = s;
    }
    env.num_objects = 5;
    env.objects = objects;
    float starts[2 * 3] = {2.0f, 3.0f, 0.3f, 1.5f, 2.0f, -1.0f};
    env.num_starts = 2;
    env.starts = starts;
    env.held = 1;

    /* ---- render mesh: the boxes plus a floor slab; planes per triangle */
    enum { MAXT = 12 * (NB + 1) };
    float verts[8 * (NB + 1) * 3];
    int32_t tris[MAXT * 3];
    float planes[MAXT * 4];
    int nt = 0;
    for (int k = 0; k < NB; ++k) nt += add_box(boxes + 6 * k, boxes + 6 * k + 3, verts, 8 * k, tris, nt, planes);
    const float flo[3] = {0.0f, 0.0f, -0.1f}, fhi[3] = {4.0f, 6.0f, 0.0f};
    nt += add_box(flo, fhi, verts, 8 * NB, tris, nt, planes);

    /* ---- steps with random, NaN and huge actions; renders of each state */
    float state[10] = {2.0f, 3.0f, 0.3f, 0, 0, 0, 0, 0, 0, 0};
    int32_t counters[2] = {0, 0};
    uint32_t ms[1], mo[1];
    uint8_t acc, done;
    float frames[96], cam[12];
    enum { W = 48, H = 48 };
    uint32_t depth[W * H], win[W * H];
    uint8_t cover[W * H];
    for (int j = 0; j < 7; ++j) state[3 + j] = rb.q_home[j];
    for (int step = 0; step < 24; ++step) {
        float a[9];
        for (int k = 0; k < 9; ++k) a[k] = urand(-0.12f, 0.12f);
        if (step == 3) a[0] = NAN;
        if (step == 5) a[4] = 1e30f;
        if (step == 6) a[1] = -INFINITY;
        o_robot_step(&rb, &pr, &env, state, counters, a, ms, mo, &acc, &done, frames, cam);
        o_rstats st;
        o_render(verts, tris, nt, (step & 1) ? planes : NULL, cam, W, H, 0.1f, 10.0f, depth,
                 (step & 2) ? win : NULL, (step & 4) ? cover : NULL, &st);
        for (int p = 0; p < W * H; ++p) checksum += depth[p] * 1e-9;
        checksum += (double)(ms[0] ^ mo[0]) + acc + done + (double)st.frags;
        if (step == 11) o_reset_env(&rb, &env, state, counters, 1);
    }
    /* a camera inside a box and looking across the near / guard planes */
    float cam2[12] = {1.0f, 1.0f, 0.2f, 0.0f, -1.0f, 0.0f, 0.0f, 0.0f, -1.0f, 1.0f, 0.0f, 0.0f};
    o_rstats st2;
    o_render(verts, tris, nt, NULL, cam2, W, H, 0.1f, 10.0f, depth, win, cover, &st2);
    checksum += (double)st2.clipped;
    for (int q = 0; q < 1000; ++q) {
        checksum += o_grid_query(&env, q & 3, urand(-0.5f, 4.5f), urand(-0.5f, 6.5f), urand(-0.2f, 2.0f));
        checksum += o_obb_query(objects + 8 * (q % 5), urand(0.0f, 4.0f), urand(0.0f, 6.0f), urand(0.0f, 0.3f), 0.1f);
    }

    /* ---- tiny MLP: forward, backward, loss, Adam */
    enum { D0 = 9, D1 = 6, ROWS = 5 };
    int dims[6] = {D0, D1, D1, D1, D1, 1};
    double *Wm[5], *bm[5], *dW[5], *db[5];
    o_mlp net;
    size_t nparam = 0;
    for (int l = 0; l < 5; ++l) {
        size_t n = (size_t)dims[l + 1] * dims[l];
        Wm[l] = malloc(sizeof(double) * n); dW[l] = malloc(sizeof(double) * n);
        bm[l] = malloc(sizeof(double) * dims[l + 1]); db[l] = malloc(sizeof(double) * dims[l + 1]);
        for (size_t i = 0; i < n; ++i) Wm[l][i] = urand(-0.5f, 0.5f);
        for (int i = 0; i < dims[l + 1]; ++i) bm[l][i] = urand(-0.1f, 0.1f);
        net.W[l] = Wm[l]; net.b[l] = bm[l];
        nparam += n;
    }
    for (int l = 0; l < 6; ++l) net.dims[l] = dims[l];
    double x[ROWS * D0], y[ROWS], z[ROWS];
    for (int i = 0; i < ROWS * D0; ++i) x[i] = o_bf16_round(urand(-1.0f, 1.0f));
    for (int i = 0; i < ROWS; ++i) y[i] = i & 1;
    o_mlp_forward(&net, x, ROWS, 1, z, NULL);
    checksum += o_mlp_backward(&net, x, y, ROWS, 4.0, 1, dW, db);
    checksum += o_mlp_loss(&net, x, y, ROWS, 4.0, 0) + z[0];
    double *m = calloc(D1 * D0, sizeof(double)), *v = calloc(D1 * D0, sizeof(double));
    o_adam(Wm[0], m, v, dW[0], D1 * D0, 1e-3, 0.9, 0.999, 1e-8, 1);
    checksum += Wm[0][0] + (double)nparam;
    for (int l = 0; l < 5; ++l) { free(Wm[l]); free(dW[l]); free(bm[l]); free(db[l]); }
    free(m); free(v);
    for (int c = 0; c < 4; ++c) { free(offs[c]); free(lays[c]); }
    printf("sanitize ok %.6f\n", checksum);
    return 0;
}
