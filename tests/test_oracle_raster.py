"""Pins of the oracle's depth rasteriser (the head-camera depth observation of
Section 4.1; the paper's batch renderer is a black box, so the rasteriser is
checked against analytic depth, FP64 ray casts and coverage invariants)."""
import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg

NEAR, FAR = 0.1, 10.0
KD64 = (2 ** 24 - 1) / (1 / np.float64(np.float32(NEAR)) - 1 / np.float64(np.float32(FAR)))


# FP32 budget of one depth value: 1/Z, (1/n - 1/Z), the constant
# (2^24-1)/(1/n - 1/f) and their product each carry a relative rounding error
# of at most 2^-24, which the cancellation in (1/n - 1/Z) can double: about
# 5 * 2^-24 relative, i.e. 5 LSB near 2^24, plus 1 for the final truncation.
REL_BUDGET = 5.0 * 2.0 ** -24


def d24_exact(z):
    """Analytic 24-bit depth of camera-space distance z (FP64)."""
    v = (1 / np.float64(np.float32(NEAR)) - 1 / np.asarray(z, np.float64)) * KD64
    return np.clip(v, 0, 2 ** 24 - 1)


def cam_look(pos, yaw, pitch=0.0):
    f = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), -np.sin(pitch)])
    r = np.array([np.sin(yaw), -np.cos(yaw), 0.0])
    d = np.cross(f, r)
    return np.concatenate([pos, r, d, f]).astype(np.float32)


def pixel_rays(cam, W, du=0.0, dv=0.0):
    """World directions (not normalised, unit forward component) through pixel
    centres, optionally offset by (du, dv) pixels."""
    hw = W / 2
    px = (np.arange(W) + 0.5 - hw) / hw
    u, v = np.meshgrid(px + du / hw, px + dv / hw, indexing="xy")
    c = cam.astype(np.float64)
    return c[9:12] + u[..., None] * c[3:6] + v[..., None] * c[6:9]


def moller_trumbore(orig, dirs, tris, return_cos=False):
    """FP64 ray/triangle intersection (Moller & Trumbore 1997): nearest t, the
    smallest barycentric margin of that hit, the second-nearest t and the
    |cosine| between the ray and the hit triangle's normal."""
    shape = dirs.shape[:-1]
    D = dirs.reshape(-1, 3)
    best = np.full(D.shape[0], np.inf)
    marg = np.zeros(D.shape[0])
    second = np.full(D.shape[0], np.inf)
    cosi = np.zeros(D.shape[0])
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    for a, b, c in tris:
        e1, e2 = b - a, c - a
        p = np.cross(D, e2)
        det = p @ e1
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / det
            s = orig - a
            u = (p @ s) * inv
            q = np.cross(s, e1)
            v = (D @ q) * inv
            t = (q @ e2) * inv
        ok = (np.abs(det) > 1e-12) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        m = np.minimum(np.minimum(u, v), 1 - u - v)
        closer = ok & (t < best)
        second = np.where(closer, best, np.where(ok, np.minimum(second, t), second))
        best = np.where(closer, t, best)
        marg = np.where(closer, m, marg)
        nrm = np.cross(e1, e2)
        nrm = nrm / np.linalg.norm(nrm)
        cosi = np.where(closer, np.abs(Dn @ nrm), cosi)
    if return_cos:
        return best.reshape(shape), marg.reshape(shape), second.reshape(shape), cosi.reshape(shape)
    return best.reshape(shape), marg.reshape(shape), second.reshape(shape)


def render(O, verts, tris, cam, W, **kw):
    return O.render(verts, tris, cam, W, W, NEAR, FAR, **kw)


def test_empty_scene(oracle_lib):
    d, _, cov, st = render(oracle_lib, np.zeros((0, 3)), np.zeros((0, 3)),
                           cam_look([0, 0, 1], 0.3), 64, want_cover=True)
    assert (d == 0xFFFFFF).all() and (cov == 0).all() and st["frags"] == 0


@pytest.mark.parametrize("D,W", [(1.0, 64), (2.5, 128), (0.45, 64), (7.0, 256)])
def test_fronto_parallel_quad_depth_and_count(oracle_lib, D, W):
    O = oracle_lib
    cam = cam_look([0, 0, 0], 0.0)
    rng = np.random.default_rng(int(D * 100) + W)
    y0, y1 = sorted(rng.uniform(-0.8, 0.8, 2) * D)
    z0, z1 = sorted(rng.uniform(-0.8, 0.8, 2) * D)
    # facing the camera (normal -x): U x V = z x y = -x
    v, t = sg.quad_mesh((D, y0, z0), (0, 0, z1 - z0), (0, y1 - y0, 0))
    depth, _, cov, _ = render(O, v, t, cam, W, want_cover=True)
    # camera-space rectangle: X = -y, Y = -z, Z = D; snapped like any vertex
    hw = np.float32(W / 2)
    Df = np.float32(np.float32(D))

    def snap(val):
        s = np.float32(hw + hw * (np.float32(val) / Df))
        return int(np.rint(np.float32(s * np.float32(16))))
    xl = min(snap(-np.float32(y)) for y in v[:, 1])
    xr = max(snap(-np.float32(y)) for y in v[:, 1])
    yt = min(snap(-np.float32(z)) for z in v[:, 2])
    yb = max(snap(-np.float32(z)) for z in v[:, 2])
    centres = 16 * np.arange(W) + 8
    inx = (centres >= xl) & (centres < xr)          # left edge in, right edge out
    iny = (centres >= yt) & (centres < yb)          # top edge in, bottom edge out
    expect = iny[:, None] & inx[None, :]
    assert np.array_equal(cov > 0, expect)
    assert cov.max() <= 1
    ref = d24_exact(np.float64(Df))
    tol = 1.0 + REL_BUDGET * ref
    assert np.all(np.abs(depth[expect].astype(np.float64) - ref) <= tol)
    assert (depth[~expect] == 0xFFFFFF).all()


def depth_tolerance(depth_img):
    """The per-value FP32 budget, 2 LSB for the plane evaluation
    d0 + (a*dx + b*dy), plus what vertices snapped by at most 1/32 pixel can
    tilt the plane: 1/8 of the local depth slope per pixel."""
    d = depth_img.astype(np.float64)
    gx = np.abs(np.diff(d, axis=1, append=d[:, -1:]))
    gy = np.abs(np.diff(d, axis=0, append=d[-1:, :]))
    return 3.0 + REL_BUDGET * d + (gx + gy) / 8.0


@pytest.mark.parametrize("pitch", [0.0, 0.3, 0.7])
def test_tilted_floor_vs_ray_plane(oracle_lib, pitch):
    O = oracle_lib
    W = 128
    cam = cam_look([2.0, 3.0, 1.1], 0.4, pitch)
    v, t = sg.quad_mesh((-20, -20, 0), (40, 0, 0), (0, 40, 0))
    depth, _, _, st = render(O, v, t, cam, W)
    assert st["clipped"] >= 1
    rays = pixel_rays(cam, W)
    tz = -1.1 / rays[..., 2]                   # distance along the forward axis
    hit = (rays[..., 2] < -1e-3) & (tz < 9.0)
    exact = d24_exact(tz)
    tol = depth_tolerance(exact)
    inner = hit.copy()
    inner[:, [0, -1]] = False
    inner[[0, -1], :] = False
    assert inner.sum() > 100
    err = np.abs(depth.astype(np.float64) - exact)
    assert np.all(err[inner] <= tol[inner])


def scene_boxes(rng, n):
    lo, hi = [], []
    for _ in range(n):
        c = rng.uniform([1.0, -1.5, 0.0], [4.0, 1.5, 1.5])
        s = rng.uniform(0.2, 0.9, 3)
        lo.append(c - s / 2)
        hi.append(c + s / 2)
    return np.array(lo), np.array(hi)


@pytest.mark.parametrize("seed", range(3))
def test_boxes_vs_moller_trumbore(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(seed)
    lo, hi = scene_boxes(rng, 4)
    v, t = sg.boxes_mesh(lo, hi, 2)
    cam = cam_look([0, 0, 0.8], rng.uniform(-0.2, 0.2), rng.uniform(-0.1, 0.3))
    W = 64
    depth, _, _, _ = render(O, v, t, cam, W)
    rays = pixel_rays(cam, W)
    tris = v.astype(np.float64)[t]
    tmin, marg, second, cosi = moller_trumbore(cam[:3].astype(np.float64), rays, tris, True)
    exact = d24_exact(tmin)
    # not at grazing incidence (there snapped slivers amplify the vertex
    # rounding beyond the slope bound), away from triangle edges, no near tie
    ok = np.isfinite(tmin) & (marg > 0.02) & (second > tmin * 1.05) & (cosi > 0.3)
    # at least 1/16 pixel away from every silhouette edge: rays shifted by
    # 1/16 pixel see the same surface
    for du, dv in ((1 / 16, 0), (-1 / 16, 0), (0, 1 / 16), (0, -1 / 16)):
        tn, _, _ = moller_trumbore(cam[:3].astype(np.float64), pixel_rays(cam, W, du, dv), tris)
        ok &= np.abs(tn - tmin) < 0.01 * tmin
    assert ok.sum() > 50
    err = np.abs(depth.astype(np.float64) - exact)
    tol = depth_tolerance(exact)
    assert np.all(err[ok] <= tol[ok])
    miss = ~np.isfinite(tmin)
    edge_free = miss.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            edge_free &= np.roll(np.roll(miss, dy, 0), dx, 1)
    assert (depth[edge_free] == 0xFFFFFF).all()


def coverage_interior(cov1):
    inside = cov1 > 0
    inner = inside.copy()
    outer = ~inside
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            sh_in = np.roll(np.roll(inside, dy, 0), dx, 1)
            inner &= sh_in
            outer &= ~sh_in
    inner[[0, -1], :] = inner[:, [0, -1]] = False
    return inner, outer


@pytest.mark.parametrize("seed", range(4))
def test_watertight_subdivided_boxes(oracle_lib, seed):
    """Front faces of closed, subdivided boxes tile the silhouette: no pixel
    is covered twice, and every pixel well inside it exactly once."""
    O = oracle_lib
    rng = np.random.default_rng(50 + seed)
    lo, hi = scene_boxes(rng, 1)
    cam = cam_look([0, 0, 0.8], rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3))
    v1, t1 = sg.boxes_mesh(lo, hi, 1)
    _, _, cov1, _ = render(O, v1, t1, cam, 128, want_cover=True)
    inner, outer = coverage_interior(cov1)
    for n in (3, 7):
        v, t = sg.boxes_mesh(lo, hi, n)
        _, _, cov, _ = render(O, v, t, cam, 128, want_cover=True)
        assert cov.max() <= 1
        assert (cov[inner] == 1).all()
        assert (cov[outer] == 0).all()


@pytest.mark.parametrize("seed", range(4))
def test_watertight_across_near_and_guard_planes(oracle_lib, seed):
    """A subdivided wall that passes behind the camera and far outside the
    viewport: clipping against the near plane and the guard band keeps the
    mesh watertight (shared clipped edges snap identically)."""
    O = oracle_lib
    rng = np.random.default_rng(70 + seed)
    cam = cam_look([0, 0, 1.0], rng.uniform(0.6, 1.1), rng.uniform(-0.3, 0.3))
    # wall in the plane y = 0.4 facing -y (toward the camera), from behind the
    # camera to far ahead: U x V = x cross z = -y
    P0, U, V = (-3.0, 0.4, -1.0), (9.0, 0, 0), (0, 0, 4.0)
    n = 12
    lo = np.array(P0)
    verts, tris = [], []
    xs = (P0[0] + U[0] * np.arange(n + 1) / n).astype(np.float32)
    zs = (P0[2] + V[2] * np.arange(n + 1) / n).astype(np.float32)
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    verts = np.stack([X, np.full_like(X, np.float32(0.4)), Z], -1).reshape(-1, 3)
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, (i + 1) * (n + 1) + j, (i + 1) * (n + 1) + j + 1, i * (n + 1) + j + 1
            tris += [[a, b, c], [a, c, d]]
    tris = np.array(tris)
    depth, _, cov, st = render(O, verts, tris, cam, 128, want_cover=True)
    assert st["clipped"] > 0
    assert cov.max() <= 1
    v1, t1 = sg.quad_mesh(P0, U, V)
    _, _, cov1, _ = render(O, v1, t1, cam, 128, want_cover=True)
    inner, outer = coverage_interior(cov1)
    assert inner.sum() > 100
    assert (cov[inner] == 1).all()
    assert (cov[outer] == 0).all()
    del lo


def test_order_invariance_and_id_tie_break(oracle_lib):
    O = oracle_lib
    cfg = sg.CONFIGS[0]
    S = sg.make_scene_set(cfg, [3])
    v, t, _ = S.env_mesh(0)
    cam = cam_look([2.0, 3.0, 1.1], 1.0, 0.2)
    d0, w0, _, _ = render(O, v, t, cam, 64, want_id=True)
    perm = np.random.default_rng(1).permutation(t.shape[0])
    d1, w1, _, _ = render(O, v, t[perm], cam, 64, want_id=True)
    assert np.array_equal(d0, d1)
    # same winners, expressed in the original ids (no exact ties in this scene
    # away from shared edges; where ties exist the smallest id must win)
    hit = w1 != 0xFFFFFFFF
    assert np.array_equal(w0 != 0xFFFFFFFF, hit)
    # exact duplicate triangle: the smaller id wins regardless of order
    tt = np.concatenate([t, t[:1]])
    dd, ww, _, _ = render(O, v, tt, cam, 64, want_id=True)
    assert not np.any(ww == t.shape[0])


def test_backfaces_are_culled(oracle_lib):
    O = oracle_lib
    cam = cam_look([0, 0, 0], 0.0)
    # facing away from the camera (normal +x)
    v, t = sg.quad_mesh((2.0, -0.5, -0.5), (0, 1.0, 0), (0, 0, 1.0))
    d, _, _, st = render(O, v, t, cam, 64)
    assert (d == 0xFFFFFF).all() and st["tris_front"] == 0


@pytest.mark.parametrize("seed", range(4))
def test_fragment_depth_within_vertex_range_for_slivers(oracle_lib, seed):
    """Depth is a convex combination of the vertex depths (barycentric
    weights from the integer edge functions): even for long, thin triangles
    spanning a large depth range, every covered pixel lies within the FP32
    budget of the analytic vertex-depth range."""
    O = oracle_lib
    rng = np.random.default_rng(900 + seed)
    cam = cam_look([0, 0, 0], 0.0)
    hits = 0
    for _ in range(150):
        a = np.array([rng.uniform(0.15, 1.0), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)])
        b = np.array([rng.uniform(3, 9.5), rng.uniform(-6, 6), rng.uniform(-6, 6)])
        c = a + (b - a) * rng.uniform(0.1, 0.9) + rng.normal(0, 10 ** rng.uniform(-6, -3), 3)
        v = np.array([a, b, c], np.float32)
        for t in (np.array([[0, 1, 2]]), np.array([[0, 2, 1]])):
            depth, _, cov, _ = render(O, v, t, cam, 128, want_cover=True)
            if cov.sum() == 0:
                continue
            hits += 1
            Z = v[:, 0].astype(np.float64)            # camera forward = world +x
            lo, hi = d24_exact(Z.min()), d24_exact(Z.max())
            got = depth[cov > 0].astype(np.float64)
            slack = 1.0 + 8.0 * REL_BUDGET * hi
            assert got.min() >= lo - slack and got.max() <= hi + slack
    assert hits > 20


def golden_constants():
    import os
    vals = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "task_constants.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = int(v)
    return vals


def test_task_constants_match_the_paper():
    g = golden_constants()
    cfg = sg.CONFIGS[1]
    consts = sg.config_constants(cfg)
    assert cfg.res0 == g["camera_resolution"]
    assert consts["episode_len"] == g["episode_horizon"]
    assert cfg.num_envs == g["envs_total"]
    robot = sg.make_robot_for(cfg)
    assert robot.dh.shape[0] == g["arm_dof"] and robot.q_home.shape[0] == g["arm_dof"]
    assert len(consts["act_lim"]) == 3   # base forward, base yaw, every joint


@pytest.mark.parametrize("half_angle_tan,W", [(0.95, 128), (0.5, 128), (1.2, 64)])
def test_field_of_view_is_ninety_degrees(oracle_lib, half_angle_tan, W):
    """A fronto-parallel strip spanning +-atan(t) horizontally covers exactly
    the pixel columns whose centre ray lies within it, the mapping of a 90
    degree FoV (the image edge at 45 degrees, Section 4.1); t > 1 covers
    every column."""
    assert golden_constants()["camera_fov_deg"] == 90
    D = 2.0
    cam = cam_look([0, 0, 0], 0.0)
    yl = half_angle_tan * D
    # facing the camera: U x V = z x y = -x; camera right = -y
    v, t = sg.quad_mesh((D, -yl, -0.2 * D), (0, 0, 0.4 * D), (0, 2 * yl, 0))
    _, _, cov, _ = render(oracle_lib, v, t, cam, W, want_cover=True)
    hw = W / 2
    u = (np.arange(W) + 0.5 - hw) / hw        # tangent of each column's centre ray
    inside = np.abs(u) < half_angle_tan - 1e-3
    outside = np.abs(u) > half_angle_tan + 1e-3
    cols = cov[W // 2]                         # middle row
    assert (cols[inside] == 1).all() and (cols[outside] == 0).all()
    if half_angle_tan > 1:
        assert (cols == 1).all()


@pytest.mark.parametrize("seed", range(4))
def test_face_plane_culling_leaves_closed_boxes_unchanged(oracle_lib, seed):
    """Culling by the camera's side of each face removes only faces that point
    away from the camera; for closed boxes seen from outside those lie behind
    front faces, so depth and winning triangles are the winding test's."""
    O = oracle_lib
    rng = np.random.default_rng(100 + seed)
    lo, hi = scene_boxes(rng, 4)
    v, t = sg.boxes_mesh(lo, hi, 2)
    pl = sg.boxes_planes(lo, hi, 2)
    cam = cam_look([0, 0, 0.8], rng.uniform(-0.3, 0.3), rng.uniform(-0.1, 0.3))
    d0, w0, _, st0 = render(O, v, t, cam, 128, want_id=True)
    d1, w1, _, st1 = render(O, v, t, cam, 128, want_id=True, planes=pl)
    assert (d0 == d1).all() and (w0 == w1).all()
    # the faces culled by their plane are exactly those the camera is behind (FP64)
    c = cam[:3].astype(np.float64)
    behind = (pl[:, :3].astype(np.float64) @ c - pl[:, 3]) <= 0
    assert behind.any() and (~behind).any()
    assert st1["tris_in"] < st0["tris_in"]


def test_face_plane_overrides_winding(oracle_lib):
    """A quad wound towards the camera but whose supplied face plane points
    away is culled; with the plane pointing at the camera it is drawn, and a
    camera exactly on the plane culls it (strictly in front is required)."""
    O = oracle_lib
    cam = cam_look([0, 0, 0], 0.0)
    v, t = sg.quad_mesh((2.0, -0.5, -0.5), (0, 0, 1.0), (0, 1.0, 0))   # U x V = z x y = -x: towards the camera
    toward = sg.quad_planes((2.0, -0.5, -0.5), (0, 0, 1.0), (0, 1.0, 0))
    assert np.allclose(toward[0, :3], [-1, 0, 0]) and toward[0, 3] == np.float32(-2.0)
    away = toward.copy()
    away[:, :4] *= -1.0
    d_none, _, _, _ = render(O, v, t, cam, 64)
    d_toward, _, _, _ = render(O, v, t, cam, 64, planes=toward)
    d_away, _, _, _ = render(O, v, t, cam, 64, planes=away)
    assert (d_none < 0xFFFFFF).sum() > 100
    assert (d_toward == d_none).all()
    assert (d_away == 0xFFFFFF).all()
    on_plane = toward.copy()
    on_plane[:, 3] = np.float32(0.0)      # the camera (origin) on the plane x = 0
    d_on, _, _, _ = render(O, v, t, cam, 64, planes=on_plane)
    assert (d_on == 0xFFFFFF).all()
