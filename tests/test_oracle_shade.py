"""Pins of the oracle's lit, textured colour (the RGB half of Section 4.1's
RGBD observation; the paper's baked textures and lighting are replaced by one
directional light with an ambient term and a world-space checker texture):
against FP64 ray casts of planar faces, and the box face normals against the
boxes' own triangles."""
import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg

NEAR, FAR = 0.1, 10.0
L = np.array([0.36, 0.48, 0.8])


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def cam_look(pos, yaw, pitch=0.0):
    f = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), -np.sin(pitch)])
    r = np.array([np.sin(yaw), -np.cos(yaw), 0.0])
    d = np.cross(f, r)
    return np.concatenate([pos, r, d, f]).astype(np.float32)


def pixel_rays(cam, W):
    hw = W / 2
    px = (np.arange(W) + 0.5 - hw) / hw
    u, v = np.meshgrid(px, px, indexing="xy")
    c = cam.astype(np.float64)
    return c[9:12] + u[..., None] * c[3:6] + v[..., None] * c[6:9]


def check_face(O, verts, tris, normal, rgb, cam, W, min_hits):
    """Render one planar face, shade it, and compare every covered pixel with
    the FP64 value along its ray: the light term from the normal, the checker
    of the exact hit point (pixels within 1 cm of a checker line skipped), and
    the rounding (pixels whose FP64 value sits within 1e-3 of a rounding
    boundary may differ by one)."""
    depth, win, _, _ = O.render(verts, tris, cam, W, W, NEAR, FAR, want_id=True)
    n = np.asarray(normal, np.float64)
    tri_n = np.tile(np.asarray(normal, np.float32), (len(tris), 1))
    tri_rgb = np.tile(np.asarray(rgb, np.uint8), (len(tris), 1))
    out = O.shade(depth, win, cam, NEAR, FAR, tri_n, tri_rgb)
    hit = depth < 0xFFFFFF
    assert (out[~hit] == 0).all()
    assert hit.sum() >= min_hits
    dirs = pixel_rays(cam, W)
    p0 = verts[0].astype(np.float64)
    pos = cam[:3].astype(np.float64)
    t = ((p0 - pos) @ n) / (dirs @ n)
    P = pos + t[..., None] * dirs
    a = np.abs(n)
    if a[2] >= a[0] and a[2] >= a[1]:
        ta, tb = P[..., 0], P[..., 1]
    elif a[0] >= a[1]:
        ta, tb = P[..., 1], P[..., 2]
    else:
        ta, tb = P[..., 0], P[..., 2]
    fa, fb = 4 * ta, 4 * tb
    near_line = (np.abs(fa - np.round(fa)) < 0.04) | (np.abs(fb - np.round(fb)) < 0.04)
    tex = np.where((np.floor(fa) + np.floor(fb)) % 2 == 1, 0.8, 1.0)
    s = 0.35 + 0.65 * max(0.0, float(n @ L))
    val = np.asarray(rgb, np.float64)[None, None, :] * (s * tex)[..., None] + 0.5
    want = np.minimum(255, np.floor(val))
    edge = np.abs(val - np.round(val)) < 1e-3
    ok = (hit & ~near_line)[..., None]
    diff = np.abs(out.astype(np.int64) - want.astype(np.int64))
    assert np.all(diff[ok & ~edge] == 0)
    assert np.all(diff[ok & edge] <= 1)
    ok = ok[..., 0]
    # both checker shades occur
    assert len(np.unique(tex[ok])) == 2
    return out


def test_face_towards_camera_is_ambient_only(O):
    """A wall facing the camera (normal -x, away from the light, n . L < 0):
    only the ambient term, 0.35, times the checker on the y-z axes."""
    v, t = sg.quad_mesh((2.0, -1.5, -1.5), (0, 0, 3.0), (0, 3.0, 0))
    check_face(O, v, t, (-1.0, 0.0, 0.0), (200, 120, 60), cam_look([0, 0, 0], 0.0), 64, 2000)


@pytest.mark.parametrize("pitch", [0.4, 0.9])
def test_floor_seen_from_above(O, pitch):
    """A floor (normal +z, n . L = 0.8, s = 0.87) under a pitched camera 1.1 m
    up: the checker on the x-y axes along every ray."""
    v, t = sg.quad_mesh((-1.0, -4.0, 0.0), (9.0, 0, 0), (0, 8.0, 0))
    check_face(O, v, t, (0.0, 0.0, 1.0), (90, 200, 250), cam_look([0.3, -0.2, 1.1], 0.4, pitch), 96, 4000)


def test_tilted_face(O):
    """A face tilted towards the light (normal (-0.6, 0, 0.8), n . L = 0.424):
    s = 0.6256; its largest normal component is z, so the checker runs on x-y."""
    n = np.array([-0.6, 0.0, 0.8])
    U = np.array([0.8, 0.0, 0.6]) * 3.0
    V = np.array([0.0, 1.0, 0.0]) * 3.0
    assert np.allclose(np.cross(U, V) / 9.0, n)
    v, t = sg.quad_mesh(np.array([1.5, -1.5, -1.2]), U, V)
    check_face(O, v, t, tuple(n), (255, 255, 255), cam_look([0, 0, 0], 0.0, 0.2), 64, 1000)


def test_box_normals_match_their_triangles(O):
    """o_box_normals gives each object / link box triangle the unit normal of
    the triangle itself (FP64 cross product), outward: the face order and the
    signs of the mesh builders."""
    import ctypes as C  # noqa: F401
    rng = np.random.default_rng(4)
    Ob = 5
    objs = np.zeros((Ob, 8), np.float32)
    frames = np.zeros((Ob, 12), np.float32)
    for o in range(Ob):
        yaw = rng.uniform(-np.pi, np.pi)
        objs[o, :3] = rng.uniform(-2, 2, 3)
        objs[o, 3:6] = rng.uniform(0.03, 0.2, 3)
        objs[o, 6:8] = (np.cos(yaw), np.sin(yaw))
        c, s = objs[o, 6], objs[o, 7]
        frames[o] = [c, -s, 0, objs[o, 0], s, c, 0, objs[o, 1], 0, 0, 1, objs[o, 2]]
    verts = np.zeros((8 * Ob, 3), np.float32)
    tris = np.zeros((12 * Ob, 3), np.int32)
    O.lib().o_object_mesh(O.ptr(frames, O._fp), O.ptr(objs, O._fp), Ob, 0, O.ptr(verts, O._fp),
                          O.ptr(tris, O._i32p))
    tri_n = np.zeros((12 * Ob, 3), np.float32)
    O.lib().o_box_normals(O.ptr(frames, O._fp), Ob, O.ptr(tri_n, O._fp))
    for k, (a, b, c) in enumerate(tris):
        A, B, Cc = (verts[i].astype(np.float64) for i in (a, b, c))
        g = np.cross(B - A, Cc - A)
        g /= np.linalg.norm(g)
        assert np.allclose(tri_n[k], g, atol=1e-5), k
