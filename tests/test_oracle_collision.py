"""Pins of the oracle's collision queries (Section 3.2, Appendix G): column
grid per sphere-radius class and sphere-vs-oriented-box, against brute-force
FP64 geometry on tiny scenes (closest point on a triangle, Ericson,
Real-Time Collision Detection, 2005, Sec. 5.1.5) and closed forms."""
import ctypes as C

import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg

H = 0.05


def closest_pt_tri(p, a, b, c):
    """Closest point on triangle abc to points p [n,3] (FP64, Voronoi regions)."""
    p = np.asarray(p, np.float64)
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = ap @ ab, ap @ ac
    bp = p - b
    d3, d4 = bp @ ab, bp @ ac
    cp = p - c
    d5, d6 = cp @ ab, cp @ ac
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    out = np.empty_like(p)
    done = np.zeros(p.shape[0], bool)

    def put(mask, val):
        nonlocal done
        m = mask & ~done
        out[m] = val[m] if np.ndim(val) == 2 else val
        done |= m
    put((d1 <= 0) & (d2 <= 0), np.broadcast_to(a, p.shape))
    put((d3 >= 0) & (d4 <= d3), np.broadcast_to(b, p.shape))
    with np.errstate(divide="ignore", invalid="ignore"):
        v = d1 / (d1 - d3)
        put((vc <= 0) & (d1 >= 0) & (d3 <= 0), a + v[:, None] * ab)
        put((d6 >= 0) & (d5 <= d6), np.broadcast_to(c, p.shape))
        w = d2 / (d2 - d6)
        put((vb <= 0) & (d2 >= 0) & (d6 <= 0), a + w[:, None] * ac)
        w2 = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        put((va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0), b + w2[:, None] * (c - b))
        den = 1.0 / (va + vb + vc)
        v3 = vb * den
        w3 = vc * den
        rest = a + v3[:, None] * ab + w3[:, None] * ac
    put(np.ones(p.shape[0], bool), rest)
    return out


def box_tris_fp64(lo, hi):
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    v, t = sg.boxes_mesh(np.zeros((1, 3)), np.ones((1, 3)), 1)
    v = lo + v.astype(np.float64) * (hi - lo)
    return v[t]


def signed_dist_box(p, lo, hi):
    """Brute force: distance to the surface triangles, negative inside."""
    tris = box_tris_fp64(lo, hi)
    d = np.full(p.shape[0], np.inf)
    for a, b, c in tris:
        q = closest_pt_tri(p, a, b, c)
        d = np.minimum(d, np.linalg.norm(p - q, axis=1))
    inside = np.all((p > lo) & (p < hi), axis=1)
    return np.where(inside, -d, d)


def tiny_scene(rng, nb):
    boxes = []
    for _ in range(nb):
        s = rng.uniform(0.2, 0.8, 3)
        x0 = rng.uniform(0.1, 1.9 - s[0])
        y0 = rng.uniform(0.1, 1.9 - s[1])
        z0 = 0.0 if rng.uniform() < 0.5 else rng.uniform(0.3, 1.0)
        boxes.append((x0, y0, z0, x0 + s[0], y0 + s[1], z0 + s[2]))
    return np.asarray(boxes, np.float32)


def make_env(O, boxes, r, nx=40, ny=40):
    offs, lay = O.grid_build(boxes, 0.0, 0.0, nx, ny, H, r)
    env = O.OEnv()
    env.grid_x0 = env.grid_y0 = 0.0
    env.grid_cell = float(np.float32(H))
    env.nx, env.ny = nx, ny
    lay = np.ascontiguousarray(lay if lay.size else np.zeros((1, 2), np.float32))
    env.grid_offsets[0] = O.ptr(offs, C.POINTER(C.c_uint32))
    env.grid_layers[0] = O.ptr(lay, C.POINTER(C.c_float))
    return env, (offs, lay)


def query(O, env, pts):
    L = O.lib()
    return np.array([L.o_grid_query(C.byref(env), 0, float(x), float(y), float(z))
                     for x, y, z in pts], bool)


def test_floor_only_closed_form(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(0)
    for r in sg.RADIUS_CLASSES:
        env, keep = make_env(O, np.zeros((0, 6), np.float32), np.float32(r), 20, 20)
        offs, lay = keep
        assert np.all(np.diff(offs) == 1) and np.all(lay[:, 0] == np.float32(r))
        assert np.all(np.isinf(lay[:, 1]))
        pts = np.stack([rng.uniform(0, 1, 500), rng.uniform(0, 1, 500),
                        rng.uniform(-0.2, 0.5, 500)], 1).astype(np.float32)
        got = query(O, env, pts)
        assert np.array_equal(got, pts[:, 2] < np.float32(r))
        # outside the grid is always contact
        assert query(O, env, [(-0.01, 0.5, 1.0), (0.5, 1.0001, 1.0)]).all()


@pytest.mark.parametrize("seed", range(6))
def test_grid_at_column_centres_equals_brute_force(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(100 + seed)
    boxes = tiny_scene(rng, 1 + seed % 3)
    for r in sg.RADIUS_CLASSES:
        rf = np.float32(r)
        env, _ = make_env(O, boxes, rf)
        i = rng.integers(0, 40, 1500)
        j = rng.integers(0, 40, 1500)
        cx = ((i + 0.5) * H).astype(np.float32)
        cy = ((j + 0.5) * H).astype(np.float32)
        z = rng.uniform(-0.1, 2.0, 1500).astype(np.float32)
        p = np.stack([cx, cy, z], 1).astype(np.float64)
        sd = np.min(np.stack([signed_dist_box(p, b[:3].astype(np.float64),
                                              b[3:].astype(np.float64)) for b in boxes]), 0)
        brute = (sd < float(rf)) | (p[:, 2] < float(rf))
        keep = (np.abs(sd - float(rf)) > 1e-5) & (np.abs(p[:, 2] - float(rf)) > 1e-5)
        got = query(O, env, p.astype(np.float32))
        assert np.array_equal(got[keep], brute[keep])


@pytest.mark.parametrize("seed", range(4))
def test_grid_anywhere_lateral_bounds(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(200 + seed)
    boxes = tiny_scene(rng, 3)
    slack = H / np.sqrt(2.0) + 1e-5
    for r in sg.RADIUS_CLASSES:
        rf = float(np.float32(r))
        env, _ = make_env(O, boxes, np.float32(r))
        p = np.stack([rng.uniform(0, 2, 1500), rng.uniform(0, 2, 1500),
                      rng.uniform(-0.1, 2.0, 1500)], 1).astype(np.float32).astype(np.float64)
        sd = np.min(np.stack([signed_dist_box(p, b[:3].astype(np.float64),
                                              b[3:].astype(np.float64)) for b in boxes]), 0)
        sd = np.minimum(sd, p[:, 2])   # floor half-space
        got = query(O, env, p.astype(np.float32))
        assert not np.any(got & ~(sd < rf + slack)), "grid contact without a nearby surface"
        assert not np.any(~got & (sd < rf - slack)), "missed contact well inside"


def test_grid_layer_invariants_and_radius_monotone(oracle_lib):
    O = oracle_lib
    cfg = sg.CONFIGS[0]
    S = sg.make_scene_set(cfg, [0, 1])
    rng = np.random.default_rng(3)
    for e in range(2):
        boxes = S.env_boxes(e)
        nx, ny = (int(v) for v in S.grid_dims[e])
        prev_env = None
        pts = np.stack([rng.uniform(0, 4, 3000), rng.uniform(0, 6, 3000),
                        rng.uniform(0, 2.5, 3000)], 1).astype(np.float32)
        prev = None
        for r in sg.RADIUS_CLASSES:
            env, (offs, lay) = make_env(O, boxes, np.float32(r), nx, ny)
            for c in range(nx * ny):
                L = lay[offs[c]:offs[c + 1]]
                assert L.shape[0] >= 1
                assert L[0, 0] >= np.float32(r)
                assert np.all(L[:, 0] < L[:, 1])
                assert np.all(L[1:, 0] > L[:-1, 1])
                assert np.isinf(L[-1, 1])
            got = query(O, env, pts)
            if prev is not None:
                assert not np.any(prev & ~got), "a bigger radius lost a contact"
            prev = got
            prev_env = env
        assert prev_env is not None


def test_multi_layer_table_column(oracle_lib):
    """A suspended slab over the floor gives two free layers per column under
    it: floor..underside and top..infinity, in sphere-centre heights."""
    O = oracle_lib
    boxes = np.array([[0.5, 0.5, 0.7, 1.5, 1.5, 0.75]], np.float32)
    r = np.float32(0.06)
    env, (offs, lay) = make_env(O, boxes, r)
    c = 20 * 40 + 20   # column centre (1.025, 1.025) is under the slab
    L = lay[offs[c]:offs[c + 1]]
    assert L.shape[0] == 2
    assert L[0, 0] == r and L[0, 1] == np.float32(np.float32(0.7) - r)
    assert L[1, 0] == np.float32(np.float32(0.75) + r) and np.isinf(L[1, 1])


def obb_fp64_mesh(o):
    c, e, cs, sn = o[:3].astype(np.float64), o[3:6].astype(np.float64), float(o[6]), float(o[7])
    tris = box_tris_fp64(-e, e)
    R = np.array([[cs, -sn, 0], [sn, cs, 0], [0, 0, 1.0]])
    return tris @ R.T + c, R


@pytest.mark.parametrize("seed", range(4))
def test_obb_vs_brute_force(oracle_lib, seed):
    O = oracle_lib
    L = O.lib()
    rng = np.random.default_rng(300 + seed)
    for _ in range(5):
        yaw = rng.uniform(-np.pi, np.pi)
        o = np.array([1, 1, 0.3, *rng.uniform(0.025, 0.3, 3), np.cos(yaw), np.sin(yaw)],
                     np.float32)
        tris, R = obb_fp64_mesh(o)
        p = rng.uniform(0.3, 1.7, (800, 3)).astype(np.float32).astype(np.float64)
        p[:, 2] = rng.uniform(-0.2, 0.8, 800).astype(np.float32)
        d = np.full(800, np.inf)
        for a, b, c in tris:
            d = np.minimum(d, np.linalg.norm(p - closest_pt_tri(p, a, b, c), axis=1))
        loc = (p - o[:3].astype(np.float64)) @ R
        inside = np.all(np.abs(loc) < o[3:6].astype(np.float64), axis=1)
        for r in sg.RADIUS_CLASSES:
            rf = float(np.float32(r))
            brute = inside | (d < rf)
            keep = inside | (np.abs(d - rf) > 1e-5)
            got = np.array([L.o_obb_query(O.ptr(o, C.POINTER(C.c_float)), *map(float, q), rf)
                            for q in p], bool)
            assert np.array_equal(got[keep], brute[keep])


def test_obb_axis_aligned_is_textbook_sphere_aabb(oracle_lib):
    """With zero yaw the test reduces to Arvo's sphere-box test (Graphics Gems, 1990)."""
    O = oracle_lib
    L = O.lib()
    rng = np.random.default_rng(9)
    o = np.array([0.5, -0.2, 0.4, 0.1, 0.2, 0.05, 1.0, 0.0], np.float32)
    lo = (o[:3] - o[3:6]).astype(np.float64)
    hi = (o[:3] + o[3:6]).astype(np.float64)
    p = rng.uniform(-0.5, 1.5, (3000, 3)).astype(np.float32)
    r = 0.08
    d2 = np.zeros(3000)
    for k in range(3):
        v = p[:, k].astype(np.float64)
        d2 += np.where(v < lo[k], (lo[k] - v) ** 2, 0) + np.where(v > hi[k], (v - hi[k]) ** 2, 0)
    brute = d2 < r * r
    keep = np.abs(np.sqrt(d2) - r) > 1e-5
    got = np.array([L.o_obb_query(O.ptr(o, C.POINTER(C.c_float)), *map(float, q),
                                  float(np.float32(r))) for q in p], bool)
    assert np.array_equal(got[keep], brute[keep])


def test_resolve_rejects_whole_move_on_contact(oracle_lib):
    """A collision disallows all robot movement for the step (Section 3.2)."""
    O = oracle_lib
    cfg = sg.CONFIGS[0]
    S = sg.make_scene_set(cfg, [0])
    robot = sg.make_robot_for(cfg)
    ob = O.OracleBatch(robot, S, sg.config_constants(cfg))
    # far from everything, tiny move: accepted
    out = ob.step(np.zeros((1, 9), np.float32))
    assert out["accepted"][0] == 1
    assert out["contact_static"].sum() == 0 and out["contact_object"].sum() == 0
    # drive the base out of the grid: the whole move (base + arm) is rejected
    ob.state[0, 0] = np.float32(0.05)
    ob.state[0, 2] = np.float32(np.pi)
    before = ob.state.copy()
    a = np.zeros((1, 9), np.float32)
    a[0, 0] = 0.1
    a[0, 2:] = 0.05
    out = ob.step(a)
    assert out["accepted"][0] == 0 and out["contact_static"].sum() > 0
    assert np.array_equal(out["state"].view(np.uint32), before.view(np.uint32))
