"""Pins of the oracle's manipulation step (Section 3.2: suction grasp with a
small sphere at the end-effector tip, the grasped object carried with the end
effector, snap-to-surface on release; Appendix I: the sliding and
object-placing heuristics) against closed forms and FP64 geometry."""
import math

import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg

CLASSES = sg.RADIUS_CLASSES_PAPER
R_HELD = float(np.float32(CLASSES[0]))
R_GRASP = float(np.float32(sg.GRASP_RADIUS))


def robot_high_sphere():
    """The seeded robot of the manipulation workload with one collision sphere
    high above the base (never in contact in an empty room)."""
    r = sg.make_robot(6, 1, False, CLASSES)
    r.sphere_link = np.array([0], np.int32)
    r.sphere_pos = np.array([[0.0, 0.0, 2.0]], np.float32)
    r.sphere_class = np.array([0], np.int32)
    r.sphere_held_only = np.array([0], np.uint8)
    return r


def scene(objects, boxes=None, mesh=None):
    """One environment: a 20 x 20 m grid around the origin (floor only unless
    boxes are given), the given object boxes, an empty render mesh."""
    objects = np.asarray(objects, np.float32).reshape(1, -1, 8)
    boxes = np.zeros((0, 6), np.float32) if boxes is None else np.asarray(boxes, np.float32)
    O = objects.shape[1]
    return sg.SceneSet(
        num_envs=1, vert_offset=np.array([0, 0], np.int64), verts=np.zeros((0, 3), np.float32),
        tri_offset=np.array([0, 0], np.int64), tris=np.zeros((0, 3), np.int32),
        tri_rgb=np.zeros((0, 3), np.uint8), box_offset=np.array([0, boxes.shape[0]], np.int64),
        boxes=boxes, num_objects=O, objects=objects,
        grid_origin=np.array([[-10.0, -10.0]], np.float32),
        grid_dims=np.array([[400, 400]], np.int32), num_starts=1,
        starts=np.zeros((1, 1, 3), np.float32), held=np.zeros(1, np.uint8),
        res=np.array([32], np.int32), tri_plane=np.zeros((0, 4), np.float32),
        obj_rgb=np.full((1, O, 3), 200, np.uint8))


def consts(slide=True, episode_len=0):
    return dict(near=0.1, far=10.0, cell=sg.CELL, radius_classes=CLASSES,
                act_lim=(0.1, 0.1, 0.05), episode_len=episode_len, res0=32, manip=True,
                slide=slide, grasp_tip=sg.GRASP_TIP, grasp_radius=sg.GRASP_RADIUS, held_class=0,
                slide_step=sg.SLIDE_STEP, place_step=sg.PLACE_STEP, seed=12345)


def action(grasp, stop=0.0, move=None):
    a = np.zeros((1, 11), np.float32)
    if move is not None:
        a[0, :9] = move
    a[0, 9] = grasp
    a[0, 10] = stop
    return a


def frame64(F):
    F = np.asarray(F, np.float64).reshape(3, 4)
    return F[:, :3], F[:, 3]


def ee_tip(O, robot, state):
    R, t = frame64(O.fk(robot, np.asarray(state, np.float32))[7])
    return R @ np.asarray(sg.GRASP_TIP, np.float64) + t, R, t


def arm_state(rng):
    s = np.zeros(10, np.float32)
    s[0:2] = rng.uniform(-1.0, 1.0, 2)
    s[2] = rng.uniform(-3.0, 3.0)
    s[3:10] = rng.uniform(-1.0, 1.0, 7)
    return s


def batch(O, robot, sc, state, **kw):
    ob = O.OracleBatch(robot, sc, consts(**kw))
    ob.set_state(np.asarray(state, np.float32)[None], np.zeros((1, 2), np.int32))
    return ob


# --------------------------------------------------------------------------
# grasp
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_grasp_attaches_iff_the_tip_sphere_overlaps(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(seed)
    robot = robot_high_sphere()
    st = arm_state(rng)
    tip, _, _ = ee_tip(O, robot, st)
    axis = np.zeros(3)
    axis[seed % 3] = 1.0 if seed % 2 == 0 else -1.0
    half = 0.03
    for gap, expect in ((R_GRASP - 2e-4, 0), (R_GRASP + 2e-4, -1)):
        c = tip + axis * (gap + half)
        obj = np.concatenate([c, [half, half, half], [1.0, 0.0]])
        ob = batch(O, robot, scene([obj]), st)
        out = ob.step(action(1.0))
        assert int(out["held"][0]) == expect, (gap, seed)
        # release intent (or a NaN) never grasps
        ob2 = batch(O, robot, scene([obj]), st)
        assert int(ob2.step(action(np.nan))["held"][0]) == -1


def test_grasp_takes_the_nearest_overlapping_object(oracle_lib):
    O = oracle_lib
    robot = robot_high_sphere()
    st = arm_state(np.random.default_rng(9))
    tip, _, _ = ee_tip(O, robot, st)
    half = 0.03
    far = np.concatenate([tip + np.array([0.0, 0.0, 0.010 + half]), [half] * 3, [1.0, 0.0]])
    near = np.concatenate([tip + np.array([0.004 + half, 0.0, 0.0]), [half] * 3, [1.0, 0.0]])
    out = batch(O, robot, scene([far, near]), st).step(action(1.0))
    assert int(out["held"][0]) == 1


@pytest.mark.parametrize("seed", range(4))
def test_carried_object_keeps_its_pose_in_the_ee_frame(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(30 + seed)
    robot = robot_high_sphere()
    st = arm_state(rng)
    tip, Re, te = ee_tip(O, robot, st)
    yaw = float(rng.uniform(-3, 3))
    obj = np.concatenate([tip + np.array([0.0, 0.0, -0.02]), [0.03, 0.04, 0.025],
                          [math.cos(yaw), math.sin(yaw)]]).astype(np.float32)
    ob = batch(O, robot, scene([obj]), st)
    out = ob.step(action(1.0))
    assert int(out["held"][0]) == 0
    # rel = F_ee^-1 F_obj (FP64)
    Ro = np.array([[obj[6], -obj[7], 0], [obj[7], obj[6], 0], [0, 0, 1]], np.float64)
    rel64 = np.concatenate([Re.T @ Ro, (Re.T @ (obj[:3].astype(np.float64) - te))[:, None]], axis=1)
    assert np.abs(out["rel"][0].reshape(3, 4) - rel64).max() < 2e-6
    for k in range(5):
        mv = np.concatenate([[0.05, 0.05], rng.uniform(-0.05, 0.05, 7)])
        out = ob.step(action(1.0, move=mv))
        assert int(out["held"][0]) == 0
        Rk, tk = frame64(out["frames"][0, 7])
        Rob, tob = frame64(out["obj_frames"][0, 0])
        assert np.abs(Rk.T @ Rob - rel64[:, :3]).max() < 1e-5
        assert np.abs(Rk.T @ (tob - tk) - rel64[:, 3]).max() < 1e-5
        # the resting record is untouched while held
        assert np.array_equal(out["objects"][0, 0], obj)


# --------------------------------------------------------------------------
# release: snap-to-surface and placing
# --------------------------------------------------------------------------
def holding(O, robot, sc, st, rel, held=0):
    ob = batch(O, robot, sc, st)
    ob.set_state(np.asarray(st, np.float32)[None], np.zeros((1, 2), np.int32),
                 held=np.array([held], np.int32), rel=np.asarray(rel, np.float32)[None])
    return ob


def rel_below_tip(z=0.0, yaw=0.3):
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([c, -s, 0, sg.GRASP_TIP[0], s, c, 0, sg.GRASP_TIP[1], 0, 0, 1,
                     sg.GRASP_TIP[2] + z], np.float32)


@pytest.mark.parametrize("seed", range(5))
def test_release_over_the_floor_lands_on_it(oracle_lib, seed):
    """The object lands upright on the floor: centre height = half height,
    x, y where it was let go, yaw = that of its carried x axis."""
    O = oracle_lib
    rng = np.random.default_rng(50 + seed)
    robot = robot_high_sphere()
    st = arm_state(rng)
    e = rng.uniform(0.025, 0.075, 3)
    obj = np.concatenate([[5.0, 5.0, e[2]], e, [1.0, 0.0]]).astype(np.float32)
    ob = holding(O, robot, scene([obj]), st, rel_below_tip(yaw=float(rng.uniform(-3, 3))))
    carried = O.fk(robot, st)  # the EE does not move under a zero action
    Re, te = frame64(carried[7])
    Rr, tr = frame64(ob.rel[0])
    Fo_R = Re @ Rr
    Fo_t = Re @ tr + te
    out = ob.step(action(0.0))
    assert int(out["held"][0]) == -1
    rec = out["objects"][0, 0].astype(np.float64)
    assert abs(rec[2] - np.float32(e[2])) < 2e-6
    assert abs(rec[0] - Fo_t[0]) < 2e-6 and abs(rec[1] - Fo_t[1]) < 2e-6
    yaw = math.atan2(Fo_R[1, 0], Fo_R[0, 0])
    assert abs(rec[6] - math.cos(yaw)) < 2e-6 and abs(rec[7] - math.sin(yaw)) < 2e-6
    assert np.array_equal(rec[3:6], obj[3:6].astype(np.float64))


@pytest.mark.parametrize("seed,below", [(7, 0.15), (8, 0.4), (11, 0.25)])
def test_release_over_a_table_lands_on_its_top(oracle_lib, seed, below):
    """Released `below` metres above a table wider than the object: the
    bottom face rests on the table top (centre = top + half height)."""
    O = oracle_lib
    robot = robot_high_sphere()
    st = arm_state(np.random.default_rng(seed))
    st[3] = 0.0
    Re, te = frame64(O.fk(robot, st)[7])
    Rr, tr = frame64(rel_below_tip())
    p = Re @ tr + te
    e = (0.04, 0.03, 0.05)
    top = float(np.float32(p[2] - e[2] - below))
    assert top > 0.05, "end effector too low for this case"
    table = [p[0] - 0.5, p[1] - 0.5, 0.0, p[0] + 0.5, p[1] + 0.5, top]
    obj = np.array([9.0, 9.0, e[2], *e, 1.0, 0.0], np.float32)
    out = holding(O, robot, scene([obj], boxes=[table]), st, rel_below_tip()).step(action(0.0))
    rec = out["objects"][0, 0]
    assert abs(float(rec[2]) - (top + float(np.float32(e[2])))) < 2e-6


def octant_spheres_hit_obb(rec, other, r):
    """FP64: does any octant sphere (radius r) of box `rec` overlap box `other`?"""
    c, e = rec[:3].astype(np.float64), rec[3:6].astype(np.float64)
    R = np.array([[rec[6], -rec[7], 0], [rec[7], rec[6], 0], [0, 0, 1]], np.float64)
    Ro = np.array([[other[6], -other[7], 0], [other[7], other[6], 0], [0, 0, 1]], np.float64)
    for k in range(8):
        o = np.array([(1 if k & 1 else -1) * e[0] / 2, (1 if k & 2 else -1) * e[1] / 2,
                      (1 if k & 4 else -1) * e[2] / 2])
        w = R @ o + c
        lp = Ro.T @ (w - other[:3].astype(np.float64))
        q = np.clip(lp, -other[3:6].astype(np.float64), other[3:6].astype(np.float64))
        if np.sum((lp - q) ** 2) < r * r - 1e-9:
            return True
    return False


@pytest.mark.parametrize("seed", range(6))
def test_release_onto_another_object_is_jittered_clear_or_restored(oracle_lib, seed):
    """Objects do not stack: a drop onto a resting object ends on the floor
    clear of it (within the jitter budget) or back at the pre-grasp record."""
    O = oracle_lib
    rng = np.random.default_rng(70 + seed)
    robot = robot_high_sphere()
    st = arm_state(rng)
    Re, te = frame64(O.fk(robot, st)[7])
    Rr, tr = frame64(rel_below_tip())
    p = Re @ tr + te
    e = (0.04, 0.04, 0.04)
    held = np.array([8.0, 8.0, e[2], *e, 1.0, 0.0], np.float32)
    other = np.array([p[0], p[1], 0.06, 0.06, 0.06, 0.06, 1.0, 0.0], np.float32)
    out = holding(O, robot, scene([held, other]), st, rel_below_tip()).step(action(0.0))
    rec = out["objects"][0, 0]
    if np.array_equal(rec, held):
        return
    assert not octant_spheres_hit_obb(rec, other, R_HELD)
    assert abs(float(rec[2]) - e[2]) < 2e-6
    d = math.hypot(float(rec[0]) - p[0], float(rec[1]) - p[1])
    assert d <= 6 * sg.PLACE_STEP + 1e-5 and d >= sg.PLACE_STEP - 1e-5


def test_release_outside_the_grid_restores_the_pre_grasp_record(oracle_lib):
    O = oracle_lib
    robot = robot_high_sphere()
    st = arm_state(np.random.default_rng(3))
    st[0:2] = (30.0, 30.0)    # far outside the 20 x 20 m grid
    held = np.array([1.0, 2.0, 0.04, 0.04, 0.04, 0.04, 1.0, 0.0], np.float32)
    out = holding(O, robot, scene([held]), st, rel_below_tip()).step(action(0.0))
    assert int(out["held"][0]) == -1
    assert np.array_equal(out["objects"][0, 0], held)


def test_release_is_deterministic(oracle_lib):
    O = oracle_lib
    robot = robot_high_sphere()
    st = arm_state(np.random.default_rng(71))
    Re, te = frame64(O.fk(robot, st)[7])
    p = Re @ frame64(rel_below_tip())[1] + te
    held = np.array([8.0, 8.0, 0.04, 0.04, 0.04, 0.04, 1.0, 0.0], np.float32)
    other = np.array([p[0], p[1], 0.06, 0.06, 0.06, 0.06, 1.0, 0.0], np.float32)
    a = holding(O, robot, scene([held, other]), st, rel_below_tip()).step(action(0.0))
    b = holding(O, robot, scene([held, other]), st, rel_below_tip()).step(action(0.0))
    assert np.array_equal(a["objects"], b["objects"])


# --------------------------------------------------------------------------
# sliding
# --------------------------------------------------------------------------
def base_sphere_robot(offset, cls=1):
    r = sg.make_robot(6, 1, False, CLASSES)
    r.sphere_link = np.array([0], np.int32)
    r.sphere_pos = np.array([offset], np.float32)
    r.sphere_class = np.array([cls], np.int32)
    r.sphere_held_only = np.array([0], np.uint8)
    return r


@pytest.mark.parametrize("seed", range(8))
def test_slide_pushes_the_base_away_from_the_contact(oracle_lib, seed):
    """A base sphere 4 cm into a wall that faces the base (more than the half
    column the grid's lateral precision allows, so the grid sees it): with
    sliding the base ends k slide steps (1 <= k <= 3) from the candidate, along
    the unit vector from the sphere's centre to the base (straight away from
    the wall here), the sphere clear of the wall to within the grid's lateral
    bound (h / sqrt 2); without sliding it stays."""
    O = oracle_lib
    rng = np.random.default_rng(90 + seed)
    off = (float(rng.uniform(0.15, 0.3)), 0.0, 0.5)
    robot = base_sphere_robot(off)
    r = float(np.float32(CLASSES[1]))
    yaw = float(np.float32((seed % 4) * (math.pi / 2) - math.pi / 2 * (seed % 4 == 3) * 4))
    st = np.zeros(10, np.float32)
    st[2] = yaw
    u = np.array([math.cos(yaw), math.sin(yaw)])
    c = u * off[0]
    ax = int(np.argmax(np.abs(u)))
    sgn = 1.0 if u[ax] > 0 else -1.0
    face = c[ax] + sgn * (r - 0.04)
    lo, hi = [-5.0, -5.0, 0.0], [5.0, 5.0, 2.0]
    if sgn > 0:
        lo[ax], hi[ax] = face, face + 0.5
    else:
        lo[ax], hi[ax] = face - 0.5, face
    wall = lo + hi
    obj = np.array([8.0, 8.0, 0.05, 0.05, 0.05, 0.05, 1.0, 0.0], np.float32)
    out = batch(O, robot, scene([obj], boxes=[wall]), st).step(action(0.0))
    assert int(out["accepted"][0]) == 2
    dxy = out["state"][0, :2].astype(np.float64)
    k = np.linalg.norm(dxy) / sg.SLIDE_STEP
    assert abs(k - round(k)) < 1e-4 and 1 <= round(k) <= 3
    assert np.abs(dxy / np.linalg.norm(dxy) + u).max() < 1e-5
    assert sgn * (face - (c[ax] + dxy[ax])) >= r - sg.CELL / math.sqrt(2.0) - 1e-6
    # without sliding the move is rejected and nothing moves
    out2 = batch(O, robot, scene([obj], boxes=[wall]), st, slide=False).step(action(0.0))
    assert int(out2["accepted"][0]) == 0
    assert np.array_equal(out2["state"][0], st)


def test_slide_gives_up_after_three_tries(oracle_lib):
    """Deep in a wall (the base sphere 20 cm inside): three 5 cm jitters
    cannot clear it, so nothing moves."""
    O = oracle_lib
    robot = base_sphere_robot((0.25, 0.0, 0.5))
    st = np.zeros(10, np.float32)
    wall = [0.25 - 0.2, -5.0, 0.0, 0.25 + 0.5, 5.0, 2.0]
    obj = np.array([8.0, 8.0, 0.05, 0.05, 0.05, 0.05, 1.0, 0.0], np.float32)
    out = batch(O, robot, scene([obj], boxes=[wall]), st).step(action(0.0))
    assert int(out["accepted"][0]) == 0
    assert np.array_equal(out["state"][0], st)


# --------------------------------------------------------------------------
# stop, reset, rendering of the objects
# --------------------------------------------------------------------------
def test_stop_ends_the_episode_and_restores_the_objects(oracle_lib):
    O = oracle_lib
    robot = robot_high_sphere()
    st = arm_state(np.random.default_rng(5))
    tip, _, _ = ee_tip(O, robot, st)
    obj = np.concatenate([tip + np.array([0.0, 0.0, -0.02]), [0.03] * 3, [1.0, 0.0]]).astype(np.float32)
    ob = batch(O, robot, scene([obj]), st)
    assert int(ob.step(action(1.0))["held"][0]) == 0
    out = ob.step(action(1.0, stop=1.0))
    assert int(out["done"][0]) == 1
    assert out["counters"][0].tolist() == [0, 1]
    assert int(out["held"][0]) == -1
    assert np.array_equal(out["objects"][0, 0], obj)
    assert np.array_equal(out["state"][0, 3:10], robot.q_home)


def d24(z, near=0.1, far=10.0):
    kd = np.float32((2 ** 24 - 1) / (1 / near - 1 / far))
    return int((1 / near - 1 / z) * float(kd))


def test_object_box_renders_its_near_face_at_analytic_depth(oracle_lib):
    """A resting object straight ahead of the head camera: the centre pixel
    holds the depth of its near face (D24, a few LSB of FP32), back faces are
    culled and nothing else is drawn."""
    O = oracle_lib
    robot = robot_high_sphere()
    st = np.zeros(10, np.float32)
    cam = O.camera(robot, st)
    p, fwd = cam[0:3].astype(np.float64), cam[9:12].astype(np.float64)
    D, half = 2.0, 0.3
    c = p + fwd * (D + half)
    obj = np.array([c[0], c[1], c[2], half, half, half, 1.0, 0.0], np.float32)
    ob = batch(O, robot, scene([obj]), st)
    out = ob.step(action(0.0))
    depth = out["depth"][0]
    W = depth.shape[0]
    centre = depth[W // 2 - 1:W // 2 + 1, W // 2 - 1:W // 2 + 1]
    assert np.all(np.abs(centre.astype(np.int64) - d24(D)) <= 4)
    assert depth[0, 0] == 0xFFFFFF
    v, t, rgb, planes = ob.env_render_mesh(0)
    assert t.shape == (12, 3) and v.shape == (8, 3)
    # every triangle is wound counter-clockwise around its outward normal
    for tri in t:
        a, b, cc = v[tri].astype(np.float64)
        n = np.cross(b - a, cc - a)
        centroid = (a + b + cc) / 3 - obj[:3]
        assert n @ centroid > 0
