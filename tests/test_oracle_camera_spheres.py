"""Pins of the oracle's head camera and sphere placement against geometry
computed independently in FP64.

* Camera (Section 4.1: a head camera, 90 degree field of view; the mount and
  the image axes are this build's reading: 0.10 m ahead of and 1.10 m above
  the base, image right = the robot's right, image down = world down when
  level, an optional downward pitch).  The camera record is exercised through
  the rasteriser: a quad perpendicular to the optical axis lands on the centre
  pixels at the analytic 24-bit depth, markers to the robot's left and above
  the axis land in the left and upper halves at the analytic pixel, and a
  downward pitch moves a horizon edge by the analytic amount.
* Sphere placement (Section 3.2 / Appendix G: sphere proxies attached to the
  links): a sphere's centre is its link frame applied to its link-local
  offset; contact with an object box flips exactly where the FP64 distance
  from that centre to the box crosses the radius.
* Held-only spheres (the grasped-object proxy): such a sphere takes part in
  the collision test only in environments that hold an object.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2306_07552_amd import scenegen as sg

NEAR, FAR = 0.1, 10.0
KD64 = (2 ** 24 - 1) / (1 / np.float64(np.float32(NEAR)) - 1 / np.float64(np.float32(FAR)))


def d24_exact(z):
    v = (1 / np.float64(np.float32(NEAR)) - 1 / np.asarray(z, np.float64)) * KD64
    return np.clip(v, 0, 2 ** 24 - 1)


def robot_with(pitch=0.0, spheres=((0, (0.0, 0.0, 0.5), 0, 0),), dh=None, mount=None):
    """A robot with the given camera pitch and spheres (link, offset, class,
    held_only)."""
    r = sg.make_robot(3, 1, False)
    r.cam_pitch_cs = np.array([np.cos(pitch), np.sin(pitch)], np.float32)
    if dh is not None:
        r.dh = np.asarray(dh, np.float32)
    if mount is not None:
        r.mount = np.asarray(mount, np.float32)
    r.sphere_link = np.array([s[0] for s in spheres], np.int32)
    r.sphere_pos = np.array([s[1] for s in spheres], np.float32).reshape(-1, 3)
    r.sphere_class = np.array([s[2] for s in spheres], np.int32)
    r.sphere_held_only = np.array([s[3] for s in spheres], np.uint8)
    return r


def head_basis_fp64(robot, state, pitch):
    """Camera position and (forward, right, down) in FP64, built from rotation
    objects: the base is turned by yaw about +z, the camera is pitched down by
    `pitch` about the base's +y axis (forward +x tips towards -z)."""
    x, y, yaw = (float(v) for v in state[:3])
    Rb = Rotation.from_euler("z", yaw).as_matrix()
    Rc = Rb @ Rotation.from_euler("y", pitch).as_matrix()
    pos = np.array([x, y, 0.0]) + Rb @ robot.cam_offset.astype(np.float64)
    fwd = Rc @ np.array([1.0, 0.0, 0.0])
    right = Rc @ np.array([0.0, -1.0, 0.0])
    down = Rc @ np.array([0.0, 0.0, -1.0])
    return pos, fwd, right, down


def facing_quad(centre, fwd, right, down, half):
    """Square of side 2*half centred on `centre`, perpendicular to `fwd`, wound
    counter-clockwise around -fwd (it faces the camera)."""
    centre = np.asarray(centre, np.float64)
    P0 = centre - half * down - half * right
    return sg.quad_mesh(P0, 2 * half * down, 2 * half * right)


def render(O, robot, state, verts, tris, W):
    cam = O.camera(robot, np.asarray(state, np.float32))
    d, _, cov, _ = O.render(verts, tris, cam, W, W, NEAR, FAR, want_cover=True)
    return d, cov


def random_state(rng):
    st = np.zeros(10, np.float32)
    st[0:2] = rng.uniform(-4, 4, 2)
    st[2] = rng.uniform(-np.pi, np.pi)
    st[3:] = rng.uniform(-1, 1, 7)
    return st


@pytest.mark.parametrize("seed,pitch,W", [(0, 0.0, 64), (1, 0.0, 128), (2, 0.35, 64),
                                          (3, -0.2, 128), (4, 0.6, 64)])
def test_camera_axis_hits_centre_pixels_at_analytic_depth(oracle_lib, seed, pitch, W):
    O = oracle_lib
    rng = np.random.default_rng(seed)
    robot = robot_with(pitch)
    st = random_state(rng)
    D = float(rng.uniform(0.6, 4.0))
    pos, fwd, right, down = head_basis_fp64(robot, st, pitch)
    v, t = facing_quad(pos + D * fwd, fwd, right, down, 0.25 * D)
    depth, cov = render(O, robot, st, v, t, W)
    h = W // 2
    centre = depth[h - 1:h + 1, h - 1:h + 1].astype(np.float64)
    # coordinates up to ~6 m carry FP32 rounding of a few 1e-7 m through the
    # camera transform: 1e-5 m of slack in distance, plus the depth budget
    ref = d24_exact(D)
    tol = 4.0 + 5.0 * 2.0 ** -24 * ref + KD64 / D ** 2 * 1e-5
    assert np.all(np.abs(centre - ref) <= tol)
    # the covered square is centred on the image: half-width 0.25 of the image
    rows = np.flatnonzero(cov.any(axis=1))
    cols = np.flatnonzero(cov.any(axis=0))
    assert abs((rows[0] + rows[-1] + 1) / 2 - h) <= 1.0
    assert abs((cols[0] + cols[-1] + 1) / 2 - h) <= 1.0
    assert abs(len(cols) - W / 4) <= 2 and abs(len(rows) - W / 4) <= 2


@pytest.mark.parametrize("seed", range(4))
def test_camera_left_and_up_land_left_and_top(oracle_lib, seed):
    """A marker to the robot's left (+y of the base) appears left of the image
    centre, one above the axis (+z, level camera) appears above it, each at the
    pixel the 90 degree pinhole projection gives."""
    O = oracle_lib
    rng = np.random.default_rng(100 + seed)
    W = 128
    robot = robot_with(0.0)
    st = random_state(rng)
    pos, fwd, right, down = head_basis_fp64(robot, st, 0.0)
    yaw = float(st[2])
    left_world = np.array([-np.sin(yaw), np.cos(yaw), 0.0])   # base +y
    up_world = np.array([0.0, 0.0, 1.0])
    D = 2.0
    for dirv, L, axis in ((left_world, 0.9, "col"), (up_world, 0.7, "row")):
        c = pos + D * fwd + L * dirv
        v, t = facing_quad(c, fwd, right, down, 0.05)
        _, cov = render(O, robot, st, v, t, W)
        ys, xs = np.nonzero(cov)
        assert len(xs) > 0
        expect = W / 2 * (1 - L / D)      # pixel coordinate of the marker's centre
        if axis == "col":
            assert abs((xs + 0.5).mean() - expect) <= 1.0 and xs.max() < W // 2
            assert abs((ys + 0.5).mean() - W / 2) <= 1.0
        else:
            assert abs((ys + 0.5).mean() - expect) <= 1.0 and ys.max() < W // 2
            assert abs((xs + 0.5).mean() - W / 2) <= 1.0


@pytest.mark.parametrize("pitch", [0.0, 0.15, 0.3, -0.25])
def test_camera_pitch_moves_the_horizon_by_its_tangent(oracle_lib, pitch):
    """A wall ahead whose lower edge is at the camera's height: with the camera
    pitched down by p that edge is the image row H/2 (1 - tan p); the wall
    covers the rows above it."""
    O = oracle_lib
    W = 64
    robot = robot_with(pitch)
    st = np.zeros(10, np.float32)          # base at the origin, heading +x
    cam_z = float(robot.cam_offset[2])
    cam_x = float(robot.cam_offset[0])
    Dw = 3.0
    # wall at x = cam_x + Dw, y in [-8, 8], z in [cam_z, cam_z + 8] (its top is
    # outside the view), facing -x
    v, t = sg.quad_mesh((cam_x + Dw, -8.0, cam_z), (0, 0, 8.0), (0, 16.0, 0))
    _, cov = render(O, robot, st, v, t, W)
    edge = W / 2 * (1 - np.tan(pitch))
    expect_rows = int(np.sum(np.arange(W) + 0.5 < edge))
    col_counts = cov.sum(axis=0)
    assert np.all(np.abs(col_counts.astype(int) - expect_rows) <= (0 if pitch == 0.0 else 1))
    # covered pixels are the top rows of each column
    for x in range(W):
        n = int(col_counts[x])
        assert cov[:n, x].all() and not cov[n:, x].any()


# --------------------------------------------------------------------------
# sphere placement and the held-only gate, through the oracle's step
# --------------------------------------------------------------------------
def tiny_sceneset(objects, held=0, boxes=None):
    """One environment: an empty render mesh, no static boxes (floor only)
    unless given, a 20 x 20 m grid around the origin, the given object boxes."""
    objects = np.asarray(objects, np.float32).reshape(1, -1, 8)
    boxes = np.zeros((0, 6), np.float32) if boxes is None else np.asarray(boxes, np.float32)
    return sg.SceneSet(
        num_envs=1, vert_offset=np.array([0, 0], np.int64), verts=np.zeros((0, 3), np.float32),
        tri_offset=np.array([0, 0], np.int64), tris=np.zeros((0, 3), np.int32),
        tri_rgb=np.zeros((0, 3), np.uint8), box_offset=np.array([0, boxes.shape[0]], np.int64),
        boxes=boxes, num_objects=objects.shape[1], objects=objects,
        grid_origin=np.array([[-10.0, -10.0]], np.float32),
        grid_dims=np.array([[400, 400]], np.int32), num_starts=1,
        starts=np.zeros((1, 1, 3), np.float32), held=np.array([held], np.uint8),
        res=np.array([8], np.int32), tri_plane=np.zeros((0, 4), np.float32))


def consts():
    return dict(near=NEAR, far=FAR, cell=sg.CELL, radius_classes=sg.RADIUS_CLASSES,
                act_lim=(0.1, 0.1, 0.05), episode_len=0, res0=8)


def step_at(O, robot, scenes, state):
    """Contact masks of `state` as the candidate (a zero action keeps every
    state bit, so the candidate is exactly `state`)."""
    ob = O.OracleBatch(robot, scenes, consts())
    ob.set_state(np.asarray(state, np.float32)[None], np.zeros((1, 2), np.int32))
    out = ob.step(np.zeros((1, 9), np.float32))
    return out


def box_at_distance(centre, direction, dist, half=0.2):
    """An axis-aligned object box (yaw 0) whose nearest face point to `centre`
    is at `dist` along unit `direction` (an axis direction)."""
    direction = np.asarray(direction, np.float64)
    c = np.asarray(centre, np.float64) + direction * (dist + half)
    return np.concatenate([c, [half, half, half], [1.0, 0.0]])


def sphere_world_fp64(state, link_pos_fn, offset):
    """World centre of a sphere from an FP64 link pose (R, t) and its offset."""
    R, tvec = link_pos_fn(state)
    return R @ np.asarray(offset, np.float64) + tvec


@pytest.mark.parametrize("seed", range(6))
def test_base_sphere_contact_flips_at_the_radius(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(200 + seed)
    off = (float(rng.uniform(-0.3, 0.3)), float(rng.uniform(-0.3, 0.3)),
           float(rng.uniform(0.4, 1.0)))
    cls = int(rng.integers(0, 4))
    r = float(np.float32(sg.RADIUS_CLASSES[cls]))
    robot = robot_with(spheres=((0, off, cls, 0),))
    st = random_state(rng)

    def base_pose(s):
        return (Rotation.from_euler("z", float(s[2])).as_matrix(),
                np.array([float(s[0]), float(s[1]), 0.0]))
    c = sphere_world_fp64(st, base_pose, np.float32(off))
    axis = [np.array(a, np.float64) for a in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0))]
    direc = axis[seed % 4]
    for gap, expect in ((r + 2e-3, 0), (r - 2e-3, 1)):
        obj = box_at_distance(c, direc, gap)
        out = step_at(O, robot, tiny_sceneset([obj]), st)
        assert int(out["contact_object"][0, 0] & 1) == expect, (gap, r)
        assert int(out["contact_static"][0, 0]) == 0
        assert int(out["accepted"][0]) == 1 - expect


def planar_arm_robot(l1, l2, h, sphere_link, offset, cls=1):
    dh = np.zeros((7, 4), np.float32)
    dh[:, 2] = 1.0                       # alpha = 0
    dh[0, 0], dh[1, 0] = l1, l2
    return robot_with(spheres=((sphere_link, offset, cls, 0),), dh=dh, mount=(0.0, 0.0, h))


@pytest.mark.parametrize("seed", range(6))
def test_arm_sphere_sits_where_the_planar_closed_form_puts_it(oracle_lib, seed):
    """A two-link planar arm on a turned base: a sphere on link 2 at offset
    (-l2, 0, 0) sits at the elbow, one at the origin of link 2 at the end
    effector (closed forms); contact with a box flips at the radius."""
    O = oracle_lib
    rng = np.random.default_rng(300 + seed)
    l1, l2 = (float(np.float32(v)) for v in rng.uniform(0.2, 0.5, 2))
    h = 0.8
    st = random_state(rng)
    st[5:] = 0.0
    x, y, yaw = (float(v) for v in st[:3])
    t1, t2 = float(st[3]), float(st[4])
    local = {"elbow": np.array([l1 * np.cos(t1), l1 * np.sin(t1), h]),
             "ee": np.array([l1 * np.cos(t1) + l2 * np.cos(t1 + t2),
                             l1 * np.sin(t1) + l2 * np.sin(t1 + t2), h])}
    Rb = Rotation.from_euler("z", yaw).as_matrix()
    cls = 1
    r = float(np.float32(sg.RADIUS_CLASSES[cls]))
    for name, offset in (("elbow", (-l2, 0.0, 0.0)), ("ee", (0.0, 0.0, 0.0))):
        robot = planar_arm_robot(l1, l2, h, 2, offset, cls)
        c = Rb @ local[name] + np.array([x, y, 0.0])
        direc = np.array([[0, 0, 1], [1, 0, 0], [0, -1, 0]][seed % 3], np.float64)
        for gap, expect in ((r + 2e-3, 0), (r - 2e-3, 1)):
            out = step_at(O, robot, tiny_sceneset([box_at_distance(c, direc, gap)]), st)
            assert int(out["contact_object"][0, 0] & 1) == expect, (name, gap)


def test_sphere_link_frame_selection(oracle_lib):
    """The same offset on different links lands at different points: a sphere
    at the origin of link j sits at joint frame j's origin, which for the
    planar arm is the FP64 closed-form position of joint j."""
    O = oracle_lib
    l1, l2 = 0.4, 0.3
    h = 0.9
    st = np.zeros(10, np.float32)
    st[3], st[4] = 0.5, -0.8
    t1, t2 = 0.5, -0.8
    pts = {0: np.array([0.0, 0.0, 0.0]),
           1: np.array([l1 * np.cos(t1), l1 * np.sin(t1), h]),
           2: np.array([l1 * np.cos(t1) + l2 * np.cos(t1 + t2),
                        l1 * np.sin(t1) + l2 * np.sin(t1 + t2), h])}
    r = float(np.float32(sg.RADIUS_CLASSES[0]))
    for link in (1, 2):
        robot = planar_arm_robot(np.float32(l1), np.float32(l2), h, link, (0.0, 0.0, 0.0), 0)
        for probe in (1, 2):
            obj = box_at_distance(pts[probe], np.array([0.0, 0.0, 1.0]), r - 5e-3, half=0.01)
            out = step_at(O, robot, tiny_sceneset([obj]), st)
            assert int(out["contact_object"][0, 0] & 1) == int(link == probe)


@pytest.mark.parametrize("held", [0, 1])
def test_held_only_sphere_is_active_only_when_holding(oracle_lib, held):
    """Sphere 0 is ordinary and free; sphere 1 is held-only and sits inside an
    object box and below the floor's reach: it makes contact iff the env holds
    an object, for the object test and the column-grid test alike."""
    O = oracle_lib
    r1 = float(np.float32(sg.RADIUS_CLASSES[1]))
    robot = robot_with(spheres=((0, (0.0, 0.0, 1.0), 0, 0), (0, (0.5, 0.0, 0.5 * r1), 1, 1)))
    st = np.zeros(10, np.float32)
    obj = np.array([0.5, 0.0, 0.03, 0.05, 0.05, 0.05, 1.0, 0.0], np.float32)
    out = step_at(O, robot, tiny_sceneset([obj], held=held), st)
    assert int(out["contact_object"][0, 0]) == (0b10 if held else 0)
    assert int(out["contact_static"][0, 0]) == (0b10 if held else 0)   # z < r: floor
    assert int(out["accepted"][0]) == 1 - held
    # the same sphere without the held-only flag is tested everywhere
    robot.sphere_held_only[:] = 0
    out = step_at(O, robot, tiny_sceneset([obj], held=0), st)
    assert int(out["contact_object"][0, 0]) == 0b10 and int(out["contact_static"][0, 0]) == 0b10
