"""Pins of the oracle's robot-link rendering: the head camera of Section 4.1
also sees the robot's own body and arm (the paper's renderer draws the robot
with the scene), each link as a box in its link frame, placed by the step's
forward kinematics."""
import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg

NEAR, FAR = 0.1, 10.0
KD64 = (2 ** 24 - 1) / (1 / np.float64(np.float32(NEAR)) - 1 / np.float64(np.float32(FAR)))
REL_BUDGET = 5.0 * 2.0 ** -24


def d24_exact(z):
    v = (1 / np.float64(np.float32(NEAR)) - 1 / np.asarray(z, np.float64)) * KD64
    return np.clip(v, 0, 2 ** 24 - 1)


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def link_mesh(O, frames, box, vbase=0):
    import ctypes as C
    fr = np.ascontiguousarray(frames, np.float32).reshape(8, 12)
    box = np.ascontiguousarray(box, np.float32)
    v = np.zeros((64, 3), np.float32)
    t = np.zeros((96, 3), np.int32)
    O.lib().o_link_mesh(O.ptr(fr, O._fp), O.ptr(box, O._fp), vbase, O.ptr(v, O._fp), O.ptr(t, O._i32p))
    return v, t


def robot_state(robot, base=(1.0, 2.0, 0.7), q=None):
    st = np.zeros(10, np.float32)
    st[:3] = base
    st[3:] = robot.q_home if q is None else q
    return st


def test_link_corners_and_winding_vs_fp64(O):
    """Every corner equals F_l (c_l +- h_l) in FP64 to FP32 rounding, and every
    triangle's normal points away from its box's centre (outward winding), at
    random arm poses."""
    robot = sg.make_robot(7, 8, True)
    rng = np.random.default_rng(5)
    for trial in range(6):
        q = rng.uniform(robot.qlim[:, 0], robot.qlim[:, 1]).astype(np.float32)
        st = robot_state(robot, (rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-3, 3)), q)
        F = O.fk(robot, st).astype(np.float64).reshape(8, 3, 4)
        v, t = link_mesh(O, F.astype(np.float32), robot.link_box, vbase=100)
        assert t.min() >= 100 and t.max() < 164
        for l in range(8):
            c, h = robot.link_box[l, :3].astype(np.float64), robot.link_box[l, 3:].astype(np.float64)
            for k in range(8):
                s = np.array([1 if k & 1 else -1, 1 if k & 2 else -1, 1 if k & 4 else -1], np.float64)
                want = F[l, :, :3] @ (c + s * h) + F[l, :, 3]
                assert np.allclose(v[8 * l + k], want, rtol=0, atol=1e-5), (trial, l, k)
            centre = F[l, :, :3] @ c + F[l, :, 3]
            for f in range(12):
                a, b, cc = (v[i - 100].astype(np.float64) for i in t[12 * l + f])
                n = np.cross(b - a, cc - a)
                assert n @ ((a + b + cc) / 3 - centre) > 0, (trial, l, f)


@pytest.mark.parametrize("yaw", [0.0, 0.7, -2.5])
def test_base_box_ahead_of_camera_closed_form(O, yaw):
    """A base-link box whose near face lies 1 m ahead of the head camera,
    square to its axis: the centre pixels read the analytic D24 of 1 m,
    wherever the base stands and however it is turned (the box rides with the
    base), and nothing else is drawn in the empty scene."""
    robot = sg.make_robot(7, 8, True)
    box = robot.link_box.copy()
    cx = float(robot.cam_offset[0])
    box[0] = (cx + 1.05, 0.0, float(robot.cam_offset[2]), 0.05, 0.3, 0.3)
    # the arm links out of view: behind the camera, far below the floor
    for l in range(1, 8):
        box[l] = (0.0, 0.0, 0.0, 0.01, 0.01, 0.01)
    st = robot_state(robot, (0.4, -1.3, yaw))
    F = O.fk(robot, st)
    cam = O.camera(robot, st)
    v, t = link_mesh(O, F, box)
    keep = [12 * 0 + f for f in range(12)]
    W = 64
    depth, win, _, _ = O.render(v, t[keep], cam, W, W, NEAR, FAR, want_id=True)
    ref = d24_exact(1.0)
    c = depth[W // 2 - 1:W // 2 + 1, W // 2 - 1:W // 2 + 1].astype(np.float64)
    assert np.all(np.abs(c - ref) <= 1.0 + REL_BUDGET * ref)
    # the face spans +-0.3 m at 1 m: +-0.3 of the half-width around the centre
    hit = depth < 0xFFFFFF
    rows, cols = np.nonzero(hit)
    assert abs(cols.min() - (W / 2 - 0.3 * W / 2)) <= 1 and abs(cols.max() + 1 - (W / 2 + 0.3 * W / 2)) <= 1
    assert abs(rows.min() - (W / 2 - 0.3 * W / 2)) <= 1 and abs(rows.max() + 1 - (W / 2 + 0.3 * W / 2)) <= 1
    # only the face towards the camera (-x of the box) wins: triangles 0 and 1
    assert set(np.unique(win[hit]).tolist()) <= {0, 1}


def test_links_in_batch_render_follow_the_base(O):
    """In a batch with links, the base-link box ahead of the camera is drawn
    after the static mesh with the link's colour, and its depth stays put while
    the base drives and turns (static scene removed so nothing else is hit)."""
    cfg = sg.scaled_config(0, 2)
    scenes = sg.make_scene_set(cfg)
    # an empty apartment: no static triangles at all
    n = scenes.num_envs
    scenes.tri_offset = np.zeros(n + 1, np.int64)
    scenes.tris = np.zeros((0, 3), np.int32)
    scenes.tri_rgb = np.zeros((0, 3), np.uint8)
    scenes.tri_plane = np.zeros((0, 4), np.float32)
    robot = sg.make_robot_for(cfg)
    box = robot.link_box.copy()
    box[0] = (float(robot.cam_offset[0]) + 1.55, 0.0, float(robot.cam_offset[2]), 0.05, 0.3, 0.3)
    for l in range(1, 8):
        box[l] = (0.0, 0.0, 0.0, 0.01, 0.01, 0.01)
    robot.link_box = box
    consts = sg.config_constants(cfg)
    consts["links"] = True
    ob = O.OracleBatch(robot, scenes, consts, color=True)
    W = int(scenes.res[0])
    ref = d24_exact(1.5)
    for k in range(4):
        a = np.zeros((n, 9), np.float32)
        a[:, 0] = 0.05 * (k % 2)
        a[:, 1] = 0.1 * k
        out = ob.step(a)
        for i in range(n):
            d = out["depth"][i].astype(np.float64)
            c = d[W // 2 - 1:W // 2 + 1, W // 2 - 1:W // 2 + 1]
            assert np.all(np.abs(c - ref) <= 1.0 + REL_BUDGET * ref), (k, i)
            rgb = out["rgb"][i]
            assert (rgb[W // 2, W // 2] == robot.link_rgb[0]).all()
            assert ((d < 0xFFFFFF) == (rgb.sum(axis=2) > 0)).all()


def test_arm_link_moves_with_its_joint(O):
    """The end-effector link's box follows joint 7: turning that joint alone
    moves only link 7's corners, by the rotation of its frame."""
    robot = sg.make_robot(7, 8, True)
    st = robot_state(robot)
    st2 = st.copy()
    st2[9] = np.float32(st[9] + 0.4)
    v1, _ = link_mesh(O, O.fk(robot, st), robot.link_box)
    v2, _ = link_mesh(O, O.fk(robot, st2), robot.link_box)
    assert np.array_equal(v1[:56], v2[:56])
    assert not np.allclose(v1[56:], v2[56:], atol=1e-4)
    # corner distances to the frame-7 origin are preserved (a rigid motion)
    o1 = O.fk(robot, st).reshape(8, 3, 4)[7][:, 3].astype(np.float64)
    o2 = O.fk(robot, st2).reshape(8, 3, 4)[7][:, 3].astype(np.float64)
    d1 = np.linalg.norm(v1[56:] - o1, axis=1)
    d2 = np.linalg.norm(v2[56:] - o2, axis=1)
    assert np.allclose(d1, d2, atol=1e-5)
