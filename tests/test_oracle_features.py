"""Pins of the oracle's definition of the surrogate's input (the learned
pre-filter is this project's extension of the kinematic step, Section 3.2):
closed forms on a floor-only column grid, the grid's edge, the scalars."""
import numpy as np

from oracle import oracle as O
from oracle import oracle_features as OF
from paper_2306_07552_amd import scenegen as sg

F32 = np.float32


def floor_grid(r, nx=80, ny=120, cell=0.05):
    """Column grid of an empty room for sphere radius r: one free layer
    [r, inf) per column."""
    offs, lay = O.grid_build(np.zeros((0, 6), F32), 0.0, 0.0, nx, ny, cell, r)
    return (offs, lay), (F32(0.0), F32(0.0)), (nx, ny)


def query(robot, grid, origin, dims, x, y, yaw, action=None, held=0):
    st = np.zeros(10, F32)
    st[0], st[1], st[2] = x, y, yaw
    st[3:] = robot.q_home
    a = np.zeros(9, F32) if action is None else np.asarray(action, F32)
    return OF.features(robot, (0.1, 0.1, 0.05), grid, origin, dims, sg.CELL, st, a, held)


def patch(x):
    return (x[OF.PATCH_BASE:].reshape(16, 16, 8) == 0x3F80)


def test_floor_only_patch_closed_form():
    """Floor only, largest radius 0.15 m: the lattice's lowest layer (sample
    heights 0.125..0.25 m) is blocked, the seven above are free."""
    robot = sg.make_robot_for(sg.CONFIGS[1])
    grid, origin, dims = floor_grid(0.15)
    p = patch(query(robot, grid, origin, dims, 2.0, 3.0, 0.3))
    assert p[:, :, 0].all() and not p[:, :, 1:].any()
    # radius 0.12: nothing below the lowest sample height, all free
    grid, origin, dims = floor_grid(0.12)
    assert not patch(query(robot, grid, origin, dims, 2.0, 3.0, 0.3)).any()


def test_patch_blocked_outside_the_grid():
    """Base 0.33 m from the grid's x = 0 edge, yaw 0: the lattice columns
    whose 0.1 m square reaches x < 0 (offsets -0.75 .. -0.35 m, five of
    sixteen) are blocked in every layer; the rest only in the floor layer."""
    robot = sg.make_robot_for(sg.CONFIGS[1])
    grid, origin, dims = floor_grid(0.15)
    p = patch(query(robot, grid, origin, dims, 0.33, 3.0, 0.0))
    assert p[:5].all()
    assert p[5:, :, 0].all() and not p[5:, :, 1:].any()
    # near the y = 0 edge the lattice's second axis is cut; turned by +90
    # degrees its first axis points along +y and is cut instead
    p = patch(query(robot, grid, origin, dims, 2.0, 0.33, 0.0))
    assert p[:, :5].all() and not p[:, 5:, 1:].any()
    p = patch(query(robot, grid, origin, dims, 2.0, 0.33, F32(np.pi / 2)))
    assert p[:5].all() and not p[5:, :, 1:].any()


def test_scalars():
    """Zero offsets, held: the joint angles themselves, zero deltas, the base
    position as fractions of the grid rectangle, yaw / pi, held = 1; a NaN
    offset counts as 0 and a large one is clamped to its limit."""
    robot = sg.make_robot_for(sg.CONFIGS[1])
    grid, origin, dims = floor_grid(0.15)
    x = query(robot, grid, origin, dims, 1.0, 1.5, F32(np.pi / 2), held=1)
    sc = (x[:20].astype(np.uint32) << 16).view(np.float32)
    from oracle.oracle_mlp import bf16_round_f32

    def bf(v):
        return bf16_round_f32(np.array([v], F32))[0]

    assert np.array_equal(sc[:7], np.array([bf(v) for v in robot.q_home], F32))
    assert not sc[7:16].any()
    assert sc[16] == bf(F32(1.0) / F32(4.0)) and sc[17] == bf(F32(1.5) / F32(6.0))
    assert sc[18] == bf(F32(np.pi / 2) * F32(0.31830988618)) and sc[19] == 1.0
    a = np.zeros(9, F32)
    a[2], a[3] = np.nan, 7.0
    y = query(robot, grid, origin, dims, 1.0, 1.5, 0.0, action=a)
    sy = (y[:20].astype(np.uint32) << 16).view(np.float32)
    assert sy[7] == 0.0 and sy[8] == 1.0   # NaN -> 0; 7 rad clamped to the 0.05 rad limit -> 1
