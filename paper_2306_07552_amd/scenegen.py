"""Seeded synthetic inputs for the batched kinematic step.

This module only *produces inputs*: procedural apartments (triangle meshes,
static collision boxes, graspable object boxes), a seeded Fetch-like robot
(DH chain + collision spheres), spawn poses and random actions.  It holds none
of the step's arithmetic (no kinematics, no collision, no rasterisation), so it
is the one module that both the CPU oracle and the HIP library consume.

The real assets of the paper (ReplicaCAD scenes, YCB objects, the Fetch robot
and its hand-authored spheres; Appendix G) are not available, so seeded
stand-ins of the same kind and scale are generated:

* static scene: a row of 4 x 6 m rooms with 2.5 m walls (Section 3.2 column
  grid covers the floor rectangle); furniture boxes with sides in [0.3, 1.5] m,
  a quarter of them suspended (shelves / cabinets) so that columns carry more
  than one free layer, as the table example of Appendix G;
* movable objects: small yaw-rotated boxes resting on the floor or on a
  furniture top (oriented boxes, Section 3.2);
* robot: planar base (x, y, yaw) + 7-DoF revolute arm with a seeded DH table,
  links proxied by spheres whose radii snap up to a small working set of radius
  classes (Appendix G);
* camera: head camera, 90 degree field of view (Section 4.1).

Coordinates are Z-up and right-handed (the paper is Y-up; this is a pure
relabelling).  Every triangle is wound counter-clockwise when seen from the
side its outward normal points to.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Working set of sphere-radius classes (metres).  The paper uses a small fixed
# working set so that one column grid per radius can be precomputed
# (Appendix G); the configs draw radii in [0.04, 0.12] m, which snap *up* to
# the next class (conservative).
RADIUS_CLASSES = (0.06, 0.08, 0.10, 0.12)
# The paper's own working set (Appendix G: 1.5, 5 and 12 cm), used by the
# manipulation workload, whose held objects need a radius that fits inside a
# 5 cm box.
RADIUS_CLASSES_PAPER = (0.015, 0.05, 0.12)

ROOM_X = 4.0
ROOM_Y = 6.0
WALL_H = 2.5
WALL_T = 0.1
CELL = 0.05


# --------------------------------------------------------------------------
# configuration records
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Robot:
    dh: np.ndarray            # f32 [7][4]: a, d, cos(alpha), sin(alpha)
    qlim: np.ndarray          # f32 [7][2]: lo, hi
    q_home: np.ndarray        # f32 [7]
    mount: np.ndarray         # f32 [3] shoulder mount in the base frame
    cam_offset: np.ndarray    # f32 [3] camera position in the base frame
    cam_pitch_cs: np.ndarray  # f32 [2] cos, sin of the downward pitch
    sphere_link: np.ndarray   # i32 [S] link frame 0..7 (0 = base)
    sphere_pos: np.ndarray    # f32 [S][3] link-local centre
    sphere_class: np.ndarray  # i32 [S] index into the radius classes
    sphere_held_only: np.ndarray  # u8 [S] 1 = active only while holding
    link_box: Optional[np.ndarray] = None   # f32 [8][6] per link frame: box centre xyz, half
                                            # extents xyz (drawn when links are rendered)
    link_rgb: Optional[np.ndarray] = None   # u8 [8][3] flat colour of each link's box

    @property
    def num_spheres(self) -> int:
        return int(self.sphere_link.shape[0])


@dataclasses.dataclass
class SceneSet:
    """Concatenated per-env arrays (CSR by env)."""
    num_envs: int
    vert_offset: np.ndarray   # i64 [N+1]
    verts: np.ndarray         # f32 [V][3]
    tri_offset: np.ndarray    # i64 [N+1]
    tris: np.ndarray          # i32 [T][3] env-local vertex indices
    tri_rgb: np.ndarray       # u8 [T][3]
    box_offset: np.ndarray    # i64 [N+1]
    boxes: np.ndarray         # f32 [B][6] static collision boxes (min xyz, max xyz)
    num_objects: int
    objects: np.ndarray       # f32 [N][O][8] centre xyz, half extents xyz, cos, sin (yaw)
    grid_origin: np.ndarray   # f32 [N][2]
    grid_dims: np.ndarray     # i32 [N][2] nx, ny
    num_starts: int
    starts: np.ndarray        # f32 [N][P][3] x, y, yaw
    held: np.ndarray          # u8 [N]
    res: np.ndarray           # i32 [N] square depth resolution per env
    tri_plane: Optional[np.ndarray] = None   # f32 [T][4] outward unit normal, offset of each
                                             # triangle's face (n . p = w on the face)
    obj_rgb: Optional[np.ndarray] = None     # u8 [N][O][3] flat colour of each movable object
                                             # (manipulation workload: objects are not in the
                                             # static mesh but drawn where they are)

    def env_mesh(self, e: int):
        v0, v1 = int(self.vert_offset[e]), int(self.vert_offset[e + 1])
        t0, t1 = int(self.tri_offset[e]), int(self.tri_offset[e + 1])
        return self.verts[v0:v1], self.tris[t0:t1], self.tri_rgb[t0:t1]

    def env_planes(self, e: int):
        """Face planes of env e's triangles, or None."""
        if self.tri_plane is None:
            return None
        t0, t1 = int(self.tri_offset[e]), int(self.tri_offset[e + 1])
        return self.tri_plane[t0:t1]

    def env_boxes(self, e: int):
        b0, b1 = int(self.box_offset[e]), int(self.box_offset[e + 1])
        return self.boxes[b0:b1]

    def num_tris(self, e: int) -> int:
        return int(self.tri_offset[e + 1] - self.tri_offset[e])


@dataclasses.dataclass
class Config:
    name: str
    seed: int
    num_envs: int
    res0: int
    num_spheres_per_link: int
    held_proxy: bool
    num_objects: int
    rooms: Sequence[int]            # inclusive range of rooms per apartment
    tri_target: Optional[Sequence[float]]  # None = no subdivision
    tri_target_log: bool = False
    res_choices: Optional[Sequence[int]] = None
    episode_len: int = 500
    steps: int = 100
    furniture_per_room: int = 20
    near: float = 0.1
    far: float = 10.0
    act_lim: Sequence[float] = (0.1, 0.1, 0.05)
    color: bool = False
    manip: bool = False              # grasp / release / place / slide, 11-float actions
    radius_set: Sequence[float] = RADIUS_CLASSES
    links: bool = False              # the head camera also sees the robot's own links


# The five workloads (sizes and distributions of the paper-scale step).
CONFIGS = {
    0: Config("plain-16env-64px", 1, 16, 64, 3, False, 5, (1, 1), None, steps=100,
              episode_len=500),
    1: Config("plain-1024env-128px-20k-80k-tris", 2, 1024, 128, 8, True, 8, (2, 6),
              (20000.0, 80000.0), steps=1000, episode_len=500),
    2: Config("uneven-4096env-2k-200k-tris-mixed-res", 3, 4096, 128, 8, True, 8, (2, 6),
              (2000.0, 200000.0), tri_target_log=True, res_choices=(64, 128, 256)),
    4: Config("mixed-8192env-2k-200k-tris-128px-rgb", 5, 8192, 128, 8, True, 8, (2, 6),
              (2000.0, 200000.0), tri_target_log=True, color=True),
    # the rest of the kinematic sim of Section 3.2 / Appendix I on the
    # paper-scale step: grasp, carry, release with snap-to-surface and the
    # placing heuristic, sliding; the paper's radius working set and its 30
    # resting objects per episode (1 target + 29 distractors, Section 4.1)
    5: Config("manip-1024env-128px-20k-80k-tris", 6, 1024, 128, 8, False, 30, (2, 6),
              (20000.0, 80000.0), steps=1000, episode_len=500, manip=True,
              radius_set=RADIUS_CLASSES_PAPER, links=True),
}

# Manipulation constants.  Section 3.2 queries a small (3 cm) sphere at the
# end-effector tip: read as 3 cm across, placed 0.25 m out along the last
# link's z axis (a suction tool clear of the arm's own spheres).  The jitter
# steps of Appendix I's heuristics are this build's choice.
GRASP_TIP = (0.0, 0.0, 0.25)
GRASP_RADIUS = 0.015
SLIDE_STEP = 0.05
PLACE_STEP = 0.10


def scaled_config(base: int, num_envs: int, **kw) -> Config:
    """A copy of a workload with fewer environments (same per-env recipe)."""
    c = dataclasses.replace(CONFIGS[base], num_envs=num_envs, **kw)
    return c


# --------------------------------------------------------------------------
# robot
# --------------------------------------------------------------------------
def make_robot(seed: int, spheres_per_link: int, held_proxy: bool,
               classes: Sequence[float] = RADIUS_CLASSES) -> Robot:
    rng = np.random.default_rng([seed, 0xB0B])
    dh = np.zeros((7, 4), np.float32)
    alpha_choices = [(0.0, -1.0), (1.0, 0.0), (0.0, 1.0)]  # -pi/2, 0, +pi/2 (exact)
    for j in range(7):
        ca, sa = alpha_choices[int(rng.integers(0, 3))]
        dh[j] = (rng.uniform(0.05, 0.15), rng.uniform(0.0, 0.12), ca, sa)
    lim = rng.uniform(1.2, 2.0, size=7)
    qlim = np.stack([-lim, lim], axis=1).astype(np.float32)
    q_home = rng.uniform(-0.3, 0.3, size=7).astype(np.float32)
    mount = np.array([0.15, 0.0, 0.95], np.float32)
    cam_offset = np.array([0.10, 0.0, 1.10], np.float32)
    cam_pitch_cs = np.array([1.0, 0.0], np.float32)  # level camera

    links, pos, radius = [], [], []
    for link in range(8):
        for _ in range(spheres_per_link):
            if link == 0:
                p = (rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), rng.uniform(0.3, 1.0))
            else:
                a = float(dh[link - 1, 0])
                p = (rng.uniform(-a, 0.0), rng.uniform(-0.04, 0.04), rng.uniform(-0.04, 0.04))
            links.append(link)
            pos.append(p)
            radius.append(rng.uniform(0.04, 0.12))
    cls = [snap_class(r, classes) for r in radius]
    held_only = [0] * len(links)
    if held_proxy:
        # one sphere for the held object, on the end-effector frame
        links.append(7)
        pos.append((0.0, 0.0, 0.10))
        cls.append(1)
        held_only.append(1)
    # render boxes of the links (no random draws): the base body below the
    # camera, and each arm link along its frame's -x over its DH length a
    # (where its spheres lie), 6 cm thick
    box = np.zeros((8, 6), np.float32)
    box[0] = (0.0, 0.0, 0.45, 0.25, 0.25, 0.45)
    for link in range(1, 8):
        a = float(dh[link - 1, 0])
        box[link] = (-0.5 * a, 0.0, 0.0, 0.5 * a + 0.02, 0.03, 0.03)
    rgb = np.array([(90, 90, 100)] + [(200, 200, 205) if k % 2 else (60, 60, 70) for k in range(1, 7)]
                   + [(180, 40, 40)], np.uint8)
    return Robot(dh=dh, qlim=qlim, q_home=q_home, mount=mount, cam_offset=cam_offset,
                 cam_pitch_cs=cam_pitch_cs,
                 sphere_link=np.asarray(links, np.int32),
                 sphere_pos=np.asarray(pos, np.float32).reshape(-1, 3),
                 sphere_class=np.asarray(cls, np.int32),
                 sphere_held_only=np.asarray(held_only, np.uint8),
                 link_box=box, link_rgb=rgb)


def snap_class(r: float, classes: Sequence[float] = RADIUS_CLASSES) -> int:
    for k, rk in enumerate(classes):
        if rk >= r:
            return k
    return len(classes) - 1


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
_FACES = (
    # (u axis, v axis, constant axis, constant at max?, flip winding)
    (0, 1, 2, True, False),    # +z: x cross y = +z
    (0, 1, 2, False, True),    # -z
    (1, 2, 0, True, False),    # +x: y cross z = +x
    (1, 2, 0, False, True),    # -x
    (2, 0, 1, True, False),    # +y: z cross x = +y
    (2, 0, 1, False, True),    # -y
)


def _face_tris(n: int) -> np.ndarray:
    """Triangle template of one n x n face grid, CCW around u x v."""
    iu, iv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a = (iu * (n + 1) + iv).ravel()
    b = ((iu + 1) * (n + 1) + iv).ravel()
    c = ((iu + 1) * (n + 1) + iv + 1).ravel()
    d = (iu * (n + 1) + iv + 1).ravel()
    return np.stack([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 1).reshape(-1, 3)


def boxes_mesh(lo, hi, n: int):
    """Closed axis-aligned boxes [B] with faces subdivided n x n and outward
    CCW winding.  Lattice coordinates are produced once per box and axis, so
    vertices on edges shared by two faces are bit-identical."""
    lo = np.asarray(lo, np.float64).reshape(-1, 3)
    hi = np.asarray(hi, np.float64).reshape(-1, 3)
    B = lo.shape[0]
    k = np.arange(n + 1, dtype=np.float64) / n
    lat = (lo[:, :, None] + (hi - lo)[:, :, None] * k[None, None, :]).astype(np.float32)  # [B,3,n+1]
    tpl = _face_tris(n)
    vpf = (n + 1) * (n + 1)
    verts = np.empty((B, 6, n + 1, n + 1, 3), np.float32)
    tris = []
    for f, (au, av, ac, at_max, flip) in enumerate(_FACES):
        verts[:, f, :, :, au] = lat[:, au, :, None]
        verts[:, f, :, :, av] = lat[:, av, None, :]
        verts[:, f, :, :, ac] = lat[:, ac, -1 if at_max else 0][:, None, None]
        t = tpl[:, [0, 2, 1]] if flip else tpl
        tris.append(t + f * vpf)
    tris = np.concatenate(tris)                                   # [12 n^2, 3]
    allt = tris[None, :, :] + (np.arange(B) * 6 * vpf)[:, None, None]
    return verts.reshape(-1, 3), allt.reshape(-1, 3)


def box_mesh(lo, hi, n: int):
    """One closed axis-aligned box (see ``boxes_mesh``)."""
    return boxes_mesh(lo, hi, n)


def quad_mesh(P0, U, V):
    """Single quad P0, P0+U, P0+U+V, P0+V as two CCW triangles (normal U x V)."""
    P0, U, V = (np.asarray(a, np.float64) for a in (P0, U, V))
    verts = np.stack([P0, P0 + U, P0 + U + V, P0 + V]).astype(np.float32)
    return verts, np.array([[0, 1, 2], [0, 2, 3]], np.int64)


def obb_mesh(centre, half, cpsi: float, spsi: float):
    """12-triangle mesh of a yaw-rotated box (outward CCW)."""
    lo = -np.asarray(half, np.float64)
    hi = np.asarray(half, np.float64)
    v, t = box_mesh(lo, hi, 1)
    v = v.astype(np.float64)
    R = np.array([[cpsi, -spsi, 0.0], [spsi, cpsi, 0.0], [0.0, 0.0, 1.0]])
    v = v @ R.T + np.asarray(centre, np.float64)
    return v.astype(np.float32), t


def _plane_row(normal, point) -> np.ndarray:
    """f32 [4]: the unit normal and the offset n . point of a face plane."""
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    return np.array([n[0], n[1], n[2], float(n @ np.asarray(point, np.float64))], np.float32)


def quad_planes(P0, U, V) -> np.ndarray:
    """Face plane of ``quad_mesh(P0, U, V)``'s two triangles, f32 [2][4]."""
    row = _plane_row(np.cross(np.asarray(U, np.float64), np.asarray(V, np.float64)), P0)
    return np.repeat(row[None, :], 2, axis=0)


def boxes_planes(lo, hi, n: int) -> np.ndarray:
    """Face planes of ``boxes_mesh(lo, hi, n)``'s triangles, f32 [B * 12 n^2][4], in its
    triangle order.  Each face's offset is the face coordinate of its vertices (the same
    float), so the plane passes exactly through them."""
    lo = np.asarray(lo, np.float64).reshape(-1, 3)
    hi = np.asarray(hi, np.float64).reshape(-1, 3)
    B = lo.shape[0]
    per_face = 2 * n * n
    rows = np.empty((B, 6, per_face, 4), np.float32)
    for f, (_au, _av, ac, at_max, _flip) in enumerate(_FACES):
        k = 1.0 if at_max else 0.0
        c = (lo[:, ac] + (hi[:, ac] - lo[:, ac]) * k).astype(np.float32)   # as in boxes_mesh
        sign = np.float32(1.0 if at_max else -1.0)
        rows[:, f, :, :3] = 0.0
        rows[:, f, :, ac] = sign
        rows[:, f, :, 3] = (sign * c)[:, None]
    return rows.reshape(-1, 4)


def obb_planes(centre, half, cpsi: float, spsi: float) -> np.ndarray:
    """Face planes of ``obb_mesh``'s 12 triangles, f32 [12][4]."""
    R = np.array([[cpsi, -spsi, 0.0], [spsi, cpsi, 0.0], [0.0, 0.0, 1.0]])
    half = np.asarray(half, np.float64)
    centre = np.asarray(centre, np.float64)
    rows = []
    for (_au, _av, ac, at_max, _flip) in _FACES:
        e = np.zeros(3)
        e[ac] = 1.0 if at_max else -1.0
        nrm = R @ e
        rows.append(_plane_row(nrm, centre + nrm * half[ac]))
        rows.append(rows[-1])
    return np.stack(rows)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------
def _rects_overlap(a, b) -> bool:
    return a[0] < b[2] and b[0] < a[2] and a[1] < b[3] and b[1] < a[3]


def make_scene(cfg: Config, env: int):
    """One procedural apartment.  Returns a dict of numpy arrays."""
    rng = np.random.default_rng([cfg.seed, env, 0x5CE])
    R = int(rng.integers(cfg.rooms[0], cfg.rooms[1] + 1))
    W, H = ROOM_X * R, ROOM_Y

    # target triangle count -> per-env subdivision level of furniture faces
    n_sub = 1
    nfurn = cfg.furniture_per_room * R
    if cfg.tri_target is not None:
        lo, hi = cfg.tri_target
        if cfg.tri_target_log:
            tt = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        else:
            tt = rng.uniform(lo, hi)
        n_sub = max(1, int(round(math.sqrt(max(tt - 200.0, 12.0 * nfurn) / (12.0 * nfurn)))))

    # spawn pad (1 x 1 m) in room 0, kept clear of furniture and objects
    px = rng.uniform(0.6, ROOM_X - 1.6)
    py = rng.uniform(0.6, ROOM_Y - 1.6)
    pad = (px, py, px + 1.0, py + 1.0)
    pad_keep = (px - 0.3, py - 0.3, px + 1.3, py + 1.3)

    static_boxes: List[tuple] = []
    # outer wall slabs, outside the floor rectangle (grid collision only)
    static_boxes.append((-WALL_T, -WALL_T, 0.0, 0.0, H + WALL_T, WALL_H))
    static_boxes.append((W, -WALL_T, 0.0, W + WALL_T, H + WALL_T, WALL_H))
    static_boxes.append((0.0, -WALL_T, 0.0, W, 0.0, WALL_H))
    static_boxes.append((0.0, H, 0.0, W, H + WALL_T, WALL_H))
    interior = []
    for k in range(1, R):
        x = ROOM_X * k
        g = rng.uniform(0.5, ROOM_Y - 1.5)
        interior.append((x - WALL_T / 2, 0.0, 0.0, x + WALL_T / 2, g, WALL_H))
        interior.append((x - WALL_T / 2, g + 1.0, 0.0, x + WALL_T / 2, H, WALL_H))
    static_boxes.extend(interior)

    furniture = []
    tops = []  # floor-standing tops that objects may rest on
    for r in range(R):
        rx0 = ROOM_X * r
        for _ in range(cfg.furniture_per_room):
            for _attempt in range(20):
                sx, sy, sz = rng.uniform(0.3, 1.5, size=3)
                x0 = rng.uniform(rx0 + 0.05, rx0 + ROOM_X - 0.05 - sx)
                y0 = rng.uniform(0.05, ROOM_Y - 0.05 - sy)
                if r == 0 and _rects_overlap((x0, y0, x0 + sx, y0 + sy), pad_keep):
                    continue
                break
            else:
                continue
            suspended = rng.uniform() < 0.25
            z0 = rng.uniform(0.5, 1.0) if suspended else 0.0
            b = (x0, y0, z0, x0 + sx, y0 + sy, z0 + sz)
            furniture.append(b)
            if not suspended:
                tops.append(b)
    static_boxes.extend(furniture)

    # movable objects: small yaw-rotated boxes on the floor or on a top
    objs = []
    for _ in range(cfg.num_objects):
        for _attempt in range(50):
            half = rng.uniform(0.05, 0.15, size=3) / 2.0
            yaw = rng.uniform(-math.pi, math.pi)
            if tops and rng.uniform() < 0.5:
                t = tops[int(rng.integers(0, len(tops)))]
                cx = rng.uniform(t[0] + 0.1, t[3] - 0.1) if t[3] - t[0] > 0.2 else (t[0] + t[3]) / 2
                cy = rng.uniform(t[1] + 0.1, t[4] - 0.1) if t[4] - t[1] > 0.2 else (t[1] + t[4]) / 2
                cz = t[5] + half[2]
            else:
                cx = rng.uniform(0.2, W - 0.2)
                cy = rng.uniform(0.2, H - 0.2)
                cz = half[2]
            if _rects_overlap((cx - 0.2, cy - 0.2, cx + 0.2, cy + 0.2), pad_keep):
                continue
            break
        objs.append((cx, cy, cz, half[0], half[1], half[2], math.cos(yaw), math.sin(yaw)))

    # ---------------- render mesh ----------------
    parts_v, parts_t, parts_p = [], [], []

    def add(v, t, pl):
        parts_v.append(v)
        parts_t.append(t)
        parts_p.append(pl)

    for q in (((0, 0, 0), (W, 0, 0), (0, H, 0)),                     # floor, +z
              ((0, 0, 0), (0, H, 0), (0, 0, WALL_H)),                # x=0 wall, +x
              ((W, 0, 0), (0, 0, WALL_H), (0, H, 0)),                # x=W wall, -x
              ((0, 0, 0), (0, 0, WALL_H), (W, 0, 0)),                # y=0 wall, +y
              ((0, H, 0), (W, 0, 0), (0, 0, WALL_H))):               # y=H wall, -y
        add(*quad_mesh(*q), quad_planes(*q))
    if interior:
        ib = np.asarray(interior, np.float64)
        add(*boxes_mesh(ib[:, :3], ib[:, 3:], 1), boxes_planes(ib[:, :3], ib[:, 3:], 1))
    if furniture:
        fb = np.asarray(furniture, np.float64)
        add(*boxes_mesh(fb[:, :3], fb[:, 3:], n_sub), boxes_planes(fb[:, :3], fb[:, 3:], n_sub))
    if not cfg.manip:
        for o in objs:
            add(*obb_mesh(o[:3], o[3:6], o[6], o[7]), obb_planes(o[:3], o[3:6], o[6], o[7]))

    verts, tris, base = [], [], 0
    for v, t in zip(parts_v, parts_t):
        verts.append(v)
        tris.append(t + base)
        base += v.shape[0]
    verts = np.concatenate(verts).astype(np.float32)
    tris = np.concatenate(tris).astype(np.int32)
    planes = np.concatenate(parts_p).astype(np.float32)
    assert planes.shape[0] == tris.shape[0]
    rgb = rng.integers(0, 256, size=(tris.shape[0], 3), dtype=np.uint8)

    starts = np.zeros((4, 3), np.float32)
    for p in range(4):
        starts[p] = (px + 0.5 + rng.uniform(-0.2, 0.2), py + 0.5 + rng.uniform(-0.2, 0.2),
                     rng.uniform(-math.pi, math.pi))

    res = cfg.res0
    if cfg.res_choices:
        res = int(cfg.res_choices[int(rng.integers(0, len(cfg.res_choices)))])
    held = int(rng.uniform() < 0.5) if cfg.held_proxy else 0
    # drawn last, so that the other workloads' scenes are unchanged
    obj_rgb = rng.integers(0, 256, size=(len(objs), 3), dtype=np.uint8) if cfg.manip else None
    nx = int(round(W / CELL))
    ny = int(round(H / CELL))
    return dict(verts=verts, tris=tris, rgb=rgb, planes=planes,
                boxes=np.asarray(static_boxes, np.float32).reshape(-1, 6),
                objects=np.asarray(objs, np.float32).reshape(-1, 8),
                grid_origin=np.array([0.0, 0.0], np.float32),
                grid_dims=np.array([nx, ny], np.int32),
                starts=starts, held=held, res=res, obj_rgb=obj_rgb)


def make_scene_set(cfg: Config, envs: Optional[Sequence[int]] = None) -> SceneSet:
    """Scenes of ``cfg`` for the env indices ``envs`` (default: all)."""
    if envs is None:
        envs = range(cfg.num_envs)
    envs = list(envs)
    scenes = [make_scene(cfg, e) for e in envs]
    N = len(scenes)
    vo = np.zeros(N + 1, np.int64)
    to = np.zeros(N + 1, np.int64)
    bo = np.zeros(N + 1, np.int64)
    for i, s in enumerate(scenes):
        vo[i + 1] = vo[i] + s["verts"].shape[0]
        to[i + 1] = to[i] + s["tris"].shape[0]
        bo[i + 1] = bo[i] + s["boxes"].shape[0]
    return SceneSet(
        num_envs=N, vert_offset=vo,
        verts=np.ascontiguousarray(np.concatenate([s["verts"] for s in scenes])),
        tri_offset=to,
        tris=np.ascontiguousarray(np.concatenate([s["tris"] for s in scenes])),
        tri_rgb=np.ascontiguousarray(np.concatenate([s["rgb"] for s in scenes])),
        box_offset=bo,
        boxes=np.ascontiguousarray(np.concatenate([s["boxes"] for s in scenes])),
        num_objects=cfg.num_objects,
        objects=np.ascontiguousarray(np.stack([s["objects"] for s in scenes])),
        grid_origin=np.ascontiguousarray(np.stack([s["grid_origin"] for s in scenes])),
        grid_dims=np.ascontiguousarray(np.stack([s["grid_dims"] for s in scenes])),
        num_starts=4,
        starts=np.ascontiguousarray(np.stack([s["starts"] for s in scenes])),
        held=np.asarray([s["held"] for s in scenes], np.uint8),
        res=np.asarray([s["res"] for s in scenes], np.int32),
        tri_plane=np.ascontiguousarray(np.concatenate([s["planes"] for s in scenes])),
        obj_rgb=(np.ascontiguousarray(np.stack([s["obj_rgb"] for s in scenes]))
                 if cfg.manip else None),
    )


def make_robot_for(cfg: Config) -> Robot:
    return make_robot(cfg.seed, cfg.num_spheres_per_link, cfg.held_proxy, tuple(cfg.radius_set))


# --------------------------------------------------------------------------
# actions
# --------------------------------------------------------------------------
def actions(cfg: Config, step: int, num_envs: Optional[int] = None,
            envs: Optional[Sequence[int]] = None) -> np.ndarray:
    """Random actions f32 [N][9] for one step: forward (m), yaw (rad), 7 joint
    deltas (rad), drawn uniformly within the action limits."""
    ids = np.arange(cfg.num_envs if num_envs is None else num_envs) if envs is None \
        else np.asarray(list(envs))
    rng = np.random.default_rng([cfg.seed, step, 0xAC7])
    lim = np.array([cfg.act_lim[0], cfg.act_lim[1]] + [cfg.act_lim[2]] * 7, np.float64)
    full_n = int(ids.max()) + 1 if ids.size else 0
    u = rng.uniform(-1.0, 1.0, size=(max(full_n, 1), 9))
    a = (u[ids] * lim).astype(np.float32)
    if cfg.manip:
        # grasp / release as a 0/1 value (grasp intent 60 % of steps, so that
        # objects are both picked and dropped), stop rarely
        d = rng.uniform(0.0, 1.0, size=(max(full_n, 1), 2))[ids]
        extra = np.stack([(d[:, 0] < 0.6), (d[:, 1] < 0.002)], axis=1).astype(np.float32)
        a = np.concatenate([a, extra], axis=1)
    return a


def config_constants(cfg: Config) -> dict:
    c = dict(near=cfg.near, far=cfg.far, cell=CELL, radius_classes=tuple(cfg.radius_set),
             act_lim=tuple(cfg.act_lim), episode_len=cfg.episode_len, res0=cfg.res0)
    if cfg.links:
        c.update(links=True)
    if cfg.manip:
        c.update(manip=True, slide=True, grasp_tip=GRASP_TIP, grasp_radius=GRASP_RADIUS,
                 held_class=0, slide_step=SLIDE_STEP, place_step=PLACE_STEP,
                 seed=cfg.seed * 1000003 + 17)
    return c
