"""Oracle of the collision surrogate's input vector (test infrastructure only).

The learned pre-filter is not part of the paper (it is this project's
extension of the kinematic step of Section 3.2): its input is defined with
it, as 2112 BF16 values per query -
  [0, 20)    scalars: the candidate joint angles q (7), the joint offsets
             divided by their limit (7), the base offsets divided by theirs
             (2), the base position within the env's grid rectangle (2,
             fractions), yaw / pi, the held flag;
  [20, 44)   the arm's pose with the base at the origin: the origins of link
             frames 1..7 and the end effector's z axis;
  [44, 64)   zero;
  [64, 2112) a 16 x 16 lattice of 0.1 m cells around the candidate base
             (rotated with its yaw), 8 layers of 0.25 m each: 1 where the
             column grid of the largest sphere class has no free layer at
             one of four heights of the layer (none below 0.125 m) anywhere
             in the grid cells the lattice cell's square covers, or where
             the square leaves the grid; else 0.
Everything is FP32 in the order written, then rounded to BF16 (1 = 0x3F80).
Candidate yaw and base offsets follow the step's action decode (Section
3.2: offsets applied directly to the state; sanitised and clamped)."""
import numpy as np

from oracle import oracle as O
from oracle.oracle_mlp import bf16_round_f32

F32 = np.float32
DIM = 2112
PATCH_BASE = 64


def lattice_cell(offs, lay, nx, i, j, k) -> bool:
    """Occupancy of grid column (i, j) in lattice layer k: blocked when at
    one of four heights inside the layer (none below 0.125 m) the column has
    no free layer."""
    c = j * nx + i
    lo_hi = lay[offs[c]:offs[c + 1]]
    for m in range(4):
        z = max(F32(F32(k) * F32(0.25)) + F32(F32(0.0625) * F32(m + 1)), F32(0.125))
        if not np.any((lo_hi[:, 0] <= z) & (z <= lo_hi[:, 1])):
            return True
    return False


def sanitize(action, act_lim):
    """NaN -> 0, then clamped to the base (m, rad) and joint (rad) limits."""
    lim = np.array([act_lim[0], act_lim[1]] + [act_lim[2]] * 7, F32)
    return np.clip(np.nan_to_num(np.asarray(action[:9], F32), nan=0.0).astype(F32), -lim, lim)


def features(robot, act_lim, grid, origin, dims, cell, state, action, held):
    """The 2112 BF16 bit patterns of one query.  grid = (offsets, layers) of
    the env's largest-class column grid; origin, dims its rectangle's corner
    and cell counts; state the env's [10] state before the step."""
    lim = [F32(v) for v in act_lim]
    st = np.asarray(state, F32)
    san = sanitize(action, act_lim)
    q = np.clip((st[3:10] + san[2:9]).astype(F32), robot.qlim[:, 0], robot.qlim[:, 1])
    x0, y0 = (F32(v) for v in origin)
    nx, ny = (int(v) for v in dims)
    cell = F32(cell)
    sc = np.concatenate([q, san[2:9] / lim[2], [san[0] / lim[0], san[1] / lim[1]],
                         [(st[0] - x0) / (F32(nx) * cell), (st[1] - y0) / (F32(ny) * cell),
                          st[2] * F32(0.31830988618), F32(held != 0)]]).astype(F32)
    out = np.zeros(DIM, np.uint16)
    out[:20] = (bf16_round_f32(sc).view(np.uint32) >> 16).astype(np.uint16)
    fr = O.fk(robot, np.concatenate([np.zeros(3, F32), q]).astype(F32)).reshape(8, 3, 4)
    arm = np.concatenate([fr[1:, :, 3].reshape(-1), fr[7, :, 2]]).astype(F32)
    out[20:44] = (bf16_round_f32(arm).view(np.uint32) >> 16).astype(np.uint16)
    # candidate base pose
    pi_f, two_pi_f = F32(np.pi), F32(2 * np.pi)
    yaw = F32(st[2] + san[1])
    if yaw > pi_f:
        yaw = F32(yaw - two_pi_f)
    elif yaw < -pi_f:
        yaw = F32(yaw + two_pi_f)
    sy, cy = (F32(v[0]) for v in O.sincos(np.array([yaw], F32)))
    bx, by = F32(st[0] + F32(san[0] * cy)), F32(st[1] + F32(san[0] * sy))
    offs, lay = grid
    cache = {}
    hx = F32(F32(0.05) * F32(abs(cy) + abs(sy)))   # half side of the rotated cell's bounding square
    for pa in range(16):
        for pb in range(16):
            px, py = F32(F32(pa) - F32(7.5)) * F32(0.1), F32(F32(pb) - F32(7.5)) * F32(0.1)
            wx = F32(bx + F32(F32(cy * px) - F32(sy * py)))
            wy = F32(by + F32(F32(sy * px) + F32(cy * py)))
            i0, i1 = (np.floor(F32(F32(F32(wx + d) - x0) / cell)) for d in (-hx, hx))
            j0, j1 = (np.floor(F32(F32(F32(wy + d) - y0) / cell)) for d in (-hx, hx))
            inside = i0 >= 0 and j0 >= 0 and i1 < nx and j1 < ny
            for k in range(8):
                blocked = not inside
                if inside:
                    for j in range(int(j0), int(j1) + 1):
                        for i in range(int(i0), int(i1) + 1):
                            if (i, j, k) not in cache:
                                cache[(i, j, k)] = lattice_cell(offs, lay, nx, i, j, k)
                            blocked = blocked or cache[(i, j, k)]
                out[PATCH_BASE + (pa * 16 + pb) * 8 + k] = 0x3F80 if blocked else 0
    return out
