"""The occlusion cull's conservativeness, checked on the host: the raster
kernel drops a cluster when the nearest possible depth of its AABB lies
behind every z-buffer maximum under the AABB's projected pixel box.  That
box is computed with the hardware's approximate reciprocal (within 1 ulp);
the kernel widens it by one pixel and lowers the depth bound by a relative
1e-5, 1e-4 m and 16 LSB.  Here the same FP32 sequence, with the reciprocal
moved by +-2 ulp, must contain every pixel a triangle with vertices in the
box can cover (the snapped vertex bbox) and stay below every vertex's D24
(interpolated depths lie above the smallest vertex depth up to a few ulp)."""
import numpy as np

F32 = np.float32


def rn_div(a, b):
    return F32(F32(a) / F32(b))


def cam_coords(cam, p):
    d = [F32(p[0] - cam["p"][0]), F32(p[1] - cam["p"][1]), F32(p[2] - cam["p"][2])]
    out = []
    for axis in ("r", "d", "f"):
        a = cam[axis]
        out.append(F32(F32(F32(a[0] * d[0]) + F32(a[1] * d[1])) + F32(a[2] * d[2])))
    return out


def make_cam(rng):
    yaw = rng.uniform(-np.pi, np.pi)
    pitch = rng.uniform(-0.3, 0.3)
    f = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), -np.sin(pitch)])
    r = np.array([np.sin(yaw), -np.cos(yaw), 0.0])
    d = np.cross(f, r)
    return {"p": rng.uniform(-3, 3, 3).astype(F32), "r": r.astype(F32), "d": d.astype(F32), "f": f.astype(F32)}


def test_cluster_bound_is_conservative():
    rng = np.random.default_rng(21)
    near, far, W = F32(0.1), F32(10.0), 128
    hw = F32(W * 0.5)
    invn = F32(F32(1.0) / near)
    kd = F32(F32(16777215.0) / F32(invn - F32(F32(1.0) / far)))
    checked = 0
    for trial in range(400):
        cam = make_cam(rng)
        centre = cam["p"] + cam["f"] * F32(rng.uniform(0.3, 6.0)) + rng.normal(scale=1.0, size=3).astype(F32)
        half = rng.uniform(0.02, 0.6, 3).astype(F32)
        lo, hi = (centre - half).astype(F32), (centre + half).astype(F32)
        # the kernel's bound, in its FP32 order
        X0, Y0, Z0 = cam_coords(cam, lo)
        e = [F32(hi[i] - lo[i]) for i in range(3)]
        terms = {ax: [F32(cam[ax][i] * e[i]) for i in range(3)] for ax in ("r", "d", "f")}
        zmin = F32(F32(F32(Z0 + min(terms["f"][0], F32(0))) + min(terms["f"][1], F32(0))) + min(terms["f"][2], F32(0)))
        if not zmin > F32(F32(1.01) * near) + F32(1e-3):
            continue
        for delta in (-2.0 ** -22, 2.0 ** -22):
            nx, ny = [], []
            for c in range(8):
                sel = [(c >> i) & 1 for i in range(3)]
                def corner(base, ax):
                    v = base
                    for i in range(3):
                        v = F32(v + (terms[ax][i] if sel[i] else F32(0)))
                    return v
                X, Y, Z = corner(X0, "r"), corner(Y0, "d"), corner(Z0, "f")
                rc = F32(rn_div(1.0, Z) * F32(1.0 + delta))
                nx.append(F32(X * rc))
                ny.append(F32(Y * rc))
            fx0, fx1 = F32(hw + F32(hw * min(nx))), F32(hw + F32(hw * max(nx)))
            fy0, fy1 = F32(hw + F32(hw * min(ny))), F32(hw + F32(hw * max(ny)))
            px0, px1 = int(np.floor(max(fx0, -1e6))) - 1, int(np.floor(min(fx1, 1e6))) + 1
            py0, py1 = int(np.floor(max(fy0, -1e6))) - 1, int(np.floor(min(fy1, 1e6))) + 1
            zlb = F32(F32(zmin * F32(1.0 - 1e-5)) - F32(1e-4))
            dlb = F32(F32(F32(invn - rn_div(1.0, zlb)) * kd) - F32(16.0))
            # points of the box: corners and random interior points
            pts = [np.where([(c >> i) & 1 for i in range(3)], hi, lo) for c in range(8)]
            pts += list(rng.uniform(lo, hi, size=(24, 3)).astype(F32))
            for p in pts:
                X, Y, Z = cam_coords(cam, np.asarray(p, F32))
                assert Z >= F32(zmin * F32(1.0 - 1e-6)) - F32(1e-6)
                xs = F32(hw + F32(hw * rn_div(X, Z)))
                ys = F32(hw + F32(hw * rn_div(Y, Z)))
                xi, yi = int(np.rint(F32(xs * F32(16)))), int(np.rint(F32(ys * F32(16))))
                # pixel centres a triangle through this vertex can cover lie
                # within ceil/floor of the snapped coordinate +- half a pixel
                assert px0 <= (xi + 7) >> 4 and ((xi - 8) >> 4) <= px1, (trial, xi, px0, px1)
                assert py0 <= (yi + 7) >> 4 and ((yi - 8) >> 4) <= py1, (trial, yi, py0, py1)
                d = F32(F32(invn - rn_div(1.0, Z)) * kd)
                assert dlb <= F32(d * F32(1.0 - 2.0 ** -20)) - F32(1.0), (trial, dlb, d)
                checked += 1
    assert checked > 10000
