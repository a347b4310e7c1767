"""Helpers shared by the GPU parity tests: build the same seeded workload for
the HIP library (through the C ABI) and for the CPU oracle, and compare."""
import numpy as np

from paper_2306_07552_amd import scenegen as sg


def u32(t):
    """torch int32 tensor -> numpy uint32 view."""
    return t.detach().cpu().numpy().view(np.uint32)


def make_pair(cfg, envs=None, oracle_envs=None, color=False):
    """(gpu Batch, OracleBatch, scenes, robot) for the envs of ``cfg``; the
    oracle covers ``oracle_envs`` (indices into the batch) only."""
    import torch  # noqa: F401
    from oracle import oracle as O
    from paper_2306_07552_amd import gal
    scenes = sg.make_scene_set(cfg, envs)
    robot = sg.make_robot_for(cfg)
    consts = sg.config_constants(cfg)
    b = gal.Batch(robot, scenes, consts, color=color)
    ob = O.OracleBatch(robot, scenes, consts, envs=oracle_envs, color=color)
    return b, ob, scenes, robot


def compare_step(b, ob, out, oout, label=""):
    """Compare one step's GPU outputs with the oracle's for the oracle envs."""
    envs = ob.envs
    st = out["state"].cpu().numpy()[envs]
    assert np.array_equal(st.view(np.uint32), oout["state"].view(np.uint32)), f"{label} state"
    assert np.array_equal(out["counters"].cpu().numpy()[envs], oout["counters"]), f"{label} counters"
    assert np.array_equal(out["accepted"].cpu().numpy()[envs], oout["accepted"]), f"{label} accepted"
    assert np.array_equal(out["done"].cpu().numpy()[envs], oout["done"]), f"{label} done"
    assert np.array_equal(u32(out["contact_static"])[envs], oout["contact_static"]), f"{label} static"
    assert np.array_equal(u32(out["contact_object"])[envs], oout["contact_object"]), f"{label} object"
    fr = out["frames"].cpu().numpy()[envs]
    # FK: bit-exact (the stated tolerance, 1e-5 m, is then met trivially)
    assert np.max(np.abs(fr - oout["frames"])) <= 1e-5, f"{label} frames tolerance"
    assert np.array_equal(fr.view(np.uint32), oout["frames"].view(np.uint32)), f"{label} frames"
    depth = u32(out["depth"])
    for i, e in enumerate(envs):
        d = b.env_depth(depth, e)
        if not np.array_equal(d, oout["depth"][i]):
            bad = np.argwhere(d != oout["depth"][i])
            y, x = bad[0]
            raise AssertionError(f"{label} depth env {e}: {len(bad)} pixels differ, first "
                                 f"({y},{x}) gpu {d[y, x]} oracle {oout['depth'][i][y, x]}")
        if "rgb" in out and oout["rgb"][i] is not None:
            rgb = out["rgb"].cpu().numpy()
            r = int(b.res[e])
            img = rgb[int(b.depth_off[e]):int(b.depth_off[e + 1])].reshape(r, r, 3)
            assert np.array_equal(img, oout["rgb"][i]), f"{label} rgb env {e}"
