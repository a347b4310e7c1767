"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.  Depth, contact masks, acceptance, counters and the
state are compared bit for bit; link frames bit for bit (and so within the
1e-5 m FK tolerance)."""
import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg
from parity_util import compare_step, make_pair, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def run_trajectory(torch, cfg, steps, envs=None, oracle_envs=None, color=False, act_fn=None):
    b, ob, scenes, robot = make_pair(cfg, envs, oracle_envs, color=color)
    out = b.alloc_outputs()
    N = b.num_envs
    for k in range(steps):
        a = sg.actions(cfg, k, num_envs=N) if act_fn is None else act_fn(k, N)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        oout = ob.step(a[ob.envs])
        compare_step(b, ob, out, oout, label=f"step {k}")
    return b, ob


def test_config0_full_trajectory(torch_cuda):
    """16 envs x 100 steps, every env, every step."""
    print("case: config 0, 16 envs x 100 steps", flush=True)
    run_trajectory(torch_cuda, sg.CONFIGS[0], 100)


def test_grid_bitwise_equal(torch_cuda):
    print("case: column grids, config 0 and 1", flush=True)
    from oracle import oracle as O
    for cfgid, envs in ((0, range(4)), (1, [0, 5])):
        cfg = sg.CONFIGS[cfgid]
        b, ob, scenes, robot = make_pair(cfg, envs, oracle_envs=[])
        for e in range(scenes.num_envs):
            nx, ny = (int(v) for v in scenes.grid_dims[e])
            for k, r in enumerate(sg.RADIUS_CLASSES):
                go, gl = b.get_grid(e, k, nx, ny)
                oo, ol = O.grid_build(scenes.env_boxes(e), *scenes.grid_origin[e], nx, ny,
                                      sg.CELL, r)
                assert np.array_equal(go, oo), f"cfg {cfgid} env {e} class {k} offsets"
                assert np.array_equal(gl.view(np.uint32), ol.view(np.uint32)), \
                    f"cfg {cfgid} env {e} class {k} layers"


def test_config1_subset_with_resets(torch_cuda):
    """Paper-scale scenes (20k-80k triangles, 128x128, 65 spheres incl. the
    held proxy), 24 envs, a short episode so auto-resets happen."""
    print("case: config 1 scenes, 24 envs x 30 steps, episode 12", flush=True)
    cfg = sg.scaled_config(1, 24, episode_len=12)
    run_trajectory(torch_cuda, cfg, 30)


def test_config1_full_batch_sampled(torch_cuda):
    """The benchmarked configuration: 1024 envs.  The oracle follows 16 of
    them for 6 steps; then one-step parity from a restored state."""
    torch = torch_cuda
    print("case: config 1, 1024 envs, 16 sampled", flush=True)
    cfg = sg.CONFIGS[1]
    sample = sorted(set(np.random.default_rng(0).choice(1024, 16, replace=False).tolist()) | {1023})
    b, ob, scenes, robot = make_pair(cfg, None, sample)
    out = b.alloc_outputs()
    for k in range(6):
        a = sg.actions(cfg, k)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        compare_step(b, ob, out, ob.step(a[sample]), label=f"step {k}")
    # one-step parity from an arbitrary restored state
    st, cnt = b.get_state()
    rng = np.random.default_rng(5)
    st[:, 3:] += rng.uniform(-0.5, 0.5, (st.shape[0], 7)).astype(np.float32)
    st[:, 3:] = np.clip(st[:, 3:], robot.qlim[:, 0], robot.qlim[:, 1])
    cnt[:, 0] = 499
    b.set_state(st, cnt)
    ob.set_state(st[sample], cnt[sample])
    a = sg.actions(cfg, 77)
    b.step(torch.from_numpy(a).cuda(), out)
    torch.cuda.synchronize()
    compare_step(b, ob, out, ob.step(a[sample]), label="restored")
    assert out["done"].cpu().numpy().all()


def test_state_roundtrip_and_reset_mask(torch_cuda):
    torch = torch_cuda
    print("case: state round trip, masked reset", flush=True)
    cfg = sg.scaled_config(0, 13)     # ragged: not a multiple of the 4 envs per block
    b, ob, scenes, robot = make_pair(cfg)
    out = b.alloc_outputs()
    for k in range(3):
        a = sg.actions(cfg, k, num_envs=13)
        b.step(torch.from_numpy(a).cuda(), out)
        ob.step(a)
    st, cnt = b.get_state()
    b.set_state(st, cnt)
    st2, cnt2 = b.get_state()
    assert np.array_equal(st.view(np.uint32), st2.view(np.uint32)) and np.array_equal(cnt, cnt2)
    mask = np.zeros(13, np.uint8)
    mask[[0, 4, 12]] = 1
    b.reset(torch.from_numpy(mask).cuda())
    ob.reset(mask)
    st3, cnt3 = b.get_state()
    assert np.array_equal(st3.view(np.uint32), ob.state.view(np.uint32))
    assert np.array_equal(cnt3, ob.counters)
    a = sg.actions(cfg, 9, num_envs=13)
    b.step(torch.from_numpy(a).cuda(), out)
    torch.cuda.synchronize()
    compare_step(b, ob, out, ob.step(a), label="after reset")


def test_degenerate_actions(torch_cuda):
    """NaN components count as zero; infinities and huge values clamp."""
    print("case: NaN / inf actions", flush=True)
    cfg = sg.scaled_config(0, 8)

    def act(k, N):
        a = sg.actions(cfg, k, num_envs=N)
        a[::2, k % 9] = np.nan
        a[1::3, (k + 4) % 9] = np.inf
        a[2::3, (k + 2) % 9] = -1e30
        return a
    run_trajectory(torch_cuda, cfg, 12, act_fn=act)


def test_mixed_resolutions_and_empty_scene(torch_cuda):
    """Per-env resolutions 64/128/256 in one batch (256 renders as four
    128x128 regions); one env with no triangles at all."""
    torch = torch_cuda
    print("case: mixed resolutions, empty env", flush=True)
    cfg = sg.scaled_config(2, 9, tri_target=(2000.0, 6000.0))
    scenes = sg.make_scene_set(cfg)
    scenes.res[:] = [64, 128, 256, 256, 64, 128, 256, 64, 128]
    # env 3: drop every triangle (and its face-plane rows, so that every other
    # env keeps the planes of its own triangles)
    t0, t1 = int(scenes.tri_offset[3]), int(scenes.tri_offset[4])
    scenes.tris = np.concatenate([scenes.tris[:t0], scenes.tris[t1:]])
    scenes.tri_rgb = np.concatenate([scenes.tri_rgb[:t0], scenes.tri_rgb[t1:]])
    scenes.tri_plane = np.concatenate([scenes.tri_plane[:t0], scenes.tri_plane[t1:]])
    scenes.tri_offset[4:] -= (t1 - t0)
    assert_triangles_on_their_planes(scenes)
    from oracle import oracle as O
    from paper_2306_07552_amd import gal
    robot = sg.make_robot_for(cfg)
    consts = sg.config_constants(cfg)
    b = gal.Batch(robot, scenes, consts)
    ob = O.OracleBatch(robot, scenes, consts)
    out = b.alloc_outputs()
    for k in range(4):
        a = sg.actions(cfg, k, num_envs=9)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        oout = ob.step(a)
        compare_step(b, ob, out, oout, label=f"step {k}")
    assert (b.env_depth(u32(out["depth"]), 3) == 0xFFFFFF).all()


def assert_triangles_on_their_planes(scenes):
    """Every triangle's vertices lie on its face plane (|n . v - w| small),
    and its winding agrees with the plane's outward normal."""
    for e in range(scenes.num_envs):
        v, t, _ = scenes.env_mesh(e)
        pl = scenes.env_planes(e).astype(np.float64)
        if t.shape[0] == 0:
            continue
        P = v.astype(np.float64)[t]                                # [T][3][3]
        dist = np.einsum("tkc,tc->tk", P, pl[:, :3]) - pl[:, 3:4]
        assert np.max(np.abs(dist)) < 1e-4, f"env {e}: triangle off its plane"
        nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        assert np.all(np.einsum("tc,tc->t", nrm, pl[:, :3]) > 0), f"env {e}: winding"


def test_without_face_planes(torch_cuda):
    """Scenes given without face planes (tri_plane NULL): back faces are
    culled by the winding of the snapped vertices alone, on both sides."""
    torch = torch_cuda
    print("case: tri_plane NULL", flush=True)
    cfg = sg.scaled_config(2, 8, tri_target=(5000.0, 40000.0))
    scenes = sg.make_scene_set(cfg)
    scenes.tri_plane = None
    from oracle import oracle as O
    from paper_2306_07552_amd import gal
    robot = sg.make_robot_for(cfg)
    consts = sg.config_constants(cfg)
    b = gal.Batch(robot, scenes, consts)
    ob = O.OracleBatch(robot, scenes, consts)
    for tuning in (dict(), dict(persistent=1, split=3, order=1, region=64, lane_max=8)):
        b.set_tuning(**tuning)
        out = b.alloc_outputs()
        for k in range(3):
            a = sg.actions(cfg, k, num_envs=8)
            b.step(torch.from_numpy(a).cuda(), out)
            torch.cuda.synchronize()
            compare_step(b, ob, out, ob.step(a), label=f"{tuning} step {k}")


def test_repeatable(torch_cuda):
    """The same inputs give the same bits on every run (no order dependence
    in the LDS z-min)."""
    torch = torch_cuda
    print("case: repeatability", flush=True)
    cfg = sg.scaled_config(1, 8)
    res = []
    for _ in range(2):
        b, _, _, _ = make_pair(cfg, oracle_envs=[])
        out = b.alloc_outputs()
        for k in range(3):
            b.step(torch.from_numpy(sg.actions(cfg, k, num_envs=8)).cuda(), out)
        torch.cuda.synchronize()
        res.append(u32(out["depth"]).copy())
    assert np.array_equal(res[0], res[1])


TUNINGS = [
    dict(block=256, region=128, lane_max=16, small_max=16, refresh=4, occlusion=0, prologue=0,
         persistent=0, robot_lanes=64),
    dict(block=512, region=64, lane_max=0, small_max=1024, refresh=16, occlusion=1, prologue=8,
         persistent=1, robot_lanes=32),
    dict(block=1024, region=32, lane_max=4096, small_max=4096, refresh=1, occlusion=1, prologue=0,
         persistent=1, robot_lanes=64),
    dict(block=512, region=128, lane_max=8, small_max=64, refresh=2, occlusion=1, prologue=64,
         persistent=0, robot_lanes=32),
    dict(block=512, region=128, lane_max=0, small_max=65536, refresh=16, occlusion=1, prologue=8,
         persistent=1, robot_lanes=64),
    # halved regions for the cheapest envs (all of them, then half)
    dict(block=256, region=64, lane_max=4, small_max=256, refresh=1, occlusion=1, prologue=256,
         persistent=1, robot_lanes=64, split=12),
    dict(block=512, region=128, lane_max=4, small_max=256, refresh=1, occlusion=1, prologue=256,
         persistent=1, robot_lanes=32, split=6),
    # queue ordered by the previous step's item times
    dict(block=512, region=128, lane_max=4, small_max=256, refresh=1, occlusion=1, prologue=128,
         persistent=1, robot_lanes=64, split=4, order=1),
    # mid-sized triangles binned per 8x8 tile in LDS
    dict(block=512, region=128, lane_max=4, small_max=256, refresh=1, occlusion=1, prologue=128,
         persistent=1, robot_lanes=64, bin=1),
    # everything but the per-lane ones binned: floors and walls over many
    # tiles, full tile lists (the overflow path draws them directly)
    dict(block=256, region=64, lane_max=0, small_max=65536, refresh=4, occlusion=1, prologue=8,
         persistent=0, robot_lanes=64, bin=1),
    dict(block=1024, region=128, lane_max=8, small_max=1024, refresh=1, occlusion=0, prologue=0,
         persistent=1, robot_lanes=32, split=4, order=1, bin=1),
    dict(block=512, region=32, lane_max=0, small_max=4096, refresh=2, occlusion=1, prologue=64,
         persistent=1, robot_lanes=64, split=12, bin=1),
]


@pytest.mark.parametrize("tuning", TUNINGS, ids=[f"t{i}" for i in range(len(TUNINGS))])
def test_tuning_invariance(torch_cuda, tuning):
    """Every launch configuration the autotuner may pick gives the oracle's bits
    (paper-scale scenes, 128x128 and 256x256)."""
    torch = torch_cuda
    print(f"case: tuning {tuning}", flush=True)
    cfg = sg.scaled_config(2, 12, tri_target=(20000.0, 80000.0))
    b, ob, scenes, robot = make_pair(cfg, oracle_envs=list(range(12)))
    b.set_tuning(**tuning)
    got = b.get_tuning()
    assert all(got[k] == v for k, v in tuning.items())
    out = b.alloc_outputs()
    for k in range(3):
        a = sg.actions(cfg, k, num_envs=12)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        compare_step(b, ob, out, ob.step(a), label=f"step {k}")


@pytest.mark.parametrize("tuning", [
    dict(block=512, region=128, lane_max=4, small_max=256, refresh=4, occlusion=0, prologue=8),
    dict(block=256, region=64, lane_max=0, small_max=64, refresh=4, occlusion=1, prologue=8),
    dict(block=512, region=128, lane_max=8, small_max=256, refresh=1, occlusion=1, prologue=256,
         persistent=1, split=5, order=1),
    dict(block=256, region=64, lane_max=0, small_max=1024, refresh=2, occlusion=1, prologue=8,
         persistent=1, bin=1),
], ids=["r128", "r64-occl", "r128-persistent-split", "r64-bin"])
def test_color_parity(torch_cuda, tuning):
    """Flat colour: the winning triangle (smallest depth, then smallest id)
    and its seeded colour, mixed scene sizes and 64/128/256 resolutions."""
    torch = torch_cuda
    print(f"case: colour {tuning}", flush=True)
    cfg = sg.scaled_config(4, 10, tri_target=(2000.0, 60000.0))
    scenes = sg.make_scene_set(cfg)
    scenes.res[:] = [128, 64, 256, 128, 128, 64, 256, 128, 64, 128]
    from oracle import oracle as O
    from paper_2306_07552_amd import gal
    robot = sg.make_robot_for(cfg)
    consts = sg.config_constants(cfg)
    b = gal.Batch(robot, scenes, consts, color=True)
    b.set_tuning(**tuning)
    ob = O.OracleBatch(robot, scenes, consts, color=True)
    out = b.alloc_outputs()
    assert "rgb" in out
    for k in range(3):
        a = sg.actions(cfg, k, num_envs=10)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        compare_step(b, ob, out, ob.step(a), label=f"step {k}")


def test_bin_lds_limit_rejected(torch_cuda):
    """With colour, a 128-pixel region's 64-bit z-buffer and the bins do not
    fit one CU's LDS: the tuning is refused and the batch keeps its own."""
    print("case: bin LDS limit", flush=True)
    from paper_2306_07552_amd import gal
    cfg = sg.scaled_config(4, 2, tri_target=(2000.0, 4000.0))
    scenes = sg.make_scene_set(cfg)
    scenes.res[:] = [128, 128]
    b = gal.Batch(sg.make_robot_for(cfg), scenes, sg.config_constants(cfg), color=True)
    before = b.get_tuning()
    with pytest.raises(gal.GalError, match="LDS"):
        b.set_tuning(region=128, bin=1)
    assert b.get_tuning() == before
    b.set_tuning(region=64, bin=1)
    assert b.get_tuning()["bin"] == 1


def test_graph_replay_matches_eager(torch_cuda):
    """The step captured as a hipGraph and replayed gives the same bits as the
    eagerly launched step, replay after replay, with eager work and
    synchronisations in between (actions refilled in place).  Both run the
    persistent queue in measured order (the queue is ordered by an extra
    workgroup of the robot-step launch, inside the graph)."""
    torch = torch_cuda
    print("case: graph replay vs eager", flush=True)
    cfg = sg.scaled_config(1, 24)
    bg, ob, scenes, robot = make_pair(cfg, oracle_envs=[0, 7, 23])
    from paper_2306_07552_amd import gal
    be = gal.Batch(robot, scenes, sg.config_constants(cfg))
    bg.set_tuning(graph=1, persistent=1, order=1)
    be.set_tuning(persistent=1, order=1)
    og, oe = bg.alloc_outputs(), be.alloc_outputs()
    act = torch.empty((24, 9), dtype=torch.float32, device="cuda")
    for k in range(6):
        a = sg.actions(cfg, k, num_envs=24)
        act.copy_(torch.from_numpy(a))
        bg.step(act, og)            # graph (captured on the first call)
        be.step(act, oe)            # eager
        junk = torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for key in ("depth", "contact_static", "contact_object", "state", "counters", "frames"):
            assert torch.equal(og[key], oe[key]), f"replay {k}: {key} differs"
        compare_step(bg, ob, og, ob.step(a[ob.envs]), label=f"graph step {k}")


def test_uneven_batch_persistent_graph(torch_cuda):
    """Uneven batching: log-uniform 2k-200k triangles and 64/128/256
    resolutions in one persistent queue kernel, captured as a graph."""
    torch = torch_cuda
    print("case: uneven batch, persistent + graph", flush=True)
    cfg = sg.scaled_config(2, 40)
    sample = [0, 3, 17, 39]
    b, ob, scenes, robot = make_pair(cfg, oracle_envs=sample)
    assert len(set(scenes.res.tolist())) > 1
    b.set_tuning(persistent=1, graph=1, region=64, order=1)
    out = b.alloc_outputs()
    act = torch.empty((40, 9), dtype=torch.float32, device="cuda")
    for k in range(4):
        a = sg.actions(cfg, k, num_envs=40)
        act.copy_(torch.from_numpy(a))
        b.step(act, out)
        torch.cuda.synchronize()
        compare_step(b, ob, out, ob.step(a[sample]), label=f"step {k}")


def test_autotune_restores_state_and_keeps_bits(torch_cuda):
    torch = torch_cuda
    print("case: autotune", flush=True)
    cfg = sg.scaled_config(1, 16)
    b, ob, scenes, robot = make_pair(cfg, oracle_envs=list(range(16)))
    out = b.alloc_outputs()
    a0 = torch.from_numpy(sg.actions(cfg, 0, num_envs=16)).cuda()
    st0, cnt0 = b.get_state()
    best, ms = b.autotune(a0, out, steps=1)
    assert ms > 0 and best["block"] in (256, 512, 1024)
    st1, cnt1 = b.get_state()
    assert np.array_equal(st0.view(np.uint32), st1.view(np.uint32)) and np.array_equal(cnt0, cnt1)
    for k in range(3):
        a = sg.actions(cfg, k, num_envs=16)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        compare_step(b, ob, out, ob.step(a), label=f"tuned step {k}")
