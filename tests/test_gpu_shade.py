"""GPU parity of the lit, textured colour (the RGB half of Section 4.1's RGBD
observation with a light and a texture standing in for the paper's baked
ones): every pixel's colour bit for bit against the oracle, through the C ABI,
for scene faces, moving objects and robot links."""
import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg
from parity_util import compare_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def shade_pair(cfg, links=True):
    from oracle import oracle as O
    from paper_2306_07552_amd import gal
    scenes = sg.make_scene_set(cfg)
    robot = sg.make_robot_for(cfg)
    consts = sg.config_constants(cfg)
    consts["shade"] = True
    if links:
        consts["links"] = True
    b = gal.Batch(robot, scenes, consts, color=True)
    ob = O.OracleBatch(robot, scenes, consts, color=True)
    return b, ob


@pytest.mark.parametrize("region,bin_", [(128, 0), (64, 0), (64, 1)])
def test_shade_parity_scenes_and_links(torch_cuda, region, bin_):
    """8 paper-scale scenes at 128x128 with links: lit, textured colour
    bit-exact, with both checker shades and lit and unlit faces present
    (also with the 8x8-tile binned raster, which with colour fits LDS at
    64^2 regions)."""
    torch = torch_cuda
    print(f"case: shade parity region={region} bin={bin_}", flush=True)
    cfg = sg.scaled_config(1, 8)
    b, ob = shade_pair(cfg)
    b.set_tuning(region=region, persistent=1 if region == 128 else 0, bin=bin_)
    out = b.alloc_outputs()
    for k in range(6):
        a = sg.actions(cfg, k) * 3.0
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        oout = ob.step(a)
        compare_step(b, ob, out, oout, f"shade step {k}")
    img = oout["rgb"][0].reshape(-1, 3).astype(np.int64)
    assert len(np.unique(img, axis=0)) > 50


def test_shade_parity_manipulation(torch_cuda):
    """The manipulation workload (objects moving, links drawn) with lit,
    textured colour: bit-exact while objects are grasped and carried."""
    torch = torch_cuda
    print("case: shade parity manipulation", flush=True)
    cfg = sg.scaled_config(5, 8, tri_target=None)
    b, ob = shade_pair(cfg)
    out = b.alloc_outputs()
    for k in range(20):
        a = sg.actions(cfg, k)
        b.step(torch.from_numpy(a).cuda(), out)
        torch.cuda.synchronize()
        oout = ob.step(a)
        compare_step(b, ob, out, oout, f"shade manip step {k}")


def test_shade_needs_planes(torch_cuda):
    """GAL_SHADE without face planes is rejected at create."""
    from paper_2306_07552_amd import gal
    cfg = sg.scaled_config(0, 2)
    scenes = sg.make_scene_set(cfg)
    scenes.tri_plane = None
    consts = sg.config_constants(cfg)
    consts["shade"] = True
    with pytest.raises(gal.GalError):
        gal.Batch(sg.make_robot_for(cfg), scenes, consts, color=True)
