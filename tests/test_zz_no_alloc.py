"""gal_mlp_forward_static, the allocation-free surrogate inference (scratch in
the library's fixed device array), against gal_mlp_forward (scratch in the
MLP object): the same logits bit for bit on two calls in a row, the second
with fewer rows, and its argument checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def bf16_rows(rng, rows):
    """Inputs shaped like the surrogate's: 64 scalars in [-1, 1], then 0/1
    occupancy values; BF16 bits as int16."""
    f = np.empty((rows, 2112), np.float32)
    f[:, :64] = rng.uniform(-1.0, 1.0, size=(rows, 64))
    f[:, 64:] = rng.integers(0, 2, size=(rows, 2048))
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def test_forward_static_matches_forward():
    import torch
    from paper_2306_07552_amd import gal
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    rng = np.random.default_rng(4)
    mlp = gal.Mlp(max_rows=4096, seed=9)
    for rows in (3000, 700):
        print(f"case: forward_static vs forward, {rows} rows", flush=True)
        x = torch.from_numpy(bf16_rows(rng, rows)).cuda()
        z_ref = torch.full((rows,), np.nan, dtype=torch.float32, device="cuda")
        z = torch.full((rows,), np.nan, dtype=torch.float32, device="cuda")
        mlp.forward(x, z_ref)
        mlp.forward_static(x, z)
        torch.cuda.synchronize()
        assert torch.isfinite(z_ref).all()
        assert torch.equal(z, z_ref), f"{rows} rows: {(z != z_ref).sum().item()} logits differ"
    # argument checks: rejected on the host before any launch
    x = torch.zeros((8, 2112), dtype=torch.int16, device="cuda")
    z = torch.zeros(8, dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        mlp.forward_static(x, z, rows=(1 << 22) + 1)
    with pytest.raises(RuntimeError):
        mlp.forward_static(x, z, rows=-1)
