"""GPU parity of the policy's PPO update (Section 4.2 trains with DD-PPO; one
GPU's step) against the FP64 oracle: GAE, the loss statistics and the whole
parameter gradient (heads, fully connected layer, the three convolutions),
with clipped and unclipped samples; Adam steps that lower the loss."""
import numpy as np
import pytest

from paper_2306_07552_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_gae_matches_oracle(torch_cuda):
    torch = torch_cuda
    print("case: gae", flush=True)
    from oracle import oracle_policy as OP
    from paper_2306_07552_amd import gal
    rng = np.random.default_rng(1)
    T, N = 16, 300
    r = rng.normal(size=(T, N)).astype(np.float32)
    v = rng.normal(size=(T, N)).astype(np.float32)
    d = (rng.uniform(size=(T, N)) < 0.1).astype(np.uint8)
    last = rng.normal(size=N).astype(np.float32)
    adv = torch.empty((T, N), device="cuda")
    ret = torch.empty((T, N), device="cuda")
    gal.gae(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda(), torch.from_numpy(d).cuda(),
            torch.from_numpy(last).cuda(), 0.99, 0.95, adv, ret)
    torch.cuda.synchronize()
    a_ref, r_ref = OP.gae(r, v, d, last, 0.99, 0.95)
    scale = 1 + np.abs(a_ref)
    assert np.all(np.abs(adv.cpu().numpy() - a_ref) <= 1e-5 * T * scale)
    assert np.all(np.abs(ret.cpu().numpy() - r_ref) <= 1e-5 * T * (1 + np.abs(r_ref)))


def rollout_samples(torch, n, seed):
    from paper_2306_07552_amd import gal
    cfg = sg.scaled_config(1, n)
    b = gal.Batch(sg.make_robot_for(cfg), sg.make_scene_set(cfg), sg.config_constants(cfg))
    out = b.alloc_outputs()
    for k in range(2):
        b.step(torch.from_numpy(sg.actions(cfg, k)).cuda(), out)
    torch.cuda.synchronize()
    dflat = out["depth"].cpu().numpy().view(np.uint32)
    depth = np.stack([b.env_depth(dflat, e) for e in range(n)])
    return out, depth


def ppo_case(torch, S, seed):
    """Samples with ratios on both sides of the clip range and advantages of
    both signs; returns the GPU gradient, stats and the oracle's result."""
    from oracle import oracle_policy as OP
    from paper_2306_07552_amd import gal
    out, depth = rollout_samples(torch, S, seed)
    A = 9
    pol = gal.Policy(S, act_dim=A, seed=seed)
    theta = pol.get_weights()
    rng = np.random.default_rng(seed)
    lay = OP.layout(A)
    off = 0
    for name, shp in lay:
        n = int(np.prod(shp))
        if name.startswith(("actor", "critic")):
            theta[off:off + n] = rng.normal(scale=0.05, size=n)
        off += n
    pol.set_weights(theta)
    noise = torch.from_numpy(rng.normal(size=(S, A)).astype(np.float32)).cuda()
    act = torch.empty((S, A), device="cuda")
    lp = torch.empty(S, device="cuda")
    pol.act(out["depth"], out["state"], act, noise=noise, logp=lp)
    torch.cuda.synchronize()
    # behaviour log-densities that put the ratio at 0.7, 0.9, 1.1 or 1.3
    ratio = np.array([0.7, 0.9, 1.1, 1.3])[np.arange(S) % 4]
    old = (lp.cpu().numpy().astype(np.float64) - np.log(ratio)).astype(np.float32)
    adv = rng.normal(size=S).astype(np.float32)
    adv[np.arange(S) % 8 < 4] = np.abs(adv[np.arange(S) % 8 < 4])
    adv[np.arange(S) % 8 >= 4] = -np.abs(adv[np.arange(S) % 8 >= 4])
    ret = rng.normal(size=S).astype(np.float32)
    grads = torch.empty(pol.num_params, device="cuda")
    stats = torch.empty(4, device="cuda")
    pol.ppo_gradients(out["depth"], out["state"], act, torch.from_numpy(old).cuda(), torch.from_numpy(adv).cuda(),
                      torch.from_numpy(ret).cuda(), 0.2, 0.5, 0.01, grads=grads, stats=stats)
    torch.cuda.synchronize()
    ref = OP.ppo_loss_and_grads(depth, out["state"].cpu().numpy(), act.cpu().numpy().astype(np.float64), old, adv,
                                ret, theta, A, 0.2, 0.5, 0.01)
    return pol, grads.cpu().numpy().astype(np.float64), stats.cpu().numpy(), ref, (out, act, old, adv, ret)


@pytest.mark.parametrize("S", [16, 96])
def test_ppo_gradients_match_oracle(torch_cuda, S):
    """Every parameter tensor's gradient within 1e-2 relative L2 (BF16
    pre-activation gradients, FP32 weight gradients; the oracle follows its
    own BF16 chain), the loss statistics within 1e-4."""
    torch = torch_cuda
    print(f"case: ppo gradients S={S}", flush=True)
    from oracle import oracle_policy as OP
    pol, g, st, ref, _ = ppo_case(torch, S, 20 + S)
    off = 0
    worst = {}
    for name, shp in OP.layout(9):
        n = int(np.prod(shp))
        a, b = g[off:off + n], ref["grad"][off:off + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        worst[name] = rel
        assert rel <= 1e-2, (name, rel, worst)
        off += n
    print(f"relative L2 per tensor: { {k: round(v, 5) for k, v in worst.items()} }", flush=True)
    assert abs(st[0] - ref["loss_pi"]) <= 1e-4 * (1 + abs(ref["loss_pi"]))
    assert abs(st[1] - ref["loss_v"]) <= 1e-4 * (1 + abs(ref["loss_v"]))
    assert abs(st[2] - ref["entropy"]) <= 1e-5 * (1 + abs(ref["entropy"]))
    assert abs(st[3] - np.mean(ref["ratio"])) <= 1e-4


def test_adam_steps_lower_the_loss(torch_cuda):
    """Small Adam steps (the update kernel is the surrogate's, checked against
    the oracle's Adam there) on one minibatch lower its PPO loss, and the
    parameters stay finite."""
    torch = torch_cuda
    print("case: ppo adam steps", flush=True)
    pol, g, st, ref, (out, act, old, adv, ret) = ppo_case(torch, 32, 77)
    old_t, adv_t, ret_t = (torch.from_numpy(x).cuda() for x in (old, adv, ret))
    stats = torch.empty(4, device="cuda")
    losses = []
    for k in range(10):
        pol.ppo_gradients(out["depth"], out["state"], act, old_t, adv_t, ret_t, stats=stats)
        pol.adam_step(1e-5)
        torch.cuda.synchronize()
        s = stats.cpu().numpy()
        losses.append(float(s[0] + 0.5 * s[1] - 0.01 * s[2]))
    print(f"PPO loss over 10 Adam steps: {[round(x, 6) for x in losses]}", flush=True)
    assert losses[-1] < losses[0]
    w = pol.get_weights()
    assert np.all(np.isfinite(w))
