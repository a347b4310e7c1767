"""Pins of the policy oracle (the network that consumes the depth stack,
Section 4.2; the SimpleCNN encoder's kernel sizes and strides from the
appendix on model sizes): the convolution against a brute-force loop and a
one-pixel input, the shape chain, the input scaling, the feature order of the
fully connected layer, the heads' linearity and the Gaussian log-density."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle_policy as OP


def brute_conv(x, w, b, s):
    N, H, W, C = x.shape
    O, k = w.shape[0], w.shape[1]
    oh, ow = (H - k) // s + 1, (W - k) // s + 1
    out = np.zeros((N, oh, ow, O))
    for n in range(N):
        for y in range(oh):
            for xx in range(ow):
                for o in range(O):
                    acc = b[o]
                    for i in range(k):
                        for j in range(k):
                            for c in range(C):
                                acc += w[o, i, j, c] * x[n, s * y + i, s * xx + j, c]
                    out[n, y, xx, o] = acc
    return out


@pytest.mark.parametrize("k,s", [(3, 1), (4, 2), (8, 4)])
def test_conv_matches_brute_force(k, s):
    rng = np.random.default_rng(k * 10 + s)
    x = rng.normal(size=(2, 17, 13, 3))
    w = rng.normal(size=(4, k, k, 3))
    b = rng.normal(size=4)
    assert np.allclose(OP.conv2d(x, w, b, s), brute_conv(x, w, b, s), rtol=1e-12, atol=1e-12)


def test_conv_of_one_pixel_reads_the_kernel_unflipped():
    """out[y][x] = sum_ij w[i][j] in[s y + i][s x + j]: a single lit pixel at
    (p, q) shows w[p - s y][q - s x] (cross-correlation, no flip)."""
    s, k = 2, 4
    x = np.zeros((1, 12, 12, 1))
    p, q = 5, 6
    x[0, p, q, 0] = 1.0
    w = np.arange(k * k, dtype=np.float64).reshape(1, k, k, 1) + 1.0
    out = OP.conv2d(x, w, np.zeros(1), s)[0, :, :, 0]
    for y in range(out.shape[0]):
        for xx in range(out.shape[1]):
            i, j = p - s * y, q - s * xx
            want = w[0, i, j, 0] if (0 <= i < k and 0 <= j < k) else 0.0
            assert out[y, xx] == want


def test_shape_chain_and_parameter_count():
    n = OP.RES
    sizes = []
    for (o, k, s, c) in OP.CONV:
        n = OP.out_size(n, k, s)
        sizes.append(n)
    assert sizes == [31, 14, 12]
    lay = dict(OP.layout(9))
    assert lay["fc.w"] == (512, 12 * 12 * 32)
    total = sum(int(np.prod(v)) for v in lay.values())
    enc = 32 * 64 + 32 + 64 * 16 * 32 + 64 + 32 * 9 * 64 + 32 + 4608 * 512 + 512
    assert total == enc + 9 * 519 + 9 + 519 + 1 + 9


def test_depth_input_scaling():
    d = np.array([[0, 1, 8388608, 16777215, 0xFFFFFFFF]], np.uint32).reshape(1, 1, 5)
    x = OP.depth_input(d)[0, 0, :, 0]
    assert x[0] == 0.0 and x[3] == 1.0 and x[4] == 1.0
    assert abs(x[2] - 0.5) < 2 ** -8 and 0 < x[1] < 1e-6
    assert np.all(np.diff(x) >= 0)


def test_fc_feature_order():
    """The fully connected layer reads the 12 x 12 x 32 map in (y, x, c) order."""
    rng = np.random.default_rng(3)
    theta = np.zeros(sum(int(np.prod(s)) for _, s in OP.layout(9)), np.float32)
    P = OP.unpack(theta, 9)
    h3 = OP.bf16(rng.uniform(0, 1, size=(1, 12, 12, 32)).astype(np.float32))
    y, x, c = 7, 2, 19
    P["fc.w"][0, (y * 12 + x) * 32 + c] = 1.0
    out = OP.encoder_layer(3, h3, P)
    assert out[0, 0] == h3[0, y, x, c]


def test_heads_linear_and_gaussian_logp():
    rng = np.random.default_rng(5)
    A = 9
    theta = rng.normal(size=sum(int(np.prod(s)) for _, s in OP.layout(A))).astype(np.float32)
    P = OP.unpack(theta, A)
    h = OP.bf16(rng.uniform(0, 1, size=(3, 512)).astype(np.float32))
    q = rng.normal(size=(3, 7)).astype(np.float32)
    mean, value = OP.heads(h, q, P)
    f = np.concatenate([h, q.astype(np.float64)], axis=1)
    for n in range(3):
        for a in range(A):
            want = sum(float(P["actor.w"][a, k]) * f[n, k] for k in range(519)) + float(P["actor.b"][a])
            assert abs(mean[n, a] - want) <= 1e-9 * (1 + abs(want))
    noise = rng.normal(size=(3, A))
    act, logp = OP.sample(mean, P["log_std"], noise)
    std = np.exp(P["log_std"].astype(np.float64))
    ref = stats.norm.logpdf(act, loc=mean, scale=std).sum(axis=1)
    assert np.allclose(logp, ref, rtol=1e-12, atol=1e-10)


def test_gae_closed_form_and_done_cut():
    """GAE with lam = 1 is the discounted return minus V; with lam = 0 the
    one-step TD error; an episode end cuts both."""
    rng = np.random.default_rng(8)
    T, N = 6, 3
    r = rng.normal(size=(T, N))
    v = rng.normal(size=(T, N))
    last = rng.normal(size=N)
    d = np.zeros((T, N))
    g = 0.9
    adv, ret = OP.gae(r, v, d, last, g, 1.0)
    for n in range(N):
        for t in range(T):
            disc = sum(g ** (k - t) * r[k, n] for k in range(t, T)) + g ** (T - t) * last[n]
            assert abs(ret[t, n] - disc) < 1e-12
    adv0, _ = OP.gae(r, v, d, last, g, 0.0)
    nxt = np.vstack([v[1:], last[None]])
    assert np.allclose(adv0, r + g * nxt - v)
    d[2, 1] = 1.0
    adv1, ret1 = OP.gae(r, v, d, last, g, 1.0)
    assert abs(ret1[2, 1] - r[2, 1]) < 1e-12          # nothing flows back across the episode end
    assert abs(ret1[1, 1] - (r[1, 1] + g * r[2, 1])) < 1e-12


def test_conv_backward_is_the_adjoint():
    """<conv(x), dy> = <x, conv_dx(dy)> and the weight gradient is the
    derivative of <conv(x; w), dy> in w (checked by central differences)."""
    rng = np.random.default_rng(9)
    for k, s in ((8, 4), (4, 2), (3, 1)):
        x = rng.normal(size=(2, 20, 20, 3))
        w = rng.normal(size=(4, k, k, 3))
        y = OP.conv2d(x, w, np.zeros(4), s)
        dy = rng.normal(size=y.shape)
        dx = OP.conv_dx(dy, w, s, x.shape)
        assert abs(np.sum(y * dy) - np.sum(x * dx)) < 1e-9 * (1 + abs(np.sum(y * dy)))
        dw = OP.conv_dw(x, dy, k, s)
        idx = (1, k - 1, 0, 2)
        e = np.zeros_like(w)
        e[idx] = 1e-6
        num = (np.sum(OP.conv2d(x, w + e, np.zeros(4), s) * dy) - np.sum(OP.conv2d(x, w - e, np.zeros(4), s) * dy)) / 2e-6
        assert abs(num - dw[idx]) < 1e-5 * (1 + abs(num))


def test_ppo_gradient_vs_central_differences():
    """The PPO loss's gradient for the heads and log_std against central
    differences of the same loss (the encoder's BF16 rounding points make
    its own gradients step-wise; they are checked by the device parity)."""
    rng = np.random.default_rng(10)
    A, S = 4, 5
    theta = (rng.normal(size=sum(int(np.prod(s)) for _, s in OP.layout(A))) * 0.05).astype(np.float32)
    depth = rng.integers(0, 2 ** 24, size=(S, 128, 128)).astype(np.uint32)
    state = rng.normal(size=(S, 10)).astype(np.float32)
    acts = rng.normal(size=(S, A))
    old = rng.normal(size=S) - 4.0
    adv = rng.normal(size=S)
    ret = rng.normal(size=S)
    args = (depth, state, acts, old, adv, ret)
    res = OP.ppo_loss_and_grads(*args, theta, A, 0.2, 0.5, 0.01)
    off = {}
    o = 0
    for name, shp in OP.layout(A):
        off[name] = o
        o += int(np.prod(shp))
    for name, k in (("actor.w", 7), ("actor.b", 1), ("critic.w", 515), ("critic.b", 0), ("log_std", 2)):
        i = off[name] + k
        t1, t2 = theta.astype(np.float64).copy(), theta.astype(np.float64).copy()
        h = 1e-3
        t1[i] += h
        t2[i] -= h
        l1 = OP.ppo_loss_and_grads(*args, t1.astype(np.float32), A, 0.2, 0.5, 0.01)["loss"]
        l2 = OP.ppo_loss_and_grads(*args, t2.astype(np.float32), A, 0.2, 0.5, 0.01)["loss"]
        # theta is stored in FP32: use the actually-applied step
        step = float(np.float32(t1[i])) - float(np.float32(t2[i]))
        num = (l1 - l2) / step
        assert abs(num - res["grad"][i]) < 2e-3 * (1 + abs(num)), (name, num, res["grad"][i])


def test_ppo_encoder_gradient_vs_central_differences():
    """With the BF16 rounding points switched off (the plain FP64 definition),
    the whole gradient chain through the fully connected layer and the three
    convolutions (their ReLU masks included) against central differences."""
    rng = np.random.default_rng(12)
    A, S = 3, 3
    theta = (rng.normal(size=sum(int(np.prod(s)) for _, s in OP.layout(A))) * 0.05).astype(np.float64)
    depth = rng.integers(0, 2 ** 24, size=(S, 128, 128)).astype(np.uint32)
    state = rng.normal(size=(S, 10)).astype(np.float32)
    acts = rng.normal(size=(S, A))
    old = rng.normal(size=S) - 6.0
    adv = rng.normal(size=S)
    ret = rng.normal(size=S)
    off, o = {}, 0
    for name, shp in OP.layout(A):
        off[name] = o
        o += int(np.prod(shp))
    OP.ROUND = False
    try:
        def run(t):
            return OP.ppo_loss_and_grads(depth, state, acts, old, adv, ret, t, A, 0.2, 0.5, 0.01)
        # unpack keeps float32 parameters: differentiate in the FP32-representable
        # neighbourhood with a step that survives the cast
        res = run(theta.astype(np.float32))
        for name, k in (("conv1.w", 37), ("conv2.w", 1000), ("conv3.w", 77), ("conv2.b", 5), ("fc.w", 12345)):
            i = off[name] + k
            base = theta.astype(np.float32).astype(np.float64)
            h = 1e-2 * max(abs(base[i]), 1e-2)
            t1, t2 = base.copy(), base.copy()
            t1[i] += h
            t2[i] -= h
            step = float(np.float32(t1[i])) - float(np.float32(t2[i]))
            num = (run(t1.astype(np.float32))["loss"] - run(t2.astype(np.float32))["loss"]) / step
            g = res["grad"][i]
            assert abs(num - g) < 5e-3 * (abs(num) + abs(g)) + 1e-9, (name, num, g)
    finally:
        OP.ROUND = True
