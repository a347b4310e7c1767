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
