"""Pins of the surrogate-MLP oracle: central finite differences (exact FP64
mode), a network constructed to compute a closed form, the logistic loss at
a known logit, BF16 rounding ties and the first Adam step."""
import numpy as np
import pytest

from oracle import oracle_mlp as M


def rand_net(rng, dims):
    W = [rng.normal(0, 1.0 / np.sqrt(dims[l]), (dims[l + 1], dims[l])) for l in range(5)]
    b = [rng.normal(0, 0.1, dims[l + 1]) for l in range(5)]
    return W, b


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_central_differences(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    dims = [7, 6, 5, 5, 4, 1]
    W, b = rand_net(rng, dims)
    x = rng.normal(0, 1, (9, dims[0]))
    y = (rng.uniform(size=9) < 0.4).astype(np.float64)
    pw = 3.0
    net = M.OracleMLP(W, b)
    loss, dW, db = net.backward(x, y, pw, round_bf16=False)
    assert abs(loss - net.loss(x, y, pw, round_bf16=False)) < 1e-12
    h = 1e-6
    for l in range(5):
        num = np.zeros_like(W[l])
        for idx in np.ndindex(W[l].shape):
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            num[idx] = (M.OracleMLP(Wp, b).loss(x, y, pw, False)
                        - M.OracleMLP(Wm, b).loss(x, y, pw, False)) / (2 * h)
        assert rel(dW[l], num) <= 1e-6
        numb = np.zeros_like(b[l])
        for j in range(b[l].size):
            bp = [v.copy() for v in b]
            bm = [v.copy() for v in b]
            bp[l][j] += h
            bm[l][j] -= h
            numb[j] = (M.OracleMLP(W, bp).loss(x, y, pw, False)
                       - M.OracleMLP(W, bm).loss(x, y, pw, False)) / (2 * h)
        assert rel(db[l], numb) <= 1e-6


def test_forward_closed_form_sum_of_abs(oracle_lib):
    """W1 = [I; -I], identities, W5 = ones: the logit is sum_k |x_k|."""
    d = 5
    W = [np.vstack([np.eye(d), -np.eye(d)]), np.eye(2 * d), np.eye(2 * d), np.eye(2 * d),
         np.ones((1, 2 * d))]
    b = [np.zeros(2 * d)] * 4 + [np.zeros(1)]
    rng = np.random.default_rng(1)
    x = rng.normal(0, 2, (20, d))
    z = M.OracleMLP(W, b).forward(x, round_bf16=False)
    assert np.allclose(z, np.abs(x).sum(1), rtol=0, atol=1e-12)
    # with BF16 rounding, inputs that are BF16 values and sums that stay exact
    xb = np.round(x * 4) / 4
    zb = M.OracleMLP(W, b).forward(xb, round_bf16=True)
    assert np.array_equal(zb, np.abs(xb).sum(1))


def test_loss_at_zero_logit(oracle_lib):
    d = 4
    W = [np.zeros((3, d)), np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((1, 3))]
    b = [np.zeros(3)] * 4 + [np.zeros(1)]
    y = np.array([1, 0, 1, 0, 0.0])
    loss = M.OracleMLP(W, b).loss(np.ones((5, d)), y, pos_weight=4.0)
    assert abs(loss - np.log(2) * (4 + 1 + 4 + 1 + 1) / 5) < 1e-15


def test_bf16_rounding(oracle_lib):
    L = M._lib()
    assert L.o_bf16_round(1.0 / 3.0) == 0.333984375
    assert L.o_bf16_round(1.0 + 2 ** -8) == 1.0                 # tie -> even
    assert L.o_bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even
    assert L.o_bf16_round(-2.5) == -2.5
    v = np.array([1 / 3, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -7.77, 1e-3], np.float32)
    assert np.array_equal(M.bf16_round_f32(v).astype(np.float64),
                          np.array([L.o_bf16_round(float(t)) for t in v]))


def test_adam_first_step(oracle_lib):
    rng = np.random.default_rng(2)
    g = rng.normal(0, 1, 50)
    w0 = rng.normal(0, 1, 50)
    w, m, v = M.adam(w0.copy(), np.zeros(50), np.zeros(50), g, 1e-3, 0.9, 0.999, 1e-8, 1)
    # bias-corrected moments are g and g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(w, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
