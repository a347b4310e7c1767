"""CPU oracle of the batched policy network -- TEST INFRASTRUCTURE ONLY.

The policy that consumes the depth stack (Section 4.2 "Approach: End-to-End
RL"; the SimpleCNN visual encoder of the appendix on model sizes): three
convolutions without padding or dilation, 8x8 stride 4, 4x4 stride 2, 3x3
stride 1 (32, 64 and 32 channels), each followed by ReLU, then a fully
connected layer to 512 with ReLU; the actor's Gaussian mean and the critic's
value are linear in [the 512 features, the 7 joint angles].  Written in FP64
with numpy, as definitions: a convolution is the sum over its window of
weight x input (cross-correlation, as the encoder is usually written), a fully
connected layer a matrix product.  Where the device keeps BF16 activations
(every ReLU output) the oracle rounds the same values to BF16, so that each
layer can be checked from the device's own input to it.

Parameter vector (FP32, in this order): conv1 W [32][8][8][1], b [32];
conv2 W [64][4][4][32], b [64]; conv3 W [32][3][3][64], b [32]; fc W [512][4608]
(input index (y * 12 + x) * 32 + c), b [512]; actor W [A][519], b [A];
critic W [519], b [1]; log_std [A].  Input: depth D24 of a 128 x 128 image,
x = D / (2^24 - 1) (no hit: 1).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

from .oracle_mlp import bf16_round_f32

CONV = ((32, 8, 4, 1), (64, 4, 2, 32), (32, 3, 1, 64))   # out, kernel, stride, in
FEAT = 512
PROPRIO = 7
RES = 128


def out_size(n: int, k: int, s: int) -> int:
    return (n - k) // s + 1


def layout(act_dim: int):
    """[(name, shape)] of the parameter vector."""
    shapes = []
    for i, (o, k, s, c) in enumerate(CONV):
        shapes += [(f"conv{i + 1}.w", (o, k, k, c)), (f"conv{i + 1}.b", (o,))]
    n = RES
    for (o, k, s, c) in CONV:
        n = out_size(n, k, s)
    flat = n * n * CONV[-1][0]
    shapes += [("fc.w", (FEAT, flat)), ("fc.b", (FEAT,)),
               ("actor.w", (act_dim, FEAT + PROPRIO)), ("actor.b", (act_dim,)),
               ("critic.w", (FEAT + PROPRIO,)), ("critic.b", (1,)), ("log_std", (act_dim,))]
    return shapes


def unpack(theta: np.ndarray, act_dim: int) -> dict:
    out, i = {}, 0
    for name, shp in layout(act_dim):
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[i:i + n], np.float32).reshape(shp)
        i += n
    assert i == theta.size, (i, theta.size)
    return out


# BF16 rounding at the device's rounding points (off only in the pins that
# differentiate the FP64 definition numerically)
ROUND = True


def bf16(a) -> np.ndarray:
    if not ROUND:
        return np.asarray(a, np.float64)
    return bf16_round_f32(np.asarray(a, np.float32)).astype(np.float64)


def depth_input(depth: np.ndarray) -> np.ndarray:
    """[N][128][128][1] BF16 values of x = D / (2^24 - 1), D in FP32 as the device divides."""
    d = np.minimum(np.asarray(depth, np.uint64), 16777215).astype(np.float32)
    x = (d / np.float32(16777215.0)).astype(np.float32)
    return bf16(x)[..., None]


def conv2d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """Valid cross-correlation, NHWC input, w [O][k][k][C]: FP64 sums over the window."""
    k = w.shape[1]
    win = sliding_window_view(x, (k, k), axis=(1, 2))[:, ::stride, ::stride]   # N, OH, OW, C, k, k
    return np.einsum("nhwcij,oijc->nhwo", win, np.asarray(w, np.float64), optimize=True) + b


def relu_bf16(v: np.ndarray) -> np.ndarray:
    return bf16(np.maximum(v, 0.0))


def encoder_layer(i: int, x: np.ndarray, P: dict) -> np.ndarray:
    """Layer i (0..2 conv, 3 fc) from its BF16 input; BF16 output."""
    if i < 3:
        o, k, s, c = CONV[i]
        return relu_bf16(conv2d(x, bf16(P[f"conv{i + 1}.w"]), P[f"conv{i + 1}.b"].astype(np.float64), s))
    flat = x.reshape(x.shape[0], -1)
    return relu_bf16(flat @ bf16(P["fc.w"]).T + P["fc.b"].astype(np.float64))


def encoder_layer_pre(i: int, x: np.ndarray, P: dict) -> np.ndarray:
    """Layer i's FP64 pre-activation (before ReLU and rounding) from its BF16 input."""
    if i < 3:
        o, k, s, c = CONV[i]
        return conv2d(x, bf16(P[f"conv{i + 1}.w"]), P[f"conv{i + 1}.b"].astype(np.float64), s)
    return x.reshape(x.shape[0], -1) @ bf16(P["fc.w"]).T + P["fc.b"].astype(np.float64)


def encoder_layer_abs(i: int, x: np.ndarray, P: dict) -> np.ndarray:
    """Sum of |terms| of layer i's pre-activation (the scale of its rounding error)."""
    if i < 3:
        o, k, s, c = CONV[i]
        return conv2d(np.abs(x), np.abs(bf16(P[f"conv{i + 1}.w"])), np.abs(P[f"conv{i + 1}.b"].astype(np.float64)), s)
    return np.abs(x.reshape(x.shape[0], -1)) @ np.abs(bf16(P["fc.w"])).T + np.abs(P["fc.b"].astype(np.float64))


def heads(h: np.ndarray, q: np.ndarray, P: dict):
    """(mean [N][A], value [N]) in FP64 from the 512 BF16 features and the joint angles."""
    f = np.concatenate([np.asarray(h, np.float64), np.asarray(q, np.float32).astype(np.float64)], axis=1)
    mean = f @ P["actor.w"].astype(np.float64).T + P["actor.b"].astype(np.float64)
    value = f @ P["critic.w"].astype(np.float64) + float(P["critic.b"][0])
    return mean, value


def forward(depth: np.ndarray, state: np.ndarray, theta: np.ndarray, act_dim: int) -> dict:
    """Every layer of the policy on N images (the oracle's own chain)."""
    P = unpack(theta, act_dim)
    acts = [depth_input(depth)]
    for i in range(4):
        acts.append(encoder_layer(i, acts[-1], P))
    mean, value = heads(acts[4], np.asarray(state)[:, 3:10], P)
    return dict(x=acts[0], h1=acts[1], h2=acts[2], h3=acts[3], h4=acts[4], mean=mean, value=value)


def sample(mean: np.ndarray, log_std: np.ndarray, noise: np.ndarray):
    """Gaussian action a = mean + exp(log_std) noise and its log-density (FP64)."""
    ls = np.asarray(log_std, np.float64)
    n = np.asarray(noise, np.float64)
    a = mean + np.exp(ls) * n
    logp = np.sum(-0.5 * n * n - ls, axis=1) - 0.5 * np.log(2 * np.pi) * n.shape[1]
    return a, logp


# ----------------------------------------------------------------------------
# PPO update (the learning half of Section 4.2's training: DD-PPO, i.e. PPO on
# each GPU with the gradients all-reduced; one GPU here)
# ----------------------------------------------------------------------------
def gae(rewards, values, dones, last_value, gamma, lam):
    """Generalised advantage estimation over a rollout [T][N] (FP64, by the
    recursion's definition): delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t,
    A_t = delta_t + gamma lam (1 - d_t) A_{t+1}; returns = A + V.  d_t = 1
    when step t ended its episode (its successor is a new episode)."""
    r = np.asarray(rewards, np.float64)
    v = np.asarray(values, np.float64)
    d = np.asarray(dones, np.float64)
    T = r.shape[0]
    adv = np.zeros_like(r)
    nxt_v = np.asarray(last_value, np.float64)
    nxt_a = np.zeros(r.shape[1])
    for t in range(T - 1, -1, -1):
        live = 1.0 - d[t]
        delta = r[t] + gamma * nxt_v * live - v[t]
        nxt_a = delta + gamma * lam * live * nxt_a
        adv[t] = nxt_a
        nxt_v = v[t]
    return adv, adv + v


def conv_dw(x, dy, k, s):
    """dW[o][i][j][c] = sum over (n, y, x) of dy[n, y, x, o] x[n, s y + i, s x + j, c]."""
    win = sliding_window_view(x, (k, k), axis=(1, 2))[:, ::s, ::s]        # N, OH, OW, C, k, k
    return np.einsum("nhwcij,nhwo->oijc", win, dy, optimize=True)


def conv_dx(dy, w, s, in_shape):
    """The adjoint of the convolution: dx[n, s y + i, s x + j, c] += sum_o dy[n, y, x, o] w[o, i, j, c]."""
    dx = np.zeros(in_shape)
    k = w.shape[1]
    oh, ow = dy.shape[1], dy.shape[2]
    for i in range(k):
        for j in range(k):
            dx[:, i:i + s * (oh - 1) + 1:s, j:j + s * (ow - 1) + 1:s, :] += np.einsum(
                "nhwo,oc->nhwc", dy, w[:, i, j, :], optimize=True)
    return dx


def ppo_loss_and_grads(depth, state, actions, old_logp, adv, ret, theta, act_dim, clip, vcoef, ecoef):
    """Loss and parameter gradient of one PPO step over S samples (the mean
    over samples), FP64, with the device's BF16 rounding points: the
    activations (ReLU outputs) and the gradients of the pre-activations of the
    encoder layers are BF16.
      r = exp(logp - old_logp); L = -mean(min(r A, clip(r, 1 - eps, 1 + eps) A))
          + vcoef mean((V - R)^2) - ecoef H,  H = sum_a (log_std_a + (1 + ln 2 pi) / 2)."""
    P = unpack(theta, act_dim)
    fw = forward(depth, state, theta, act_dim)
    S = depth.shape[0]
    ls = P["log_std"].astype(np.float64)
    std = np.exp(ls)
    a = np.asarray(actions, np.float64)
    mean, V = fw["mean"], fw["value"]
    z = (a - mean) / std
    logp = np.sum(-0.5 * z * z - ls, axis=1) - 0.5 * np.log(2 * np.pi) * act_dim
    r = np.exp(logp - np.asarray(old_logp, np.float64))
    A_ = np.asarray(adv, np.float64)
    s1 = r * A_
    s2 = np.clip(r, 1.0 - clip, 1.0 + clip) * A_
    use1 = s1 <= s2
    R = np.asarray(ret, np.float64)
    H = float(np.sum(ls + 0.5 * (1.0 + np.log(2 * np.pi))))
    loss_pi = -np.mean(np.where(use1, s1, s2))
    loss_v = np.mean((V - R) ** 2)
    loss = loss_pi + vcoef * loss_v - ecoef * H
    # gradients
    dlogp = np.where(use1, -A_ * r, 0.0) / S                  # dL / dlogp per sample
    g_mean = dlogp[:, None] * (z / std)                       # dlogp/dmean = (a - mean) / std^2
    g_ls = np.sum(dlogp[:, None] * (z * z - 1.0), axis=0) - ecoef * np.ones(act_dim)
    g_v = vcoef * 2.0 * (V - R) / S
    q = np.asarray(state, np.float32)[:, 3:10].astype(np.float64)
    f = np.concatenate([fw["h4"], q], axis=1)
    G = {}
    G["actor.w"] = g_mean.T @ f
    G["actor.b"] = g_mean.sum(axis=0)
    G["critic.w"] = g_v @ f
    G["critic.b"] = np.array([g_v.sum()])
    G["log_std"] = g_ls
    df = g_mean @ P["actor.w"].astype(np.float64) + np.outer(g_v, P["critic.w"].astype(np.float64))
    # fc (ReLU mask on its output h4); the device keeps dpre in BF16
    d4 = bf16(df[:, :FEAT] * (fw["h4"] > 0))
    h3 = fw["h3"].reshape(S, -1)
    G["fc.w"] = d4.T @ h3
    G["fc.b"] = d4.sum(axis=0)
    d3 = bf16((d4 @ bf16(P["fc.w"])) * (h3 > 0)).reshape(fw["h3"].shape)
    ins = [fw["x"], fw["h1"], fw["h2"]]
    dpre = d3
    for i in (2, 1, 0):
        o, k, s, c = CONV[i]
        G[f"conv{i + 1}.w"] = conv_dw(ins[i], dpre, k, s)
        G[f"conv{i + 1}.b"] = dpre.sum(axis=(0, 1, 2))
        if i > 0:
            dx = conv_dx(dpre, bf16(P[f"conv{i + 1}.w"]), s, ins[i].shape)
            dpre = bf16(dx * (ins[i] > 0))
    grad = np.concatenate([np.asarray(G[name], np.float64).reshape(-1) for name, _ in layout(act_dim)])
    return dict(loss=loss, loss_pi=loss_pi, loss_v=loss_v, entropy=H, grad=grad, ratio=r, logp=logp)
