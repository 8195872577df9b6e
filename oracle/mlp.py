"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

A multilayer perceptron (x, t) -> (v, Dv): input normalisation, `depth`
hidden layers of width `width` with SiLU, a linear output layer, output
de-normalisation.  Loss on a batch of B rows, in normalised output units:

    L = (1/B) sum_rows [ (y_0 - T_0)^2 + (lambda/n) sum_{j>=1} (y_j - T_j)^2 ]

Parameters are a list of (W [out][in], b [out]) per layer.  Written from the
definitions (chain rule by hand); pinned by finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, rng):
    """He-style uniform init: U(-sqrt(6/fan_in), sqrt(6/fan_in)) * 0.5, zero biases."""
    params = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        lim = 0.5 * np.sqrt(6.0 / fin)
        params.append((rng.uniform(-lim, lim, (fout, fin)), np.zeros(fout)))
    return params


def forward(params, X):
    """X [B][in] (normalised).  Returns (Y [B][out], cache)."""
    acts, pre = [X], []
    h = X
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        pre.append(z)
        h = silu(z) if li < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def loss_and_grads(params, X, T, lam: float):
    """Loss and its gradient w.r.t. every W and b."""
    B, nout = T.shape
    n = nout - 1
    wts = np.full(nout, lam / n)
    wts[0] = 1.0
    Y, (acts, pre) = forward(params, X)
    diff = Y - T
    loss = np.sum(wts * diff * diff) / B
    dY = 2.0 * wts * diff / B
    grads = [None] * len(params)
    d = dY
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        grads[li] = (d.T @ acts[li], d.sum(axis=0))
        if li > 0:
            d = (d @ W) * dsilu(pre[li - 1])
    return loss, grads


def normalise(x, mean, std):
    return (x - mean) / std


def predict(params, xt, in_mean, in_std, out_mean, out_std):
    """Raw (x, t) rows -> raw (v, Dv) rows."""
    Y, _ = forward(params, normalise(xt, in_mean, in_std))
    return Y * out_std + out_mean


def round_bf16(a):
    """Round float64 values to the nearest bfloat16 (8 significant bits, ties
    to even), returned as float64 (normal range only)."""
    m, e = np.frexp(np.asarray(a, dtype=np.float64))
    return np.ldexp(np.round(m * 256.0), e - 8)


def forward_bf16_storage(params, X):
    """Forward pass with the storage rounding of a bfloat16 network: weights,
    inputs and every hidden activation rounded to bfloat16; products, sums,
    biases and SiLU in float64; the output layer is not rounded."""
    h = round_bf16(X)
    L = len(params)
    for li, (W, b) in enumerate(params):
        z = h @ round_bf16(W).T + b
        h = round_bf16(silu(z)) if li < L - 1 else z
    return h


def value_at(params, norm, y, t):
    """Value head of the network at states y [..., n] and time t (raw units).

    norm: [4][n + 1] (input mean, input std, output mean, output std)."""
    y = np.asarray(y, dtype=np.float64)
    shape = y.shape[:-1]
    rows = y.reshape(-1, y.shape[-1])
    xt = np.concatenate([rows, np.full((rows.shape[0], 1), float(t))], axis=1)
    out = forward_bf16_storage(params, (xt - norm[0]) / norm[1])
    return (out[:, 0] * norm[3][0] + norm[2][0]).reshape(shape)


def value_grad_at(params, norm, x, t):
    """(v, Dv) outputs of the network at x [Q, n], time t (raw units)."""
    x = np.asarray(x, dtype=np.float64)
    xt = np.concatenate([x, np.full((x.shape[0], 1), float(t))], axis=1)
    out = forward_bf16_storage(params, (xt - norm[0]) / norm[1]) * norm[3] + norm[2]
    return out[:, 0], out[:, 1:]


def loss_and_grads_bf16_storage(params, X, T, lam: float, rnd=round_bf16):
    """loss_and_grads with the storage rounding of a bfloat16 network.

    What a network whose matrix operands live in bfloat16 computes, with every
    product and sum in float64: weights, inputs and hidden activations rounded
    (as in forward_bf16_storage); the output error dY = 2 w (Y - T) / B and
    each back-propagated error dz = (dY W) silu'(z) rounded before they enter
    a product; the output layer, the loss and the parameter gradients not
    rounded.  rnd = identity gives loss_and_grads exactly.
    """
    B, nout = T.shape
    n = nout - 1
    wts = np.full(nout, lam / n)
    wts[0] = 1.0
    Wr = [rnd(W) for W, _ in params]
    acts, pre = [rnd(X)], []
    h = acts[0]
    L = len(params)
    for li, (_, b) in enumerate(params):
        z = h @ Wr[li].T + b
        pre.append(z)
        h = rnd(silu(z)) if li < L - 1 else z
        acts.append(h)
    diff = h - T
    loss = np.sum(wts * diff * diff) / B
    d = rnd(2.0 * wts * diff / B)
    grads = [None] * L
    for li in range(L - 1, -1, -1):
        grads[li] = (d.T @ acts[li], d.sum(axis=0))
        if li > 0:
            d = rnd((d @ Wr[li]) * dsilu(pre[li - 1]))
    return loss, grads
