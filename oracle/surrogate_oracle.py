"""FP64 CPU oracle of the learned surrogate: a stack of 3x3 convolutions.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the product path
never imports it and it imports nothing from the product.

The network: layers l = 0..L-1, each y = conv3x3(x, W_l) + b_l with zero
padding (same spatial size), ReLU after every layer but the last.  Shapes:
x [C_in, H, W], W_l [C_out, C_in, 3, 3], b_l [C_out].  The GPU runs it with
BF16 weights and activations and FP32 accumulation; `bf16_round` reproduces
the BF16 storage here (round to nearest even of the top 16 bits), products
and sums stay exact-ish in FP64.  Loss: mean squared error.  Optimiser: Adam
(Kingma & Ba 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def conv3x3(x, W, b):
    """y[o, i, j] = b[o] + sum_c sum_{di, dj in 0..2} W[o, c, di, dj] x[c, i+di-1, j+dj-1],
    with x taken as zero outside the image."""
    C, H, Wd = x.shape
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:H + 1, 1:Wd + 1] = x
    y = np.zeros((W.shape[0], H, Wd))
    for di in range(3):
        for dj in range(3):
            y += np.tensordot(W[:, :, di, dj], xp[:, di:di + H, dj:dj + Wd], axes=(1, 0))
    return y + b[:, None, None]


def conv3x3_backward(x, W, dy):
    """Gradients of sum(dy * conv3x3(x, W, b)) with respect to x, W and b."""
    C, H, Wd = x.shape
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:H + 1, 1:Wd + 1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for di in range(3):
        for dj in range(3):
            patch = xp[:, di:di + H, dj:dj + Wd]
            dW[:, :, di, dj] = np.tensordot(dy, patch, axes=([1, 2], [1, 2]))
            dxp[:, di:di + H, dj:dj + Wd] += np.tensordot(W[:, :, di, dj], dy, axes=(0, 0))
    db = dy.sum(axis=(1, 2))
    return dxp[:, 1:H + 1, 1:Wd + 1], dW, db


def forward(x, weights, biases, bf16=True):
    """Network forward.  Returns the output and the per-layer inputs/pre-activations
    kept for the backward pass.  With bf16=True, weights and every stored
    activation (the input and each layer's output) are rounded to BF16."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    acts = [r(x)]
    pre = []
    h = acts[0]
    L = len(weights)
    for l in range(L):
        z = conv3x3(h, r(weights[l]), np.asarray(biases[l], dtype=np.float64))
        pre.append(z)
        if l < L - 1:
            h = r(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, (acts, pre)


def mse(pred, target):
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(weights, cache, dout, bf16=True):
    """Gradients of the loss with respect to all weights and biases, given
    dL/d(output) and the forward cache."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    acts, pre = cache
    L = len(weights)
    gW, gb = [None] * L, [None] * L
    g = dout
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            g = g * (pre[l] > 0.0)
        dx, gW[l], gb[l] = conv3x3_backward(acts[l], r(weights[l]), g)
        g = dx
    return gW, gb


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (in place on params, m, v); t is the 1-based step count."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1.0 - beta1) * g
        vv *= beta2
        vv += (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** t)
        vhat = vv / (1.0 - beta2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)


def init_weights(channels, seed):
    """He-uniform initial weights for the layer widths `channels` (e.g. 5,48,...,4)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for cin, cout in zip(channels[:-1], channels[1:]):
        bound = np.sqrt(6.0 / (9 * cin))
        Ws.append(rng.uniform(-bound, bound, size=(cout, cin, 3, 3)))
        bs.append(np.zeros(cout))
    return Ws, bs
