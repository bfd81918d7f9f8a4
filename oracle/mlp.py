"""FP64 reference of the start-vector network (test infrastructure only).

Multilayer perceptron 32 -> 64 -> 64 -> 16 with SiLU hidden activations and a
linear output, mean-squared-error loss, and Adam updates (Kingma & Ba 2015:
beta1 = 0.9, beta2 = 0.999, eps = 1e-8). Its inputs are coefficients on a POD
basis of recent stage solutions and the projection of the stage right-hand
side (Sec. IV's POD start vectors); its output are the coefficients of the
start vector on that basis.

Parameters are a dict {W1 [64,32], b1 [64], W2 [64,64], b2 [64],
W3 [16,64], b3 [16]}; y = W x + b for each layer.
"""

from __future__ import annotations

import numpy as np

LAYERS = (32, 64, 64, 16)
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def _q(a, bf16):
    """A matmul operand: rounded to bfloat16 in the BF16 form, else as is."""
    return round_bf16(a) if bf16 else a


def forward(p, x, bf16=False):
    """Returns the output [B,16] and the cache of pre-activations.

    bf16: the BF16 form of the network (BF16 weights with FP32 accumulation):
    both operands of every matrix product, the weights and the layer inputs,
    are rounded to bfloat16 first; biases and the sums are not."""
    h1 = _q(x, bf16) @ _q(p["W1"], bf16).T + p["b1"]
    a1 = silu(h1)
    h2 = _q(a1, bf16) @ _q(p["W2"], bf16).T + p["b2"]
    a2 = silu(h2)
    y = _q(a2, bf16) @ _q(p["W3"], bf16).T + p["b3"]
    return y, (x, h1, a1, h2, a2)


def loss(p, x, t, bf16=False):
    y, _ = forward(p, x, bf16)
    return float(np.mean((y - t) ** 2))


def backward(p, x, t, bf16=False):
    """Loss and gradients of L = mean((y - t)^2) over batch and outputs.

    bf16: as in forward, every operand of the backward matrix products (the
    output error, the layer errors, the activations, the inputs and the
    weights) is rounded to bfloat16; the bias gradients sum unrounded errors."""
    y, (x, h1, a1, h2, a2) = forward(p, x, bf16)
    B, K = y.shape
    dy = 2.0 * (y - t) / (B * K)
    g = {}
    g["W3"] = _q(dy, bf16).T @ _q(a2, bf16)
    g["b3"] = dy.sum(axis=0)
    da2 = _q(dy, bf16) @ _q(p["W3"], bf16)
    dh2 = da2 * silu_grad(h2)
    g["W2"] = _q(dh2, bf16).T @ _q(a1, bf16)
    g["b2"] = dh2.sum(axis=0)
    da1 = _q(dh2, bf16) @ _q(p["W2"], bf16)
    dh1 = da1 * silu_grad(h1)
    g["W1"] = _q(dh1, bf16).T @ _q(x, bf16)
    g["b1"] = dh1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = {"t": int, "m": {...}, "v": {...}}."""
    state["t"] += 1
    t = state["t"]
    for k in NAMES:
        m = state["m"][k] = b1 * state["m"][k] + (1 - b1) * g[k]
        v = state["v"][k] = b2 * state["v"][k] + (1 - b2) * g[k] ** 2
        mhat = m / (1 - b1 ** t)
        vhat = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)


def adam_state(p):
    return {"t": 0, "m": {k: np.zeros_like(p[k]) for k in NAMES}, "v": {k: np.zeros_like(p[k]) for k in NAMES}}


def round_bf16(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64.

    bfloat16 keeps the top 16 bits of an IEEE binary32; rounding goes through
    binary32 first (as a GPU that converts FP32 accumulators does)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
