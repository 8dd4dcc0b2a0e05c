"""FP64 oracle of the surrogate MLP (test infrastructure only).

Network: inputs (alpha, log S_b, log S_s, b, omega), z-scored; 4 hidden layers
of width 256 with the exact GELU, x Phi(x) = x (1 + erf(x / sqrt 2)) / 2; a
linear output layer of 33 (32 head-displacement summaries and the mean
speed, z-scored).  Loss: mean squared error over the batch and the 33
outputs.  Optimizer: Adam (Kingma & Ba 2015) with beta = (0.9, 0.999),
eps = 1e-8, bias-corrected moments.

bf16=True reproduces "BF16 weights and activations with higher-precision
accumulation" literally: every GEMM operand is rounded to bfloat16
(round-to-nearest-even) and the products are accumulated in FP64; biases,
activations and the elementwise parts stay FP64.  bf16=False is the plain
FP64 network.
"""
import math

import numpy as np

LAYERS = (5, 256, 256, 256, 256, 33)
SQRT1_2 = 1.0 / math.sqrt(2.0)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def _erf(x):
    v = np.vectorize(math.erf, otypes=[np.float64])
    return v(x)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x * SQRT1_2))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x * SQRT1_2))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def _op(a, use_bf16):
    return bf16(a) if use_bf16 else np.asarray(a, dtype=np.float64)


def forward(params, X, bf16_ops=True):
    """params: list of (W (fan_in x fan_out), b (fan_out)).  Returns outputs and
    the pre-activations of every hidden layer."""
    h = np.asarray(X, dtype=np.float64)
    pre = []
    hs = []
    for l, (W, b) in enumerate(params):
        hs.append(h)
        a = _op(h, bf16_ops) @ _op(W, bf16_ops) + np.asarray(b, dtype=np.float64)
        if l < len(params) - 1:
            pre.append(a)
            h = gelu(a)
        else:
            out = a
    return out, pre, hs


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(params, X, T, bf16_ops=True):
    """Loss and gradients (dW, db) of the MSE loss."""
    Y, pre, hs = forward(params, X, bf16_ops)
    B, M = Y.shape
    dA = 2.0 * (Y - T) / (B * M)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        dW = _op(hs[l], bf16_ops).T @ _op(dA, bf16_ops)
        db = dA.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            dH = _op(dA, bf16_ops) @ _op(W, bf16_ops).T
            dA = dH * gelu_grad(pre[l - 1])
    return mse(Y, T), grads


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1, 2, ...); returns new params, m, v."""
    newp, newm, newv = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = b1 * mm + (1 - b1) * g
            vv = b2 * vv + (1 - b2) * g * g
            mh = mm / (1 - b1 ** t)
            vh = vv / (1 - b2 ** t)
            out.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        newp.append((out[0][0], out[1][0]))
        newm.append((out[0][1], out[1][1]))
        newv.append((out[0][2], out[1][2]))
    return newp, newm, newv


def zeros_like(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]


def n_params():
    return sum(a * b + b for a, b in zip(LAYERS[:-1], LAYERS[1:]))
