"""FP64 reference of the surrogate network: forward, backward and Adam.

TEST INFRASTRUCTURE ONLY: checks the GPU training and inference kernels.

Network: x (6 features) -> 256 -> 256 -> 256 -> 1, SiLU after each hidden
layer, mean-squared-error loss. Parameters are stored the way the GPU library
stores them: W_l as (fan_out, fan_in) row-major, b_l as (fan_out,).
"""
from __future__ import annotations

import numpy as np

LAYERS = (6, 256, 256, 256, 1)


def init_params(seed: int, layers=LAYERS):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(layers[:-1], layers[1:]):
        bound = 1.0 / np.sqrt(fi)
        params.append(rng.uniform(-bound, bound, size=(fo, fi)))
        params.append(rng.uniform(-bound, bound, size=(fo,)))
    return params


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """Returns (y (B,), cache)."""
    h = np.asarray(x, dtype=np.float64)
    pre = []
    acts = [h]
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W.T + b
        pre.append(z)
        h = silu(z) if l < nl - 1 else z
        acts.append(h)
    return h[:, 0], (pre, acts)


def loss_and_grads(params, x, y):
    """MSE loss 0.5 * mean((f(x) - y)^2)... as mean((f - y)^2), and its gradients."""
    out, (pre, acts) = forward(params, x)
    B = out.shape[0]
    r = out - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    g = (2.0 / B) * r[:, None]                 # dL/d(output pre-activation)
    nl = len(params) // 2
    grads = [None] * len(params)
    for l in range(nl - 1, -1, -1):
        W = params[2 * l]
        grads[2 * l] = g.T @ acts[l]
        grads[2 * l + 1] = g.sum(axis=0)
        if l > 0:
            g = (g @ W) * silu_grad(pre[l - 1])
    return loss, grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place on params, m, v; t starts at 1."""
    for k in range(len(params)):
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] * grads[k]
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params, m, v
