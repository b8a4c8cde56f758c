"""FP64 CPU reference of the small multilayer perceptron used for the learned
warm start (TEST INFRASTRUCTURE: only tests/ and the cpu_baseline leg of
bench.py may import it; it shares no code with the GPU path).

Network: x [B][w0] -> hidden layers h_l = tanh(h_{l-1} W_l^T + b_l) -> linear
output y = h_{L-1} W_L^T + b_L. Weights are used as bf16 (rounded to nearest
even from the FP32 master values), biases and activations in full precision.
Loss: mean over all B * wL outputs of (y - t)^2. Parameters are packed layer by
layer as [W_l (out x in, row-major), b_l (out)].

Pinned by tests/test_oracle_mlp.py: the analytic gradient against central
finite differences of the loss (in FP64 with unrounded weights), the bf16
rounding against exactly representable values and ties, and Adam against its
closed form after one step (m-hat = g, v-hat = g^2).
"""
from __future__ import annotations

import numpy as np


def param_count(widths):
    return sum(widths[i + 1] * widths[i] + widths[i + 1] for i in range(len(widths) - 1))


def unpack(p, widths):
    out, off = [], 0
    for i in range(len(widths) - 1):
        o, n = widths[i + 1], widths[i]
        W = p[off:off + o * n].reshape(o, n)
        off += o * n
        b = p[off:off + o]
        off += o
        out.append((W, b))
    return out


def bf16_round(x):
    """Round float32 values to the nearest bf16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, widths, x, bf16=True):
    """All layer outputs [h_1, ..., h_{L-1}, y] for inputs x [B][w0]."""
    acts = []
    h = np.asarray(x, dtype=np.float64)
    layers = unpack(np.asarray(p, dtype=np.float64), widths)
    for i, (W, b) in enumerate(layers):
        Wu = bf16_round(W) if bf16 else W
        z = h @ Wu.T + b
        h = np.tanh(z) if i < len(layers) - 1 else z
        acts.append(h)
    return acts


def loss_and_grad(p, widths, x, t, bf16=True):
    """MSE loss and its gradient with respect to the packed parameters (the
    weight gradient is taken at the bf16 weights used in the forward pass)."""
    x = np.asarray(x, dtype=np.float64)
    acts = forward(p, widths, x, bf16)
    layers = unpack(np.asarray(p, dtype=np.float64), widths)
    y = acts[-1]
    B, wl = y.shape
    loss = float(np.mean((y - t) ** 2))
    d = 2.0 * (y - t) / (B * wl)                      # dL/dz of the linear output
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, b = layers[i]
        Wu = bf16_round(W) if bf16 else W
        h_in = x if i == 0 else acts[i - 1]
        gW = d.T @ h_in
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        if i > 0:
            d = (d @ Wu) * (1.0 - acts[i - 1] ** 2)      # through tanh of the previous layer
    grads.reverse()
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, g


def adam(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), bias-corrected; returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
