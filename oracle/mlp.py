"""CPU oracle for the selector's MLP -- TEST INFRASTRUCTURE ONLY.

The network: 16 inputs -> 64 -> 64 -> K, ReLU between layers, parameters
packed [W1 16x64 | b1 64 | W2 64x64 | b2 64 | W3 64xK | b3 K] (row-major,
input index first).  The device stores parameters, inputs and hidden
activations in BF16 and accumulates in FP32; this reference rounds the same
values to BF16 (round to nearest even) at the same points and does all
arithmetic in float64.  Loss: mean squared error over the B x K outputs.
Backward: BF16 rounding is treated as identity, ReLU'(0) = 0.

Not from the paper (the paper has no learned component); pinned by finite
differences of this module's own loss (which checks the analytic gradient
against the definition of a derivative, not against a second copy of the
formula) and by a hand-computed two-layer example in the tests.
"""
from __future__ import annotations

import numpy as np

IN, H = 16, 64


def param_count(K: int) -> int:
    return IN * H + H + H * H + H + H * K + K


def bf16_round(x):
    """Round float64/float32 values to the nearest BF16 (ties to even), as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p, K: int):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + IN * H].reshape(IN, H); o += IN * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H * K].reshape(H, K); o += H * K
    b3 = p[o:o + K]; o += K
    return W1, b1, W2, b2, W3, b3


def forward(params_bf16_values, X, K: int):
    """params_bf16_values: the parameters as already-BF16 values (float64 array)."""
    W1, b1, W2, b2, W3, b3 = unpack(params_bf16_values, K)
    x = bf16_round(X)
    z1 = x @ W1 + b1
    a1 = bf16_round(np.maximum(z1, 0.0))
    z2 = a1 @ W2 + b2
    a2 = bf16_round(np.maximum(z2, 0.0))
    y = a2 @ W3 + b3
    return y, dict(x=x, z1=z1, a1=a1, z2=z2, a2=a2)


def loss_and_grads(params_bf16_values, X, T, K: int):
    W1, b1, W2, b2, W3, b3 = unpack(params_bf16_values, K)
    y, c = forward(params_bf16_values, X, K)
    B = X.shape[0]
    d = y - T
    loss = float(np.mean(d * d))
    dY = 2.0 * d / (B * K)
    gW3 = c["a2"].T @ dY
    gb3 = dY.sum(0)
    dZ2 = (dY @ W3.T) * (c["z2"] > 0)
    gW2 = c["a1"].T @ dZ2
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * (c["z1"] > 0)
    gW1 = c["x"].T @ dZ1
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def finite_difference(params_bf16_values, X, T, K: int, idx, h: float = 1e-6):
    """Central differences of the loss, with the BF16 roundings of the
    activations frozen (the same straight-through convention)."""
    p = np.asarray(params_bf16_values, np.float64)

    def loss_frozen(q):
        W1, b1, W2, b2, W3, b3 = unpack(q, K)
        _, c = forward(p, X, K)
        x = c["x"]
        z1 = x @ W1 + b1
        a1 = np.maximum(z1, 0.0) + (c["a1"] - np.maximum(c["z1"], 0.0))   # keep the rounding offsets fixed
        z2 = a1 @ W2 + b2
        a2 = np.maximum(z2, 0.0) + (c["a2"] - np.maximum(c["z2"], 0.0))
        y = a2 @ W3 + b3
        return float(np.mean((y - T) ** 2))

    out = []
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        out.append((loss_frozen(p + e) - loss_frozen(p - e)) / (2 * h))
    return np.array(out)


def adam_step(w, g, m1, m2, lr, b1, b2, eps, step):
    """One Adam step (Kingma and Ba, 2015) on float64 arrays: returns (w, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, m2
