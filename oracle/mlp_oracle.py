"""FP64 reference of the surrogate MLP (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to check the GPU surrogate
kernels; never by the library or its binding.

The network: layers l = 0..L-1 with weights W_l [out, in] and bias b_l;
hidden layers z = x W^T + b, x' = GELU(z) (exact, erf form); the last layer
is linear.  Loss: mean squared error over the batch and the outputs.

``bf16=True`` rounds, at the same points as the GPU path, the values it
stores in bfloat16: the inputs, the weights, every hidden activation x' and
every back-propagated dL/dz; all arithmetic in between is FP64.
"""
from __future__ import annotations

import math

import numpy as np


def bf16_round(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), via FP32."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    z = np.asarray(z, np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(Ws, bs, X, bf16=False):
    """Returns (output, cache) with the per-layer inputs and pre-activations."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    x = r(X)
    xs, zs = [], []
    L = len(Ws)
    for l in range(L):
        xs.append(x)
        z = x @ r(Ws[l]).T + np.asarray(bs[l], np.float64)
        zs.append(z)
        if l < L - 1:
            x = r(gelu(z))
    return zs[-1], (xs, zs)


def loss_and_grads(Ws, bs, X, Y, bf16=False):
    """MSE loss and its gradients with respect to every W_l and b_l."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    out, (xs, zs) = forward(Ws, bs, X, bf16)
    B, O = out.shape
    diff = out - np.asarray(Y, np.float64)
    loss = float(np.mean(diff * diff))
    dz = r(2.0 * diff / (B * O))
    gW = [None] * len(Ws)
    gb = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        gW[l] = dz.T @ xs[l]
        gb[l] = dz.sum(axis=0)
        if l > 0:
            dx = dz @ r(Ws[l])
            dz = r(dx * gelu_grad(zs[l - 1]))
    return loss, gW, gb


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
