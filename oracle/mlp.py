"""Fully connected GELU network, forward / backward / Adam -- oracle, FP64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The learned form's surrogate maps the 128 leading Karhunen-Loeve
coefficients of the log-modulus and log-thickness fields to the per-node
peak radial displacement: layers W_l [out, in], b_l [out]; every hidden
layer is z = W h + b, h' = GELU(z) with the exact erf form
GELU(x) = x/2 (1 + erf(x / sqrt 2)); the output layer is linear.  Loss:
mean squared error over the batch and outputs, L = 1/(B n) sum (y - t)^2.
Adam (Kingma & Ba 2015) with bias correction; optional decoupled weight
decay on the weight matrices (AdamW, Loshchilov & Hutter 2019): the step
adds lr * wd * W to the Adam update of W, biases are not decayed.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss
against backward() on a small network; GELU identities
GELU(x) - GELU(-x) = x and GELU(0) = 0 and its derivative against a finite
difference; a linear single-layer network whose gradient is X^T dY in closed
form; one Adam step against the update written from its definition; weight
decay alone (zero gradient) shrinks W by exactly (1 - lr wd) and leaves b.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + special.erf(x / SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + special.erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) * INV_SQRT_2PI


def init_params(sizes, rng):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; sizes = [n_in, h1, ..., n_out]."""
    return [(rng.standard_normal((o, i)) * math.sqrt(2.0 / i), np.zeros(o))
            for i, o in zip(sizes[:-1], sizes[1:])]


def forward(params, X):
    """Returns outputs Y [B, n_out] and the cache (inputs and pre-activations)."""
    h = X
    cache = []
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if li < len(params) - 1 else z
    return h, cache


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(params, cache, Y, T):
    """Gradients [(dW, db)] of the mean squared error."""
    B, n = Y.shape
    d = 2.0 * (Y - T) / (B * n)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        h, z = cache[li]
        if li < len(params) - 1:
            d = d * gelu_grad(z)
        W, _ = params[li]
        grads[li] = (d.T @ h, d.sum(axis=0))
        d = d @ W
    return grads


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, weight_decay=0.0):
    """One Adam step (t counts from 1).  m, v: lists like params.
    weight_decay: decoupled decay of the weight matrices (not the biases)."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for p, g, mm, vv, wd in ((W, gW, mW, vW, weight_decay), (b, gb, mb, vb, 0.0)):
            mm = b1 * mm + (1.0 - b1) * g
            vv = b2 * vv + (1.0 - b2) * g * g
            mhat = mm / (1.0 - b1 ** t)
            vhat = vv / (1.0 - b2 ** t)
            new.append((p - lr * (mhat / (np.sqrt(vhat) + eps) + wd * p), mm, vv))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v
