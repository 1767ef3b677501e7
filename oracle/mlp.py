"""CPU oracle of the learned PST proposal network (binary64 numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: x (1216 = 40x30 depth residual + 6D previous velocity + 10 zeros)
-> 256 GELU -> 256 GELU -> 12 = (mu in R^6, log-scale l in R^6).
Loss: heteroscedastic Gaussian negative log-likelihood per sample,
sum_d [ (y_d - mu_d)^2 / (2 exp(2 l_d)) + l_d ], averaged over the batch.
GELU(z) = z Phi(z) with the standard normal CDF Phi (exact, erf-based).
Adam (Kingma & Ba 2015) on binary64 copies of the parameters.

Parameter layout (shared with the GPU binding): W1 (1216, 256), b1 (256),
W2 (256, 256), b2 (256), W3 (256, 12), b3 (12); y = x W + b (row vectors).

bf16=True: every matrix product takes its two operands rounded to bfloat16
first (binary32, then round to nearest even on the upper 16 bits: the
rounding the matrix cores' inputs go through), then multiplies them in
binary64; everything else is unchanged.  Pinned: the rounding's ties go to
even and it is the identity on bfloat16 values; products of bfloat16-exact
operands equal the plain ones.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def bf16_round(a) -> np.ndarray:
    """a rounded to binary32, then to bfloat16 (nearest, ties to even), as
    binary64 values."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mm(A, B, bf16: bool = False):
    """A @ B in binary64; bf16: operands rounded to bfloat16 first."""
    if bf16:
        return bf16_round(A) @ bf16_round(B)
    return A @ B


def forward(p, X, bf16: bool = False):
    """Returns (out (B, 12), cache)."""
    X = np.asarray(X, np.float64)
    Z1 = mm(X, p["W1"], bf16) + p["b1"]
    H1 = gelu(Z1)
    Z2 = mm(H1, p["W2"], bf16) + p["b2"]
    H2 = gelu(Z2)
    out = mm(H2, p["W3"], bf16) + p["b3"]
    return out, (X, Z1, H1, Z2, H2)


def loss_and_dout(out, Y):
    """Mean Gaussian NLL over the batch and its gradient w.r.t. out."""
    Y = np.asarray(Y, np.float64)
    B = out.shape[0]
    mu, ls = out[:, :6], out[:, 6:]
    r = Y - mu
    inv = np.exp(-2.0 * ls)
    loss = float(np.sum(0.5 * r * r * inv + ls) / B)
    dmu = -r * inv / B
    dls = (1.0 - r * r * inv) / B
    return loss, np.concatenate([dmu, dls], axis=1)


def backward(p, cache, dout, bf16: bool = False):
    X, Z1, H1, Z2, H2 = cache
    g = {}
    g["W3"] = mm(H2.T, dout, bf16)
    g["b3"] = dout.sum(0)
    dZ2 = mm(dout, p["W3"].T, bf16) * gelu_grad(Z2)
    g["W2"] = mm(H1.T, dZ2, bf16)
    g["b2"] = dZ2.sum(0)
    dZ1 = mm(dZ2, p["W2"].T, bf16) * gelu_grad(Z1)
    g["W1"] = mm(X.T, dZ1, bf16)
    g["b1"] = dZ1.sum(0)
    return g


def loss_and_grads(p, X, Y, bf16: bool = False):
    out, cache = forward(p, X, bf16)
    loss, dout = loss_and_dout(out, Y)
    return loss, backward(p, cache, dout, bf16)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place on every entry of p; t is the 1-based step count."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1**t)
        vh = v[k] / (1 - b2**t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
