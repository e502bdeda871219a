"""Learned low-rank factor: MLP forward, loss, manual backward and Adam, FP64.

Not in the paper.  Section 3.2 preconditions with P = Phi Phi^T + lambda I for
any factor Phi with Phi Phi^T ~= K; here Phi = U is the output of a small
network applied to every input row, so P stays symmetric positive definite
and PCG stays exact whatever the network outputs.

    h1 = gelu(X W1 + b1),  h2 = gelu(h1 W2 + b2),  U = h2 W3 + b3
    gelu(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2      (exact, erf form)

Training data are probe pairs (Z, K Z) with Rademacher Z, which the kernel
product already produces.  Because E[Z Z^T] = I, the loss
    L = |U (U^T Z) - K Z|_F^2 / |K Z|_F^2
is, up to the constant normaliser, an unbiased estimate of |U U^T - K|_F^2.
Its gradient with R = U (U^T Z) - K Z is
    dL/dU = 2 (R (U^T Z)^T + Z (R^T U)) / |K Z|_F^2,
then back through the layers by the chain rule.  Adam follows Kingma & Ba
(bias-corrected first and second moments).

``round_bf16=True`` rounds weights and every matmul input to bfloat16
(round-to-nearest-even) before the float64 product, which mirrors a
bfloat16-weight, wider-accumulation implementation.

Pinned by (tests/test_oracle_mlp.py): backward against central finite
differences of the loss; a zero network gives U = 0, i.e. P = lambda I; the
exact-factor case U U^T = K gives zero loss; Adam's first step moves each
weight by lr * sign(gradient) (closed form).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / _SQRT2))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a / _SQRT2)) + a * _INV_SQRT_2PI * np.exp(-0.5 * a * a)


def round_bf16(a):
    """Round float64 values to the nearest bfloat16 (ties to even) via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(params, X, bf16=False):
    """Returns U and the cache of pre-activations for the backward pass."""
    q = round_bf16 if bf16 else (lambda a: a)
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], dtype=np.float64) for k in PARAM_NAMES)
    X = np.asarray(X, dtype=np.float64)
    a1 = q(X) @ q(W1) + b1
    h1 = gelu(a1)
    a2 = q(h1) @ q(W2) + b2
    h2 = gelu(a2)
    U = q(h2) @ q(W3) + b3
    return U, (X, a1, h1, a2, h2)


def loss(U, Z, KZ):
    R = U @ (U.T @ Z) - KZ
    return float(np.sum(R * R) / np.sum(KZ * KZ))


def loss_grad_U(U, Z, KZ):
    M = U.T @ Z
    R = U @ M - KZ
    c = np.sum(KZ * KZ)
    return float(np.sum(R * R) / c), 2.0 * (R @ M.T + Z @ (R.T @ U)) / c


def backward(params, cache, dU):
    X, a1, h1, a2, h2 = cache
    W2 = np.asarray(params["W2"], dtype=np.float64)
    W3 = np.asarray(params["W3"], dtype=np.float64)
    g = {}
    g["W3"] = h2.T @ dU
    g["b3"] = dU.sum(axis=0)
    da2 = (dU @ W3.T) * gelu_grad(a2)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ W2.T) * gelu_grad(a1)
    g["W1"] = X.T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def loss_and_grad(params, X, Z, KZ, bf16=False):
    U, cache = forward(params, X, bf16=bf16)
    L, dU = loss_grad_U(U, Z, KZ)
    return L, backward(params, cache, dU)


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in params.items()}
        self.v = {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in params.items()}

    def step(self, params, grads):
        self.t += 1
        out = {}
        for k, w in params.items():
            g = grads[k]
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g * g
            mhat = self.m[k] / (1.0 - self.b1 ** self.t)
            vhat = self.v[k] / (1.0 - self.b2 ** self.t)
            out[k] = np.asarray(w, dtype=np.float64) - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return out
