"""ADAGRAD ascent on the log-hyperparameters (Section 5), FP64.

Section 5 optimises theta by stochastic-gradient ascent with ADAGRAD (Duchi,
Hazan & Singer) and a single step size of one:
    G_t = G_{t-1} + g_t^2,   theta_{t+1} = theta_t + eta g_t / (sqrt(G_t) + eps)
elementwise, on the log parameters of ``oracle.gradient``.

Pinned by (tests/test_oracle_gradient.py): the first step moves each
coordinate by eta * sign(g) (up to eps), a closed form.
"""
from __future__ import annotations

import numpy as np


class Adagrad:
    def __init__(self, eta=1.0, eps=1e-8):
        self.eta, self.eps = eta, eps
        self.G = None

    def step(self, theta, g):
        g = np.asarray(g, dtype=np.float64)
        self.G = g * g if self.G is None else self.G + g * g
        return np.asarray(theta, dtype=np.float64) + self.eta * g / (np.sqrt(self.G) + self.eps)
