"""Direct (Cholesky) solve and log-marginal likelihood, FP64.

Section 2.1: with a Gaussian likelihood y_i ~ N(f_i, lambda) the
log-marginal likelihood is
    log p(y | theta, X) = -1/2 log|K_y| - 1/2 y^T K_y^{-1} y - n/2 log(2 pi),
K_y = K + lambda I, and the traditional route factorises K_y = L L^T.  The
method under test reaches K_y^{-1} B exactly in the limit of iterations, so
this plain definition is the reference for every solution.

Pinned by (tests/test_oracle_direct.py): n = 1 and n = 2 closed forms of the
log-marginal likelihood (scalar Gaussian density, 2x2 determinant and
inverse); residual of the returned solution through the independent
row-blocked product of ``oracle.kernel``; prediction: at a training input
with tiny noise the mean reproduces the target and the variance vanishes,
far from the data the mean is 0 and the variance sigma2, and the n = 1
closed form k* y / (sigma2 + lambda), sigma2 - k*^2 / (sigma2 + lambda).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .kernel import kernel_matrix, rbf_block


def _factor(X, sigma2, lengthscales, lam):
    Ky = kernel_matrix(X, sigma2, lengthscales) + lam * np.eye(X.shape[0])
    return sla.cho_factor(Ky, lower=True)


def solve(X, sigma2, lengthscales, lam, B):
    """K_y^{-1} B through the Cholesky factor of K_y."""
    c = _factor(X, sigma2, lengthscales, lam)
    return sla.cho_solve(c, np.asarray(B, dtype=np.float64))


def log_marginal_likelihood(X, sigma2, lengthscales, lam, y):
    """-1/2 log|K_y| - 1/2 y^T K_y^{-1} y - n/2 log 2 pi."""
    c = _factor(X, sigma2, lengthscales, lam)
    L = c[0]
    alpha = sla.cho_solve(c, y)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    n = X.shape[0]
    return -0.5 * logdet - 0.5 * float(y @ alpha) - 0.5 * n * math.log(2.0 * math.pi)


def predict(X, sigma2, lengthscales, lam, y, Xs):
    """GP predictive mean K(X_*, X) K_y^-1 y and latent variance
    sigma2 - diag(K(X_*, X) K_y^-1 K(X, X_*)) by Cholesky (the predictive
    equations the paper refers to for test data, Section 2.1)."""
    X = np.asarray(X, dtype=np.float64)
    Xs = np.asarray(Xs, dtype=np.float64)
    c = _factor(X, sigma2, lengthscales, lam)
    Ks = rbf_block(Xs, X, sigma2, lengthscales)
    mean = Ks @ sla.cho_solve(c, np.asarray(y, dtype=np.float64))
    var = sigma2 - np.sum(Ks * sla.cho_solve(c, Ks.T).T, axis=1)
    return mean, var
