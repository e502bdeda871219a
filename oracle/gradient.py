"""Gradient of the log-marginal likelihood: exact (Eq. 2) and Hutchinson estimate, FP64.

Parameterisation (the paper lists theta = {sigma^2, l_r^2} without fixing one
for the optimiser): log sigma^2, log l_1 .. log l_d, log lambda, in that order.
With Delta_r = x_ir - x_jr the derivatives of K_y = K + lambda I are
    dK_y / dlog sigma^2 = K
    dK_y / dlog l_r     = K o (Delta_r^2 / l_r^2)          (o: elementwise)
    dK_y / dlog lambda  = lambda I.

Eq. (2): g_i = -1/2 Tr(K_y^{-1} dK_y_i) + 1/2 y^T K_y^{-1} dK_y_i K_y^{-1} y.

Section 2.1 replaces the trace by (1/N) sum_c r_c^T K_y^{-1} dK_y_i r_c with
Rademacher r_c (unbiased because E[r r^T] = I).  With alpha = K_y^{-1} y and
s_c = K_y^{-1} r_c this gives
    g_i ~= 1/2 alpha^T dK_y_i alpha - 1/(2N) sum_c s_c^T dK_y_i r_c.

Pinned by (tests/test_oracle_gradient.py): central finite differences of the
Cholesky log-marginal likelihood in the same log space; the n = 1 closed form;
Sylvester-Hadamard probes (H H^T = n I) make the estimate equal the exact
trace; the mean over many probe draws lies within 3 standard errors of the
exact gradient, with the variance of r^T M r for Rademacher r taken from
its closed form 2 (|M_s|_F^2 - sum_i (M_s)_ii^2), M_s = (M + M^T)/2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .kernel import kernel_matrix, rbf_block


def derivative_matrices(X, sigma2, lengthscales, lam):
    """List of the d + 2 dense matrices dK_y / dlog(theta_i).  Small n only."""
    X = np.asarray(X, dtype=np.float64)
    ls = np.asarray(lengthscales, dtype=np.float64)
    K = kernel_matrix(X, sigma2, ls)
    mats = [K]
    for r in range(X.shape[1]):
        diff = (X[:, r][:, None] - X[:, r][None, :]) / ls[r]
        mats.append(K * diff * diff)
    mats.append(lam * np.eye(X.shape[0]))
    return mats


def exact_gradient(X, sigma2, lengthscales, lam, y):
    """Eq. (2) with the trace taken exactly from the Cholesky inverse."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Ky = kernel_matrix(X, sigma2, lengthscales) + lam * np.eye(n)
    c = sla.cho_factor(Ky, lower=True)
    alpha = sla.cho_solve(c, y)
    Kinv = sla.cho_solve(c, np.eye(n))
    g = []
    for dK in derivative_matrices(X, sigma2, lengthscales, lam):
        g.append(-0.5 * np.sum(Kinv * dK.T) + 0.5 * float(alpha @ dK @ alpha))
    return np.array(g)


def bilinear_forms(X, sigma2, lengthscales, lam, U, V, block=256):
    """F[c, i] = U[:, c]^T (dK_y / dlog theta_i) V[:, c], without storing dK_y.

    Row blocks of K and of the squared scaled differences are regenerated
    from X, as in the product of ``oracle.kernel``.
    """
    X = np.asarray(X, dtype=np.float64)
    ls = np.asarray(lengthscales, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64).reshape(X.shape[0], -1)
    V = np.asarray(V, dtype=np.float64).reshape(X.shape[0], -1)
    n, d = X.shape
    kcols = U.shape[1]
    F = np.zeros((kcols, d + 2))
    for s in range(0, n, block):
        rows = slice(s, min(s + block, n))
        Kb = rbf_block(X[rows], X, sigma2, ls)
        F[:, 0] += np.sum(U[rows] * (Kb @ V), axis=0)
        for r in range(d):
            diff = (X[rows, r][:, None] - X[None, :, r]) / ls[r]
            F[:, 1 + r] += np.sum(U[rows] * ((Kb * diff * diff) @ V), axis=0)
    F[:, d + 1] = lam * np.sum(U * V, axis=0)
    return F


def hutchinson_gradient(X, sigma2, lengthscales, lam, alpha, S, Z):
    """1/2 alpha^T dK alpha - 1/(2N) sum_c s_c^T dK z_c for every parameter."""
    Z = np.asarray(Z, dtype=np.float64)
    N = Z.shape[1]
    data = bilinear_forms(X, sigma2, lengthscales, lam, alpha, alpha)[0]
    trace = bilinear_forms(X, sigma2, lengthscales, lam, S, Z).sum(axis=0)
    return 0.5 * data - trace / (2.0 * N)


def hutchinson_terms(X, sigma2, lengthscales, lam, alpha, S, Z):
    """Magnitudes |1/2 alpha^T dK alpha| + 1/(2N) sum_c |s_c^T dK z_c| per parameter."""
    Z = np.asarray(Z, dtype=np.float64)
    N = Z.shape[1]
    data = bilinear_forms(X, sigma2, lengthscales, lam, alpha, alpha)[0]
    trace = bilinear_forms(X, sigma2, lengthscales, lam, S, Z)
    return 0.5 * np.abs(data) + np.abs(trace).sum(axis=0) / (2.0 * N)
