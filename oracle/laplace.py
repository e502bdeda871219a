"""Laplace approximation for GP classification with a probit likelihood, FP64.

Test infrastructure (like the rest of ``oracle/``).  Follows the paper's
non-Gaussian-likelihood section (Section 2.2) and its supplementary
derivations: Newton iterations written with B = I + W^1/2 K W^1/2, the
approximate log-marginal likelihood, its stochastic gradient (explicit trace
term, data-fit term, implicit term) and the predictive class probability.

Likelihood p(y_i | f_i) = Phi(y_i f_i), y_i in {-1, +1}.  With z = y f and
the inverse Mills ratio r(z) = N(z) / Phi(z) (N the standard normal density),
r'(z) = -r (z + r) and r''(z) = r (z^2 + 3 z r + 2 r^2 - 1), so
    d/df   log p = y r(z)
    W  =  -d^2/df^2 log p = r(z) (z + r(z))          (> 0: log p is concave)
    d^3/df^3 log p = y r''(z).
W is the negative Hessian, so dW/df_j = -d^3 log p / df_j^3 (the supplement
prints the derivative without the minus sign; the finite-difference pin of
the gradient below settles the sign).

Newton step (the paper's Laplace algorithm): b = W f + d log p,
c = W^1/2 K b, solve B z = c, a = b - W^1/2 z, f_new = K a.  At the mode
a = K^-1 f_hat = d log p(f_hat).  Approximate log-marginal likelihood
    log q = -1/2 log|B| - 1/2 f_hat^T a + sum log Phi(y f_hat).
Stochastic gradient in theta = (log sigma2, log l_1 .. log l_d) with probes
r_c (E[r r^T] = I):
    g_i = -1/(2N) sum_c (W^1/2 B^-1 r_c)^T dK_i (W^1/2 r_c)
          + 1/2 a^T dK_i a
          - 1/2 (W^1/2 B^-1 W^-1/2 u)^T dK_i (d log p)
    u_j = (1/N) sum_c r_cj [(K^-1 + W)^-1 r_c]_j (dW/df_j),
    (K^-1 + W)^-1 r = K (r - W^1/2 B^-1 W^1/2 K r).
Prediction: m_* = k_*^T a, s_*^2 = k_** - (W^1/2 k_*)^T B^-1 (W^1/2 k_*),
p(y_* = 1) = Phi(m_* / sqrt(1 + s_*^2)).

Pinned by (tests/test_oracle_laplace.py): the probit derivatives against
central differences of log Phi; the mode satisfies f_hat = K d log p(f_hat)
and maximises Psi; with Sylvester-Hadamard probes (exact traces) the
stochastic gradient equals central finite differences of log q; the
predictive variance equals the textbook form k_** - k_*^T (K + W^-1)^-1 k_*
and the mean k_*^T d log p(f_hat).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.special import erfcx, log_ndtr, ndtr

from .gradient import derivative_matrices
from .kernel import kernel_matrix, rbf_block

_SQRT2 = np.sqrt(2.0)
_SQRT2PI = np.sqrt(2.0 * np.pi)


def mills(z):
    """r(z) = N(z) / Phi(z), stable for large negative z (erfcx form)."""
    z = np.asarray(z, dtype=np.float64)
    return 2.0 / (_SQRT2PI * erfcx(-z / _SQRT2))


def probit_derivatives(y, f):
    """(log p, d1, W, d3) elementwise: log Phi(y f), its first derivative,
    W = -second derivative, and the third derivative in f."""
    z = y * f
    r = mills(z)
    logp = log_ndtr(z)
    d1 = y * r
    W = r * (z + r)
    d3 = y * r * (z * z + 3.0 * z * r + 2.0 * r * r - 1.0)
    return logp, d1, W, d3


def mode(K, y, tol=1e-12, max_newton=100):
    """Newton iterations of the paper's Laplace algorithm, dense.  Returns
    (f_hat, a, iterations)."""
    n = K.shape[0]
    f = np.zeros(n)
    psi_old = -np.inf
    for it in range(1, max_newton + 1):
        _, d1, W, _ = probit_derivatives(y, f)
        sw = np.sqrt(W)
        b = W * f + d1
        B = np.eye(n) + sw[:, None] * K * sw[None, :]
        z = np.linalg.solve(B, sw * (K @ b))
        a = b - sw * z
        f = K @ a
        logp = log_ndtr(y * f)
        psi = logp.sum() - 0.5 * a @ f
        if abs(psi - psi_old) <= tol * max(1.0, abs(psi)):
            break
        psi_old = psi
    # a at the returned f (the fixed point: a = d log p(f_hat))
    return f, a, it


def log_marginal(X, sigma2, lengthscales, y, tol=1e-13):
    """Approximate log-marginal likelihood log q at the mode."""
    K = kernel_matrix(X, sigma2, lengthscales)
    f, a, _ = mode(K, y, tol=tol)
    _, _, W, _ = probit_derivatives(y, f)
    sw = np.sqrt(W)
    B = np.eye(len(y)) + sw[:, None] * K * sw[None, :]
    logdet = 2.0 * np.sum(np.log(np.diag(sla.cholesky(B, lower=True))))
    return -0.5 * logdet - 0.5 * a @ f + log_ndtr(y * f).sum()


def stochastic_gradient(X, sigma2, lengthscales, y, f, R):
    """The paper's three-term gradient estimate at the mode f with probes R
    (n x N), dense solves.  Components (log sigma2, log l_1 .. log l_d)."""
    X = np.asarray(X, dtype=np.float64)
    n, N = R.shape
    K = kernel_matrix(X, sigma2, lengthscales)
    _, d1, W, d3 = probit_derivatives(y, f)
    a = d1                                        # K^-1 f_hat at the mode
    sw = np.sqrt(W)
    B = np.eye(n) + sw[:, None] * K * sw[None, :]
    Bc = sla.cho_factor(B, lower=True)
    binv = lambda V: sla.cho_solve(Bc, V)
    dW = -d3                                      # W is the negative Hessian
    S1 = sw[:, None] * binv(R)                    # W^1/2 B^-1 r_c
    V1 = sw[:, None] * R                          # W^1/2 r_c
    KR = K @ R
    post = K @ (R - sw[:, None] * binv(sw[:, None] * KR))   # (K^-1 + W)^-1 r_c
    u = np.mean(R * post, axis=1) * dW
    s3 = sw * binv(u / sw)                        # W^1/2 B^-1 W^-1/2 u
    g = []
    for dK in derivative_matrices(X, sigma2, lengthscales, 0.0)[:-1]:
        t1 = -0.5 / N * np.sum(S1 * (dK @ V1))
        t2 = 0.5 * a @ dK @ a
        t3 = -0.5 * s3 @ dK @ d1
        g.append(t1 + t2 + t3)
    return np.array(g)


def predict(X, sigma2, lengthscales, y, f, Xs):
    """(m_*, s_*^2, p(y_* = +1)) at test inputs Xs, B-form (dense)."""
    K = kernel_matrix(X, sigma2, lengthscales)
    _, d1, W, _ = probit_derivatives(y, f)
    sw = np.sqrt(W)
    B = np.eye(len(y)) + sw[:, None] * K * sw[None, :]
    Ks = rbf_block(np.asarray(Xs, dtype=np.float64), X, sigma2, lengthscales)  # n_* x n
    m = Ks @ d1
    V = sw[:, None] * Ks.T
    s2 = sigma2 - np.sum(V * np.linalg.solve(B, V), axis=0)
    return m, s2, ndtr(m / np.sqrt(1.0 + s2))
