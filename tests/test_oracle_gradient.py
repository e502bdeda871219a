"""Pins of the oracle's LML gradient, exact (Eq. (2)) and Hutchinson (Section 2.1)."""
import math

import numpy as np
import scipy.linalg as sla

from oracle import direct as od
from oracle import gradient as og
from oracle import kernel as ok
from oracle.adagrad import Adagrad
from pkm_inputs import make, rademacher


def _lml_logspace(X, theta, y):
    d = X.shape[1]
    s2 = math.exp(theta[0])
    ls = np.exp(theta[1:1 + d])
    lam = math.exp(theta[1 + d])
    return od.log_marginal_likelihood(X, s2, ls, lam, y)


def test_exact_gradient_vs_central_differences():
    p = make("block_fp32", seed=0, n=120, n_probes=0)
    d = p.d
    theta = np.concatenate([[math.log(1.3)], np.log(p.lengthscales), [math.log(0.05)]])
    g = og.exact_gradient(p.X, math.exp(theta[0]), np.exp(theta[1:1 + d]),
                          math.exp(theta[-1]), p.y)
    h = 1e-5
    for i in range(d + 2):
        e = np.zeros_like(theta)
        e[i] = h
        fd = (_lml_logspace(p.X, theta + e, p.y) - _lml_logspace(p.X, theta - e, p.y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_n1_closed_form_gradient():
    X = np.array([[0.2, 0.4]])
    y = np.array([0.8])
    s2, lam = 1.5, 0.2
    v = s2 + lam
    dv = -0.5 / v + 0.5 * y[0] ** 2 / v ** 2
    g = og.exact_gradient(X, s2, np.array([0.7, 0.3]), lam, y)
    assert np.allclose(g, [s2 * dv, 0.0, 0.0, lam * dv], rtol=1e-14, atol=1e-15)


def _sylvester(n):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def test_hadamard_probes_make_estimate_exact():
    p = make("block_fp32", seed=1, n=64, n_probes=0)
    H = _sylvester(64)
    assert np.array_equal(H @ H.T, 64 * np.eye(64))
    alpha = od.solve(p.X, p.sigma2, p.lengthscales, p.lam, p.y)
    S = od.solve(p.X, p.sigma2, p.lengthscales, p.lam, H)
    est = og.hutchinson_gradient(p.X, p.sigma2, p.lengthscales, p.lam, alpha, S, H)
    ex = og.exact_gradient(p.X, p.sigma2, p.lengthscales, p.lam, p.y)
    assert np.allclose(est, ex, rtol=1e-10, atol=1e-10)


def test_estimator_mean_within_standard_errors():
    p = make("block_fp32", seed=2, n=32, n_probes=0)
    n = p.n
    Ky = ok.kernel_matrix(p.X, p.sigma2, p.lengthscales) + p.lam * np.eye(n)
    c = sla.cho_factor(Ky, lower=True)
    alpha = sla.cho_solve(c, p.y)
    ex = og.exact_gradient(p.X, p.sigma2, p.lengthscales, p.lam, p.y)
    rng = np.random.default_rng(7)
    draws, N = 300, 4
    ests = []
    for _ in range(draws):
        Z = rademacher(rng, n, N)
        S = sla.cho_solve(c, Z)
        ests.append(og.hutchinson_gradient(p.X, p.sigma2, p.lengthscales, p.lam, alpha, S, Z))
    ests = np.array(ests)
    Kinv = sla.cho_solve(c, np.eye(n))
    for i, dK in enumerate(og.derivative_matrices(p.X, p.sigma2, p.lengthscales, p.lam)):
        M = Kinv @ dK
        Ms = 0.5 * (M + M.T)
        var1 = 2.0 * (np.sum(Ms * Ms) - np.sum(np.diag(Ms) ** 2))
        # estimate of g_i has variance var1 / (4 N) per draw
        se = math.sqrt(var1 / (4.0 * N) / draws)
        assert abs(ests[:, i].mean() - ex[i]) <= 3.0 * se + 1e-12, (i, ests[:, i].mean(), ex[i], se)


def test_bilinear_forms_match_dense_derivatives():
    p = make("block_fp32", seed=3, n=90, n_probes=2)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((p.n, 2))
    V = rng.standard_normal((p.n, 2))
    F = og.bilinear_forms(p.X, p.sigma2, p.lengthscales, p.lam, U, V, block=16)
    for i, dK in enumerate(og.derivative_matrices(p.X, p.sigma2, p.lengthscales, p.lam)):
        for c in range(2):
            assert np.isclose(F[c, i], U[:, c] @ dK @ V[:, c], rtol=1e-12, atol=1e-12)


def test_adagrad_first_step_is_sign():
    a = Adagrad(eta=0.7)
    theta = np.array([0.1, -0.2, 0.3])
    g = np.array([2.0, -1e-3, 5.0])
    out = a.step(theta, g)
    assert np.allclose(out - theta, 0.7 * np.sign(g), rtol=1e-4)
    out2 = a.step(out, g)
    assert np.allclose(out2 - out, 0.7 * g / np.sqrt(2 * g * g), rtol=1e-4)
