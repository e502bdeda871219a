"""Pins of the oracle's Laplace approximation for probit GP classification."""
import numpy as np
import pytest
from scipy.linalg import hadamard
from scipy.special import log_ndtr

from oracle import laplace as ol
from oracle.kernel import kernel_matrix, rbf_block


def _data(n=32, d=2, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    y = np.where(np.sin(3 * X[:, 0]) + np.cos(2 * X[:, 1]) + 0.3 * rng.standard_normal(n) > 1.0,
                 1.0, -1.0)
    return X, y


def test_probit_derivatives_match_finite_differences():
    f = np.linspace(-8, 8, 41)
    h = 1e-5
    for y in (1.0, -1.0):
        yv = np.full_like(f, y)
        logp, d1, W, d3 = ol.probit_derivatives(yv, f)
        np.testing.assert_allclose(logp, log_ndtr(y * f), rtol=1e-14)
        fd1 = (log_ndtr(y * (f + h)) - log_ndtr(y * (f - h))) / (2 * h)
        np.testing.assert_allclose(d1, fd1, rtol=1e-6, atol=1e-9)
        fW = -(ol.probit_derivatives(yv, f + h)[1] - ol.probit_derivatives(yv, f - h)[1]) / (2 * h)
        np.testing.assert_allclose(W, fW, rtol=1e-6, atol=1e-9)
        fd3 = -(ol.probit_derivatives(yv, f + h)[2] - ol.probit_derivatives(yv, f - h)[2]) / (2 * h)
        np.testing.assert_allclose(d3, fd3, rtol=1e-5, atol=1e-8)
        assert np.all(W > 0)


def test_mode_is_the_fixed_point_and_maximiser():
    X, y = _data()
    K = kernel_matrix(X, 1.5, np.array([0.4, 0.6]))
    f, a, it = ol.mode(K, y)
    d1 = ol.probit_derivatives(y, f)[1]
    np.testing.assert_allclose(f, K @ d1, rtol=0, atol=1e-9)
    np.testing.assert_allclose(a, d1, rtol=0, atol=1e-9)
    Kj = K + 1e-10 * np.eye(len(y))
    psi = lambda g: log_ndtr(y * g).sum() - 0.5 * g @ np.linalg.solve(Kj, g)
    rng = np.random.default_rng(1)
    for _ in range(5):
        assert psi(f) >= psi(f + 1e-3 * rng.standard_normal(len(y))) - 1e-12
    assert it < 30


def test_stochastic_gradient_with_exact_traces_matches_finite_differences():
    """Sylvester-Hadamard probes (H H^T = n I) make every trace estimate in the
    three-term gradient exact, so it must equal central differences of the
    approximate log-marginal likelihood (this fixes the sign of dW/df)."""
    X, y = _data(n=32)
    s2, ls = 1.3, np.array([0.5, 0.7])
    K = kernel_matrix(X, s2, ls)
    f, _, _ = ol.mode(K, y, tol=1e-14)
    R = hadamard(32).astype(float)
    g = ol.stochastic_gradient(X, s2, ls, y, f, R)
    theta = np.concatenate([[np.log(s2)], np.log(ls)])
    h = 1e-5
    fd = []
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = ol.log_marginal(X, np.exp(tp[0]), np.exp(tp[1:]), y)
        lm = ol.log_marginal(X, np.exp(tm[0]), np.exp(tm[1:]), y)
        fd.append((lp - lm) / (2 * h))
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-7)


def test_prediction_matches_textbook_form():
    X, y = _data(n=40, seed=2)
    s2, ls = 1.0, np.array([0.3, 0.5])
    K = kernel_matrix(X, s2, ls)
    f, _, _ = ol.mode(K, y)
    Xs = np.random.default_rng(3).random((7, 2))
    m, v, p = ol.predict(X, s2, ls, y, f, Xs)
    _, d1, W, _ = ol.probit_derivatives(y, f)
    Ks = rbf_block(Xs, X, s2, ls)
    np.testing.assert_allclose(m, Ks @ d1, rtol=1e-12)
    vt = s2 - np.sum(Ks.T * np.linalg.solve(K + np.diag(1.0 / W), Ks.T), axis=0)
    np.testing.assert_allclose(v, vt, rtol=1e-9, atol=1e-12)
    assert np.all((p > 0) & (p < 1))
