"""Pins of the oracle's Cholesky solve and log-marginal likelihood (Section 2.1)."""
import math

import numpy as np
import pytest

from oracle import direct as od
from oracle import kernel as ok
from pkm_inputs import make


def test_lml_n1_closed_form():
    X = np.array([[0.3, 0.1]])
    for s2, lam, y in [(1.0, 0.01, 0.7), (2.5, 0.3, -1.2)]:
        v = s2 + lam
        want = -0.5 * math.log(v) - 0.5 * y * y / v - 0.5 * math.log(2 * math.pi)
        got = od.log_marginal_likelihood(X, s2, np.array([0.5, 0.5]), lam, np.array([y]))
        assert abs(got - want) < 1e-14


def test_lml_n2_closed_form():
    X = np.array([[0.0], [0.6]])
    s2, l, lam = 1.4, 0.8, 0.2
    y = np.array([0.9, -0.4])
    c = s2 * math.exp(-0.5 * 0.36 / 0.64)
    a = s2 + lam
    det = a * a - c * c
    quad = (a * y[0] ** 2 - 2 * c * y[0] * y[1] + a * y[1] ** 2) / det
    want = -0.5 * math.log(det) - 0.5 * quad - math.log(2 * math.pi)
    got = od.log_marginal_likelihood(X, s2, np.array([l]), lam, y)
    assert abs(got - want) < 1e-13


def test_solution_residual_through_independent_product():
    p = make("small_fp64", seed=0, n=512, n_probes=3)
    x = od.solve(p.X, p.sigma2, p.lengthscales, p.lam, p.B)
    r = p.B - ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, x)
    assert np.all(np.linalg.norm(r, axis=0) / np.linalg.norm(p.B, axis=0) < 1e-12)


def test_predict_closed_forms():
    """n = 1 closed form; interpolation at a training input with tiny noise;
    prior mean and variance far from the data."""
    import math
    from oracle import direct as od2
    x = np.array([[0.3, 0.1]])
    ls = np.array([0.5, 0.8])
    s2, lam, yv = 1.7, 0.2, 0.9
    xs = np.array([[0.5, -0.2]])
    k = s2 * math.exp(-0.5 * ((0.2 / 0.5) ** 2 + (0.3 / 0.8) ** 2))
    m, v = od2.predict(x, s2, ls, lam, np.array([yv]), xs)
    assert m[0] == pytest.approx(k * yv / (s2 + lam), rel=1e-13)
    assert v[0] == pytest.approx(s2 - k * k / (s2 + lam), rel=1e-13)
    rng = np.random.default_rng(7)
    X = rng.random((30, 2))
    y = np.sin(3 * X).sum(axis=1)
    m, v = od2.predict(X, 1.0, ls, 1e-10, y, X[:5])
    # m = y - lambda K_y^-1 y: off by lambda |alpha| (K_y is ill-conditioned)
    np.testing.assert_allclose(m, y[:5], rtol=0, atol=1e-5)
    assert np.all(np.abs(v) < 1e-5)
    m, v = od2.predict(X, 1.0, ls, 1e-2, y, X[:3] + 100.0)
    np.testing.assert_allclose(m, 0.0, atol=1e-12)
    np.testing.assert_allclose(v, 1.0, rtol=1e-12)
