"""Pins of the oracle's learned-factor MLP: backward, special cases, Adam."""
import numpy as np

from oracle import kernel as ok
from oracle import mlp
from oracle import precond as op


def _params(rng, d, h, r, scale=0.5):
    return {
        "W1": rng.standard_normal((d, h)) * scale, "b1": rng.standard_normal(h) * 0.1,
        "W2": rng.standard_normal((h, h)) * scale / np.sqrt(h), "b2": rng.standard_normal(h) * 0.1,
        "W3": rng.standard_normal((h, r)) * scale / np.sqrt(h), "b3": rng.standard_normal(r) * 0.1,
    }


def test_backward_vs_central_differences():
    rng = np.random.default_rng(0)
    n, d, h, r, nz = 30, 3, 7, 4, 5
    X = rng.random((n, d))
    Z = rng.choice([-1.0, 1.0], size=(n, nz))
    KZ = ok.kernel_matrix(X, 1.0, np.full(d, 0.6)) @ Z
    params = _params(rng, d, h, r)
    L, g = mlp.loss_and_grad(params, X, Z, KZ)
    eps = 1e-6
    for name in mlp.PARAM_NAMES:
        w = params[name]
        flat = w.reshape(-1)
        for t in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[t]
            flat[t] = old + eps
            lp = mlp.loss(mlp.forward(params, X)[0], Z, KZ)
            flat[t] = old - eps
            lm = mlp.loss(mlp.forward(params, X)[0], Z, KZ)
            flat[t] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].reshape(-1)[t]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, t, fd, an)


def test_gelu_grad_vs_differences():
    a = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(a), fd, atol=1e-8)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0


def test_zero_network_gives_lambda_identity():
    rng = np.random.default_rng(1)
    d, h, r = 3, 5, 4
    params = {k: np.zeros_like(v) for k, v in _params(rng, d, h, r).items()}
    X = rng.random((20, d))
    U, _ = mlp.forward(params, X)
    assert np.all(U == 0)
    P = op.lowrank(U, 0.25)
    R = rng.standard_normal((20, 2))
    assert np.allclose(P(R), R / 0.25, rtol=1e-15)


def test_exact_factor_has_zero_loss():
    rng = np.random.default_rng(2)
    X = rng.random((25, 2))
    K = ok.kernel_matrix(X, 1.0, np.array([0.2, 0.3])) + 1e-9 * np.eye(25)
    L = np.linalg.cholesky(K)
    Z = rng.choice([-1.0, 1.0], size=(25, 6))
    assert mlp.loss(L, Z, K @ Z) < 1e-24


def test_adam_first_step_is_lr_sign():
    rng = np.random.default_rng(3)
    params = _params(rng, 2, 3, 2)
    grads = {k: rng.standard_normal(v.shape) for k, v in params.items()}
    opt = mlp.Adam(params, lr=1e-2)
    new = opt.step(params, grads)
    for k in params:
        assert np.allclose(new[k] - params[k], -1e-2 * np.sign(grads[k]), rtol=1e-5)


def test_round_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between bf16 neighbours 1 and 1 + 2^-7: ties go to even (1).
    assert mlp.round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even (1 + 2^-6).
    assert mlp.round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    assert mlp.round_bf16(np.array([3.0]))[0] == 3.0
