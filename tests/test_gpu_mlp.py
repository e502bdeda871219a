"""Parity of the learned-factor network kernels against the FP64 oracle (same
BF16 rounding of weights and products' inputs), and its use as a preconditioner."""
import numpy as np
import pytest

from gpu_util import ctx, dev, host, rel_err  # noqa: F401
from oracle import kernel as ok
from oracle import mlp as om
from oracle.pcg import pcg
from oracle import precond as op
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make, mlp_params, rademacher

pytestmark = pytest.mark.gpu
HID = 128


def _setup(n, d, r, seed, nz=16):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    ls = np.full(d, 0.5)
    params = mlp_params(seed, d_in=d, hidden=HID, rank=r)
    # the library keeps FP32 master weights: give the oracle the same values
    params = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    params["b1"] = rng.standard_normal(HID).astype(np.float32).astype(np.float64) * 0.1
    Xs = X / ls
    Z = rademacher(rng, n, nz)
    KZ = ok.rbf_block(X, X, 1.0, ls) @ Z
    return X, ls, Xs, params, Z, KZ


@pytest.mark.parametrize("n,d,r", [(300, 8, 128), (77, 3, 48), (513, 16, 16)])
def test_forward_matches_oracle(ctx, n, d, r):
    X, ls, Xs, params, _, _ = _setup(n, d, r, seed=n)
    prob = pk.Problem(dev(X), ls, 1.0, 1e-3)
    net = pk.pkm_mlp_create(ctx, params, d, HID, r)
    try:
        U = host(pk.pkm_mlp_forward(ctx, net, prob, r))
    finally:
        pk.pkm_mlp_destroy(net)
    want, _ = om.forward(params, Xs, bf16=True)
    # FP32 accumulation vs FP64, plus occasional flips of a BF16 rounding of
    # hidden activations: well below 2e-3 norm-wise
    assert rel_err(U, want, axis=None) < 2e-3


def test_loss_and_gradient_match_oracle(ctx):
    n, d, r = 256, 8, 64
    X, ls, Xs, params, Z, KZ = _setup(n, d, r, seed=3)
    prob = pk.Problem(dev(X), ls, 1.0, 1e-3)
    net = pk.pkm_mlp_create(ctx, params, d, HID, r)
    try:
        L, g = pk.pkm_mlp_loss_grad(ctx, net, prob, dev(Z), dev(KZ), d, HID, r)
    finally:
        pk.pkm_mlp_destroy(net)
    Lo, go = om.loss_and_grad(params, Xs, Z, KZ, bf16=True)
    assert abs(L - Lo) <= 1e-3 * Lo
    for k in om.PARAM_NAMES:
        assert rel_err(g[k], go[k], axis=None) < 1e-2, k


def test_adam_step_and_training_progress(ctx):
    n, d, r = 512, 8, 32
    X, ls, Xs, params, Z, KZ = _setup(n, d, r, seed=4)
    prob = pk.Problem(dev(X), ls, 1.0, 1e-3)
    net = pk.pkm_mlp_create(ctx, params, d, HID, r)
    try:
        L0 = pk.pkm_mlp_train_step(ctx, net, prob, dev(Z), dev(KZ), 1e-3)
        p1 = pk.pkm_mlp_params(ctx, net, d, HID, r)
        _, go = om.loss_and_grad(params, Xs, Z, KZ, bf16=True)
        # first Adam step: every weight with a clear gradient moves by lr * sign(g)
        for k in om.PARAM_NAMES:
            delta = p1[k] - params[k]
            big = np.abs(go[k]) > 1e-3 * np.abs(go[k]).max()
            if big.any():
                agree = np.mean(np.sign(delta[big]) == -np.sign(go[k][big]))
                assert agree > 0.99, k
                assert np.allclose(np.abs(delta[big]), 1e-3, rtol=2e-2), k
        losses = [L0]
        for _ in range(60):
            losses.append(pk.pkm_mlp_train_step(ctx, net, prob, dev(Z), dev(KZ), 3e-3))
    finally:
        pk.pkm_mlp_destroy(net)
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_learned_factor_reduces_pcg_steps(ctx):
    """Train on K Z probe pairs, then precondition with the Nystrom factor of
    the learned sketch, P = K U (U^T K U)^-1 U^T K + lambda I: fewer CG steps
    than without a preconditioner, and the solution still meets the FP64
    tolerance (P only changes the path, not the answer)."""
    p = make("learned", seed=1, n=2048, n_probes=2)
    d, r = p.d, 64
    prob_np = p
    X = dev(p.X)
    prob = pk.Problem(X, p.lengthscales, p.sigma2, p.lam)
    rng = np.random.default_rng(9)
    Zt = rademacher(rng, p.n, 64)
    KZ = ok.rbf_block(p.X, p.X, p.sigma2, p.lengthscales) @ Zt
    net = pk.pkm_mlp_create(ctx, mlp_params(5, d_in=d, hidden=HID, rank=r), d, HID, r)
    try:
        for _ in range(150):
            pk.pkm_mlp_train_step(ctx, net, prob, dev(Zt), dev(KZ), 3e-3)
        U = pk.pkm_mlp_forward(ctx, net, prob, r)
    finally:
        pk.pkm_mlp_destroy(net)
    pc = pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_SKETCH, r, Phi=U, jitter=1e-8)
    try:
        Xl, il = pk.pkm_solve(ctx, prob, dev(p.B), pc=pc,
                              opts=pk.make_opts(tol=1e-6, prec=pk.PKM_FP64, max_iter=20000))
    finally:
        pk.pkm_precond_destroy(pc)
    Xc, ic = pk.pkm_solve(ctx, prob, dev(p.B), opts=pk.make_opts(tol=1e-6, prec=pk.PKM_FP64,
                                                                   max_iter=20000))
    assert np.all(il.col_status == pk.PKM_COL_CONVERGED)
    # The learned/plain step ratio of this recipe, measured over seeds 1-8
    # (network seed 5 + s - 1): 0.501, 0.633, 0.528, 0.502, 0.506, 0.601,
    # 0.589, 0.483 (mean 0.54); this test's seed 1 gives 0.501 (836 / 1669).
    # The bound is the largest of the eight, rounded up: 0.65.  Against
    # Nystrom of equal rank (m = 64) the same factor ranged 0.84-1.04, so it
    # is not asserted to beat it (the hybrid test in test_gpu_learned.py does
    # assert that against a rank-matched control).
    assert il.iters.max() < 0.65 * ic.iters.max(), (il.iters, ic.iters)
    r_true = p.B - ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, host(Xl))
    assert np.all(np.linalg.norm(r_true, axis=0) / np.linalg.norm(p.B, axis=0) <= 1e-6)
