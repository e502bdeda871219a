"""Prediction at test inputs: the cross-kernel product and the predictive
mean and variance (one PCG solve per test point) against the oracle."""
import numpy as np
import pytest

from gpu_util import GpuProblem, ctx, dev, host  # noqa: F401
from oracle import direct as od
from oracle import kernel as ok
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,ns,k,d", [(700, 130, 3, 8), (257, 1, 1, 4), (1000, 300, 17, 16),
                                      (333, 77, 5, 32)])
def test_cross_product_matches_oracle(ctx, n, ns, k, d):
    rng = np.random.default_rng(n + ns)
    X = rng.random((n, d))
    Xs = rng.random((ns, d)) * 1.2 - 0.1
    ls = np.exp(rng.uniform(np.log(0.3), np.log(1.5), size=d))
    V = rng.standard_normal((n, k))
    prob = pk.Problem(dev(X), ls, 1.4, 1e-3)
    got = host(pk.pkm_cross_mvm(ctx, prob, dev(Xs), dev(V)))
    want = ok.rbf_block(Xs, X, 1.4, ls) @ V
    err = np.linalg.norm(got - want, axis=0) / np.linalg.norm(want, axis=0)
    assert np.all(err < 1e-13), err


def test_predict_mean_and_variance_match_cholesky(ctx):
    p = make("block_fp32", seed=51, n=1500, m=64, n_probes=0)
    g = GpuProblem(p)
    Xs = np.random.default_rng(52).random((40, p.d))
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 64, idx=g.idx, jitter=1e-8)
    try:
        mean, var, im, iv = pk.pkm_predict(ctx, g.prob, dev(p.y), dev(Xs), pc=pc,
                                           opts=pk.make_opts(tol=1e-10, prec=pk.PKM_FP64))
    finally:
        pk.pkm_precond_destroy(pc)
    wm, wv = od.predict(p.X, p.sigma2, p.lengthscales, p.lam, p.y, Xs)
    assert np.all(im.col_status == pk.PKM_COL_CONVERGED)
    assert np.all(iv.col_status == pk.PKM_COL_CONVERGED)
    # solves to 1e-10 relative residual; K_y^-1 amplifies by at most 1/lambda
    # relative to |b|, and the mean/variance are bilinear forms of the solution
    scale_m = np.abs(ok.rbf_block(Xs, p.X, p.sigma2, p.lengthscales)).sum(axis=1).max()
    tol_m = 1e-10 / p.lam * np.linalg.norm(p.y) * scale_m / np.sqrt(p.n) + 1e-12
    np.testing.assert_allclose(host(mean), wm, rtol=0, atol=tol_m)
    np.testing.assert_allclose(host(var), wv, rtol=0, atol=1e-7 * p.sigma2)
    assert np.all(host(var) > -1e-9) and np.all(host(var) <= p.sigma2 + 1e-12)


def test_predict_mean_only_many_points(ctx):
    p = make("small_fp64", seed=53, n=800, n_probes=0)
    g = GpuProblem(p)
    Xs = np.random.default_rng(54).random((1000, p.d))
    mean, var, im, iv = pk.pkm_predict(ctx, g.prob, dev(p.y), dev(Xs), variance=False,
                                       opts=pk.make_opts(tol=1e-12, prec=pk.PKM_FP64))
    assert var is None and iv is None
    wm, _ = od.predict(p.X, p.sigma2, p.lengthscales, p.lam, p.y, Xs[:5])
    np.testing.assert_allclose(host(mean)[:5], wm, rtol=1e-8, atol=1e-9)


def test_predict_rejects_too_many_variance_points(ctx):
    p = make("small_fp64", seed=55, n=300, n_probes=0)
    g = GpuProblem(p)
    Xs = dev(np.zeros((257, p.d)))
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_predict(ctx, g.prob, dev(p.y), Xs)
    assert e.value.code == pk.PKM_ERR_INVALID
