"""Parity of the HIP gradient pass (Eq. (2) with the probe trace estimate)."""
import numpy as np
import pytest

from gpu_util import GpuProblem, ctx, dev, host  # noqa: F401
from oracle import direct as od
from oracle import gradient as og
from oracle import precond as op  # noqa: F401
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,N,d", [(600, 4, 8), (257, 16, 3), (400, 1, 16), (300, 20, 32),
                                   (5000, 16, 8), (700, 40, 5), (300, 3, 1), (300, 3, 10),
                                   (300, 3, 12), (300, 3, 18), (300, 3, 20), (300, 3, 24),
                                   (300, 3, 26), (300, 3, 28), (1, 2, 4), (17, 1, 6)])
def test_grad_pass_matches_oracle_on_same_solutions(ctx, n, N, d):
    rng = np.random.default_rng(n + N)
    X = rng.random((n, d))
    ls = np.exp(rng.uniform(np.log(0.2 * np.sqrt(d)), np.log(np.sqrt(d)), size=d))
    s2, lam = 1.2, 5e-3
    y = rng.standard_normal(n)
    Z = rng.choice([-1.0, 1.0], size=(n, N))
    alpha = od.solve(X, s2, ls, lam, y)
    S = od.solve(X, s2, ls, lam, Z)
    want = og.hutchinson_gradient(X, s2, ls, lam, alpha, S, Z)
    scale = og.hutchinson_terms(X, s2, ls, lam, alpha, S, Z)
    AS = np.concatenate([alpha[:, None], S], axis=1)
    YZ = np.concatenate([alpha[:, None], Z], axis=1)
    prob = pk.Problem(dev(X), ls, s2, lam)
    got = pk.pkm_grad_pass(ctx, prob, N, dev(AS), dev(YZ))
    # FP64 on both sides; different summation order only
    assert np.all(np.abs(got - want) <= 1e-10 * scale + 1e-12), (got, want)


def test_lml_grad_end_to_end(ctx):
    p = make("block_fp32", seed=7, n=2000, m=80, n_probes=8)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, len(p.idx), idx=g.idx, jitter=1e-8)
    sol = dev(np.zeros((p.n, 9)))
    try:
        grad, info = pk.pkm_lml_grad(ctx, g.prob, dev(p.y), dev(p.Z), pc=pc,
                                     opts=pk.make_opts(tol=1e-8, prec=pk.PKM_FP32), sol=sol)
    finally:
        pk.pkm_precond_destroy(pc)
    alpha = od.solve(p.X, p.sigma2, p.lengthscales, p.lam, p.y)
    S = od.solve(p.X, p.sigma2, p.lengthscales, p.lam, p.Z)
    want = og.hutchinson_gradient(p.X, p.sigma2, p.lengthscales, p.lam, alpha, S, p.Z)
    scale = og.hutchinson_terms(p.X, p.sigma2, p.lengthscales, p.lam, alpha, S, p.Z)
    # solutions certified to 1e-8 true residual; kappa ~ 1/lambda amplifies to
    # <~1e-5 relative error in s_c, which bounds the gradient error per term
    assert np.all(np.abs(grad - want) <= 1e-4 * scale), (grad, want, scale)
    assert np.all(info.col_status == pk.PKM_COL_CONVERGED)
