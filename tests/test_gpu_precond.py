"""Parity of the HIP Nystrom / FITC / factor preconditioners against the oracle."""
import numpy as np
import pytest

from gpu_util import GpuProblem, ctx, dev, host, rel_err  # noqa: F401
from oracle import precond as op
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu

JIT = 1e-8
# FP64 setup on both sides, factorised differently (the oracle solves the
# lambda K_UU + K_UX K_XU core directly, the library goes through the Cholesky
# factor of K_UU + jitter I).  The two setups differ by about u cond(K_UU)
# relative (FITC's diag(K - Q) cancels to that absolute level), and P^-1
# amplifies a relative change of P by up to cond(P): bound 64 u cond(K_UU)
# cond(P), floored at 1e-11.
TOL = 1e-9


def _tol(P):
    c = np.linalg.cond(P.info["Kuu"]) * np.linalg.cond(P.dense())
    return max(1e-11, 64 * 2.2e-16 * c)


@pytest.mark.parametrize("kind,n,m", [(pk.PKM_PC_NYSTROM, 700, 64), (pk.PKM_PC_NYSTROM, 1000, 130),
                                      (pk.PKM_PC_FITC, 700, 64), (pk.PKM_PC_FITC, 333, 200),
                                      (pk.PKM_PC_NYSTROM, 50, 1)])
def test_apply_matches_oracle(ctx, kind, n, m):
    p = make("block_fp32", seed=21, n=n, m=m, n_probes=4)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, kind, m, idx=g.idx, jitter=JIT)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        make_o = op.nystrom if kind == pk.PKM_PC_NYSTROM else op.fitc
        P = make_o(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=JIT)
        want = P(p.B)
        assert np.all(rel_err(got, want) < _tol(P)), (rel_err(got, want), _tol(P))
        D = pk.pkm_precond_diag(ctx, pc, n)
        if kind == pk.PKM_PC_FITC:
            assert np.allclose(D, P.info["D"], rtol=1e-9, atol=1e-12)
            assert np.allclose(D[p.idx], p.lam, rtol=0, atol=1e-7)
        else:
            assert np.all(D == p.lam)
    finally:
        pk.pkm_precond_destroy(pc)


def test_lowrank_apply_matches_oracle(ctx):
    rng = np.random.default_rng(3)
    n, r, lam = 900, 70, 1e-3
    Phi = rng.standard_normal((n, r)) * 0.3
    p = make("block_fp32", seed=22, n=n, n_probes=5)
    g = GpuProblem(p)
    prob = pk.Problem(g.X, p.lengthscales, p.sigma2, lam)
    pc = pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_LOWRANK, r, Phi=dev(Phi))
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        want = op.lowrank(Phi, lam)(p.B)
        assert np.all(rel_err(got, want) < TOL)
    finally:
        pk.pkm_precond_destroy(pc)


def test_zero_factor_is_lambda_identity(ctx):
    p = make("block_fp32", seed=23, n=200, n_probes=2)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_LOWRANK, 8, Phi=dev(np.zeros((200, 8))))
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        assert np.allclose(got, p.B / p.lam, rtol=1e-15, atol=0)
    finally:
        pk.pkm_precond_destroy(pc)


def test_duplicate_inducing_points_without_jitter_is_breakdown(ctx):
    p = make("block_fp32", seed=24, n=100, n_probes=0)
    g = GpuProblem(p)
    idx = dev(np.array([3, 3, 7], np.int32))
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 3, idx=idx, jitter=0.0)
    assert e.value.code == pk.PKM_ERR_BREAKDOWN


def test_out_of_range_index_is_invalid(ctx):
    p = make("block_fp32", seed=25, n=100, n_probes=0)
    g = GpuProblem(p)
    idx = dev(np.array([3, 100], np.int32))
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 2, idx=idx, jitter=JIT)
    assert e.value.code == pk.PKM_ERR_INVALID


@pytest.mark.parametrize("n,m", [(700, 48), (333, 20)])
def test_sketch_apply_matches_oracle(ctx, n, m):
    rng = np.random.default_rng(n)
    p = make("block_fp32", seed=26, n=n, n_probes=3)
    S = rng.standard_normal((n, m))
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_SKETCH, m, Phi=dev(S), jitter=1e-10)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
    finally:
        pk.pkm_precond_destroy(pc)
    P = op.sketch(p.X, p.sigma2, p.lengthscales, p.lam, S, jitter=1e-10)
    want = P(p.B)
    # K S comes from the FP32 product (relative error <= 1e-5): the factor and
    # hence P^-1 inherit that level, amplified by at most cond(P)
    tol = 1e-5 * np.linalg.cond(P.dense()) ** 0.5
    assert np.all(rel_err(got, want) < tol), (rel_err(got, want), tol)
