"""Parity of the FP64-class int8-digit product (PKM_I8X) against the FP64
oracle and against the oracle's model of its rounding points
(oracle/precision.int8_digit_product)."""
import numpy as np
import pytest

from gpu_util import GpuProblem, ctx, dev, host, rel_err  # noqa: F401
from oracle import kernel as ok
from oracle import precision as pr
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu

# Against the exact product: K in steps of 2^-30 sigma2 and V in steps of
# 2^-30 of each column's largest magnitude (rounded to nearest: half a step
# each), the dropped digit pairs (p + q < 2) add ~2^-36 per term; norm-wise
# that is ~2^-30 relative on these inputs (random-sign probe columns
# included), so 2^-26 leaves a factor 16.
TOL_EXACT = 2.0 ** -26
# Against the model of the same arithmetic: the GPU's FP64 exponent and exp2
# differ from the oracle's in the last bits only, so kint = rint(2^30 K) can
# differ by one where 2^30 K falls within a few 1e-7 of a half-integer (about
# one entry in a million), moving one output by 2^-30 |v_j|; the epilogue's
# FP64 sums differ in order.  1e-10 norm-wise, ten times below the model's
# own error against the exact product.
TOL_MODEL = 1e-10


def _model(p, V, shift):
    return pr.int8_digit_product(p.X, p.sigma2, p.lengthscales, V, shift=shift, min_class=2)


@pytest.mark.parametrize("n,k", [(1000, 1), (777, 17), (600, 33), (300, 34), (513, 64),
                                 (257, 7), (1000, 16), (1, 1), (40, 2), (2047, 3)])
def test_i8_product_against_oracle_and_model(ctx, n, k):
    p = make("mixed", seed=21, n=n, n_probes=max(k - 1, 0))
    g = GpuProblem(p)
    V = p.B[:, :k]
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, dev(V), pk.PKM_I8X))
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    assert np.all(rel_err(got, want) < TOL_EXACT), rel_err(got, want)
    model = _model(p, V, p.lam)
    assert np.all(rel_err(got, model) < TOL_MODEL), rel_err(got, model)


@pytest.mark.parametrize("d", [1, 4, 13, 16, 32])
def test_i8_product_dimensions(ctx, d):
    rng = np.random.default_rng(200 + d)
    n, k = 700, 9
    X = rng.standard_normal((n, d))
    ls = np.exp(rng.uniform(np.log(0.5 * np.sqrt(d)), np.log(2 * np.sqrt(d)), size=d))
    V = rng.standard_normal((n, k))
    prob = pk.Problem(dev(X), ls, 0.7, 1e-4)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), pk.PKM_I8X))
    want = ok.kernel_mvm(X, 0.7, ls, 1e-4, V)
    assert np.all(rel_err(got, want) < TOL_EXACT), rel_err(got, want)
    model = pr.int8_digit_product(X, 0.7, ls, V, shift=1e-4, min_class=2)
    assert np.all(rel_err(got, model) < TOL_MODEL)


@pytest.mark.parametrize("sigma2", [1e-6, 1.0, 3e5])
def test_i8_column_scales_and_signal_variance(ctx, sigma2):
    """Columns 1e-25 and 1e+25 in size, an all-zero column and a column with
    one nonzero entry: each column's power-of-two scale keeps the bound (the
    zero column stays exactly zero), at tiny and large sigma2."""
    p = make("mixed", seed=22, n=900, n_probes=5)
    g = GpuProblem(p)
    V = p.B.copy()
    V[:, 1] *= 1e-25
    V[:, 2] *= 1e25
    V[:, 3] = 0.0
    V[:, 4] = 0.0
    V[123, 4] = -7.5
    lam = 1e-4 * sigma2
    prob = pk.Problem(g.X, p.lengthscales, sigma2, lam)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), pk.PKM_I8X))
    want = ok.kernel_mvm(p.X, sigma2, p.lengthscales, lam, V)
    assert np.all(got[:, 3] == 0.0)
    keep = [0, 1, 2, 4, 5]
    err = rel_err(got[:, keep], want[:, keep])
    assert np.all(err < TOL_EXACT), err


def test_i8_kernel_column_entries(ctx):
    """V = e_j returns a column of K + lambda I: every entry within half a
    fixed-point step (2^-31 sigma2) plus FP64 rounding of the exact value."""
    p = make("mixed", seed=23, n=640, n_probes=0)
    g = GpuProblem(p)
    V = np.zeros((p.n, 2))
    V[17, 0] = 1.0
    V[600, 1] = -3.0
    got = host(pk.pkm_kernel_mvm_shift(ctx, g.prob, dev(V), 0.0, pk.PKM_I8X))
    K = ok.rbf_block(p.X, p.X[[17, 600]], p.sigma2, p.lengthscales)
    want = K * np.array([1.0, -3.0])
    err = np.abs(got - want) / (p.sigma2 * np.array([1.0, 3.0]))
    assert np.max(err) <= 2.0 ** -31 * (1 + 1e-6), np.max(err) * 2 ** 31


def test_i8_product_is_deterministic(ctx):
    p = make("mixed", seed=24, n=5000, n_probes=16)
    g = GpuProblem(p)
    a = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, pk.PKM_I8X))
    b = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, pk.PKM_I8X))
    assert np.array_equal(a, b)


def test_i8_mixed_workload_full_size_sampled_rows(ctx):
    """The 262,144-point, d = 16 workload with 1 + 32 right-hand sides in the
    launch shape its solves use (8 j-splits of 32,768 rows: the int32 range
    limit); 32 sampled rows recomputed by the oracle."""
    p = make("mixed", seed=0)
    g = GpuProblem(p)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, pk.PKM_I8X))
    rows = np.random.default_rng(8).choice(p.n, size=32, replace=False)
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows)
    assert rel_err(got[rows], want, axis=None) < TOL_EXACT


def test_i8_beyond_eight_splits_sampled_rows(ctx):
    """n = 300,000 > 8 x 32,768: the j range takes two launches whose partial
    planes the finishing pass adds; sampled rows against the oracle."""
    rng = np.random.default_rng(25)
    n, d = 300_000, 4
    X = rng.standard_normal((n, d))
    ls = np.full(d, 1.5)
    V = rng.standard_normal((n, 2))
    prob = pk.Problem(dev(X), ls, 1.0, 1e-4)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), pk.PKM_I8X))
    rows = np.concatenate([[0, n - 1], rng.choice(n, size=30, replace=False)])
    want = ok.kernel_mvm(X, 1.0, ls, 1e-4, V, rows=rows)
    assert rel_err(got[rows], want, axis=None) < TOL_EXACT


def test_i8_solve_certifies_small_lambda(ctx):
    """A 3,000-point problem of the 262,144-point recipe (d = 16, lambda =
    1e-4) solved with the int8-digit product inside PCG: every column
    certified by the FP64 true residual at 1e-8, without escalation, and the
    oracle's residual of the returned x agrees."""
    p = make("mixed", seed=26, n=3000, m=64, n_probes=4)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 64, idx=g.idx, jitter=1e-8)
    try:
        X, info = pk.pkm_solve(ctx, g.prob, g.B, pc=pc,
                               opts=pk.make_opts(tol=1e-8, prec=pk.PKM_I8X, reliable_every=-50))
    finally:
        pk.pkm_precond_destroy(pc)
    assert np.all(info.col_status == pk.PKM_COL_CONVERGED)
    assert info.prec_final == pk.PKM_I8X
    r = p.B - ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, host(X))
    tr = np.linalg.norm(r, axis=0) / np.linalg.norm(p.B, axis=0)
    assert np.all(tr <= 1.01e-8), tr


def test_i8_rejects_large_d(ctx):
    rng = np.random.default_rng(27)
    X = rng.random((50, 33))
    prob = pk.Problem(dev(X), np.ones(33), 1.0, 1e-3)
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_kernel_mvm(ctx, prob, dev(np.ones((50, 1))), pk.PKM_I8X)
    assert e.value.code == pk.PKM_ERR_INVALID
