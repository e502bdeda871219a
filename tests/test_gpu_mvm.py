"""Parity of the HIP kernel product (K + lambda I) V against the FP64 oracle."""
import numpy as np
import pytest

from gpu_util import GpuProblem, ctx, dev, host, rel_err  # noqa: F401
from oracle import kernel as ok
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu

# FP64: the GPU's augmented FP64 contraction leaves each base-2 exponent with
# an absolute error of a few 2^-53 (|a_i| + |b_j|) (|xh|^2 <= ~40 after
# centring), i.e. ~1e-14 relative per entry; its exp2 adds a few ulp and the
# sums differ from the oracle's only in order: 1e-13 norm-wise.
TOL64 = 1e-13
# FP32: each entry's base-2 exponent carries about 2^-24 (|a_i| + |b_j|) absolute
# error from the FP32 contraction (|xh|^2 <= ~40 after centring), exp2 adds ~2
# ulp, and the FP32 sum over n terms adds ~2^-24 sqrt(n) relative: < 1e-5 norm-wise.
TOL32 = 1e-5


@pytest.mark.parametrize("n,k", [(1000, 1), (1000, 3), (777, 17), (300, 33), (1, 2), (17, 5)])
def test_fp64_product(ctx, n, k):
    p = make("block_fp32", seed=11, n=n, n_probes=max(k - 1, 0))
    g = GpuProblem(p)
    V = p.B[:, :k]
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, dev(V), pk.PKM_FP64))
    assert np.all(rel_err(got, want) < TOL64), rel_err(got, want)


@pytest.mark.parametrize("n,k", [(1000, 1), (1000, 16), (777, 17), (600, 33), (513, 64),
                                 (300, 65), (1, 1), (40, 2), (257, 7)])
def test_fp32_product(ctx, n, k):
    p = make("block_fp32", seed=12, n=n, n_probes=max(k - 1, 0))
    g = GpuProblem(p)
    V = p.B[:, :k]
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, dev(V), pk.PKM_FP32))
    err = rel_err(got, want)
    assert np.all(err < TOL32), err


@pytest.mark.parametrize("d", [1, 4, 16, 32, 34])
def test_fp32_product_dimensions(ctx, d):
    rng = np.random.default_rng(d)
    n, k = 700, 9
    X = rng.random((n, d))
    ls = np.exp(rng.uniform(np.log(0.2 * np.sqrt(d)), np.log(np.sqrt(d)), size=d))
    V = rng.standard_normal((n, k))
    Xd = dev(X)
    prob = pk.Problem(Xd, ls, 1.3, 3e-3)
    want = ok.kernel_mvm(X, 1.3, ls, 3e-3, V)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), pk.PKM_FP32))
    assert np.all(rel_err(got, want) < TOL32)
    got64 = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), pk.PKM_FP64))
    assert np.all(rel_err(got64, want) < TOL64)


def test_fp32_product_full_size_sampled_rows(ctx):
    """The 65,536-point block workload in the launch shape the solver uses;
    64 sampled output rows recomputed by the oracle."""
    p = make("block_fp32", seed=0)
    g = GpuProblem(p)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, pk.PKM_FP32))
    rows = np.random.default_rng(5).choice(p.n, size=64, replace=False)
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows)
    assert rel_err(got[rows], want, axis=None) < TOL32


@pytest.mark.parametrize("prec", [pk.PKM_FP32, pk.PKM_F16X3])
def test_product_is_deterministic(ctx, prec):
    p = make("block_fp32", seed=13, n=5000, n_probes=16)
    g = GpuProblem(p)
    a = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, prec))
    b = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, prec))
    assert np.array_equal(a, b)


def test_invalid_arguments_rejected(ctx):
    p = make("block_fp32", seed=14, n=100, n_probes=0)
    g = GpuProblem(p)
    bad = pk.Problem(g.X, p.lengthscales, p.sigma2, -1.0)
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_kernel_mvm(ctx, bad, g.B, pk.PKM_FP32)
    assert e.value.code == pk.PKM_ERR_INVALID
    ls = p.lengthscales.copy()
    ls[2] = 0.0
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_kernel_mvm(ctx, pk.Problem(g.X, ls, p.sigma2, p.lam), g.B, pk.PKM_FP32)
    assert e.value.code == pk.PKM_ERR_INVALID


# 16-bit products.  Exponents keep FP32-class accuracy (exact 3-part splits);
# K and V are rounded to BF16: relative 2^-9 per entry (split 1), or carried
# as two parts with ~2^-17 relative error (split 3); FP16 parts of K / sigma2
# and of the power-of-two-scaled V columns carry ~2^-22, so the FP32-class
# exponent dominates as in the FP32 product.  Norm-wise bounds with margin for
# the random-sign probe columns: 1e-2, 1e-4 and the FP32 bound.
@pytest.mark.parametrize("prec,tol", [(pk.PKM_BF16X1, 1e-2), (pk.PKM_BF16X3, 1e-4),
                                      (pk.PKM_F16X3, TOL32)])
@pytest.mark.parametrize("n,k", [(1000, 1), (777, 17), (600, 33), (513, 64), (300, 65), (1, 1),
                                 (40, 2), (257, 7), (400, 81), (333, 100), (300, 129), (260, 144),
                                 (200, 145), (150, 300)])
def test_bf16_product(ctx, prec, tol, n, k):
    p = make("block_fp32", seed=15, n=n, n_probes=max(k - 1, 0))
    g = GpuProblem(p)
    V = p.B[:, :k]
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, dev(V), prec))
    err = rel_err(got, want)
    assert np.all(err < tol), err


@pytest.mark.parametrize("prec,tol", [(pk.PKM_BF16X3, 1e-4), (pk.PKM_F16X3, TOL32)])
@pytest.mark.parametrize("d", [1, 4, 16, 32, 36])
def test_16bit_product_dimensions(ctx, d, prec, tol):
    rng = np.random.default_rng(100 + d)
    n, k = 700, 9
    X = rng.random((n, d))
    ls = np.exp(rng.uniform(np.log(0.2 * np.sqrt(d)), np.log(np.sqrt(d)), size=d))
    V = rng.standard_normal((n, k))
    prob = pk.Problem(dev(X), ls, 0.7, 1e-3)
    want = ok.kernel_mvm(X, 0.7, ls, 1e-3, V)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), prec))
    assert np.all(rel_err(got, want) < tol)


@pytest.mark.parametrize("prec,tol", [(pk.PKM_BF16X3, 1e-4), (pk.PKM_F16X3, TOL32)])
@pytest.mark.parametrize("d,k", [(8, 112), (36, 112), (8, 137), (36, 137)])
def test_16bit_product_wide_blocks(ctx, d, k, prec, tol):
    """k = 112 (one pass of seven 16-column tiles) and k = 137 (two passes),
    at the smallest and the largest exponent-slice count, with columns of
    very different scales."""
    rng = np.random.default_rng(200 + d + k)
    n = 900
    X = rng.random((n, d))
    ls = np.exp(rng.uniform(np.log(0.2 * np.sqrt(d)), np.log(np.sqrt(d)), size=d))
    V = rng.standard_normal((n, k)) * np.exp(rng.uniform(-3, 3, size=k))
    prob = pk.Problem(dev(X), ls, 1.3, 1e-3)
    want = ok.kernel_mvm(X, 1.3, ls, 1e-3, V)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), prec))
    assert np.all(rel_err(got, want) < tol)


@pytest.mark.parametrize("sigma2", [1e-6, 1.0, 3e5])
def test_f16x3_column_scales_and_signal_variance(ctx, sigma2):
    """FP16 parts need K / sigma2 (in (0, 1]) and power-of-two column scales:
    columns 1e-25 and 1e+25 in size, an all-zero column and a column with one
    nonzero entry all keep the FP32-class bound, at tiny and large sigma2
    (where K itself would leave FP16's range); the zero column stays zero."""
    p = make("block_fp32", seed=18, n=900, n_probes=5)
    g = GpuProblem(p)
    V = p.B.copy()
    V[:, 1] *= 1e-25
    V[:, 2] *= 1e25
    V[:, 3] = 0.0
    V[:, 4] = 0.0
    V[123, 4] = -7.5
    lam = 1e-3 * sigma2
    prob = pk.Problem(g.X, p.lengthscales, sigma2, lam)
    want = ok.kernel_mvm(p.X, sigma2, p.lengthscales, lam, V)
    got = host(pk.pkm_kernel_mvm(ctx, prob, dev(V), pk.PKM_F16X3))
    assert np.all(got[:, 3] == 0.0)
    keep = [0, 1, 2, 4, 5]
    err = rel_err(got[:, keep], want[:, keep])
    assert np.all(err < TOL32), err


def test_bf16_exponent_matches_fp32_path(ctx):
    """With V = e_j the product returns a kernel column; BF16X3 and FP32 share
    the exponent's accuracy, so the column entries agree to ~2^-16 relative."""
    p = make("block_fp32", seed=16, n=640, n_probes=0)
    g = GpuProblem(p)
    V = np.zeros((p.n, 2))
    V[17, 0] = 1.0
    V[600, 1] = 1.0
    a = host(pk.pkm_kernel_mvm(ctx, g.prob, dev(V), pk.PKM_BF16X3))
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    big = np.abs(want) > 1e-3
    assert np.max(np.abs(a - want)[big] / np.abs(want)[big]) < 2e-5


@pytest.mark.parametrize("prec,tol", [(pk.PKM_BF16X3, 1e-4), (pk.PKM_F16X3, TOL32)])
def test_16bit_full_size_sampled_rows(ctx, prec, tol):
    p = make("block_fp32", seed=0)
    g = GpuProblem(p)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, prec))
    rows = np.random.default_rng(6).choice(p.n, size=64, replace=False)
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows)
    assert rel_err(got[rows], want, axis=None) < tol


@pytest.mark.parametrize("prec,tol", [(pk.PKM_FP64, TOL64), (pk.PKM_FP32, TOL32),
                                      (pk.PKM_BF16X3, 1e-4), (pk.PKM_F16X3, TOL32)])
def test_mixed_workload_full_size_sampled_rows(ctx, prec, tol):
    """The 262,144-point, d = 16 workload with its 1 + 32 right-hand sides, in
    the launch shape its solves use; 32 sampled output rows recomputed by the
    oracle (FP64 product: about 0.15 s per launch)."""
    p = make("mixed", seed=0)
    g = GpuProblem(p)
    got = host(pk.pkm_kernel_mvm(ctx, g.prob, g.B, prec))
    rows = np.random.default_rng(7).choice(p.n, size=32, replace=False)
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows)
    assert rel_err(got[rows], want, axis=None) < tol


@pytest.mark.parametrize("prec,tol", [(pk.PKM_FP64, TOL64), (pk.PKM_FP32, TOL32)])
def test_shifted_product_zero_shift_is_plain_K(ctx, prec, tol):
    p = make("block_fp32", seed=17, n=900, n_probes=6)
    g = GpuProblem(p)
    want = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, 0.0, p.B)
    got = host(pk.pkm_kernel_mvm_shift(ctx, g.prob, g.B, 0.0, prec))
    assert np.all(rel_err(got, want) < tol)
    want2 = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, 0.25, p.B)
    got2 = host(pk.pkm_kernel_mvm_shift(ctx, g.prob, g.B, 0.25, prec))
    assert np.all(rel_err(got2, want2) < tol)
