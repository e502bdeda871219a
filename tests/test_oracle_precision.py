"""Pins of the precision emulator (oracle/precision.py): closed forms for the
rounding and contraction helpers, then the numerical-feasibility facts the
solver's precision policy rests on, reproduced at small n."""
import numpy as np
import pytest

from oracle import precision as pr
from oracle.kernel import kernel_matrix


def test_round_fp32_ties_to_even():
    u = 2.0 ** -24
    assert pr.round_fp32(np.array([1.0 + u]))[0] == 1.0            # tie -> even
    assert pr.round_fp32(np.array([1.0 + 3 * u]))[0] == 1.0 + 4 * u  # tie -> even (up)
    assert pr.round_fp32(np.array([1.0 + 1.5 * u]))[0] == 1.0 + 2 * u
    assert pr.round_fp32(np.array([0.5]))[0] == 0.5


def test_fp16_split_of_one_third_by_hand():
    """binary16 keeps 11 significant bits: 1/3 = 1.0101010101...b x 2^-2
    rounds down to 1365/4096; the remainder 1/(3 * 4096) = (1/3) 2^-12 lies in
    the normal range (>= 2^-14) and rounds the same way to 1365 / 2^24; the
    pair then misses 1/3 by exactly 1 / (3 * 2^24)."""
    h, l = pr.split_fp16(np.array([1.0 / 3.0]))
    assert h[0] == 1365 / 4096
    assert l[0] == 1365 / 2.0 ** 24
    assert 1.0 / 3.0 - (h[0] + l[0]) == pytest.approx(1.0 / (3 * 2.0 ** 24), rel=1e-9)


def test_round_fp16_format_limits():
    assert pr.round_fp16(np.array([65504.0]))[0] == 65504.0            # largest finite
    assert np.isinf(pr.round_fp16(np.array([65520.0]))[0])             # rounds past it
    assert pr.round_fp16(np.array([2.0 ** -24]))[0] == 2.0 ** -24      # smallest subnormal
    assert pr.round_fp16(np.array([2.0 ** -26]))[0] == 0.0             # below half of it
    assert pr.round_fp16(np.array([1.0 + 2.0 ** -11]))[0] == 1.0       # tie -> even
    assert pr.round_fp16(np.array([1.0 + 3 * 2.0 ** -11]))[0] == 1.0 + 2.0 ** -9


def test_fp16_split_error_bound_on_kernel_entries():
    """Entry-wise bound of the two-part FP16 split of K / sigma2 in (0, 1]:
    max(2^-23 K, 2^-25) (relative 2^-11 per part where normal, half the
    2^-24 subnormal spacing below).  Dropping the low part would leave
    2^-12 relative; a BF16 split leaves ~2^-17."""
    rng = np.random.default_rng(3)
    X = rng.random((300, 4))
    K = kernel_matrix(X, 1.0, np.full(4, 0.3))
    assert K.min() < 2.0 ** -14 < K.max()          # spans the subnormal range
    h, l = pr.split_fp16(K)
    err = np.abs(h + l - K)
    assert np.all(err <= np.maximum(2.0 ** -23 * K, 2.0 ** -25))
    assert np.max(np.abs(h - K) / K) > 2.0 ** -13  # the low part is needed
    bf = pr.perturbed_kernel(X, 1.0, np.full(4, 0.3), "bf16x2")
    assert np.max(np.abs(bf - K)) > 8 * np.max(err)


def test_fp16_split_scales_with_sigma2():
    rng = np.random.default_rng(4)
    X = rng.random((120, 3))
    ls = np.full(3, 0.4)
    K1 = pr.perturbed_kernel(X, 1.0, ls, "f16x2")
    K2 = pr.perturbed_kernel(X, 3.0e5, ls, "f16x2")
    np.testing.assert_allclose(K2, 3.0e5 * K1, rtol=1e-15, atol=0)


def test_rho_closed_form():
    K = np.diag([1.0, 2.0, 3.0])
    eps, lam = 1e-3, 1e-2
    Kh = K + np.diag([eps, -2 * eps, 0.0])
    assert pr.rho(Kh, K, lam) == pytest.approx(2 * eps / lam, rel=1e-12)


@pytest.mark.parametrize("c", [0.3, -0.2, -0.75])
def test_refinement_contraction_closed_form(c):
    """1x1 system: the error shrinks by c / (mu + lam + c) per refinement
    step, so |r_t| / |b| = |c / (mu + lam + c)|^t (divergent for c = -0.75)."""
    mu, lam = 1.0, 0.0
    K = np.array([[mu]])
    Kh = K + c * (mu + lam)
    hist = pr.refine(Kh, K, lam, np.array([2.0]), steps=5)
    q = abs(c * (mu + lam) / (mu + lam + c * (mu + lam)))
    for t, h in enumerate(hist, start=1):
        assert h == pytest.approx(q ** t, rel=1e-9)


def test_exact_operator_refines_in_one_step():
    rng = np.random.default_rng(0)
    X = rng.random((200, 3))
    K = kernel_matrix(X, 1.0, np.full(3, 0.7))
    b = rng.standard_normal(200)
    # one backward-stable dense solve: residual at the level n u ||A|| ||x|| / ||b||
    assert pr.refine(K, K, 1e-3, b, steps=1)[0] < 1e-10


@pytest.fixture(scope="module")
def c1_like():
    """1024 points of the 2048-point FP64 workload's recipe (d = 8, U[0,1],
    lengthscales 0.5, sigma2 = 1)."""
    rng = np.random.default_rng(0)
    X = rng.random((1024, 8))
    ls = np.full(8, 0.5)
    return X, ls, kernel_matrix(X, 1.0, ls), np.sin(3 * X).sum(axis=1)


def test_bf16_entries_make_the_operator_indefinite(c1_like):
    """BF16-rounded K at lambda = 1e-4: rho far above 1, K_hat + lambda I has
    a negative eigenvalue and refinement diverges."""
    X, ls, K, b = c1_like
    Kh = pr.perturbed_kernel(X, 1.0, ls, "bf16")
    assert pr.rho(Kh, K, 1e-4) > 10
    assert np.linalg.eigvalsh(Kh + 1e-4 * np.eye(len(b))).min() < 0
    assert pr.refine(Kh, K, 1e-4, b, steps=4)[-1] > 1.0


@pytest.mark.parametrize("model", ["fp32", "bf16x2", "f16x2", "augmented_fp32"])
def test_fp32_class_products_refine_to_fp64_accuracy(c1_like, model):
    X, ls, K, b = c1_like
    Kh = pr.perturbed_kernel(X, 1.0, ls, model)
    assert pr.rho(Kh, K, 1e-4) < 1
    assert pr.refine(Kh, K, 1e-4, b, steps=6)[-1] < 1e-12


def test_fp32_rounded_solution_misses_1e6(c1_like):
    """The exact solution rounded to FP32 leaves probe columns above a 1e-6
    relative residual at lambda = 1e-4: x has to be accumulated in FP64."""
    X, ls, K, b = c1_like
    Z = np.random.default_rng(1).integers(0, 2, (len(b), 4)) * 2.0 - 1.0
    res = pr.fp32_solution_residual(K, 1e-4, np.column_stack([b, Z]))
    assert np.all(res[1:] > 1e-6)


def test_augmented_fp32_error_grows_with_n_not_sqrt_n():
    """The FP32 exponent's per-row norm roundings scale E with K itself:
    for a smooth kernel rho doubles when n doubles (entry rounding alone
    grows about sqrt(2)-fold).  This is why FP32-class products stop
    certifying 1e-6 for large smooth problems at lambda = 1e-4."""
    rhos, rhos_entry = [], []
    for n in (512, 1024):
        X = np.random.default_rng(1).random((n, 4))
        ls = np.full(4, 1.5)
        K = kernel_matrix(X, 1.0, ls)
        rhos.append(pr.rho(pr.perturbed_kernel(X, 1.0, ls, "augmented_fp32"), K, 1e-4))
        rhos_entry.append(pr.rho(pr.perturbed_kernel(X, 1.0, ls, "fp32"), K, 1e-4))
    assert 1.6 < rhos[1] / rhos[0] < 2.6
    assert rhos_entry[1] / rhos_entry[0] < 1.6
    assert rhos[1] > 3 * rhos_entry[1]


def test_fp16_split_perturbs_less_than_bf16_split(c1_like):
    """At the 1024-point size of the FP64 workload's recipe the FP16x2
    entries' rho is an order of magnitude below the BF16x2 entries' and below
    the FP32 exponent's: the K V part no longer dominates the product's error."""
    X, ls, K, b = c1_like
    r16 = pr.rho(pr.perturbed_kernel(X, 1.0, ls, "f16x2"), K, 1e-4)
    rb = pr.rho(pr.perturbed_kernel(X, 1.0, ls, "bf16x2"), K, 1e-4)
    ra = pr.rho(pr.perturbed_kernel(X, 1.0, ls, "augmented_fp32"), K, 1e-4)
    print("rho f16x2 %.3e bf16x2 %.3e augmented_fp32 %.3e" % (r16, rb, ra))
    assert r16 < rb / 10
    assert r16 < ra


# ---- int8-digit product model ---------------------------------------------

def test_signed_digits_reconstruct_and_stay_in_range():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.integers(-2 ** 30, 2 ** 30, 2000).astype(float),
                        [0, 1, -1, 127, 128, -128, -129, 255, 256, 2 ** 30, -2 ** 30 + 1]])
    d = pr.signed_digits(x)
    assert d.min() >= -128 and d.max() <= 127
    assert np.all((d * 256.0 ** np.arange(4)[:, None]).sum(axis=0) == x)


def test_signed_digits_unique_by_brute_force():
    """Every two-digit value v in [-128 - 127*256, 127 + 127*256] has exactly
    one pair (s0, s1) in [-128, 127]^2 with s0 + 256 s1 = v, and the
    recursion returns it."""
    s = np.arange(-128, 128)
    vals = (s[:, None] + 256 * s[None, :]).ravel()
    assert len(np.unique(vals)) == vals.size              # unique representation
    pick = np.random.default_rng(12).choice(vals.size, 3000, replace=False)
    d = pr.signed_digits(vals[pick].astype(float), ndig=2)
    s0, s1 = np.divmod(pick, 256)                          # pick = i0 * 256 + i1
    assert np.all(d[0] == s[s0]) and np.all(d[1] == s[s1])


def test_column_exponents_bracket():
    V = np.array([[1.0, -2.0 ** 40, 0.0, np.nextafter(4.0, 0.0), 3.0e-300],
                  [0.5, 3.0, 0.0, -1.0, 0.0]])
    e = pr._column_exponents(V)
    m = np.max(np.abs(V), axis=0)
    sc = np.ldexp(m, e)
    nz = m > 0
    assert np.all((sc[nz] >= 2.0 ** 29) & (sc[nz] < 2.0 ** 30))
    assert e[2] == 0


def test_int8_all_pairs_equal_exact_integer_product():
    """With every digit pair kept (min_class 0), the model is the exact
    product of the fixed-point integers kint = rint(2^30 K / sigma2) and
    vint = rint(2^e V), here recomputed with Python integers."""
    rng = np.random.default_rng(13)
    X = rng.random((9, 3))
    ls = np.array([0.3, 0.5, 0.8])
    s2 = 2.5
    V = rng.standard_normal((9, 2)) * np.array([1e-3, 40.0])
    got = pr.int8_digit_product(X, s2, ls, V, min_class=0)
    K = kernel_matrix(X, s2, ls)
    e = pr._column_exponents(V)
    for c in range(2):
        vint = [int(np.rint(np.ldexp(v, int(e[c])))) for v in V[:, c]]
        for i in range(9):
            kint = [int(np.rint(np.ldexp(K[i, j] / s2, 30))) for j in range(9)]
            exact = sum(a * b for a, b in zip(kint, vint))
            assert got[i, c] == pytest.approx(s2 * exact * 2.0 ** (-30 - int(e[c])), rel=1e-15)


@pytest.mark.parametrize("min_class", [2, 3])
def test_int8_truncation_within_bound(min_class):
    """Dropping the digit pairs with p + q < min_class moves each output by
    at most n x the per-term bound (in units of sigma2 2^(-30 - e))."""
    rng = np.random.default_rng(14)
    n = 200
    X = rng.standard_normal((n, 4))
    ls = np.full(4, 1.5)
    V = rng.standard_normal((n, 3))
    full = pr.int8_digit_product(X, 1.0, ls, V, min_class=0)
    part = pr.int8_digit_product(X, 1.0, ls, V, min_class=min_class)
    e = pr._column_exponents(V)
    bound = n * pr.int8_truncation_bound(min_class) * 2.0 ** (-30.0 - e)
    assert np.all(np.abs(part - full) <= bound[None, :])
    assert np.max(np.abs(part - full) / bound[None, :]) > 1e-4   # the bound is not vacuous


def test_int8_model_error_against_exact_product():
    """Norm-wise error of the model against the FP64 product: K in steps of
    2^-30 and V in steps of 2^-30 of its column maximum leave about 2^-30
    relative (the pairs with p + q < 2 add ~2^-36 per term), over an order
    below FP32-rounded entries and V on the same product (whose K V sums
    cancel: V is random).  Dropping the pairs with p + q = 2 as well would
    cost a factor ~4."""
    rng = np.random.default_rng(15)
    n = 512
    X = rng.standard_normal((n, 8))
    ls = np.exp(rng.uniform(np.log(2), np.log(8), 8))
    V = rng.standard_normal((n, 5))
    K = kernel_matrix(X, 1.7, ls)
    exact = K @ V + 1e-4 * V
    got = pr.int8_digit_product(X, 1.7, ls, V, shift=1e-4, min_class=2, K=K)
    err = np.linalg.norm(got - exact, axis=0) / np.linalg.norm(exact, axis=0)
    f32 = pr.round_fp32(K) @ pr.round_fp32(V) + 1e-4 * V
    err32 = np.linalg.norm(f32 - exact, axis=0) / np.linalg.norm(exact, axis=0)
    assert np.all(err < 2.0 ** -29), err
    assert np.all(err < err32 / 10), (err, err32)
    got3 = pr.int8_digit_product(X, 1.7, ls, V, shift=1e-4, min_class=3, K=K)
    err3 = np.linalg.norm(got3 - exact, axis=0) / np.linalg.norm(exact, axis=0)
    assert np.all(err3 > 2 * err), (err3, err)


# ---- stored-FP32 Psi in the Woodbury apply ----------------------------------

def _nystrom_factor(X, sigma2, ls, idx, jitter=1e-8):
    """Phi = K_XU L^-T with K_UU + jitter I = L L^T (so Phi Phi^T = Q)."""
    from oracle.kernel import rbf_block
    Xu = X[idx]
    L = np.linalg.cholesky(rbf_block(Xu, Xu, sigma2, ls) + jitter * np.eye(len(idx)))
    return np.linalg.solve(L, rbf_block(X, Xu, sigma2, ls).T).T


def _c2_like(seed, n=900, d=8, m=64, lam=1e-3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    ls = np.full(d, 1.5)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    return X, 1.0, ls, lam, _nystrom_factor(X, 1.0, ls, idx)


def test_woodbury_psi_apply_is_the_dense_inverse():
    """D^-1 - Psi Psi^T from woodbury_psi is (diag(D) + Phi Phi^T)^-1 itself
    (brute force: a dense solve), for a FITC-like varying D."""
    rng = np.random.default_rng(3)
    n, m = 300, 20
    Phi = rng.standard_normal((n, m)) * 0.7
    D = 1e-2 + rng.random(n)
    R = rng.standard_normal((n, 5))
    Psi = pr.woodbury_psi(D, Phi)
    want = np.linalg.solve(np.diag(D) + Phi @ Phi.T, R)
    got = pr.woodbury_apply(D, Psi, R)
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def test_fp32_psi_apply_is_symmetric_and_within_its_bound():
    """The stored-FP32 apply of a C2-like Nystrom preconditioner (lambda =
    1e-3): symmetric as an operator (both factors rounded alike), changed by
    no more than the entrywise bound, and changed (the rounding bites at a
    visible fraction of the bound)."""
    X, s2, ls, lam, Phi = _c2_like(5)
    n = X.shape[0]
    D = np.full(n, lam)
    Psi = pr.woodbury_psi(D, Phi)
    R = np.random.default_rng(6).standard_normal((n, 7))
    z64 = pr.woodbury_apply(D, Psi, R)
    z32 = pr.woodbury_apply(D, Psi, R, round_psi=True)
    bound = pr.psi_rounding_bound(Psi, R)
    slack = 1e-13 * (np.abs(R) / lam + np.abs(Psi) @ (np.abs(Psi).T @ np.abs(R)))
    dev = np.abs(z32 - z64)
    assert np.all(dev <= bound + slack)
    assert dev.max() >= 1e-3 * bound.max()
    E = np.eye(n)
    M = pr.woodbury_apply(D, Psi, E, round_psi=True)
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))


@pytest.mark.parametrize("lam,changes", [(1e-2, False), (1e-3, True)])
def test_fp32_psi_step_effect_follows_its_perturbation(lam, changes):
    """PCG (oracle, FP64) to 1e-6 on a 900-point system with the exact and the
    stored-FP32 Nystrom apply (m = 64).  The rounding moves the preconditioned
    operator by at most eta = (2u + u^2) || |Psi| ||^2 ||K_y|| (from the
    entrywise bound); where eta is small (lambda = 1e-2) the step counts agree
    within 10 % + 2, where it is not (lambda = 1e-3: Psi grows like
    lambda^-1/2) the rounded preconditioner costs more than 10 % more steps.
    Either way it stays positive definite and PCG converges."""
    from oracle.pcg import pcg
    X, s2, ls, _, Phi = _c2_like(7)
    n = X.shape[0]
    K = kernel_matrix(X, s2, ls) + lam * np.eye(n)
    D = np.full(n, lam)
    Psi = pr.woodbury_psi(D, Phi)
    u = 2.0 ** -24
    eta = (2 * u + u * u) * np.linalg.norm(np.abs(Psi), 2) ** 2 * np.linalg.norm(K, 2)
    B = np.random.default_rng(8).standard_normal((n, 4))
    r64 = pcg(lambda V: K @ V, B, precond=lambda R: pr.woodbury_apply(D, Psi, R), tol=1e-6)
    r32 = pcg(lambda V: K @ V, B, precond=lambda R: pr.woodbury_apply(D, Psi, R, round_psi=True),
              tol=1e-6)
    Pinv32 = pr.woodbury_apply(D, Psi, np.eye(n), round_psi=True)
    assert np.linalg.eigvalsh(0.5 * (Pinv32 + Pinv32.T)).min() > 0
    assert np.all(r32.relres <= 1e-6) and np.all(r64.relres <= 1e-6)
    i32, i64 = int(r32.iters.max()), int(r64.iters.max())
    if changes:
        assert eta > 0.1 and i32 > 1.1 * i64, (eta, i32, i64)
    else:
        assert eta < 0.05 and abs(i32 - i64) <= 0.1 * i64 + 2, (eta, i32, i64)
