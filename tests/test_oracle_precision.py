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


@pytest.mark.parametrize("model", ["fp32", "bf16x2", "augmented_fp32"])
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
