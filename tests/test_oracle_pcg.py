"""Pins of the oracle's PCG (Algorithm 1, textbook reading)."""
import numpy as np
import scipy.linalg as sla

from conftest import read_golden
from oracle import direct as od
from oracle import kernel as ok
from oracle.pcg import pcg
from pkm_inputs import make


def _golden():
    out = {}
    for line in read_golden("cg_2x2.txt"):
        f = line.split()
        out[f[0]] = np.array(f[1:], float)
    return out


def test_hand_worked_2x2():
    g = _golden()
    A = np.array([[4.0, 1.0], [1.0, 3.0]])
    b = np.array([1.0, 2.0])
    steps = []

    def mv(P):
        steps.append(P.copy())
        return A @ P

    res1 = pcg(mv, b, tol=0.0, max_iter=1)
    assert np.allclose(res1.x, g["x1"], rtol=0, atol=1e-16)
    res2 = pcg(lambda P: A @ P, b, tol=1e-15, max_iter=10)
    assert res2.iters[0] == 2
    assert np.allclose(res2.x, g["x2"], rtol=0, atol=1e-15)
    # the second search direction seen by the product is p1
    steps.clear()
    pcg(mv, b, tol=0.0, max_iter=2)
    assert np.allclose(steps[1][:, 0], g["p1"], rtol=0, atol=1e-16)


def test_cg_distinct_eigenvalues_terminates():
    rng = np.random.default_rng(0)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    eig = np.repeat([1.0, 3.0, 10.0, 40.0], n // 4)
    A = (Q * eig) @ Q.T
    b = rng.standard_normal(n)
    res = pcg(lambda P: A @ P, b, tol=1e-10, max_iter=50)
    assert res.iters[0] <= 4


def test_pcg_three_distinct_preconditioned_eigenvalues():
    # P^{-1} A has 3 distinct eigenvalues: A = P^{1/2} Q diag(mu) Q^T P^{1/2}.
    rng = np.random.default_rng(1)
    n = 48
    G = rng.standard_normal((n, n))
    P = G @ G.T + n * np.eye(n)
    w, E = np.linalg.eigh(P)
    Ph = (E * np.sqrt(w)) @ E.T
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    mu = np.repeat([0.5, 2.0, 7.0], n // 3)
    A = Ph @ ((Q * mu) @ Q.T) @ Ph
    A = 0.5 * (A + A.T)
    b = rng.standard_normal((n, 2))
    res = pcg(lambda V: A @ V, b, precond=lambda R: np.linalg.solve(P, R),
              tol=1e-9, max_iter=50)
    assert np.all(res.iters <= 3)
    assert np.allclose(res.x, np.linalg.solve(A, b), rtol=1e-7, atol=1e-9)
    # without the preconditioner the same system needs many more steps
    plain = pcg(lambda V: A @ V, b, tol=1e-9, max_iter=200)
    assert np.all(plain.iters > 6)


def test_exact_preconditioner_one_step():
    p = make("small_fp64", seed=1, n=400, n_probes=4)
    Ky = ok.kernel_matrix(p.X, p.sigma2, p.lengthscales) + p.lam * np.eye(p.n)
    c = sla.cho_factor(Ky, lower=True)
    res = pcg(lambda V: Ky @ V, p.B, precond=lambda R: sla.cho_solve(c, R),
              tol=1e-10, max_iter=20)
    assert np.all(res.iters == 1)


def test_matches_cholesky_and_monotone_energy_error():
    p = make("small_fp64", seed=2, n=512, n_probes=2)
    mv = lambda V: ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    xs = od.solve(p.X, p.sigma2, p.lengthscales, p.lam, p.B)
    res = pcg(mv, p.B, tol=1e-10, max_iter=5000)
    assert np.all(np.linalg.norm(res.x - xs, axis=0) / np.linalg.norm(xs, axis=0) < 1e-6)
    # K_y-norm of the error decreases monotonically (CG minimises it over Krylov spaces)
    Ky = ok.kernel_matrix(p.X, p.sigma2, p.lengthscales) + p.lam * np.eye(p.n)
    errs = []
    for t in (1, 5, 20, 60, 150):
        e = pcg(mv, p.B[:, 0], tol=0.0, max_iter=t).x - xs[:, 0]
        errs.append(float(e @ Ky @ e))
    assert all(a > b for a, b in zip(errs, errs[1:]))


def test_absolute_threshold_and_frozen_columns():
    p = make("small_fp64", seed=3, n=256, n_probes=3)
    mv = lambda V: ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    B = p.B.copy()
    B[:, 2] *= 1e-6      # this column meets the absolute test much earlier
    res = pcg(mv, B, tol_abs=1e-3, max_iter=5000)
    assert res.iters[2] < res.iters[0]
    r = B - mv(res.x)
    assert np.all(np.linalg.norm(r, axis=0) < 1.001e-3)
