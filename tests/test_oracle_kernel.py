"""Pins of the oracle's ARD-RBF kernel and product (Eq. (1), Section 2.1)."""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import kernel as ok
from pkm_inputs import make


def test_golden_hand_values():
    for line in read_golden("rbf_hand.txt"):
        f = [s.strip() for s in line.split("|")]
        d = int(f[0])
        x = np.array(f[1].split(), float).reshape(1, d)
        xp = np.array(f[2].split(), float).reshape(1, d)
        ls = np.array(f[3].split(), float)
        s2 = float(f[4])
        want = float(f[5])
        got = ok.rbf_block(x, xp, s2, ls)[0, 0]
        assert got == pytest.approx(want, rel=1e-15, abs=0), line
        # symmetric in its two arguments
        assert ok.rbf_block(xp, x, s2, ls)[0, 0] == got


def test_diagonal_symmetry_psd():
    p = make("block_fp32", seed=3, n=300)
    K = ok.kernel_matrix(p.X, 1.7, p.lengthscales)
    assert np.all(np.diag(K) == 1.7)
    assert np.array_equal(K, K.T)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -1e-12 * ev.max()


def test_long_lengthscale_limit():
    rng = np.random.default_rng(0)
    X = rng.random((50, 4))
    V = rng.standard_normal((50, 3))
    got = ok.kernel_mvm(X, 2.5, np.full(4, 1e9), 0.0, V)
    want = 2.5 * np.ones((50, 1)) * V.sum(axis=0)[None, :]
    assert np.allclose(got, want, rtol=1e-14, atol=1e-14)


def test_short_lengthscale_limit():
    rng = np.random.default_rng(1)
    X = rng.random((40, 3))
    V = rng.standard_normal((40, 2))
    got = ok.kernel_mvm(X, 0.8, np.full(3, 1e-6), 0.3, V)
    assert np.allclose(got, 1.1 * V, rtol=1e-14, atol=0)


def test_brute_force_triple_loop():
    rng = np.random.default_rng(2)
    n, d, k = 9, 3, 2
    X = rng.random((n, d))
    ls = np.array([0.3, 0.9, 1.7])
    V = rng.standard_normal((n, k))
    s2, lam = 1.3, 0.05
    want = np.zeros((n, k))
    for i in range(n):
        for j in range(n):
            e = 0.0
            for r in range(d):
                e += (X[i, r] - X[j, r]) ** 2 / ls[r] ** 2
            kij = s2 * math.exp(-0.5 * e) + (lam if i == j else 0.0)
            for c in range(k):
                want[i, c] += kij * V[j, c]
    got = ok.kernel_mvm(X, s2, ls, lam, V, block=4)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-15)


def test_row_subset_and_threads_agree():
    p = make("block_fp32", seed=4, n=700, n_probes=3)
    full = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, threads=4, block=64)
    one = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, threads=1, block=128)
    assert np.allclose(full, one, rtol=1e-13, atol=1e-13)
    rows = np.array([0, 5, 699, 350])
    sub = ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, p.B, rows=rows)
    assert np.allclose(sub, full[rows], rtol=1e-13, atol=1e-13)
