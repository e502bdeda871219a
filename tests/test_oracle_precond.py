"""Pins of the oracle's Nystrom / FITC / factor preconditioners (Sections 3.1, 3.2)."""
import numpy as np

from oracle import kernel as ok
from oracle.kernel import kernel_matrix
from oracle import precond as op
from oracle.pcg import pcg
from pkm_inputs import make


def _case(n=300, m=40, seed=0):
    p = make("block_fp32", seed=seed, n=n, m=m, n_probes=3)
    return p


def test_nystrom_apply_equals_dense_solve():
    p = _case()
    P = op.nystrom(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=1e-8)
    dense = P.dense()
    assert np.allclose(dense, dense.T, atol=1e-12)
    assert np.linalg.eigvalsh(dense).min() > 0
    R = p.B
    assert np.allclose(P(R), np.linalg.solve(dense, R), rtol=1e-8, atol=1e-8)


def test_fitc_apply_equals_dense_solve_and_diagonal():
    p = _case(seed=1)
    P = op.fitc(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=1e-8)
    dense = P.dense()
    # diag(P) = diag(K) + lambda exactly (up to the clip at zero)
    assert np.allclose(np.diag(dense), p.sigma2 + p.lam, rtol=1e-10, atol=0)
    D = P.info["D"]
    assert np.all(D >= p.lam)
    # at inducing points K - Q vanishes on the diagonal
    assert np.allclose(D[p.idx], p.lam, rtol=0, atol=1e-6)
    assert np.allclose(P(p.B), np.linalg.solve(dense, p.B), rtol=1e-8, atol=1e-8)


def test_full_inducing_set_reproduces_K_and_one_step_pcg():
    # A smooth-enough, well-conditioned case so that K_UU = K can be inverted.
    rng = np.random.default_rng(5)
    n, d = 64, 3
    X = rng.random((n, d)) * 4.0
    ls = np.array([0.3, 0.4, 0.5])
    s2, lam = 1.0, 1e-2
    idx = np.arange(n)
    K = ok.kernel_matrix(X, s2, ls)
    assert np.linalg.cond(K) < 1e6
    Pn = op.nystrom(X, s2, ls, lam, idx)
    assert np.allclose(Pn.dense(), K + lam * np.eye(n), rtol=1e-10, atol=1e-10)
    Pf = op.fitc(X, s2, ls, lam, idx)
    assert np.allclose(Pf.dense(), Pn.dense(), rtol=1e-10, atol=1e-10)
    B = rng.standard_normal((n, 2))
    res = pcg(lambda V: ok.kernel_mvm(X, s2, ls, lam, V), B, precond=Pn, tol=1e-9, max_iter=20)
    assert np.all(res.iters == 1)


def test_factor_form_with_top_eigenpairs():
    p = _case(n=200, seed=2)
    K = ok.kernel_matrix(p.X, p.sigma2, p.lengthscales)
    w, V = np.linalg.eigh(K)
    r = 12
    Phi = V[:, -r:] * np.sqrt(w[-r:])
    P = op.lowrank(Phi, p.lam)
    Ky = K + p.lam * np.eye(p.n)
    PinvKy = P(Ky)
    # on the top-r eigenvectors P^{-1} K_y acts as the identity
    assert np.allclose(PinvKy @ V[:, -r:], V[:, -r:], atol=1e-8)
    assert np.allclose(P(p.B), np.linalg.solve(P.dense(), p.B), rtol=1e-8, atol=1e-8)


def test_nystrom_reduces_iterations():
    p = make("small_fp64", seed=0, n=1024, m=64)
    mv = lambda V: ok.kernel_mvm(p.X, p.sigma2, p.lengthscales, p.lam, V)
    P = op.nystrom(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=1e-8)
    plain = pcg(mv, p.y, tol=1e-8, max_iter=5000)
    pre = pcg(mv, p.y, precond=P, tol=1e-8, max_iter=5000)
    assert pre.iters[0] < plain.iters[0]


def test_sketch_with_identity_columns_is_nystrom():
    p = _case(n=250, m=30, seed=3)
    S = np.zeros((p.n, len(p.idx)))
    S[p.idx, np.arange(len(p.idx))] = 1.0
    Ps = op.sketch(p.X, p.sigma2, p.lengthscales, p.lam, S, jitter=0.0)
    Pn = op.nystrom(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=0.0)
    assert np.allclose(Ps.dense(), Pn.dense(), rtol=1e-8, atol=1e-8)
    assert np.allclose(Ps(p.B), Pn(p.B), rtol=1e-7, atol=1e-7)


def test_sketch_never_exceeds_K_and_full_sketch_is_exact():
    rng = np.random.default_rng(4)
    p = _case(n=120, m=10, seed=4)
    S = rng.standard_normal((p.n, 15))
    Ps = op.sketch(p.X, p.sigma2, p.lengthscales, p.lam, S, jitter=0.0)
    K = ok.kernel_matrix(p.X, p.sigma2, p.lengthscales)
    # K_y - P = K - K S C^-1 S^T K is positive semi-definite
    gap = K + p.lam * np.eye(p.n) - Ps.dense()
    assert np.linalg.eigvalsh(0.5 * (gap + gap.T)).min() > -1e-8
    # a full-rank sketch reproduces K_y: one PCG step
    X2 = rng.random((40, 3))
    Pf = op.sketch(X2, 1.0, np.array([0.3, 0.4, 0.5]), 1e-2, np.eye(40), jitter=0.0)
    B = rng.standard_normal((40, 2))
    res = pcg(lambda V: ok.kernel_mvm(X2, 1.0, np.array([0.3, 0.4, 0.5]), 1e-2, V), B,
              precond=Pf, tol=1e-9, max_iter=20)
    assert np.all(res.iters == 1)


def test_pitc_apply_equals_dense_solve_and_blocks_match_K():
    """PITC (Section 3.1.1): apply equals a dense solve with P = Q +
    blockdiag(K - Q) + lambda I, and P's diagonal blocks are K's plus lambda I
    exactly (the correction restores them)."""
    rng = np.random.default_rng(21)
    X = rng.random((150, 3))
    ls = np.array([0.4, 0.7, 1.1])
    idx = np.sort(rng.choice(150, 20, replace=False))
    lam, blk = 1e-2, 32
    P = op.pitc(X, 1.3, ls, lam, idx, blk, jitter=1e-8)
    Pd = P.dense()
    R = rng.standard_normal((150, 3))
    want = np.linalg.solve(Pd, R)
    # both sides go through K_UU^-1 (condition ~1e8 with this jitter)
    np.testing.assert_allclose(P(R), want, rtol=0, atol=1e-8 * np.abs(want).max())
    K = ok.kernel_matrix(X, 1.3, ls)
    for s0 in range(0, 150, blk):
        s1 = min(150, s0 + blk)
        np.testing.assert_allclose(Pd[s0:s1, s0:s1], K[s0:s1, s0:s1] + lam * np.eye(s1 - s0),
                                   rtol=0, atol=1e-10)


def test_pitc_limits_fitc_and_exact():
    """Block size 1 is FITC; a single block of all rows is K + lambda I, so
    PCG with it stops after one step."""
    rng = np.random.default_rng(22)
    X = rng.random((90, 2))
    ls = np.array([0.5, 0.8])
    idx = np.sort(rng.choice(90, 12, replace=False))
    lam = 1e-2
    P1 = op.pitc(X, 1.0, ls, lam, idx, 1, jitter=1e-10)
    F = op.fitc(X, 1.0, ls, lam, idx, jitter=1e-10)
    np.testing.assert_allclose(P1.dense(), F.dense(), rtol=0, atol=1e-9)
    Pn = op.pitc(X, 1.0, ls, lam, idx, 90, jitter=1e-10)
    Ky = ok.kernel_matrix(X, 1.0, ls) + lam * np.eye(90)
    np.testing.assert_allclose(Pn.dense(), Ky, rtol=0, atol=1e-10)
    b = np.sin(3 * X).sum(axis=1)
    res = pcg(lambda v: Ky @ v, b, precond=Pn, tol=1e-10)
    assert res.iters <= 2


def test_spectral_features_closed_forms():
    """Section 3.2 spectral approximation: (Phi Phi^T)_ij equals the printed
    sum of cosines of frequency-projected differences; its diagonal is sigma^2
    exactly (cos^2 + sin^2 = 1); with many frequencies it approaches K (the
    RBF kernel is the expectation of cos(omega^T (x - x')) for omega ~
    N(0, diag(1/l^2)))."""
    rng = np.random.default_rng(31)
    X = rng.random((40, 3))
    ls = np.array([0.6, 0.9, 1.4])
    s2 = 1.7
    W = rng.standard_normal((25, 3))
    Phi = op.spectral_features(X, s2, ls, W)
    Khat = Phi @ Phi.T
    omega = W / ls
    D = X[:, None, :] - X[None, :, :]
    printed = s2 / 25 * np.cos(np.einsum("ijd,rd->ijr", D, omega)).sum(axis=2)
    np.testing.assert_allclose(Khat, printed, rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.diag(Khat), s2, rtol=1e-14)
    Wbig = np.random.default_rng(32).standard_normal((200000, 3))
    Kbig = op.spectral_features(X, s2, ls, Wbig)
    err = np.abs(Kbig @ Kbig.T - ok.kernel_matrix(X, s2, ls)).max()
    assert err < 5 * s2 / np.sqrt(200000)   # Monte Carlo, ~1/sqrt(m)


# ---- randomised truncated SVD (Section 3.2, partial SVD) --------------------

def test_rsvd_recovers_a_low_rank_kernel_exactly():
    """X with c distinct points (each repeated) gives rank(K) = c; a sketch of
    l >= c columns spans K's range, so with r >= c the factor reproduces K
    and P = K + lambda I (PCG needs one step)."""
    from oracle.pcg import pcg
    rng = np.random.default_rng(11)
    c, rep, d = 12, 9, 3
    X = np.repeat(rng.random((c, d)), rep, axis=0)
    ls = np.full(d, 0.4)
    K = kernel_matrix(X, 1.3, ls)
    Omega = rng.standard_normal((X.shape[0], 16))
    Phi = op.rsvd_factor(X, 1.3, ls, Omega, r=14, q=0)
    assert np.max(np.abs(Phi @ Phi.T - K)) <= 1e-10 * np.max(np.abs(K))
    P = op.rsvd(X, 1.3, ls, 1e-2, Omega, r=14)
    b = rng.standard_normal(X.shape[0])
    res = pcg(lambda V: K @ V + 1e-2 * V, b, precond=P, tol=1e-10)
    assert int(res.iters[0]) <= 2


def test_rsvd_with_power_iterations_is_near_the_best_rank_r():
    """Eckart-Young: no rank-r Phi Phi^T gets closer to K (2-norm) than the
    (r+1)-th eigenvalue; with 4 power iterations and 10 oversampling columns
    the randomised factor comes within 1 % of it."""
    rng = np.random.default_rng(12)
    X = rng.random((300, 4))
    ls = np.full(4, 0.35)
    K = kernel_matrix(X, 1.0, ls)
    lam_K = np.sort(np.linalg.eigvalsh(K))[::-1]
    r = 20
    Phi = op.rsvd_factor(X, 1.0, ls, rng.standard_normal((300, r + 10)), r=r, q=4)
    err = np.linalg.norm(K - Phi @ Phi.T, 2)
    assert lam_K[r] * (1 - 1e-9) <= err <= 1.01 * lam_K[r], (err, lam_K[r])
    # Rayleigh-Ritz: the factor's eigenvalues (Ritz values) never exceed the
    # corresponding eigenvalues of K and here come within 0.1 % of them
    w = np.sort(np.linalg.eigvalsh(Phi.T @ Phi))[::-1]
    assert np.all(w <= lam_K[:r] * (1 + 1e-12))
    assert np.allclose(w, lam_K[:r], rtol=1e-3)


def test_rsvd_is_the_factor_form():
    """P from the randomised SVD is the factor form P = Phi Phi^T + lambda I
    (dense solve), symmetric positive definite with P >= lambda I; unlike
    Nystrom it is a projection Pi K Pi of K, which may exceed K in some
    directions."""
    rng = np.random.default_rng(13)
    X = rng.random((120, 2))
    ls = np.full(2, 0.3)
    K = kernel_matrix(X, 0.8, ls)
    lam = 1e-3
    P = op.rsvd(X, 0.8, ls, lam, rng.standard_normal((120, 30)), r=24, q=1)
    R = rng.standard_normal((120, 3))
    dense = P.dense()
    assert np.allclose(P(R), np.linalg.solve(dense, R), rtol=1e-8, atol=1e-10)
    assert np.allclose(dense, dense.T, atol=1e-12)
    assert np.linalg.eigvalsh(dense).min() >= lam * (1 - 1e-9)
