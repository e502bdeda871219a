"""Low-rank preconditioners applied through the matrix inversion lemma, FP64.

Section 3.1 (Nystrom): with inducing set U (m rows of X),
    P = K_XU K_UU^{-1} K_UX + lambda I,
    P^{-1} v = lambda^{-1} [ v - K_XU (lambda K_UU + K_UX K_XU)^{-1} K_UX v ].
The printed inverse omits the factor lambda in front of K_UU; the form above
is the matrix inversion lemma applied to the stated P (the two agree only at
lambda = 1).

Section 3.1.1 (FITC): P = Q + diag(K - Q) + lambda I with Q = K_XU K_UU^{-1}
K_UX.  The diagonal D = diag(K - Q) + lambda I takes the place of lambda I:
    P^{-1} v = D^{-1} v - D^{-1} K_XU (K_UU + K_UX D^{-1} K_XU)^{-1} K_UX D^{-1} v.
diag(K - Q) is clipped at zero against rounding.

Section 3.1.1 (PITC): the same with the diagonal correction widened to
blocks of consecutive rows B_1, B_2, ... (size ``block``, the last one
ragged): D = blockdiag(K_BB - Q_BB) + lambda I, P = Q + D, and
    P^{-1} v = D^{-1} v - D^{-1} K_XU (K_UU + K_UX D^{-1} K_XU)^{-1} K_UX D^{-1} v
with D^{-1} applied block by block.  Block size 1 is FITC (up to FITC's
clipping); one block of all n rows is K + lambda I itself.

Section 3.2 (factor form): P = Phi Phi^T + lambda I,
    P^{-1} v = lambda^{-1} [ v - Phi (lambda I + Phi^T Phi)^{-1} Phi^T v ],
again with lambda restored in the core (printed as I + Phi^T Phi).

Section 3.2 (spectral approximation, random Fourier features): with m
frequencies s_r drawn from N(0, Lambda / (4 pi^2)), Lambda = diag(1 / l^2),
    K_hat_ij = sigma^2 / m sum_r cos(2 pi s_r^T (x_i - x_j)) = (Phi Phi^T)_ij,
    Phi = sqrt(sigma^2 / m) [cos(2 pi S X^T)^T, sin(2 pi S X^T)^T]  (n x 2m),
and P = Phi Phi^T + lambda I as in the factor form.  The caller passes
standard normal draws W (m x d); 2 pi s_r = W_r / l.

K_UU carries a jitter delta I (the caller's value; the same on both sides),
which changes P but never the solution of the preconditioned system.

Section 3.2 (partial SVD, randomised truncated form): with m standard
normal sketch columns Omega (n x l), q power iterations and the r largest
eigenpairs,
    Y = K Omega;  q times: Q = orth(Y), Y = K Q;  Q = orth(Y),
    B = Q^T K Q = V diag(w) V^T,   Phi = Q V_r diag(w_r)^1/2,
so Phi Phi^T approximates K by its leading eigenpairs, and P = Phi Phi^T +
lambda I as in the factor form.  Negative eigenvalues of B (rounding)
are clipped to zero.

Pinned by (tests/test_oracle_precond.py): each apply against a direct solve
with the dense P it defines; m = n Nystrom reproduces K (so PCG stops after
one step); FITC has diag(P) = diag(K) + lambda exactly and D_u = lambda at
inducing points; m = n FITC equals Nystrom; Phi built from the top
eigenpairs of K leaves unit eigenvalues of P^{-1} K_y on that subspace.
"""
from __future__ import annotations

import numpy as np

from .kernel import rbf_block


class Preconditioner:
    """P^{-1} as a callable, plus the dense P for small-n checks."""

    def __init__(self, apply, dense, info=None):
        self._apply = apply
        self._dense = dense
        self.info = info or {}

    def __call__(self, R):
        return self._apply(np.asarray(R, dtype=np.float64))

    def dense(self):
        return self._dense()


def nystrom(X, sigma2, lengthscales, lam, idx, jitter=0.0):
    X = np.asarray(X, dtype=np.float64)
    Xu = X[np.asarray(idx)]
    Kuu = rbf_block(Xu, Xu, sigma2, lengthscales) + jitter * np.eye(len(idx))
    Kxu = rbf_block(X, Xu, sigma2, lengthscales)
    core = lam * Kuu + Kxu.T @ Kxu

    def apply(R):
        return (R - Kxu @ np.linalg.solve(core, Kxu.T @ R)) / lam

    def dense():
        return Kxu @ np.linalg.solve(Kuu, Kxu.T) + lam * np.eye(X.shape[0])

    return Preconditioner(apply, dense, {"Kxu": Kxu, "Kuu": Kuu})


def fitc_diagonal(X, sigma2, lengthscales, lam, idx, jitter=0.0):
    """D = max(diag(K - K_XU K_UU^{-1} K_UX), 0) + lambda."""
    X = np.asarray(X, dtype=np.float64)
    Xu = X[np.asarray(idx)]
    Kuu = rbf_block(Xu, Xu, sigma2, lengthscales) + jitter * np.eye(len(idx))
    Kxu = rbf_block(X, Xu, sigma2, lengthscales)
    qdiag = np.sum(Kxu * np.linalg.solve(Kuu, Kxu.T).T, axis=1)
    kdiag = np.full(X.shape[0], float(sigma2))   # k(x, x) = sigma^2, Eq. (1)
    return np.maximum(kdiag - qdiag, 0.0) + lam


def fitc(X, sigma2, lengthscales, lam, idx, jitter=0.0):
    X = np.asarray(X, dtype=np.float64)
    Xu = X[np.asarray(idx)]
    Kuu = rbf_block(Xu, Xu, sigma2, lengthscales) + jitter * np.eye(len(idx))
    Kxu = rbf_block(X, Xu, sigma2, lengthscales)
    D = fitc_diagonal(X, sigma2, lengthscales, lam, idx, jitter)
    core = Kuu + Kxu.T @ (Kxu / D[:, None])

    def apply(R):
        DR = R / D[:, None] if R.ndim == 2 else R / D
        inner = Kxu @ np.linalg.solve(core, Kxu.T @ DR)
        return DR - (inner / D[:, None] if R.ndim == 2 else inner / D)

    def dense():
        return Kxu @ np.linalg.solve(Kuu, Kxu.T) + np.diag(D)

    return Preconditioner(apply, dense, {"D": D, "Kxu": Kxu, "Kuu": Kuu})


def pitc(X, sigma2, lengthscales, lam, idx, block, jitter=0.0):
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Xu = X[np.asarray(idx)]
    Kuu = rbf_block(Xu, Xu, sigma2, lengthscales) + jitter * np.eye(len(idx))
    Kxu = rbf_block(X, Xu, sigma2, lengthscales)
    starts = list(range(0, n, block))
    Dblocks = []
    for s0 in starts:
        s1 = min(n, s0 + block)
        Kbb = rbf_block(X[s0:s1], X[s0:s1], sigma2, lengthscales)
        Qbb = Kxu[s0:s1] @ np.linalg.solve(Kuu, Kxu[s0:s1].T)
        Dblocks.append(Kbb - Qbb + lam * np.eye(s1 - s0))

    def dinv(R):
        out = np.empty_like(R)
        for s0, Db in zip(starts, Dblocks):
            out[s0:s0 + Db.shape[0]] = np.linalg.solve(Db, R[s0:s0 + Db.shape[0]])
        return out

    DKxu = dinv(Kxu)
    core = Kuu + Kxu.T @ DKxu

    def apply(R):
        R2 = R if R.ndim == 2 else R[:, None]
        DR = dinv(R2)
        out = DR - DKxu @ np.linalg.solve(core, Kxu.T @ DR)
        return out if R.ndim == 2 else out[:, 0]

    def dense():
        D = np.zeros((n, n))
        for s0, Db in zip(starts, Dblocks):
            D[s0:s0 + Db.shape[0], s0:s0 + Db.shape[0]] = Db
        return Kxu @ np.linalg.solve(Kuu, Kxu.T) + D

    return Preconditioner(apply, dense, {"Dblocks": Dblocks, "Kxu": Kxu, "Kuu": Kuu})


def sketch(X, sigma2, lengthscales, lam, S, jitter=0.0):
    """Nystrom with a general sketch S (n x m): P = K S C^{-1} S^T K + lambda I,
    C = S^T K S + jitter * diag(S^T K S) (a relative jitter, so rescaling a
    sketch column changes nothing).  With S = columns of the identity at the
    inducing indices (and the jitter scaled by sigma^2) this is the
    Section 3.1 preconditioner; inverted by the same matrix inversion lemma,
    P^{-1} v = lambda^{-1} [ v - A (lambda C + A^T A)^{-1} A^T v ],  A = K S."""
    X = np.asarray(X, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    K = rbf_block(X, X, sigma2, lengthscales)
    A = K @ S
    C = S.T @ A
    C = 0.5 * (C + C.T)
    C = C + jitter * np.diag(np.diag(C))
    core = lam * C + A.T @ A

    def apply(R):
        return (R - A @ np.linalg.solve(core, A.T @ R)) / lam

    def dense():
        return A @ np.linalg.solve(C, A.T) + lam * np.eye(X.shape[0])

    return Preconditioner(apply, dense, {"C": C, "A": A})


def spectral_features(X, sigma2, lengthscales, W):
    """Phi (n x 2m): columns cos(omega_r^T x) then sin(omega_r^T x) for each r,
    times sqrt(sigma2 / m), omega_r = W_r / l (= 2 pi s_r)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    m = W.shape[0]
    omega = W / np.asarray(lengthscales, dtype=np.float64)[None, :]
    A = X @ omega.T                               # (n, m): omega_r^T x_i
    scale = np.sqrt(sigma2 / m)
    return np.concatenate([np.cos(A), np.sin(A)], axis=1) * scale


def spectral(X, sigma2, lengthscales, lam, W):
    return lowrank(spectral_features(X, sigma2, lengthscales, W), lam)


def lowrank(Phi, lam):
    Phi = np.asarray(Phi, dtype=np.float64)
    core = lam * np.eye(Phi.shape[1]) + Phi.T @ Phi

    def apply(R):
        return (R - Phi @ np.linalg.solve(core, Phi.T @ R)) / lam

    def dense():
        return Phi @ Phi.T + lam * np.eye(Phi.shape[0])

    return Preconditioner(apply, dense, {"Phi": Phi})


def rsvd_factor(X, sigma2, lengthscales, Omega, r, q=0):
    """Phi (n x r) of the randomised truncated SVD of K (Section 3.2):
    range of K^(q+1) Omega, Rayleigh-Ritz on it, the r largest eigenpairs."""
    X = np.asarray(X, dtype=np.float64)
    K = rbf_block(X, X, sigma2, lengthscales)
    Y = K @ np.asarray(Omega, dtype=np.float64)
    for _ in range(q):
        Q, _ = np.linalg.qr(Y)
        Y = K @ Q
    Q, _ = np.linalg.qr(Y)
    B = Q.T @ K @ Q
    w, V = np.linalg.eigh(0.5 * (B + B.T))
    order = np.argsort(w)[::-1][:r]
    return Q @ (V[:, order] * np.sqrt(np.maximum(w[order], 0.0)))


def rsvd(X, sigma2, lengthscales, lam, Omega, r, q=0):
    return lowrank(rsvd_factor(X, sigma2, lengthscales, Omega, r, q), lam)
