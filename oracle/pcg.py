"""Preconditioned conjugate gradients, Algorithm 1, FP64.

Algorithm 1 is adapted from Golub & Van Loan's textbook PCG; its printed
listing has four slips (alpha's denominator, the sign of the residual update,
beta's numerator and denominator, the direction update).  This oracle takes
the textbook reading that the algorithm's citation fixes:

    r_0 = v - K_y x_0,  z_0 = P^{-1} r_0,  p_0 = z_0
    for i = 0, 1, ...:
        alpha_i   = r_i^T z_i / p_i^T K_y p_i
        x_{i+1}   = x_i + alpha_i p_i
        r_{i+1}   = r_i - alpha_i K_y p_i
        stop if |r_{i+1}|_2 <= tol |v|_2        (relative reading of the
                                                 paper's |r| < epsilon)
        z_{i+1}   = P^{-1} r_{i+1}
        beta_i    = r_{i+1}^T z_{i+1} / r_i^T z_i
        p_{i+1}   = z_{i+1} + beta_i p_i

A block of right-hand sides (targets plus probe vectors) runs as independent
recurrences per column that share one product K_y [p_1 ... p_k]; a column
that has met its stop test is frozen.  ``tol_abs`` gives the paper's absolute
test |r| < epsilon instead.

Pinned by (tests/test_oracle_pcg.py): with P = I it is textbook CG and
terminates in at most q steps on a diagonal matrix with q distinct
eigenvalues; with P = K_y it stops after one step; its solution matches the
Cholesky solve; the K_y-norm error decreases monotonically; a hand-worked
2x2 example (tests/golden/cg_2x2.txt).
"""
from __future__ import annotations

import numpy as np


class PCGResult:
    def __init__(self, x, iters, relres, history):
        self.x = x                # (n, k) solution
        self.iters = iters        # (k,) steps taken per column
        self.relres = relres      # (k,) final recursive relative residual
        self.history = history    # list of (k,) relative residuals per step


def pcg(matvec, B, precond=None, tol=1e-6, max_iter=100000, x0=None,
        tol_abs=None):
    """Solve K_y X = B column by column.

    matvec(P) must return K_y P for an (n, k) block; precond(R) returns
    P^{-1} R (identity when None).
    """
    B = np.asarray(B, dtype=np.float64)
    squeeze = B.ndim == 1
    if squeeze:
        B = B[:, None]
    n, k = B.shape
    Pinv = (lambda R: R.copy()) if precond is None else precond
    x = np.zeros((n, k)) if x0 is None else np.array(x0, dtype=np.float64).reshape(n, k)
    bnorm = np.linalg.norm(B, axis=0)
    thresh = tol * bnorm if tol_abs is None else np.full(k, float(tol_abs))

    r = B - matvec(x) if np.any(x) else B.copy()
    z = Pinv(r)
    p = z.copy()
    rz = np.sum(r * z, axis=0)
    iters = np.zeros(k, dtype=np.int64)
    active = np.linalg.norm(r, axis=0) > thresh
    history = []
    for _ in range(max_iter):
        if not active.any():
            break
        Ap = matvec(p)
        pAp = np.sum(p * Ap, axis=0)
        alpha = np.where(active, rz / np.where(active, pAp, 1.0), 0.0)
        x += alpha * p
        r -= alpha * Ap
        iters += active
        rnorm = np.linalg.norm(r, axis=0)
        history.append(rnorm / np.where(bnorm > 0, bnorm, 1.0))
        active &= rnorm > thresh
        if not active.any():
            break
        z = Pinv(r)
        rz_new = np.sum(r * z, axis=0)
        beta = np.where(active, rz_new / np.where(active, rz, 1.0), 0.0)
        p = z + beta * p
        rz = np.where(active, rz_new, rz)
    relres = np.linalg.norm(r, axis=0) / np.where(bnorm > 0, bnorm, 1.0)
    if squeeze:
        return PCGResult(x[:, 0], iters[:1], relres[:1], history)
    return PCGResult(x, iters, relres, history)
