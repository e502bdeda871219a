"""ARD-RBF kernel blocks and the (K + lambda I) V product, FP64, direct differences.

Follows Eq. (1): k(x_i, x_j) = sigma^2 exp(-1/2 sum_r (x_ir - x_jr)^2 / l_r^2),
and K_y = K + lambda I (Section 2.1).  Distances are formed from direct
coordinate differences (never the |a|^2 + |b|^2 - 2 a.b expansion), so the
only rounding is that of float64 arithmetic.

Pinned by (tests/test_oracle_kernel.py): K_ii = sigma^2; symmetry; positive
semi-definiteness; the hand example k(0, 1 | l=1, sigma^2=1) = e^{-1/2};
the two limits l -> infinity (K -> sigma^2 11^T) and l -> 0 (K -> sigma^2 I);
a pure-Python triple loop on tiny inputs; the golden fixture
tests/golden/rbf_hand.txt.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def rbf_block(Xa: np.ndarray, Xb: np.ndarray, sigma2: float,
              lengthscales: np.ndarray) -> np.ndarray:
    """Gram block K[a, b] of Eq. (1) for row sets Xa (p, d) and Xb (q, d)."""
    Xa = np.asarray(Xa, dtype=np.float64)
    Xb = np.asarray(Xb, dtype=np.float64)
    ls = np.asarray(lengthscales, dtype=np.float64)
    sq = np.zeros((Xa.shape[0], Xb.shape[0]))
    for r in range(Xa.shape[1]):
        diff = (Xa[:, r][:, None] - Xb[:, r][None, :]) / ls[r]
        sq += diff * diff
    return sigma2 * np.exp(-0.5 * sq)


def kernel_matrix(X, sigma2, lengthscales):
    """Dense K (n, n).  Only for small n."""
    return rbf_block(X, X, sigma2, lengthscales)


def _threads():
    return max(1, int(os.environ.get("PKM_ORACLE_THREADS", os.cpu_count() or 1)))


def kernel_mvm(X, sigma2, lengthscales, lam, V, rows=None, block=256,
               threads=None):
    """(K + lambda I) V for V (n, k), without storing K.

    ``rows`` restricts the output to a subset of row indices (the product's
    rows are independent), which lets a caller sample a large product.
    Row blocks of K are regenerated from X and multiplied into V; blocks run
    on a thread pool (NumPy releases the GIL inside its kernels).
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None]
    rows = np.arange(X.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((rows.shape[0], V.shape[1]))

    def work(s):
        r = rows[s:s + block]
        Kb = rbf_block(X[r], X, sigma2, lengthscales)
        out[s:s + block] = Kb @ V + lam * V[r]

    starts = range(0, rows.shape[0], block)
    nthr = threads or _threads()
    if nthr == 1 or rows.shape[0] <= block:
        for s in starts:
            work(s)
    else:
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, starts))
    return out[:, 0] if squeeze else out
