"""Seeded synthetic inputs for kernel-matrix PCG workloads.

This module only draws random inputs (points, lengthscales, targets, probe
vectors, inducing-point indices).  It holds none of the method's arithmetic:
no kernel evaluation, no solve, no preconditioner.  Both the FP64 oracle and
the HIP path receive the very same arrays from here.

Workloads (all regression with a Gaussian likelihood, ARD-RBF kernel of
Eq. (1), noise variance lambda, Section 2):

  small_fp64   n=2048,   d=8,  X ~ U[0,1], l_r = 0.5, lambda = 1e-2, k = 1,
               Nystrom m = 64, tol 1e-8 (FP64 end to end)
  block_fp32   n=65536,  d=8,  X ~ U[0,1], l_r ~ LogU[0.1, 1], lambda = 1e-3,
               k = 1 + 16 Rademacher probes, Nystrom / FITC m = 512
  mixed        n=262144, d=16, X ~ N(0, I), l_r ~ LogU[2, 8], lambda = 1e-4,
               k = 1 + 32, Nystrom m = 1024
  batched      64 problems, n ~ LogU[1000, 32000], d in {4,8,16,32},
               l_r ~ LogU[0.2 sqrt(d), sqrt(d)], lambda ~ LogU[1e-4, 1e-2],
               k = 1 + 8, Nystrom m = min(n, 64 ceil(4 sqrt(n) / 64))
  learned      n=131072, d=8,  X ~ U[0,1], l_r = 0.5, lambda = 1e-4,
               64 training probes, k = 1 + 16 for solves

Targets follow y = sum_k sin(3 x_k) + 0.1 eps with eps ~ N(0, 1).  Probe
vectors are Rademacher (+-1 with probability 1/2), as the stochastic trace
estimate of Section 2.1 requires.  Inducing points are drawn uniformly
without replacement (Section 5 draws them at random from the inputs).

Every workload takes an optional ``n`` override so that parity tests can run
the same recipe at sizes a CPU oracle finishes in seconds.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Problem", "make", "WORKLOADS", "rademacher", "inducing_indices",
           "batched_problems", "mlp_params", "classification"]


@dataclasses.dataclass
class Problem:
    """One GP regression problem: inputs, hyperparameters, right-hand sides."""
    name: str
    X: np.ndarray            # (n, d) float64, row-major
    lengthscales: np.ndarray  # (d,) float64
    sigma2: float
    lam: float
    y: np.ndarray            # (n,) float64 targets
    Z: np.ndarray            # (n, N) float64 Rademacher probes (may be N = 0)
    idx: np.ndarray          # (m,) int32 inducing-point indices (may be m = 0)
    tol: float

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def B(self) -> np.ndarray:
        """Right-hand-side block [y, Z] as an (n, 1 + N) row-major array."""
        return np.ascontiguousarray(np.concatenate([self.y[:, None], self.Z], axis=1))


def rademacher(rng: np.random.Generator, n: int, N: int) -> np.ndarray:
    """(n, N) matrix of independent +-1 entries with probability 1/2 each."""
    if N == 0:
        return np.zeros((n, 0))
    return rng.integers(0, 2, size=(n, N)).astype(np.float64) * 2.0 - 1.0


def inducing_indices(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    """m distinct indices drawn uniformly from range(n)."""
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)


def _targets(rng: np.random.Generator, X: np.ndarray) -> np.ndarray:
    return np.sin(3.0 * X).sum(axis=1) + 0.1 * rng.standard_normal(X.shape[0])


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def make(name: str, seed: int = 0, n: int | None = None, m: int | None = None,
         n_probes: int | None = None) -> Problem:
    """Draw workload ``name`` with ``seed``; ``n``, ``m``, ``n_probes`` override sizes."""
    rng = np.random.default_rng(seed)
    if name == "small_fp64":
        n = 2048 if n is None else n
        d = 8
        X = rng.random((n, d))
        ls = np.full(d, 0.5)
        sigma2, lam, tol = 1.0, 1e-2, 1e-8
        N = 0 if n_probes is None else n_probes
        m = 64 if m is None else m
    elif name == "block_fp32":
        n = 65536 if n is None else n
        d = 8
        X = rng.random((n, d))
        ls = _loguniform(rng, 0.1, 1.0, size=d)
        sigma2, lam, tol = 1.0, 1e-3, 1e-6
        N = 16 if n_probes is None else n_probes
        m = 512 if m is None else m
    elif name == "mixed":
        n = 262144 if n is None else n
        d = 16
        X = rng.standard_normal((n, d))
        ls = _loguniform(rng, 2.0, 8.0, size=d)
        sigma2, lam, tol = 1.0, 1e-4, 1e-6
        N = 32 if n_probes is None else n_probes
        m = 1024 if m is None else m
    elif name == "learned":
        n = 131072 if n is None else n
        d = 8
        X = rng.random((n, d))
        ls = np.full(d, 0.5)
        sigma2, lam, tol = 1.0, 1e-4, 1e-6
        N = 16 if n_probes is None else n_probes
        m = 512 if m is None else m
    else:
        raise KeyError(f"unknown workload {name!r}")
    y = _targets(rng, X)
    Z = rademacher(rng, n, N)
    m = min(m, n)
    idx = inducing_indices(rng, n, m) if m > 0 else np.zeros(0, np.int32)
    return Problem(name, np.ascontiguousarray(X), ls, sigma2, lam, y, Z, idx, tol)


def batched_problems(seed: int = 0, count: int = 64, n_lo: int = 1000,
                     n_hi: int = 32000, n_probes: int = 8,
                     dims=(4, 8, 16, 32)) -> list[Problem]:
    """Many independent GP problems of uneven size, dimension and hyperparameters."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(round(_loguniform(rng, n_lo, n_hi)))
        d = int(rng.choice(dims))
        X = rng.random((n, d))
        ls = _loguniform(rng, 0.2 * math.sqrt(d), math.sqrt(d), size=d)
        lam = float(_loguniform(rng, 1e-4, 1e-2))
        y = _targets(rng, X)
        Z = rademacher(rng, n, n_probes)
        m = min(n, 64 * math.ceil(4.0 * math.sqrt(n) / 64.0))
        idx = inducing_indices(rng, n, m)
        out.append(Problem(f"batched[{b}]", np.ascontiguousarray(X), ls, 1.0, lam,
                           y, Z, idx, 1e-6))
    return out


def mlp_params(seed: int = 0, d_in: int = 8, hidden: int = 128, rank: int = 128,
               out_scale: float = 1.0) -> dict:
    """Initial weights of the factor network: W ~ N(0, 1/fan_in) (the output
    layer additionally times ``out_scale``), zero biases."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((d_in, hidden)) / math.sqrt(d_in),
        "b1": np.zeros(hidden),
        "W2": rng.standard_normal((hidden, hidden)) / math.sqrt(hidden),
        "b2": np.zeros(hidden),
        "W3": rng.standard_normal((hidden, rank)) / math.sqrt(hidden) * out_scale,
        "b3": np.zeros(rank),
    }


def classification(seed: int = 0, n: int = 4096, d: int = 14, m: int | None = None):
    """Binary labels for GP classification: X ~ U[0,1]^d, latent
    g = sum_k sin(3 x_k) + 0.3 eps, y = +1 where g is above its median, -1
    below (balanced classes); lengthscales LogU[0.5 sqrt(d), sqrt(d)],
    sigma2 = 1; m = sqrt(n) inducing indices (rounded to 16).  Returns
    (X, y, lengthscales, sigma2, idx)."""
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    g = np.sin(3.0 * X).sum(axis=1) + 0.3 * rng.standard_normal(n)
    y = np.where(g > np.median(g), 1.0, -1.0)
    ls = _loguniform(rng, 0.5 * math.sqrt(d), math.sqrt(d), size=d)
    m = m if m is not None else max(16, 16 * round(math.sqrt(n) / 16))
    idx = inducing_indices(rng, n, min(m, n))
    return np.ascontiguousarray(X), y, ls, 1.0, idx


WORKLOADS = ("small_fp64", "block_fp32", "mixed", "learned")
