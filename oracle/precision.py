"""Precision emulator: what reduced-precision kernel products do to the
solve, in FP64 arithmetic on the CPU.  Test infrastructure only (like the
rest of ``oracle/``); nothing in the library calls it.

Not in the paper.  The paper's products are exact (stored K, FP64 BLAS).  A
product computed with reduced precision applies a perturbed operator
    A_hat = (K + E) + lambda I,      A = K + lambda I,
and iterative refinement around it (x <- x + A_hat^-1 (b - A x), with the
residual b - A x in FP64) contracts the error by the spectral radius of
    I - A_hat^-1 A = A_hat^-1 E,
bounded by rho = ||E||_2 / lambda_min(A_hat) ~ ||E||_2 / lambda.  Once
rho > 1, A_hat may even be indefinite (lambda_min(K + E) < -lambda) and no
refinement on A_hat reaches the true solution.

Rounding points emulated here (what the GPU products round):
  * ``entries``: every K_ij rounded (to FP32, or to BF16, or carried as a
    two-part BF16 split K_h + K_l, or as a two-part FP16 split of K_ij / sigma2
    -- IEEE binary16 with its subnormals -- times sigma2), exact sums;
  * ``augmented_fp32``: the FP32 kernel's own exponent, the augmented dot
    product a_i . b_j accumulated in FP32 over FP32 operands, then exp2 in
    FP32 -- its per-row norm roundings make E proportional to K row by row,
    so ||E|| grows with ||K|| (about n for smooth kernels) rather than with
    sqrt(n).

Functions:
  round_fp32, round_bf16,         elementwise rounding (RNE)
  round_fp16
  perturbed_kernel(...)           K + E for one of the rounding models
  rho(Khat, K, lam)               ||Khat - K||_2 / lam
  refine(Khat, K, lam, b, ...)    FP64-residual refinement on A_hat, history
  fp32_solution_residual(...)     true residual of the exact solution rounded
                                  to FP32 (why x must stay FP64)
"""
from __future__ import annotations

import math

import numpy as np

from .kernel import kernel_matrix
from .mlp import round_bf16

__all__ = ["round_fp32", "round_bf16", "round_fp16", "split_fp16", "perturbed_kernel",
           "rho", "refine",
           "fp32_solution_residual", "augmented_fp32_kernel"]


def round_fp32(a):
    """Round FP64 values to the nearest FP32 (ties to even), returned as FP64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_fp16(a):
    """Round FP64 values to the nearest IEEE binary16 (ties to even, gradual
    underflow below 2^-14, overflow to inf above 65504), returned as FP64."""
    with np.errstate(over="ignore"):
        return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def split_fp16(a):
    """Two-part FP16 split: h = fp16(a), l = fp16(a - h) (a - h is exact in
    FP64).  For |a| <= 1 the carried value h + l is within
    max(2^-23 |a|, 2^-25) of a."""
    a = np.asarray(a, dtype=np.float64)
    h = round_fp16(a)
    return h, round_fp16(a - h)


def augmented_fp32_kernel(X, sigma2, lengthscales):
    """K_ij = 2^(a_i . b_j) with the contraction done in FP32 the way an FP32
    MFMA accumulates it (operands rounded to FP32, running FP32 sum over the
    augmented slots in order), exp2 in FP32.

    xh = (x - mean) / l * sqrt(log2(e) / 2),
    a_i = [2 xh_i, log2 sigma2 - |xh_i|^2, 1],  b_j = [xh_j, 1, -|xh_j|^2],
    so a_i . b_j = log2 sigma2 - |xh_i - xh_j|^2 (Eq. (1) in base 2)."""
    X = np.asarray(X, dtype=np.float64)
    c = math.sqrt(0.5 * math.log2(math.e))
    xh = ((X - X.mean(axis=0)) / np.asarray(lengthscales, float) * c).astype(np.float32)
    nrm = (xh.astype(np.float64) ** 2).sum(axis=1)
    n = X.shape[0]
    a = np.concatenate([2.0 * xh, (math.log2(sigma2) - nrm)[:, None].astype(np.float32),
                        np.ones((n, 1), np.float32)], axis=1).astype(np.float32)
    b = np.concatenate([xh, np.ones((n, 1), np.float32),
                        (-nrm)[:, None].astype(np.float32)], axis=1).astype(np.float32)
    S = np.zeros((n, n), dtype=np.float32)
    for r in range(a.shape[1]):
        S = (S + np.outer(a[:, r], b[:, r]).astype(np.float32)).astype(np.float32)
    return np.exp2(S).astype(np.float64)


def perturbed_kernel(X, sigma2, lengthscales, model):
    """K + E under rounding ``model``: 'fp32', 'bf16', 'bf16x2', 'f16x2'
    (entries), or 'augmented_fp32' (the FP32 product's exponent arithmetic)."""
    if model == "augmented_fp32":
        return augmented_fp32_kernel(X, sigma2, lengthscales)
    K = kernel_matrix(X, sigma2, lengthscales)
    if model == "fp32":
        return round_fp32(K)
    if model == "bf16":
        return round_bf16(K)
    if model == "bf16x2":
        hi = round_bf16(K)
        return hi + round_bf16(K - hi)
    if model == "f16x2":
        hi, lo = split_fp16(K / sigma2)
        return sigma2 * (hi + lo)
    raise ValueError(f"unknown rounding model {model!r}")


def rho(Khat, K, lam):
    """||Khat - K||_2 / lambda (spectral norm of the symmetric part of E)."""
    E = np.asarray(Khat) - np.asarray(K)
    E = 0.5 * (E + E.T)
    return float(np.max(np.abs(np.linalg.eigvalsh(E))) / lam)


def refine(Khat, K, lam, b, steps=8):
    """Iterative refinement: x_{t+1} = x_t + A_hat^-1 (b - A x_t), x_0 = 0,
    with exact (dense) solves on A_hat and the residual in FP64.  Returns the
    list of true relative residuals |b - A x_t| / |b|, t = 1..steps."""
    n = K.shape[0]
    A = K + lam * np.eye(n)
    Ah = Khat + lam * np.eye(n)
    x = np.zeros_like(b, dtype=np.float64)
    hist = []
    bn = np.linalg.norm(b)
    for _ in range(steps):
        r = b - A @ x
        x = x + np.linalg.solve(Ah, r)
        hist.append(float(np.linalg.norm(b - A @ x) / bn))
    return hist


def fp32_solution_residual(K, lam, B):
    """Per column: true relative residual of the exact solution of
    (K + lambda I) x = b after rounding x to FP32."""
    A = K + lam * np.eye(K.shape[0])
    X = np.linalg.solve(A, B)
    R = B - A @ round_fp32(X)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
