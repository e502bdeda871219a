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

  * ``int8 digits``: an FP64-class product on integer matrix cores.  K / sigma2
    in (0, 1] is carried as the fixed-point integer kint = rint(2^30 K / sigma2)
    (absolute error <= 2^-31), each V column as vint = rint(2^e V) with the
    power of two e that puts its largest magnitude in [2^29, 2^30); both
    integers are written in signed base-256 digits (four digits in
    [-128, 127] each), digit products are summed exactly (integers), and only
    the digit pairs whose weight 256^(p + q) has p + q >= 3 are kept.  There is
    no structured (row- or column-wise) error: the exponent and exp2 are FP64
    and every rounding is of a single entry, at 2^-30 of its scale.

Functions:
  round_fp32, round_bf16,         elementwise rounding (RNE)
  round_fp16
  perturbed_kernel(...)           K + E for one of the rounding models
  rho(Khat, K, lam)               ||Khat - K||_2 / lam
  refine(Khat, K, lam, b, ...)    FP64-residual refinement on A_hat, history
  fp32_solution_residual(...)     true residual of the exact solution rounded
                                  to FP32 (why x must stay FP64)
  signed_digits(x, ndig)          base-256 digits in [-128, 127] of integers
  int8_digit_product(...)         (K + shift I) V under the int8-digit model
  int8_truncation_bound(...)      largest per-term error of the dropped pairs
  refinement_factor(apply, ...)   |E(d)| / |r| for d = A^-1 r: the contraction
                                  one refinement step achieves on residual r
  woodbury_psi(D, Phi)            Psi of P^-1 = D^-1 - Psi Psi^T, P = D + Phi Phi^T
  woodbury_apply(D, Psi, R, ...)  D^-1 R - Psi~ (Psi~^T R), Psi~ = Psi or its
                                  FP32 rounding (the stored-FP32 apply)
  psi_rounding_bound(Psi, R)      entrywise bound on what the rounding changes

  * ``stored-FP32 Psi``: the Woodbury apply (Section 3.2's matrix inversion
    lemma written as P^-1 = D^-1 - Psi Psi^T) with Psi rounded once to FP32
    and everything else FP64.  Since Psi~ = Psi (1 + delta), |delta| <= u =
    2^-24 entrywise, (Psi~ Psi~^T - Psi Psi^T)_ij = sum_a Psi_ia Psi_ja
    (delta_ia + delta_ja + delta_ia delta_ja): the operator stays symmetric,
    and it moves by at most (2u + u^2) |Psi| |Psi|^T entrywise.  It is a
    different preconditioner, not a product error: PCG stays exact in FP64
    around it, only its step count can change.
"""
from __future__ import annotations

import math

import numpy as np

from .kernel import kernel_matrix
from .mlp import round_bf16

__all__ = ["round_fp32", "round_bf16", "round_fp16", "split_fp16", "perturbed_kernel",
           "rho", "refine",
           "fp32_solution_residual", "augmented_fp32_kernel", "signed_digits",
           "int8_digit_product", "int8_truncation_bound", "refinement_factor",
           "woodbury_psi", "woodbury_apply", "psi_rounding_bound"]


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


def signed_digits(x, ndig=4):
    """Digits s_0 .. s_{ndig-1} in [-128, 127] with x = sum_p s_p 256^p, for
    integer-valued x (array, |x| well below 2^(8 ndig - 1)).  Textbook
    signed-digit recursion: s = ((x + 128) mod 256) - 128, x <- (x - s) / 256.
    Returns an array of shape (ndig,) + x.shape (float64, exact integers)."""
    x = np.asarray(x, dtype=np.float64).copy()
    out = np.empty((ndig,) + x.shape)
    for p in range(ndig):
        s = np.mod(x + 128.0, 256.0) - 128.0
        out[p] = s
        x = (x - s) / 256.0
    if np.any(x != 0):
        raise ValueError("value needs more digits")
    return out


def _column_exponents(V):
    """Power of two e_c per column with max |V_c| 2^e_c in [2^29, 2^30);
    0 for an all-zero column."""
    m = np.max(np.abs(V), axis=0)
    e = np.zeros(V.shape[1], dtype=np.int64)
    nz = m > 0
    e[nz] = 29 - np.floor(np.log2(m[nz])).astype(np.int64)
    # log2 of a value just below a power of two can round up: fix the bracket
    scaled = np.ldexp(m, e)
    e[nz & (scaled >= 2.0 ** 30)] -= 1
    e[nz & (np.ldexp(m, e) < 2.0 ** 29)] += 1
    return e


def int8_digit_product(X, sigma2, lengthscales, V, shift=0.0, min_class=3, K=None):
    """(K + shift I) V under the int8-digit model (see the module header).

    kint = rint(2^30 K / sigma2) and vint = rint(2^e_c V) in four signed
    base-256 digits each; G_c = sum over digit pairs with p + q = c of the
    exact integer products ks_p @ vs_q; the result is
        sigma2 2^(-30 - e_c) sum_{c >= min_class} 256^c G_c  +  shift V
    (min_class = 0 keeps every pair: then the K V part is exactly
    sigma2 kint vint 2^(-30 - e) up to the final FP64 rounding)."""
    V = np.asarray(V, dtype=np.float64)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None]
    if K is None:
        K = kernel_matrix(X, sigma2, lengthscales)
    kint = np.rint(np.ldexp(K / sigma2, 30))
    e = _column_exponents(V)
    vint = np.rint(np.ldexp(V, e[None, :]))
    ks = signed_digits(kint)
    vs = signed_digits(vint)
    n, k = V.shape
    acc = np.zeros((n, k))
    for c in range(6, min_class - 1, -1):   # largest weight first
        G = np.zeros((n, k))
        for p in range(4):
            q = c - p
            if 0 <= q < 4:
                G += ks[p] @ vs[q]          # integers below 2^53: exact
        acc += G * 256.0 ** c
    Y = sigma2 * np.ldexp(acc, -30 - e[None, :]) + shift * V
    return Y[:, 0] if squeeze else Y


def int8_truncation_bound(min_class=3):
    """Largest |sum over dropped digit pairs| per (i, j) term, in units of
    2^(-30 - e) sigma2: pairs with p + q < min_class, every digit magnitude at
    most 128.  Relative to a column's largest scaled value (2^30) this is
    about 2^-28.4 for min_class = 3."""
    tot = 0.0
    for c in range(min_class):
        npairs = sum(1 for p in range(4) if 0 <= c - p < 4)
        tot += npairs * 128.0 * 128.0 * 256.0 ** c
    return tot


def refinement_factor(apply, K, lam, R):
    """Per column |E(d)| / |r| with d = A^-1 r, A = K + lam I and
    E(d) = apply(d) - A d: one step of FP64-residual refinement around the
    approximate product turns residual r into about E(A_hat^-1 r) ~ E(d), so
    this is the contraction it achieves on r (below 1: refinement converges;
    above 1: it cannot)."""
    A = K + lam * np.eye(K.shape[0])
    D = np.linalg.solve(A, R)
    E = apply(D) - A @ D
    return np.linalg.norm(E, axis=0) / np.linalg.norm(R, axis=0)


def woodbury_psi(D, Phi):
    """Psi with P^-1 = D^-1 - Psi Psi^T for P = diag(D) + Phi Phi^T (the
    matrix inversion lemma, Section 3.2): C = I + Phi^T D^-1 Phi = L L^T
    (Cholesky), Psi = D^-1 Phi L^-T."""
    D = np.asarray(D, dtype=np.float64)
    Phi = np.asarray(Phi, dtype=np.float64)
    DPhi = Phi / D[:, None]
    C = np.eye(Phi.shape[1]) + Phi.T @ DPhi
    L = np.linalg.cholesky(C)
    return np.linalg.solve(L, DPhi.T).T          # D^-1 Phi L^-T


def woodbury_apply(D, Psi, R, round_psi=False):
    """D^-1 R - Psi~ (Psi~^T R), Psi~ = round_fp32(Psi) when round_psi (the
    apply from Psi stored in FP32), else Psi; FP64 arithmetic throughout."""
    D = np.asarray(D, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    P = round_fp32(Psi) if round_psi else np.asarray(Psi, dtype=np.float64)
    return R / D[:, None] - P @ (P.T @ R)


def psi_rounding_bound(Psi, R):
    """Entrywise bound on |apply(Psi~) - apply(Psi)| for R, from
    |Psi~ Psi~^T - Psi Psi^T| <= (2u + u^2) |Psi| |Psi|^T, u = 2^-24 (exact
    arithmetic; the FP64 sums add ~1e-16 relative on top)."""
    u = 2.0 ** -24
    A = np.abs(np.asarray(Psi, dtype=np.float64))
    return (2 * u + u * u) * (A @ (A.T @ np.abs(np.asarray(R, dtype=np.float64))))
