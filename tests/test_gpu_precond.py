"""Parity of the HIP Nystrom / FITC / factor preconditioners against the oracle."""
import numpy as np
import pytest

from gpu_util import GpuProblem, ctx, dev, host, rel_err  # noqa: F401
from oracle import kernel as ok
from oracle import precond as op
from paper_1602_06693_amd import binding as pk
from pkm_inputs import make

pytestmark = pytest.mark.gpu

JIT = 1e-8
# FP64 setup on both sides, factorised differently (the oracle solves the
# lambda K_UU + K_UX K_XU core directly, the library goes through the Cholesky
# factor of K_UU + jitter I).  The two setups differ by about u cond(K_UU)
# relative (FITC's diag(K - Q) cancels to that absolute level), and P^-1
# amplifies a relative change of P by up to cond(P): bound 64 u cond(K_UU)
# cond(P), floored at 1e-11.
TOL = 1e-9


def _tol(P):
    c = np.linalg.cond(P.info["Kuu"]) * np.linalg.cond(P.dense())
    return max(1e-11, 64 * 2.2e-16 * c)


@pytest.mark.parametrize("kind,n,m", [(pk.PKM_PC_NYSTROM, 700, 64), (pk.PKM_PC_NYSTROM, 1000, 130),
                                      (pk.PKM_PC_FITC, 700, 64), (pk.PKM_PC_FITC, 333, 200),
                                      (pk.PKM_PC_NYSTROM, 50, 1)])
def test_apply_matches_oracle(ctx, kind, n, m):
    p = make("block_fp32", seed=21, n=n, m=m, n_probes=4)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, kind, m, idx=g.idx, jitter=JIT)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        make_o = op.nystrom if kind == pk.PKM_PC_NYSTROM else op.fitc
        P = make_o(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, jitter=JIT)
        want = P(p.B)
        assert np.all(rel_err(got, want) < _tol(P)), (rel_err(got, want), _tol(P))
        D = pk.pkm_precond_diag(ctx, pc, n)
        if kind == pk.PKM_PC_FITC:
            assert np.allclose(D, P.info["D"], rtol=1e-9, atol=1e-12)
            assert np.allclose(D[p.idx], p.lam, rtol=0, atol=1e-7)
        else:
            assert np.all(D == p.lam)
    finally:
        pk.pkm_precond_destroy(pc)


def test_lowrank_apply_matches_oracle(ctx):
    rng = np.random.default_rng(3)
    n, r, lam = 900, 70, 1e-3
    Phi = rng.standard_normal((n, r)) * 0.3
    p = make("block_fp32", seed=22, n=n, n_probes=5)
    g = GpuProblem(p)
    prob = pk.Problem(g.X, p.lengthscales, p.sigma2, lam)
    pc = pk.pkm_precond_setup(ctx, prob, pk.PKM_PC_LOWRANK, r, Phi=dev(Phi))
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        want = op.lowrank(Phi, lam)(p.B)
        assert np.all(rel_err(got, want) < TOL)
    finally:
        pk.pkm_precond_destroy(pc)


def test_zero_factor_is_lambda_identity(ctx):
    p = make("block_fp32", seed=23, n=200, n_probes=2)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_LOWRANK, 8, Phi=dev(np.zeros((200, 8))))
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        assert np.allclose(got, p.B / p.lam, rtol=1e-15, atol=0)
    finally:
        pk.pkm_precond_destroy(pc)


def test_duplicate_inducing_points_without_jitter_is_breakdown(ctx):
    p = make("block_fp32", seed=24, n=100, n_probes=0)
    g = GpuProblem(p)
    idx = dev(np.array([3, 3, 7], np.int32))
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 3, idx=idx, jitter=0.0)
    assert e.value.code == pk.PKM_ERR_BREAKDOWN


def test_out_of_range_index_is_invalid(ctx):
    p = make("block_fp32", seed=25, n=100, n_probes=0)
    g = GpuProblem(p)
    idx = dev(np.array([3, 100], np.int32))
    with pytest.raises(pk.PkmError) as e:
        pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 2, idx=idx, jitter=JIT)
    assert e.value.code == pk.PKM_ERR_INVALID


@pytest.mark.parametrize("n,m", [(700, 48), (333, 20)])
def test_sketch_apply_matches_oracle(ctx, n, m):
    rng = np.random.default_rng(n)
    p = make("block_fp32", seed=26, n=n, n_probes=3)
    S = rng.standard_normal((n, m))
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_SKETCH, m, Phi=dev(S), jitter=1e-10)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
    finally:
        pk.pkm_precond_destroy(pc)
    P = op.sketch(p.X, p.sigma2, p.lengthscales, p.lam, S, jitter=1e-10)
    want = P(p.B)
    # K S comes from the FP32 product (relative error <= 1e-5): the factor and
    # hence P^-1 inherit that level, amplified by at most cond(P)
    tol = 1e-5 * np.linalg.cond(P.dense()) ** 0.5
    assert np.all(rel_err(got, want) < tol), (rel_err(got, want), tol)


@pytest.mark.parametrize("n,m,block", [(700, 64, 32), (333, 40, 64), (200, 16, 1), (257, 30, 17)])
def test_pitc_apply_matches_oracle(ctx, n, m, block):
    """PITC (Section 3.1.1): block-diagonal correction over consecutive rows,
    ragged last block included."""
    p = make("block_fp32", seed=23, n=n, m=m, n_probes=4)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup_pitc(ctx, g.prob, m, g.idx, block, jitter=JIT)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
        P = op.pitc(p.X, p.sigma2, p.lengthscales, p.lam, p.idx, block, jitter=JIT)
        want = P(p.B)
        assert np.all(rel_err(got, want) < _tol(P)), (rel_err(got, want), _tol(P))
        D = pk.pkm_precond_diag(ctx, pc, n)
        Dw = np.concatenate([np.diag(Db) for Db in P.info["Dblocks"]])
        assert np.allclose(D, Dw, rtol=1e-9, atol=1e-12)
    finally:
        pk.pkm_precond_destroy(pc)


def test_pitc_solve_with_ordered_blocks(ctx):
    """Rows sorted along the first coordinate make the blocks local; PCG with
    PITC reaches the FP64 tolerance and takes no more steps than the
    oracle's PCG with the same preconditioner (+10 % + 2)."""
    from oracle import kernel as ok
    from oracle.pcg import pcg
    p = make("small_fp64", seed=24, n=1500, m=48, n_probes=2)
    order = np.argsort(p.X[:, 0], kind="stable")
    X = np.ascontiguousarray(p.X[order])
    B = np.ascontiguousarray(p.B[order])
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    idx = np.sort(inv[p.idx]).astype(np.int32)
    prob = pk.Problem(dev(X), p.lengthscales, p.sigma2, p.lam)
    pc = pk.pkm_precond_setup_pitc(ctx, prob, len(idx), dev(idx), 32, jitter=JIT)
    try:
        Xs, info = pk.pkm_solve(ctx, prob, dev(B), pc=pc,
                                opts=pk.make_opts(tol=1e-8, prec=pk.PKM_FP64),
                                allow_warning=False)
    finally:
        pk.pkm_precond_destroy(pc)
    r = B - ok.kernel_mvm(X, p.sigma2, p.lengthscales, p.lam, host(Xs))
    assert np.all(np.linalg.norm(r, axis=0) / np.linalg.norm(B, axis=0) <= 1e-8 * 1.001)
    P = op.pitc(X, p.sigma2, p.lengthscales, p.lam, idx, 32, jitter=JIT)
    res = pcg(lambda v: ok.kernel_mvm(X, p.sigma2, p.lengthscales, p.lam, v), B, precond=P,
              tol=1e-8)
    assert np.all(info.iters <= 1.1 * res.iters + 2), (info.iters, res.iters)


def test_pitc_rejected_by_batched_solve(ctx):
    p = make("block_fp32", seed=25, n=300, m=20, n_probes=1)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup_pitc(ctx, g.prob, 20, g.idx, 16, jitter=JIT)
    try:
        with pytest.raises(pk.PkmError) as e:
            pk.pkm_solve_batched(ctx, [g.prob], [g.B], pcs=[pc],
                                 opts=pk.make_opts(tol=1e-6, prec=pk.PKM_FP64))
        assert e.value.code == pk.PKM_ERR_UNSUPPORTED
    finally:
        pk.pkm_precond_destroy(pc)


def test_spectral_features_and_apply_match_oracle(ctx):
    """Spectral approximation (Section 3.2): the library's Phi Phi^T (read back
    through pkm_precond_sub_lowrank) equals the oracle's random-Fourier-feature
    kernel, with diagonal sigma^2, and the Woodbury apply matches."""
    p = make("block_fp32", seed=26, n=300, n_probes=3)
    g = GpuProblem(p)
    rng = np.random.default_rng(26)
    W = rng.standard_normal((40, p.d))
    pc = pk.pkm_precond_setup_spectral(ctx, g.prob, dev(W))
    try:
        Y = dev(np.zeros((p.n, p.n)))
        pk.pkm_precond_sub_lowrank(ctx, pc, dev(np.eye(p.n)), Y)
        Khat = -host(Y)
        got = host(pk.pkm_precond_apply(ctx, pc, g.B))
    finally:
        pk.pkm_precond_destroy(pc)
    Phi = op.spectral_features(p.X, p.sigma2, p.lengthscales, W)
    np.testing.assert_allclose(Khat, Phi @ Phi.T, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.diag(Khat), p.sigma2, rtol=1e-12)
    P = op.spectral(p.X, p.sigma2, p.lengthscales, p.lam, W)
    want = P(p.B)
    c = np.linalg.cond(P.dense())
    err = np.linalg.norm(got - want, axis=0) / np.linalg.norm(want, axis=0)
    assert np.all(err < max(1e-11, 64 * 2.2e-16 * c)), (err, c)


def test_spectral_preconditioner_cuts_cg_steps_for_smooth_kernels(ctx):
    """m = sqrt(n) frequencies (the paper's setting) on the 2048-point recipe
    with long lengthscales (l = 3, lambda = 1e-4), where 45 random features
    capture K's leading spectrum: fewer PCG steps than plain CG, both
    certified to 1e-8 (oracle PCG: 254 vs 361).  With l = 0.5 the same
    features overshoot K and PCG needs about 5x more steps than plain CG --
    the paper likewise finds the spectral preconditioner the weakest for short
    lengthscales."""
    p = make("small_fp64", seed=27, n_probes=2)
    X = dev(p.X)
    prob = pk.Problem(X, np.full(p.d, 3.0), 1.0, 1e-4)
    B = dev(p.B)
    W = np.random.default_rng(27).standard_normal((int(np.sqrt(p.n)), p.d))
    opts = pk.make_opts(tol=1e-8, prec=pk.PKM_FP64)
    pc = pk.pkm_precond_setup_spectral(ctx, prob, dev(W))
    try:
        _, with_pc = pk.pkm_solve(ctx, prob, B, pc=pc, opts=opts, allow_warning=False)
    finally:
        pk.pkm_precond_destroy(pc)
    _, plain = pk.pkm_solve(ctx, prob, B, opts=opts, allow_warning=False)
    assert np.all(with_pc.relres_true <= 1e-8) and np.all(plain.relres_true <= 1e-8)
    print("spectral m=45:", with_pc.iters, "plain CG:", plain.iters)
    assert with_pc.iters.max() < plain.iters.max()


# ---- Psi stored in FP32 (pkm_precond_psi_f32) --------------------------------

def _nystrom_phi(p, jitter=JIT):
    """Phi = K_XU L^-T, K_UU + jitter I = L L^T: the factor whose Psi the
    library forms (for the rounding bound, which needs |Psi| only)."""
    from oracle.kernel import rbf_block
    Xu = p.X[p.idx]
    L = np.linalg.cholesky(rbf_block(Xu, Xu, p.sigma2, p.lengthscales) + jitter * np.eye(len(p.idx)))
    return np.linalg.solve(L, rbf_block(p.X, Xu, p.sigma2, p.lengthscales).T).T


@pytest.mark.parametrize("kind,n,m,k", [(pk.PKM_PC_NYSTROM, 3000, 128, 17),   # m % 4 == 0
                                        (pk.PKM_PC_NYSTROM, 2000, 130, 33),   # m even only
                                        (pk.PKM_PC_FITC, 1500, 97, 1),        # m odd
                                        (pk.PKM_PC_FITC, 1031, 64, 4)])
def test_psi_f32_apply_within_rounding_bound(ctx, kind, n, m, k):
    """The apply from FP32-rounded Psi moves each entry by no more than the
    derived bound (2u + u^2) |Psi| (|Psi|^T |R|) (plus FP64-sum slack), moves
    it visibly, and switching back gives the FP64 apply bit for bit."""
    from oracle import precision as pr
    p = make("small_fp64", seed=24, n=n, m=m, n_probes=k - 1)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, kind, m, idx=g.idx, jitter=JIT)
    try:
        z64 = host(pk.pkm_precond_apply(ctx, pc, g.B))
        pk.pkm_precond_psi_f32(ctx, pc, True)
        z32 = host(pk.pkm_precond_apply(ctx, pc, g.B))
        pk.pkm_precond_psi_f32(ctx, pc, False)
        z64b = host(pk.pkm_precond_apply(ctx, pc, g.B))
        D = pk.pkm_precond_diag(ctx, pc, n)
    finally:
        pk.pkm_precond_destroy(pc)
    assert np.array_equal(z64, z64b)
    Psi = pr.woodbury_psi(D, _nystrom_phi(p))
    R = p.B
    bound = pr.psi_rounding_bound(Psi, R)
    slack = 1e-12 * (np.abs(R) / D[:, None] + np.abs(Psi) @ (np.abs(Psi).T @ np.abs(R)))
    dev_ = np.abs(z32 - z64)
    assert np.all(dev_ <= 1.001 * bound + slack), np.max(dev_ / (bound + slack))
    assert dev_.max() > 0


@pytest.mark.parametrize("lam", [1e-2, 1e-3])
def test_psi_f32_solve_is_certified(ctx, lam):
    """Solves with the FP32-stored Psi are exact PCG around a slightly
    different preconditioner: certified at 1e-6 either way; at lambda = 1e-2
    (small rounding perturbation) the step count stays within 10 % + 2 of the
    FP64 Psi's.  (At 1e-3 it rises, as the oracle's pin predicts.)"""
    import dataclasses
    p = dataclasses.replace(make("block_fp32", seed=25, n=12000, m=256, n_probes=8), lam=lam)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 256, idx=g.idx, jitter=JIT)
    opts = pk.make_opts(tol=1e-6, prec=pk.PKM_FP64)
    try:
        _, i64 = pk.pkm_solve(ctx, g.prob, g.B, pc=pc, opts=opts)
        pk.pkm_precond_psi_f32(ctx, pc, True)
        _, i32 = pk.pkm_solve(ctx, g.prob, g.B, pc=pc, opts=opts)
    finally:
        pk.pkm_precond_destroy(pc)
    print(f"lambda {lam:g}: PCG steps FP64 Psi {i64.total_iters}, FP32 Psi {i32.total_iters}")
    for info in (i64, i32):
        assert np.all(info.col_status == pk.PKM_COL_CONVERGED)
        assert np.all(info.relres_true <= 1e-6)
    if lam >= 1e-2:
        assert abs(i32.total_iters - i64.total_iters) <= 0.1 * i64.total_iters + 2


def test_psi_f32_rejects_bad_flag(ctx):
    p = make("small_fp64", seed=26, n=300, m=20, n_probes=1)
    g = GpuProblem(p)
    pc = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 20, idx=g.idx, jitter=JIT)
    try:
        rc = pk.load().pkm_precond_psi_f32(ctx, pc, 2)
        assert rc == pk.PKM_ERR_INVALID
    finally:
        pk.pkm_precond_destroy(pc)


# ---- randomised truncated SVD (Section 3.2) ---------------------------------

def _rsvd_case(seed, n, d, ls, l):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    Omega = rng.standard_normal((n, l))
    R = rng.standard_normal((n, 5))
    return X, np.full(d, ls), Omega, R


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rsvd_apply_matches_oracle_without_truncation(ctx, q):
    """r = l: P = Q Q^T K Q Q^T + lambda I depends only on span(K^(q+1) Omega),
    so the GPU (FP64 products, Cholesky QR) and the oracle (Householder QR)
    agree to within the span's sensitivity, ~u cond(Y) cond(P)."""
    X, ls, Omega, R = _rsvd_case(40 + q, 600, 3, 0.3, 40)
    lam, s2 = 1e-2, 1.1
    prob = pk.Problem(dev(X), ls, s2, lam)
    pc = pk.pkm_precond_setup_rsvd(ctx, prob, 40, dev(Omega), q=q, prec=pk.PKM_FP64)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, dev(R)))
    finally:
        pk.pkm_precond_destroy(pc)
    P = op.rsvd(X, s2, ls, lam, Omega, r=40, q=q)
    want = P(R)
    K = ok.kernel_matrix(X, s2, ls)
    Y = np.linalg.matrix_power(K, q + 1) @ Omega
    tol = max(1e-11, 64 * 2.2e-16 * np.linalg.cond(Y) * np.linalg.cond(P.dense()))
    assert np.all(rel_err(got, want) < tol), (rel_err(got, want), tol)


def test_rsvd_truncation_with_a_spectral_gap(ctx):
    """Eight tight clusters give eight dominant eigenvalues; r = 8 of l = 24
    keeps exactly them (a wide gap makes the truncated factor well defined):
    the GPU apply matches the oracle's."""
    rng = np.random.default_rng(50)
    centres = rng.random((8, 4))
    X = np.repeat(centres, 60, axis=0) + 0.01 * rng.standard_normal((480, 4))
    ls = np.full(4, 0.5)
    Omega = rng.standard_normal((480, 24))
    R = rng.standard_normal((480, 3))
    lam, s2 = 5e-2, 1.0
    prob = pk.Problem(dev(X), ls, s2, lam)
    pc = pk.pkm_precond_setup_rsvd(ctx, prob, 8, dev(Omega), q=1, prec=pk.PKM_FP64)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, dev(R)))
    finally:
        pk.pkm_precond_destroy(pc)
    want = op.rsvd(X, s2, ls, lam, Omega, r=8, q=1)(R)
    assert np.all(rel_err(got, want) < 1e-8), rel_err(got, want)


def test_rsvd_recovers_a_rank_deficient_kernel(ctx):
    """Twelve distinct points, each repeated nine times: rank(K) = 12 < l = 16
    (the sketch is rank-deficient, the Cholesky QR's later passes need their
    fallback shift), and r = 14 reproduces K, so PCG converges in a few
    steps."""
    rng = np.random.default_rng(51)
    X = np.repeat(rng.random((12, 3)), 9, axis=0)
    ls = np.full(3, 0.4)
    Omega = rng.standard_normal((108, 16))
    lam, s2 = 1e-2, 1.3
    prob = pk.Problem(dev(X), ls, s2, lam)
    B = rng.standard_normal((108, 2))
    pc = pk.pkm_precond_setup_rsvd(ctx, prob, 14, dev(Omega), q=0, prec=pk.PKM_FP64)
    try:
        Xs, info = pk.pkm_solve(ctx, prob, dev(B), pc=pc,
                                opts=pk.make_opts(tol=1e-10, prec=pk.PKM_FP64),
                                allow_warning=False)
    finally:
        pk.pkm_precond_destroy(pc)
    assert info.total_iters <= 4, info.total_iters
    K = ok.kernel_matrix(X, s2, ls) + lam * np.eye(108)
    assert np.allclose(host(Xs), np.linalg.solve(K, B), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("n", [1, 17, 300])
def test_rsvd_full_sketch_is_exact(ctx, n):
    """l = r = n (one point, a ragged 17, several MFMA tiles): Q spans the
    whole space, so P = Q (Q^T K Q) Q^T + lambda I is K + lambda I up to
    rounding; its apply is the dense solve and PCG stops after one or two
    steps."""
    rng = np.random.default_rng(60 + n)
    X = rng.random((n, 2))
    ls = np.array([0.5, 0.7])
    lam, s2 = 1e-2, 1.2
    Omega = rng.standard_normal((n, n))
    R = rng.standard_normal((n, 3))
    prob = pk.Problem(dev(X), ls, s2, lam)
    pc = pk.pkm_precond_setup_rsvd(ctx, prob, n, dev(Omega), q=0, prec=pk.PKM_FP64)
    try:
        got = host(pk.pkm_precond_apply(ctx, pc, dev(R)))
        Xs, info = pk.pkm_solve(ctx, prob, dev(R), pc=pc,
                                opts=pk.make_opts(tol=1e-9, prec=pk.PKM_FP64),
                                allow_warning=False)
    finally:
        pk.pkm_precond_destroy(pc)
    Ky = ok.kernel_matrix(X, s2, ls) + lam * np.eye(n)
    want = np.linalg.solve(Ky, R)
    assert np.all(rel_err(got, want) < 1e-8), rel_err(got, want)
    assert np.all(info.col_status == pk.PKM_COL_CONVERGED)
    assert info.total_iters <= 2 * 3, info.total_iters
    assert np.allclose(host(Xs), want, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("sketch_prec", ["fp32", "f16x3"])
def test_rsvd_solve_certifies_and_cuts_steps(ctx, sketch_prec):
    """Randomised SVD (r = 200 of l = 220, one power iteration, FP32 or FP16x3
    products for the sketch, two passes of 110 columns) preconditioning an 8000-point solve of the smooth
    learned-workload recipe (l = 0.5 on [0, 1]^8, lambda = 1e-3): certified
    at 1e-6 and far fewer PCG steps than no preconditioner.  (Like every
    low-rank preconditioner here it helps smooth kernels; on the rougher
    65,536-point recipe it costs steps, as the paper finds for short
    lengthscales.)"""
    import dataclasses
    p = dataclasses.replace(make("learned", seed=52, n=8000, m=200, n_probes=4), lam=1e-3)
    g = GpuProblem(p)
    Omega = dev(np.random.default_rng(53).standard_normal((p.n, 220)))
    opts = pk.make_opts(tol=1e-6, prec=pk.PKM_FP32)
    sp = {"fp32": pk.PKM_FP32, "f16x3": pk.PKM_F16X3}[sketch_prec]
    pc = pk.pkm_precond_setup_rsvd(ctx, g.prob, 200, Omega, q=1, prec=sp)
    try:
        _, info = pk.pkm_solve(ctx, g.prob, g.B, pc=pc, opts=opts)
    finally:
        pk.pkm_precond_destroy(pc)
    _, plain = pk.pkm_solve(ctx, g.prob, g.B, opts=opts)
    pcn = pk.pkm_precond_setup(ctx, g.prob, pk.PKM_PC_NYSTROM, 200, idx=g.idx, jitter=JIT)
    try:
        _, nys = pk.pkm_solve(ctx, g.prob, g.B, pc=pcn, opts=opts)
    finally:
        pk.pkm_precond_destroy(pcn)
    print(f"8000 points: randomised SVD r = 200 ({sketch_prec} sketch): {info.total_iters} PCG steps, "
          f"Nystrom m = 200: {nys.total_iters}, none: {plain.total_iters}")
    assert np.all(info.col_status == pk.PKM_COL_CONVERGED)
    assert np.all(info.relres_true <= 1e-6)
    assert info.total_iters < 0.75 * plain.total_iters


def test_rsvd_rejects_bad_arguments(ctx):
    X, ls, Omega, _ = _rsvd_case(54, 100, 2, 0.3, 10)
    prob = pk.Problem(dev(X), ls, 1.0, 1e-2)
    Om = dev(Omega)
    lib = pk.load()
    out = pk.C.c_void_p()
    for r, l, q in ((11, 10, 0), (0, 10, 0), (5, 10, 9), (5, 101, 0)):
        rc = lib.pkm_precond_setup_rsvd(ctx, prob.ref, r, l, pk._ptr(Om), q, pk.PKM_FP64,
                                        pk.C.byref(out))
        assert rc == pk.PKM_ERR_INVALID, (r, l, q)
    rc = lib.pkm_precond_setup_rsvd(ctx, prob.ref, 5, 10, None, 0, pk.PKM_FP64, pk.C.byref(out))
    assert rc == pk.PKM_ERR_INVALID
